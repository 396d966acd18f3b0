"""GPU parity: the HIP sweep, initial grains and grain statistics against the
CPU oracle, element by element (bit-exact: every quantity here is integer).

Sizes span several tiles plus ragged edges; the full-size cases use the
launch configuration the benchmark times (default tiling).
"""
import os

import numpy as np
import pytest

import oracle
import paper_1007_3509_amd as hmc
import synth

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))


def say(*a):
    print(*a, flush=True)


def gpu_run(dims, nbr, Q, B, kT, n_mcs, seed, *, spin=hmc.HMC_I16, init=None, vseed=None,
            proposal=hmc.HMC_PROP_NEIGHBOUR, tiling=None, chunks=None):
    say(f"[gpu] dims={dims} nbr={nbr} Q={Q} kT={kT} mcs={n_mcs} seed={seed} spin={spin} prop={proposal} "
        f"tiling={tiling} chunks={chunks}")
    with hmc.Lattice(dims, nbr, Q, voronoi_seed=vseed, spin=spin, proposal=proposal) as lat:
        if init is not None:
            lat.set_spins(init)
        lat.set_grain_energy(B)
        if tiling is not None:
            lat.set_tiling(*tiling)
        start = lat.spins().astype(np.int32)
        for n in (chunks or [n_mcs]):
            lat.sweep(kT, n, seed)
        assert lat.mcs == n_mcs
        return start, lat.spins().astype(np.int32)


def assert_same(got, want, label):
    bad = int(np.sum(got != want))
    assert bad == 0, f"{label}: {bad} of {want.size} sites differ"


# ------------------------------------------------------------ initial grains

@pytest.mark.parametrize("dims,G,seed,spin", [
    ((64, 64), 40, 1, hmc.HMC_I32), ((36, 20), 7, 9, hmc.HMC_I16), ((4, 4), 3, 2, hmc.HMC_I16),
    ((1024, 1024), 2000, 2, hmc.HMC_I16), ((12, 10, 8), 5, 4, hmc.HMC_I32),
    ((256, 256, 256), 20000, 3, hmc.HMC_I16), ((2048, 1024), 32000, 8, hmc.HMC_I32),
])
def test_voronoi_init_matches_oracle(dims, G, seed, spin):
    nbr = hmc.HMC_VN4 if len(dims) == 2 else hmc.HMC_VN6
    say(f"[gpu] voronoi dims={dims} G={G}")
    with hmc.Lattice(dims, nbr, G, voronoi_seed=seed, spin=spin) as lat:
        got = lat.spins().astype(np.int32)
    want = oracle.voronoi(dims, G, seed, threads=THREADS)
    assert_same(got, want, "voronoi")


# ------------------------------------------------------- small / ragged sweeps

def _energies(Q, seed, lo=-20000, hi=30000):
    return np.random.default_rng(seed).integers(lo, hi, size=Q).astype(np.int32)


SMALL = [
    # dims, nbr, Q, kT, mcs, spin, proposal
    ((100, 36), hmc.HMC_VN4, 30, 0.5, 37, hmc.HMC_I16, 0),
    ((100, 36), hmc.HMC_VN4, 30, 1.3, 11, hmc.HMC_I32, 1),
    ((4, 4), hmc.HMC_VN4, 2, 1.0, 25, hmc.HMC_I16, 1),
    ((100, 36), hmc.HMC_MOORE8, 30, 0.7, 23, hmc.HMC_I16, 0),
    ((50, 22), hmc.HMC_MOORE8, 9, 2.0, 9, hmc.HMC_I32, 1),
    ((20, 14, 12), hmc.HMC_VN6, 20, 0.6, 15, hmc.HMC_I16, 0),
    ((20, 14, 12), hmc.HMC_VN6, 5, 1.5, 6, hmc.HMC_I32, 1),
    ((12, 10, 8), hmc.HMC_MOORE26, 12, 0.8, 7, hmc.HMC_I16, 0),
    ((8, 6, 10), hmc.HMC_MOORE26, 4, 3.0, 3, hmc.HMC_I32, 1),
    # degenerate temperatures: almost every uphill trial rejected, almost every one accepted
    ((64, 48), hmc.HMC_VN4, 40, 1e-3, 9, hmc.HMC_I16, 0),
    ((64, 48), hmc.HMC_MOORE8, 40, 40.0, 9, hmc.HMC_I16, 0),
    ((16, 12, 8), hmc.HMC_VN6, 20, 1e-3, 6, hmc.HMC_I32, 0),
    ((64, 32, 32), hmc.HMC_VN6, 50, 40.0, 5, hmc.HMC_I16, 0),
    ((64, 32, 32), hmc.HMC_VN6, 50, 1e-3, 5, hmc.HMC_I16, 0),
]


@pytest.mark.parametrize("dims,nbr,Q,kT,mcs,spin,prop", SMALL)
def test_small_sweeps_match_oracle(dims, nbr, Q, kT, mcs, spin, prop):
    B = _energies(Q, Q + mcs)
    vseed = 100 + Q
    start, got = gpu_run(dims, nbr, Q, B, kT, mcs, seed=77 + Q, spin=spin, vseed=vseed, proposal=prop)
    want = oracle.sweep(start, nbr, dims, B, kT, mcs, 77 + Q, proposal=prop, threads=THREADS)
    assert not np.array_equal(want, start)
    assert_same(got, want, "small sweep")


def test_uniform_trials_from_random_spins_int16_max_q():
    dims, Q = (16, 12), 32767
    init = synth.random_spins(dims, Q, 4)
    B = _energies(Q, 5, -3000, 3000)
    start, got = gpu_run(dims, hmc.HMC_VN4, Q, B, 0.9, 5, 123, init=init, proposal=1)
    want = oracle.sweep(init, hmc.HMC_VN4, dims, B, 0.9, 5, 123, proposal=1)
    assert_same(got, want, "Q=32767 symmetric trials")


def test_single_grain_never_changes():
    start, got = gpu_run((8, 8), hmc.HMC_VN4, 1, [0], 5.0, 10, 3, vseed=1)
    assert np.all(start == 0) and np.all(got == 0)


# ------------------------------------------------------ determinism contract

@pytest.mark.parametrize("dims,nbr,tilings", [
    ((128, 96), hmc.HMC_VN4, [(64, 32, 0, 1), (32, 32, 0, 3), (128, 96, 0, 1), (16, 48, 0, 5), (2, 2, 0, 1),
                              (32, 32, 0, -1), (64, 32, 0, -3)]),
    ((38, 20), hmc.HMC_VN4, [(38, 20, 0, 1), (2, 10, 0, 1), (38, 4, 0, 2)]),   # Lx = 2 mod 4: 2-byte rows
    ((96, 64), hmc.HMC_MOORE8, [(32, 32, 0, 1), (96, 16, 0, 2), (8, 8, 0, 1), (32, 32, 0, -2), (32, 16, 0, -3)]),
    ((24, 20, 16), hmc.HMC_VN6, [(8, 10, 4, 1), (24, 20, 2, 1), (12, 4, 16, 2), (4, 4, 4, 3), (8, 10, 4, -1)]),
    ((16, 12, 8), hmc.HMC_MOORE26, [(4, 4, 4, 1), (8, 6, 8, 1), (16, 2, 2, 1), (4, 4, 4, -2), (8, 6, 8, -4),
                                    (16, 2, 2, -3)]),
])
def test_result_independent_of_tiling(dims, nbr, tilings):
    Q = 40
    B = _energies(Q, 3)
    results = []
    for t in tilings:
        start, got = gpu_run(dims, nbr, Q, B, 0.75, 9, 5, vseed=11, tiling=t)
        results.append(got)
    want = oracle.sweep(start, nbr, dims, B, 0.75, 9, 5, threads=THREADS)
    for t, r in zip(tilings, results):
        assert_same(r, want, f"tiling {t}")


def test_split_calls_equal_one_call():
    dims, Q = (64, 48), 25
    B = _energies(Q, 8)
    _, one = gpu_run(dims, hmc.HMC_VN4, Q, B, 0.6, 40, 9, vseed=5)
    _, split = gpu_run(dims, hmc.HMC_VN4, Q, B, 0.6, 40, 9, vseed=5, chunks=[13, 1, 0, 26])
    assert_same(split, one, "split calls")


def test_checkpoint_resume_and_mcs_counter():
    dims, Q = (64, 64), 30
    B = _energies(Q, 9)
    with hmc.Lattice(dims, hmc.HMC_VN4, Q, voronoi_seed=4) as lat:
        lat.set_grain_energy(B)
        s0 = lat.spins().astype(np.int32)
        lat.sweep(0.5, 10, 21)
        hmc.hmc_snapshot(lat.h)
        mid = lat.spins()
        lat.sweep(0.5, 15, 21)
        end = lat.spins().astype(np.int32)
        hmc.hmc_restore(lat.h)
        assert lat.mcs == 10 and np.array_equal(lat.spins(), mid)
        lat.sweep(0.5, 15, 21)
        assert_same(lat.spins().astype(np.int32), end, "restore + resume")
        # host round trip and an explicit MC counter
        lat.set_spins(mid)
        lat.mcs = 10
        lat.sweep(0.5, 15, 21)
        assert_same(lat.spins().astype(np.int32), end, "set_spins + set_mcs")
    want = oracle.sweep(s0, hmc.HMC_VN4, dims, B, 0.5, 25, 21)
    assert_same(end, want, "checkpointed run vs oracle")
    want_mid = oracle.sweep(s0, hmc.HMC_VN4, dims, B, 0.5, 10, 21)
    want_end = oracle.sweep(want_mid, hmc.HMC_VN4, dims, B, 0.5, 15, 21, mcs0=10)
    assert np.array_equal(want_end, want)


def test_device_side_errors():
    with hmc.Lattice((16, 16), hmc.HMC_VN4, 5, voronoi_seed=1) as lat:
        with pytest.raises(hmc.HmcError) as ei:
            lat.set_spins(np.full((16, 16), 5, np.int16))
        assert ei.value.status == hmc.HMC_E_INVAL
        with pytest.raises(hmc.HmcError):
            lat.set_grain_energy(np.zeros(4, np.int32))
        with pytest.raises(hmc.HmcError) as ei:
            lat.set_grain_energy(np.array([0, 2 ** 30, -2 ** 30, 0, 0], np.int32))
        assert ei.value.status == hmc.HMC_E_RANGE
        with pytest.raises(hmc.HmcError):
            lat.set_tiling(6, 16, 0, 1)        # 6 does not divide 16
        with pytest.raises(hmc.HmcError):
            lat.sweep(0.0, 1, 1)
        with pytest.raises(hmc.HmcError):
            lat.sweep(float("nan"), 1, 1)
        with pytest.raises(hmc.HmcError):
            lat.sweep(0.5, -1, 1)
        with pytest.raises(hmc.HmcError) as ei:
            hmc.hmc_restore(lat.h)
        assert ei.value.status == hmc.HMC_E_STATE
        with pytest.raises(hmc.HmcError):
            lat.texture_stats(np.full(5, 3, np.int32), 2)


# ------------------------------------------------------------ workload sizes

def test_voronoi_2d_64_full():
    w = synth.voronoi_2d_64()
    start, got = gpu_run(w.dims, w.nbr, w.n_grains, w.B, w.kT, w.n_mcs, w.sweep_seed, spin=w.spin,
                         vseed=w.voronoi_seed)
    want = oracle.sweep(start, w.nbr, w.dims, w.B, w.kT, w.n_mcs, w.sweep_seed, threads=THREADS)
    assert_same(got, want, w.name)


def test_schmid_2d_1024_full_1000_mcs():
    w = synth.schmid_2d_1024()
    start, got = gpu_run(w.dims, w.nbr, w.n_grains, w.B, w.kT, w.n_mcs, w.sweep_seed, spin=w.spin,
                         vseed=w.voronoi_seed)
    want = oracle.sweep(start, w.nbr, w.dims, w.B, w.kT, w.n_mcs, w.sweep_seed, threads=THREADS)
    assert_same(got, want, w.name)
    # grain statistics of the final state
    with hmc.Lattice(w.dims, w.nbr, w.n_grains, spin=w.spin) as lat:
        lat.set_spins(got)
        ng, mean, frac = lat.texture_stats(w.grain_bin, w.n_bins)
        areas = lat.grain_areas()
    a_o, ng_o, mean_o, frac_o = oracle.texture(want, w.n_grains, w.grain_bin, w.n_bins)
    assert np.array_equal(areas, a_o)
    assert ng == ng_o and mean == mean_o
    assert np.array_equal(frac, frac_o)


def test_schmid_3d_256_full_lattice_100_mcs():
    w = synth.schmid_3d_256()
    start, got = gpu_run(w.dims, w.nbr, w.n_grains, w.B, w.kT, 100, w.sweep_seed, spin=w.spin,
                         vseed=w.voronoi_seed)
    want = oracle.sweep(start, w.nbr, w.dims, w.B, w.kT, 100, w.sweep_seed, threads=THREADS)
    assert_same(got, want, w.name)
    a_o, ng_o, mean_o, frac_o = oracle.texture(want, w.n_grains, w.grain_bin, w.n_bins)
    with hmc.Lattice(w.dims, w.nbr, w.n_grains, spin=w.spin) as lat:
        lat.set_spins(got)
        ng, mean, frac = lat.texture_stats(w.grain_bin, w.n_bins)
    assert ng == ng_o and np.array_equal(frac, frac_o)


def test_moore8_member_full_1000_mcs():
    members = [m for m in synth.ensemble_moore8() if m.dims[0] <= 256]
    w = members[0]
    start, got = gpu_run(w.dims, w.nbr, w.n_grains, w.B, w.kT, w.n_mcs, w.sweep_seed, spin=w.spin,
                         vseed=w.voronoi_seed)
    want = oracle.sweep(start, w.nbr, w.dims, w.B, w.kT, w.n_mcs, w.sweep_seed, threads=THREADS)
    assert_same(got, want, w.name)


# ------------------------------------------------ grain-energy placement

@pytest.mark.parametrize("Q,spread", [(5000, 0.9), (50, 3.0), (7, 0.0)])
def test_grain_energy_placement(Q, spread):
    # spread < 1 (2^16 fixed-point units): energies staged in LDS as 16-bit
    # offsets; wider spreads are read from global memory; both exact
    rng = np.random.default_rng(Q)
    B = synth.quantise(rng.uniform(-spread / 2, spread / 2, size=Q))
    dims = (96, 64)
    start, got = gpu_run(dims, hmc.HMC_VN4, Q, B, 0.9, 12, 77, vseed=5)
    want = oracle.sweep(start, hmc.HMC_VN4, dims, B, 0.9, 12, 77, threads=THREADS)
    assert_same(got, want, f"Q={Q} spread={spread}")


@pytest.mark.parametrize("nbr,k", [(hmc.HMC_VN4, 6), (hmc.HMC_MOORE8, 3)])
def test_large_lattice_default_takes_128_tiles(nbr, k):
    """A 2048^2 int16 lattice splits into one 128x128 tile per CU of an
    MI355X, so the default takes them; the result equals the oracle's and a
    64x64 tiling's."""
    dims, Q, n_mcs = (2048, 2048), 3000, 13
    B = synth.quantise(0.2 * (0.27 + 0.23 * np.random.default_rng(21).random(Q)))
    say(f"[gpu] 2048^2 nbr={nbr} default tiling")
    with hmc.Lattice(dims, nbr, Q, voronoi_seed=21) as a, hmc.Lattice(dims, nbr, Q, voronoi_seed=21) as b:
        a.set_grain_energy(B)
        b.set_grain_energy(B)
        start = a.spins().astype(np.int32)
        assert tuple(hmc.hmc_get_tiling(a.h)) == (128, 128, 1, k)
        b.set_tiling(64, 64, 1, 2)
        a.sweep(0.5, n_mcs, 9)
        b.sweep(0.5, n_mcs, 9)
        got = a.spins()
        assert np.array_equal(got, b.spins())
        want = oracle.sweep(start, nbr, dims, B, 0.5, n_mcs, 9, threads=THREADS)
        assert np.array_equal(got.astype(np.int32), want)


@pytest.mark.parametrize("nbr,k", [(hmc.HMC_VN4, 4), (hmc.HMC_MOORE8, 3)])
def test_larger_lattice_default_takes_256x128_tiles(nbr, k):
    """A 4096^2 int16 lattice splits into two 256x128 tiles per CU of an
    MI355X, so the default takes them; the result equals the oracle's and a
    64x64 tiling's."""
    dims, Q, n_mcs = (4096, 4096), 8000, 5
    B = synth.quantise(0.2 * (0.27 + 0.23 * np.random.default_rng(23).random(Q)))
    say(f"[gpu] 4096^2 nbr={nbr} default tiling")
    with hmc.Lattice(dims, nbr, Q, voronoi_seed=23) as a, hmc.Lattice(dims, nbr, Q, voronoi_seed=23) as b:
        a.set_grain_energy(B)
        b.set_grain_energy(B)
        start = a.spins().astype(np.int32)
        assert tuple(hmc.hmc_get_tiling(a.h)) == (256, 128, 1, k)
        b.set_tiling(64, 64, 1, 2)
        a.sweep(0.5, n_mcs, 4)
        b.sweep(0.5, n_mcs, 4)
        got = a.spins()
        assert np.array_equal(got, b.spins())
        want = oracle.sweep(start, nbr, dims, B, 0.5, n_mcs, 4, threads=THREADS)
        assert np.array_equal(got.astype(np.int32), want)
