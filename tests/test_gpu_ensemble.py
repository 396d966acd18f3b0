"""GPU: the batched ensemble (one persistent kernel over a ragged tile table,
launch sequence replayed from a HIP graph) gives every member exactly what a
single-lattice sweep gives, and that matches the oracle; the autotuner picks
a valid tiling without changing results."""
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


def _members(specs, nbr=hmc.HMC_MOORE8, spin=hmc.HMC_I16):
    lats = []
    for dims, G, vseed in specs:
        lat = hmc.Lattice(dims, nbr, G, voronoi_seed=vseed, spin=spin)
        m = 0.27 + 0.23 * np.random.default_rng(vseed).random(G)
        lat.set_grain_energy(synth.quantise(0.2 * m))
        lats.append(lat)
    return lats


def test_ensemble_matches_singles_and_oracle():
    specs = [((128, 128), 50, 7), ((64, 192), 300, 8), ((256, 128), 900, 9), ((64, 64), 20, 10)]
    kT = np.array([0.3, 0.55, 1.0, 0.8], np.float32)
    seeds = np.array([4000, 4001, 4002, 2 ** 40 + 5], np.uint64)
    n_mcs = 37
    say("[gpu] ensemble of", len(specs))
    lats = _members(specs)
    starts = [l.spins().astype(np.int32) for l in lats]
    E = hmc.hmc_ensemble_create(lats)
    try:
        hmc.hmc_ensemble_sweep(E, kT, seeds, n_mcs)
        hmc.hmc_ensemble_synchronize(E)
        got = [l.spins().astype(np.int32) for l in lats]
        assert all(l.mcs == n_mcs for l in lats)
    finally:
        hmc.hmc_ensemble_free(E)
    for i, ((dims, G, vseed), lat) in enumerate(zip(specs, lats)):
        B = synth.quantise(0.2 * (0.27 + 0.23 * np.random.default_rng(vseed).random(G)))
        want = oracle.sweep(starts[i], hmc.HMC_MOORE8, dims, B, float(kT[i]), n_mcs, int(seeds[i]), threads=THREADS)
        assert np.array_equal(got[i], want), f"member {i}: {int(np.sum(got[i] != want))} sites differ"
        with hmc.Lattice(dims, hmc.HMC_MOORE8, G, spin=hmc.HMC_I16) as single:
            single.set_spins(starts[i])
            single.set_grain_energy(B)
            single.sweep(float(kT[i]), n_mcs, int(seeds[i]))
            assert np.array_equal(single.spins().astype(np.int32), got[i])
        lat.close()


def test_ensemble_graph_replay_and_split_calls():
    specs = [((64, 64), 30, 1), ((128, 64), 60, 2)]
    kT = np.array([0.6, 0.9], np.float32)
    seeds = np.array([11, 12], np.uint64)
    a = _members(specs)
    b = _members(specs)
    Ea, Eb = hmc.hmc_ensemble_create(a), hmc.hmc_ensemble_create(b)
    try:
        hmc.hmc_ensemble_set_tiling(Ea, 32, 32, 0, 3)
        for _ in range(3):                      # the same captured graph, replayed
            hmc.hmc_ensemble_sweep(Ea, kT, seeds, 10)
        hmc.hmc_ensemble_sweep(Eb, kT, seeds, 30)
        hmc.hmc_ensemble_synchronize(Ea)
        hmc.hmc_ensemble_synchronize(Eb)
        for x, y in zip(a, b):
            assert x.mcs == y.mcs == 30
            assert np.array_equal(x.spins(), y.spins())
        # members keep working on their own afterwards
        a[0].sweep(0.6, 5, 11)
        b[0].sweep(0.6, 5, 11)
        assert np.array_equal(a[0].spins(), b[0].spins())
    finally:
        hmc.hmc_ensemble_free(Ea)
        hmc.hmc_ensemble_free(Eb)
        for l in a + b:
            l.close()


def test_ensemble_profile_counts_launches_and_updates():
    """Events around each graph replay: the launch and site-update counts are
    exact, the time is positive and below the host's wall time, profiling
    changes nothing in the result, and a read resets the sums."""
    import time
    specs = [((64, 64), 30, 1), ((128, 64), 60, 2)]
    kT = np.array([0.6, 0.9], np.float32)
    seeds = np.array([11, 12], np.uint64)
    a = _members(specs)
    b = _members(specs)
    Ea, Eb = hmc.hmc_ensemble_create(a), hmc.hmc_ensemble_create(b)
    try:
        hmc.hmc_ensemble_set_tiling(Ea, 32, 32, 0, 3)
        hmc.hmc_ensemble_set_tiling(Eb, 32, 32, 0, 3)
        say("[gpu] ensemble profile")
        hmc.hmc_ensemble_profile(Ea, True)
        t0 = time.perf_counter()
        for _ in range(2):
            hmc.hmc_ensemble_sweep(Ea, kT, seeds, 10)
        hmc.hmc_ensemble_synchronize(Ea)
        wall_ms = (time.perf_counter() - t0) * 1e3
        ms, launches, su = hmc.hmc_ensemble_profile_read(Ea)
        assert launches == 2 * 4                       # ceil(10 / 3) per call
        assert su == 2 * 10 * (64 * 64 + 128 * 64)
        assert 0.0 < ms <= wall_ms
        assert hmc.hmc_ensemble_profile_read(Ea) == (0.0, 0, 0)
        hmc.hmc_ensemble_profile(Ea, False)
        hmc.hmc_ensemble_sweep(Ea, kT, seeds, 10)
        hmc.hmc_ensemble_synchronize(Ea)
        assert hmc.hmc_ensemble_profile_read(Ea) == (0.0, 0, 0)
        hmc.hmc_ensemble_sweep(Eb, kT, seeds, 30)
        hmc.hmc_ensemble_synchronize(Eb)
        for x, y in zip(a, b):
            assert np.array_equal(x.spins(), y.spins())
    finally:
        hmc.hmc_ensemble_free(Ea)
        hmc.hmc_ensemble_free(Eb)
        for l in a + b:
            l.close()


def test_ensemble_vn4_and_vn6_members():
    for nbr, specs in [(hmc.HMC_VN4, [((64, 96), 40, 3), ((128, 64), 70, 4)]),
                       (hmc.HMC_VN6, [((16, 16, 32), 40, 5), ((32, 16, 16), 70, 6)])]:
        say("[gpu] ensemble nbr", nbr)
        lats = _members(specs, nbr=nbr)
        starts = [l.spins().astype(np.int32) for l in lats]
        E = hmc.hmc_ensemble_create(lats)
        kT = np.array([0.5, 0.7], np.float32)
        seeds = np.array([21, 22], np.uint64)
        hmc.hmc_ensemble_sweep(E, kT, seeds, 9)
        hmc.hmc_ensemble_synchronize(E)
        for i, ((dims, G, vseed), lat) in enumerate(zip(specs, lats)):
            B = synth.quantise(0.2 * (0.27 + 0.23 * np.random.default_rng(vseed).random(G)))
            want = oracle.sweep(starts[i], nbr, dims, B, float(kT[i]), 9, int(seeds[i]), threads=THREADS)
            assert np.array_equal(lat.spins().astype(np.int32), want)
        hmc.hmc_ensemble_free(E)
        for l in lats:
            l.close()


def test_ensemble_rejects_mixed_members():
    a = hmc.Lattice((16, 16), hmc.HMC_VN4, 4, voronoi_seed=1)
    b = hmc.Lattice((16, 16), hmc.HMC_MOORE8, 4, voronoi_seed=1)
    with pytest.raises(hmc.HmcError):
        hmc.hmc_ensemble_create([a, b])
    with pytest.raises(hmc.HmcError):
        hmc.hmc_ensemble_create([a, a])
    E = hmc.hmc_ensemble_create([a])
    with pytest.raises(hmc.HmcError):
        hmc.hmc_ensemble_set_tiling(E, 6, 16, 0, 1)
    hmc.hmc_ensemble_free(E)
    a.close()
    b.close()


def test_autotuners_keep_results():
    desc = hmc.make_desc((128, 128), hmc.HMC_VN4)
    best, us = hmc.hmc_autotune(desc, 100, 0.5, 8)
    assert best[0] > 0 and us > 0
    w = synth.schmid_2d(side=128, G=100, n_mcs=12)
    with hmc.Lattice(w.dims, w.nbr, w.n_grains, voronoi_seed=w.voronoi_seed) as lat:
        assert lat.tiling() == best            # the tuned shape is used for this lattice shape
        start = lat.spins().astype(np.int32)
        lat.set_grain_energy(w.B)
        lat.sweep(w.kT, 12, w.sweep_seed)
        want = oracle.sweep(start, w.nbr, w.dims, w.B, w.kT, 12, w.sweep_seed)
        assert np.array_equal(lat.spins().astype(np.int32), want)
    lats = _members([((128, 128), 50, 7), ((256, 128), 300, 8)])
    starts = [l.spins() for l in lats]
    E = hmc.hmc_ensemble_create(lats)
    kT = np.array([0.5, 0.8], np.float32)
    seeds = np.array([1, 2], np.uint64)
    best_e = hmc.hmc_ensemble_autotune(E, kT, seeds, 4)
    assert hmc.hmc_ensemble_get_tiling(E) == best_e
    for l, s in zip(lats, starts):                # members restored
        assert l.mcs == 0 and np.array_equal(l.spins(), s)
    hmc.hmc_ensemble_free(E)
    for l in lats:
        l.close()


def test_large_ensemble_takes_128_tiles_and_matches_singles():
    """Sixteen 512^2 Moore8 members give one 128x128 tile per CU of an
    MI355X, so the ensemble takes them (3 MC steps per launch); every member
    equals its single run (64x64 tiles) and the oracle."""
    specs = [((512, 512), 300 + 10 * i, 60 + i) for i in range(16)]
    kT = np.linspace(0.3, 1.0, 16).astype(np.float32)
    seeds = np.arange(7000, 7016, dtype=np.uint64)
    n_mcs = 7
    say("[gpu] large ensemble 16 x 512^2")
    a = _members(specs)
    b = _members(specs)
    starts = [l.spins().astype(np.int32) for l in a]
    E = hmc.hmc_ensemble_create(a)
    try:
        assert tuple(hmc.hmc_ensemble_get_tiling(E)) == (128, 128, 1, 3)
        hmc.hmc_ensemble_sweep(E, kT, seeds, n_mcs)
        hmc.hmc_ensemble_synchronize(E)
        for i, (x, y) in enumerate(zip(a, b)):
            y.set_tiling(64, 64, 1, 2)
            y.sweep(float(kT[i]), n_mcs, int(seeds[i]))
            assert np.array_equal(x.spins(), y.spins()), i
        for i in (0, 9, 15):
            lat = a[i]
            B = synth.quantise(0.2 * (0.27 + 0.23 * np.random.default_rng(specs[i][2]).random(specs[i][1])))
            want = oracle.sweep(starts[i], hmc.HMC_MOORE8, specs[i][0], B, float(kT[i]), n_mcs, int(seeds[i]),
                                threads=THREADS)
            assert np.array_equal(lat.spins().astype(np.int32), want), i
    finally:
        hmc.hmc_ensemble_free(E)
        for l in a + b:
            l.close()


@pytest.mark.parametrize("Q", [300, 6000])
def test_compiled_moore8_ensemble_tiles_equal_oracle(Q):
    """16-bit Moore8 members in 128x128 tiles with 3 MC steps per launch run
    the ensemble kernel compiled for that tile (grain energies in LDS for
    Q = 300, from global memory for Q = 6000); 7 MC steps = two such
    launches and a short general one.  Every member equals the oracle."""
    specs = [((256, 256), Q, 21), ((128, 384), Q, 22), ((384, 128), Q, 23)]
    kT = np.array([0.4, 0.7, 1.1], np.float32)
    seeds = np.array([71, 72, 73], np.uint64)
    n_mcs = 7
    say(f"[gpu] compiled Moore8 ensemble tiles, Q={Q}")
    lats = _members(specs)
    starts = [l.spins().astype(np.int32) for l in lats]
    E = hmc.hmc_ensemble_create(lats)
    try:
        hmc.hmc_ensemble_set_tiling(E, 128, 128, 1, 3)
        hmc.hmc_ensemble_sweep(E, kT, seeds, n_mcs)
        hmc.hmc_ensemble_synchronize(E)
        got = [l.spins().astype(np.int32) for l in lats]
    finally:
        hmc.hmc_ensemble_free(E)
    for i, ((dims, G, vseed), lat) in enumerate(zip(specs, lats)):
        B = synth.quantise(0.2 * (0.27 + 0.23 * np.random.default_rng(vseed).random(G)))
        want = oracle.sweep(starts[i], hmc.HMC_MOORE8, dims, B, float(kT[i]), n_mcs, int(seeds[i]), threads=THREADS)
        assert not np.array_equal(want, starts[i])
        assert np.array_equal(got[i], want), f"member {i}: {int(np.sum(got[i] != want))} sites differ"
        lat.close()
