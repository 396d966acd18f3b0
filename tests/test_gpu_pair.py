"""GPU parity of the sweep with a bond energy per pair of grains (Eq. (7)'s
J_{q_i,q_n}) against the oracle, element by element (integer: bit-exact),
and of the GPU Read-Shockley table against the oracle's (within one unit of
2^-16, the rounding of a device transcendental).  Pair tables fed to both
paths come from the oracle or from a seeded generator, never from the GPU.
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


def _random_table(Q, seed, hi=70000):
    A = np.random.default_rng(seed).integers(0, hi, size=(Q, Q))
    T = np.triu(A, 1)
    return (T + T.T).astype(np.int32)


def _orientations(Q, seed):
    rng = np.random.default_rng(seed)
    return synth.matrix_to_bunge(synth.quat_to_matrix(synth.shoemake_quaternions(rng, Q)))


def _gpu_pair_run(dims, nbr, Q, B, Jp, kT, n_mcs, seed, vseed, spin=hmc.HMC_I16, proposal=0, tiling=None,
                  chunks=None):
    say(f"[gpu] pair dims={dims} nbr={nbr} Q={Q} spin={spin} prop={proposal} tiling={tiling} chunks={chunks}")
    with hmc.Lattice(dims, nbr, Q, voronoi_seed=vseed, spin=spin, proposal=proposal) as lat:
        lat.set_grain_energy(B)
        lat.set_pair_energy(Jp)
        if tiling is not None:
            lat.set_tiling(*tiling)
        start = lat.spins().astype(np.int32)
        for n in (chunks or [n_mcs]):
            lat.sweep(kT, n, seed)
        return start, lat.spins().astype(np.int32)


CASES = [
    # dims, nbr, Q, spin, proposal, tiling
    ((100, 36), hmc.HMC_VN4, 30, hmc.HMC_I16, 0, None),
    ((64, 48), hmc.HMC_VN4, 20, hmc.HMC_I32, 1, (16, 16, 0, 3)),
    ((96, 64), hmc.HMC_MOORE8, 40, hmc.HMC_I16, 0, None),
    ((24, 20, 16), hmc.HMC_VN6, 25, hmc.HMC_I16, 0, (8, 10, 4, 1)),
    ((32, 16, 12), hmc.HMC_VN6, 25, hmc.HMC_I32, 0, None),
    ((16, 12, 8), hmc.HMC_MOORE26, 15, hmc.HMC_I16, 0, None),
]


@pytest.mark.parametrize("dims,nbr,Q,spin,prop,tiling", CASES)
def test_pair_sweep_matches_oracle(dims, nbr, Q, spin, prop, tiling):
    B = synth.quantise(np.random.default_rng(Q).uniform(0.0, 0.2, size=Q))
    Jp = _random_table(Q, Q + 1)
    start, got = _gpu_pair_run(dims, nbr, Q, B, Jp, 0.7, 11, 17, vseed=4, spin=spin, proposal=prop, tiling=tiling,
                               chunks=[4, 7])
    want = oracle.sweep_pair(start, nbr, dims, Jp, B, 0.7, 11, 17, proposal=prop, threads=THREADS)
    assert np.array_equal(got, want), f"{int(np.sum(got != want))} sites differ"


def test_read_shockley_sweep_matches_oracle_1024():
    w = synth.schmid_2d_1024()
    euler = _orientations(w.n_grains, 77)
    Jp = oracle.pair_table(euler, 1.0, 15.0)
    say("[gpu] read-shockley 1024^2, 40 MCS")
    start, got = _gpu_pair_run(w.dims, w.nbr, w.n_grains, w.B, Jp, w.kT, 40, w.sweep_seed, vseed=w.voronoi_seed)
    want = oracle.sweep_pair(start, w.nbr, w.dims, Jp, w.B, w.kT, 40, w.sweep_seed, threads=THREADS)
    assert np.array_equal(got, want), f"{int(np.sum(got != want))} sites differ"


def test_uniform_table_equals_uniform_mode():
    dims, Q = (128, 96), 40
    B = synth.quantise(np.linspace(0.0, 0.2, Q))
    Jp = (65536 * (1 - np.eye(Q))).astype(np.int32)
    with hmc.Lattice(dims, hmc.HMC_VN4, Q, voronoi_seed=3) as a, hmc.Lattice(dims, hmc.HMC_VN4, Q, voronoi_seed=3) as b:
        for lat in (a, b):
            lat.set_grain_energy(B)
        b.set_pair_energy(Jp)
        a.sweep(0.6, 13, 5)
        b.sweep(0.6, 13, 5)
        assert np.array_equal(a.spins(), b.spins())
        # back to the uniform bond energy
        b.set_pair_energy(None)
        a.sweep(0.6, 5, 6)
        b.sweep(0.6, 5, 6)
        assert np.array_equal(a.spins(), b.spins())


def test_misorientation_table_matches_oracle():
    Q = 300
    e = _orientations(Q, 5)
    got = hmc.hmc_misorientation_energy(e, 1.0, 15.0)
    want = oracle.pair_table(e, 1.0, 15.0)
    assert np.array_equal(got, got.T) and np.all(np.diag(got) == 0)
    diff = np.abs(got.astype(np.int64) - want)
    assert diff.max() <= 1
    assert np.mean(diff == 0) > 0.999
    # identical orientations and a twin pair
    e2 = np.array([[0.1, 0.2, 0.3], [0.1, 0.2, 0.3], [0.0, 0.0, 0.0]])
    t = hmc.hmc_misorientation_energy(e2, 2.0, 15.0)
    assert t[0, 1] == 0 and t[0, 2] > 0


def test_pair_energy_validation():
    with hmc.Lattice((32, 32), hmc.HMC_VN4, 4, voronoi_seed=1) as lat:
        good = _random_table(4, 2)
        bad = good.copy()
        bad[0, 1] += 1                         # not symmetric
        with pytest.raises(hmc.HmcError):
            lat.set_pair_energy(bad)
        bad = good.copy()
        bad[2, 2] = 5                          # nonzero diagonal
        with pytest.raises(hmc.HmcError):
            lat.set_pair_energy(bad)
        bad = good.copy()
        bad[1, 3] = bad[3, 1] = -1             # negative
        with pytest.raises(hmc.HmcError):
            lat.set_pair_energy(bad)
        with pytest.raises(hmc.HmcError):
            lat.set_pair_energy(_random_table(5, 2))   # wrong Q
        lat.set_pair_energy(good)
        with pytest.raises(hmc.HmcError):       # ensembles take uniform bonds only
            hmc.hmc_ensemble_create([lat])
    with pytest.raises(hmc.HmcError):
        hmc.hmc_misorientation_energy(np.zeros((3, 3)), -1.0, 15.0)
