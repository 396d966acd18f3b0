"""GPU parity of the sweep with a per-site bulk field (Eq. (7)'s b_i inside
grains) and both carry-over rules against the oracle, element by element
(spins and field: integers, bit-exact), plus the reductions, checkpoints and
argument checks."""
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


CASES = [
    # dims, nbr, Q, spin, rule, tiling
    ((100, 36), hmc.HMC_VN4, 30, hmc.HMC_I16, 0, None),
    ((64, 48), hmc.HMC_VN4, 20, hmc.HMC_I32, 1, (16, 16, 0, 3)),
    ((128, 96), hmc.HMC_VN4, 40, hmc.HMC_I16, 1, (64, 32, 0, -3)),
    ((96, 64), hmc.HMC_MOORE8, 40, hmc.HMC_I16, 0, (32, 32, 0, -2)),
    ((24, 20, 16), hmc.HMC_VN6, 25, hmc.HMC_I16, 0, (8, 10, 4, 1)),
    ((32, 16, 12), hmc.HMC_VN6, 25, hmc.HMC_I32, 1, None),
    ((16, 12, 8), hmc.HMC_MOORE26, 15, hmc.HMC_I16, 0, None),
]


@pytest.mark.parametrize("dims,nbr,Q,spin,rule,tiling", CASES)
def test_field_sweep_matches_oracle(dims, nbr, Q, spin, rule, tiling):
    say(f"[gpu] field dims={dims} nbr={nbr} spin={spin} rule={rule} tiling={tiling}")
    B = synth.quantise(np.random.default_rng(Q).uniform(0.0, 0.2, size=Q))
    with hmc.Lattice(dims, nbr, Q, voronoi_seed=6, spin=spin) as lat:
        start = lat.spins().astype(np.int32)
        field = synth.heterogeneous_field(start, B, 0.3, 8.0)
        lat.set_grain_energy(np.zeros(Q, np.int32) + 1000)
        lat.set_site_energy(field, rule)
        if tiling is not None:
            lat.set_tiling(*tiling)
        for n in (4, 7):
            lat.sweep(0.7, n, 19)
        got, gotf = lat.spins().astype(np.int32), lat.site_energy()
    want, wantf = oracle.sweep_field(start, field, rule, nbr, dims, np.zeros(Q, np.int32) + 1000, 0.7, 11, 19,
                                     threads=THREADS)
    assert np.array_equal(got, want), f"{int(np.sum(got != want))} sites differ"
    assert np.array_equal(gotf, wantf), f"{int(np.sum(gotf != wantf))} field values differ"


def test_grain_energy_field_is_the_per_grain_model_1024():
    w = synth.schmid_2d_1024()
    say("[gpu] field = grain energies, 1024^2, 60 MCS")
    with hmc.Lattice(w.dims, w.nbr, w.n_grains, voronoi_seed=w.voronoi_seed) as a, \
            hmc.Lattice(w.dims, w.nbr, w.n_grains, voronoi_seed=w.voronoi_seed) as b:
        a.set_grain_energy(w.B)
        b.set_site_energy(w.B[b.spins()])
        a.sweep(w.kT, 60, w.sweep_seed)
        b.sweep(w.kT, 60, w.sweep_seed)
        sa, sb = a.spins(), b.spins()
        assert np.array_equal(sa, sb)
        assert np.array_equal(b.site_energy(), w.B[sb])


def test_field_checkpoint_and_removal():
    dims, Q = (64, 64), 12
    with hmc.Lattice(dims, hmc.HMC_VN4, Q, voronoi_seed=2) as lat:
        f0 = synth.heterogeneous_field(lat.spins(), synth.quantise(np.full(Q, 0.1)), 0.5, 16.0)
        lat.set_site_energy(f0, hmc.HMC_FIELD_RECRYSTALLISE)
        hmc.hmc_snapshot(lat.h)
        lat.sweep(0.8, 10, 3)
        f1, s1 = lat.site_energy(), lat.spins()
        assert not np.array_equal(f1, f0)
        hmc.hmc_restore(lat.h)
        assert np.array_equal(lat.site_energy(), f0)
        lat.sweep(0.8, 10, 3)
        assert np.array_equal(lat.site_energy(), f1) and np.array_equal(lat.spins(), s1)
        lat.set_site_energy(None)
        with pytest.raises(hmc.HmcError):
            lat.site_energy()


def test_field_argument_checks():
    with hmc.Lattice((32, 32), hmc.HMC_VN4, 4, voronoi_seed=1, proposal=hmc.HMC_PROP_UNIFORM) as lat:
        with pytest.raises(hmc.HmcError):         # needs neighbour trials
            lat.set_site_energy(np.zeros((32, 32), np.int32))
    with hmc.Lattice((32, 32), hmc.HMC_VN4, 4, voronoi_seed=1) as lat:
        with pytest.raises(hmc.HmcError):         # wrong size
            lat.set_site_energy(np.zeros((32, 16), np.int32))
        with pytest.raises(hmc.HmcError):         # out of range
            lat.set_site_energy(np.full((32, 32), 1 << 25, np.int32))
        with pytest.raises(hmc.HmcError):         # unknown rule
            lat.set_site_energy(np.zeros((32, 32), np.int32), 7)
        lat.set_site_energy(np.zeros((32, 32), np.int32))
        with pytest.raises(hmc.HmcError):         # not combined with pair energies
            lat.set_pair_energy((65536 * (1 - np.eye(4))).astype(np.int32))
        with pytest.raises(hmc.HmcError):         # ensembles take plain lattices
            hmc.hmc_ensemble_create([lat])
