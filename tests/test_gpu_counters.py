"""GPU: the boundary-site count against the oracle, and the profiling trial
counter against the exact number of queued trials of the temporally blocked
kernel in the symmetric-trial mode (every site of a pass's region queued).
"""
import numpy as np
import pytest

import oracle
import paper_1007_3509_amd as hmc
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("dims,nbr,G,spin", [
    ((64, 48), hmc.HMC_VN4, 30, hmc.HMC_I16), ((128, 64), hmc.HMC_MOORE8, 70, hmc.HMC_I32),
    ((24, 16, 20), hmc.HMC_VN6, 40, hmc.HMC_I16), ((16, 16, 12), hmc.HMC_MOORE26, 25, hmc.HMC_I32),
    ((1024, 1024), hmc.HMC_VN4, 2000, hmc.HMC_I16),
])
def test_boundary_sites_match_oracle(dims, nbr, G, spin):
    say(f"[gpu] boundary dims={dims} nbr={nbr}")
    with hmc.Lattice(dims, nbr, G, voronoi_seed=4, spin=spin) as lat:
        B = synth.quantise(np.linspace(0.0, 0.2, G))
        lat.set_grain_energy(B)
        for n in (0, 6):
            if n:
                lat.sweep(0.8, n, 9)
            s = lat.spins()
            assert lat.boundary_sites() == oracle.boundary_sites(s, nbr, dims, G)


def _queued_per_tile(tile, passes, ndim):
    """Sites of each pass's colour in the region it computes: the tile grown
    by (passes - 1 - p) rings at pass p (every region side is even, so a
    2-colour class is exactly half of it)."""
    tot = 0
    for p in range(passes):
        grow = 2 * (passes - 1 - p)
        vol = 1
        for a in range(ndim):
            vol *= tile[a] + grow
        tot += vol // 2
    return tot


@pytest.mark.parametrize("dims,nbr,tiling,n_mcs", [
    ((64, 48), hmc.HMC_VN4, (16, 16, 0, 2), 4), ((64, 48), hmc.HMC_VN4, (32, 16, 0, 1), 3),
    ((32, 32, 16), hmc.HMC_VN6, (16, 16, 8, 1), 2),
])
def test_trial_counter_uniform_mode(dims, nbr, tiling, n_mcs):
    say(f"[gpu] trial counter dims={dims} tiling={tiling}")
    ndim = len(dims)
    with hmc.Lattice(dims, nbr, 5, voronoi_seed=2, proposal=hmc.HMC_PROP_UNIFORM) as lat:
        lat.set_tiling(*tiling)
        hmc.hmc_profile(lat.h, True)
        hmc.hmc_profile_trials(lat.h)
        lat.sweep(1.0, n_mcs, 3)
        got = hmc.hmc_profile_trials(lat.h)
        _, launches, su = hmc.hmc_profile_read(lat.h)
        hmc.hmc_profile(lat.h, False)
    k = tiling[3]
    ntiles = int(np.prod([dims[a] // tiling[a] for a in range(ndim)]))
    want = 0
    for m in [k] * (n_mcs // k) + ([n_mcs % k] if n_mcs % k else []):
        want += ntiles * _queued_per_tile(tiling[:ndim], 2 * m, ndim)
    assert launches == -(-n_mcs // k) and su == n_mcs * int(np.prod(dims))
    assert got == want


def test_trial_counter_is_off_without_profiling():
    with hmc.Lattice((64, 64), hmc.HMC_VN4, 10, voronoi_seed=1) as lat:
        lat.sweep(0.5, 2, 1)
        assert hmc.hmc_profile_trials(lat.h) == 0
