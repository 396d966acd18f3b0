"""GPU: the two largest lattices against the oracle, element by element
(Sec. 3 Metropolis trials, Sec. 4 Red/Black half steps, Sec. 6 grain
energy), in the launch configuration the benchmark times:

* 16384^2 VN4 int16 (512 MiB per buffer, beyond the Infinity Cache) with its
  default 256x128 tiles and 4 MC steps per launch;
* 512^3 VN6 int32 (512 MiB per buffer) with its default tiles.

Each: the Voronoi initial state built on the GPU equals the oracle's, and the
spins after 12 MC steps (several launches, the last one short) and the grain
statistics equal the oracle's.
"""
import os

import numpy as np
import pytest

import oracle
import paper_1007_3509_amd as hmc
import synth

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, len(os.sched_getaffinity(0))))
N_MCS = 12


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("make", [synth.stress_2d_16384, synth.stress_3d_512], ids=["2d_16384", "3d_512"])
def test_largest_lattices_equal_oracle(make):
    w = make()
    say(f"[gpu] {w.name}: Voronoi init and {N_MCS} MC steps")
    with hmc.Lattice(w.dims, w.nbr, w.n_grains, voronoi_seed=w.voronoi_seed, spin=w.spin) as lat:
        lat.set_grain_energy(w.B)
        tiling = tuple(hmc.hmc_get_tiling(lat.h))
        start = lat.spins().astype(np.int32)
        lat.sweep(w.kT, N_MCS, w.sweep_seed)
        got = lat.spins().astype(np.int32)
        ng, mean, frac = lat.texture_stats(w.grain_bin, w.n_bins)
    say(f"[cpu] {w.name}: oracle (tiling {tiling})")
    init = oracle.voronoi(w.dims, w.n_grains, w.voronoi_seed, threads=THREADS)
    assert np.array_equal(start, init.reshape(start.shape)), f"{int(np.sum(start != init))} initial sites differ"
    del init
    want = oracle.sweep(start, w.nbr, w.dims, w.B, w.kT, N_MCS, w.sweep_seed, threads=THREADS)
    assert np.array_equal(got, want), f"{int(np.sum(got != want))} sites differ after {N_MCS} steps"
    _, ng_o, mean_o, frac_o = oracle.texture(want, w.n_grains, w.grain_bin, w.n_bins)
    assert ng == ng_o and mean == mean_o and np.array_equal(frac, frac_o)
