"""GPU: the threshold table a sweep reads, copied back from device memory,
equals the host builder's and the oracle's T(d) for every reachable (dn, dB)
(bucketed table of the uniform-bond model) or every d up to the largest
possible (direct table of pair bond energies and per-site fields).  Sec. 3
(Metropolis rule)."""
import numpy as np
import pytest

import oracle
import paper_1007_3509_amd as hmc
import synth
from test_table import table_problems

pytestmark = pytest.mark.gpu

J = 65536


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("make", [synth.voronoi_2d_64, synth.schmid_2d_1024, synth.schmid_3d_256,
                                  synth.moore26_3d_128], ids=lambda f: f.__name__)
def test_device_table_equals_oracle(make):
    w = make()
    say(f"[gpu] table {w.name}")
    M = oracle.num_neighbours(w.nbr)
    with hmc.Lattice(w.dims, w.nbr, w.n_grains, spin=w.spin) as lat:
        lat.set_grain_energy(w.B)
        for kT in (w.kT, 0.3, 2.5):
            lay, table, bounds = hmc.hmc_threshold_table(lat.h, kT)
            assert lay["kind"] == 0
            lo, hi = int(w.B.min()), int(w.B.max())
            assert table_problems(oracle, kT, M, J, lo, hi, lay, table, bounds) == []
            lay_h, table_h, bounds_h = hmc.hmc_threshold_table_host(kT, M, J, lo, hi)
            assert lay_h == lay and np.array_equal(table_h, table) and np.array_equal(bounds_h, bounds)


def test_ensemble_member_tables_equal_oracle():
    members = synth.ensemble_moore8()[:8]
    for w in members:
        with hmc.Lattice(w.dims, w.nbr, w.n_grains, spin=w.spin) as lat:
            lat.set_grain_energy(w.B)
            lay, table, bounds = hmc.hmc_threshold_table(lat.h, w.kT)
            assert table_problems(oracle, w.kT, 8, J, int(w.B.min()), int(w.B.max()), lay, table, bounds) == []


@pytest.mark.parametrize("mode", ["pair", "field"])
def test_direct_table_equals_oracle(mode):
    dims, Q, kT = (64, 64), 30, 0.7
    say(f"[gpu] direct table {mode}")
    rng = np.random.default_rng(9)
    B = synth.quantise(np.linspace(0.0, 0.2, Q))
    with hmc.Lattice(dims, hmc.HMC_VN4, Q, voronoi_seed=4) as lat:
        lat.set_grain_energy(B)
        if mode == "pair":
            A = np.triu(rng.integers(10000, 80000, size=(Q, Q)), 1)
            Jp = (A + A.T).astype(np.int32)
            lat.set_pair_energy(Jp)
            Dmax = 4 * int(Jp.max()) + int(B.max() - B.min())
        else:
            field = rng.integers(-3000, 9000, size=dims[0] * dims[1]).astype(np.int32)
            lat.set_site_energy(field, hmc.HMC_FIELD_CARRY)
            Dmax = 4 * J + int(B.max() - B.min()) + int(field.max() - field.min())
        lay, table, _ = hmc.hmc_threshold_table(lat.h, kT)
        assert lay["kind"] == 1 and lay["Dmax"] == Dmax and table.size == Dmax + 1
        want = oracle.threshold_many(np.arange(Dmax + 1), kT)
        assert table[0] == 0xFFFFFFFF and np.array_equal(table[1:], want[1:])
