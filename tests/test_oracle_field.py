"""Pins of the oracle's per-site bulk field (Eq. (7)'s b_i varying inside a
grain) and its two carry-over rules (the paper's closing discussion):

* a constant field changes nothing (it cancels from every energy change);
* a field equal to its grain's energy, carried from the neighbour whose spin
  a site adopts, reproduces the per-grain model exactly and stays equal to
  its grain's energy (catches a field taken from the wrong site);
* under recrystallisation every swept site ends dislocation-free and no
  site's field ever grows.
"""
import numpy as np
import pytest

import synth


@pytest.mark.parametrize("nbr,dims", [(0, (32, 24)), (1, (24, 32)), (2, (12, 10, 8)), (3, (8, 6, 8))])
def test_constant_field_is_inert(orc, nbr, dims):
    Q = 9
    s = orc.voronoi(dims, Q, 3)
    B = synth.quantise(np.linspace(0.0, 0.3, Q))
    field = np.full(s.shape, 12345, np.int32)
    a, f = orc.sweep_field(s, field, orc.FIELD_CARRY, nbr, dims, B, 0.8, 9, 21)
    b = orc.sweep(s, nbr, dims, B, 0.8, 9, 21)
    assert np.array_equal(a, b) and np.all(f == 12345)


@pytest.mark.parametrize("nbr,dims", [(0, (32, 24)), (1, (24, 32)), (2, (12, 10, 8))])
def test_field_of_grain_energies_reproduces_per_grain_model(orc, nbr, dims):
    Q = 12
    s = orc.voronoi(dims, Q, 5)
    B = synth.quantise(np.random.default_rng(nbr).uniform(0.0, 0.4, size=Q))
    a, f = orc.sweep_field(s, B[s], orc.FIELD_CARRY, nbr, dims, np.zeros(Q, np.int32), 0.7, 15, 4)
    b = orc.sweep(s, nbr, dims, B, 0.7, 15, 4)
    assert np.array_equal(a, b)
    assert np.array_equal(f, B[a])


def test_recrystallised_sites_are_dislocation_free(orc):
    dims, Q = (48, 40), 10
    s = orc.voronoi(dims, Q, 8)
    rng = np.random.default_rng(2)
    field = rng.integers(1000, 20000, size=s.shape).astype(np.int32)
    a, f = orc.sweep_field(s, field, orc.FIELD_RECRYSTALLISE, 0, dims, np.zeros(Q, np.int32), 0.9, 20, 6)
    assert np.all((f == 0) | (f == field))
    assert np.all(f[a != s] == 0)
    assert np.count_nonzero(f == 0) > 0
    # a stored field drives boundaries into the deformed matrix: more sites sweep than without it
    a0 = orc.sweep(s, 0, dims, np.zeros(Q, np.int32), 0.9, 20, 6)
    assert np.count_nonzero(a != s) > np.count_nonzero(a0 != s)
