"""Pins of the oracle's initial microstructure, grain statistics and sweep
invariants.

* Voronoi labelling: the bucket-grid search equals brute force exactly, and
  agrees with scipy's periodic k-d tree wherever the nearest point is unique.
* grain statistics: areas sum to N, the number of grains equals the number of
  distinct spins, bin fractions sum to the fraction of binned area.
* sweep invariants that follow from the counter-based random numbers and the
  synchronous half step: splitting a run, thread count, zero steps.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import synth


@pytest.mark.parametrize("dims,G,seed", [((4, 4), 3, 1), ((8, 6), 5, 2), ((64, 64), 40, 1),
                                         ((30, 18), 200, 9), ((6, 4, 8), 7, 3), ((16, 16, 16), 60, 4),
                                         ((12, 10, 8), 1, 5)])
def test_voronoi_grid_equals_brute(orc, dims, G, seed):
    a = orc.voronoi(dims, G, seed, method="brute")
    b = orc.voronoi(dims, G, seed, method="grid", threads=4)
    assert a.dtype == np.int32 and a.shape == tuple(reversed(dims))
    assert np.array_equal(a, b)
    assert a.min() >= 0 and a.max() < G


@pytest.mark.parametrize("dims,G,seed", [((256, 256), 500, 2), ((48, 40, 32), 900, 3)])
def test_voronoi_vs_periodic_kdtree(orc, dims, G, seed):
    lab = orc.voronoi(dims, G, seed, threads=8).ravel()
    pts = orc.voronoi_points(len(dims), dims, G, seed).astype(np.float64)
    box = np.array(dims, dtype=np.float64) * 256
    tree = cKDTree(pts, boxsize=box)
    grids = np.meshgrid(*[np.arange(L) for L in reversed(dims)], indexing="ij")
    sites = np.stack([g.ravel() for g in reversed(grids)], 1).astype(np.float64) * 256
    d, idx = tree.query(sites, k=2)
    unique = d[:, 1] > d[:, 0]
    assert unique.mean() > 0.99
    assert np.array_equal(lab[unique], idx[unique, 0])
    # on ties the lower index wins
    tie = ~unique
    assert np.all(lab[tie] == np.minimum(idx[tie, 0], idx[tie, 1]))


def test_voronoi_points_in_box(orc):
    pts = orc.voronoi_points(3, (10, 20, 30), 1000, 77)
    assert pts.min() >= 0
    assert np.all(pts < np.array([10, 20, 30]) * 256)


def test_texture_identities(orc):
    rng = np.random.default_rng(3)
    Q = 50
    s = rng.integers(0, Q - 5, size=(40, 60)).astype(np.int32)
    gb = rng.integers(-1, 7, size=Q).astype(np.int32)
    areas, ng, mean, frac = orc.texture(s, Q, gb, 7)
    assert areas.sum() == s.size
    assert ng == len(np.unique(s))
    assert np.array_equal(areas, np.bincount(s.ravel(), minlength=Q))
    assert mean == pytest.approx(s.size / ng, rel=0, abs=1e-12)
    binned = sum(areas[q] for q in range(Q) if gb[q] >= 0)
    assert frac.sum() == pytest.approx(binned / s.size, abs=1e-12)
    for b in range(7):
        assert frac[b] == pytest.approx(areas[gb == b].sum() / s.size, abs=1e-15)
    with pytest.raises(ValueError):
        orc.texture(np.array([[Q]], np.int32), Q)


def test_sweep_split_equals_whole(orc):
    w = synth.schmid_2d(side=32, G=30, n_mcs=40)
    s0 = orc.voronoi(w.dims, w.n_grains, w.voronoi_seed)
    whole = orc.sweep(s0, w.nbr, w.dims, w.B, w.kT, 40, w.sweep_seed)
    part = orc.sweep(s0, w.nbr, w.dims, w.B, w.kT, 13, w.sweep_seed)
    part = orc.sweep(part, w.nbr, w.dims, w.B, w.kT, 27, w.sweep_seed, mcs0=13)
    assert np.array_equal(whole, part)
    assert not np.array_equal(whole, s0)


@pytest.mark.parametrize("nbr,dims", [(0, (24, 20)), (1, (24, 20)), (2, (12, 10, 8)), (3, (8, 10, 6))])
def test_sweep_thread_count_invariant(orc, nbr, dims):
    G = 25
    s0 = orc.voronoi(dims, G, 4)
    B = synth.quantise(0.2 * (0.27 + 0.23 * np.random.default_rng(1).random(G)))
    a = orc.sweep(s0, nbr, dims, B, 0.7, 6, seed=5, threads=1)
    b = orc.sweep(s0, nbr, dims, B, 0.7, 6, seed=5, threads=7)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, s0)
    assert np.array_equal(orc.sweep(s0, nbr, dims, B, 0.7, 0, seed=5), s0)


def test_sweep_rejects_bad_arguments(orc):
    s = np.zeros((4, 4), np.int32)
    with pytest.raises(ValueError):
        orc.sweep(s, 0, (4, 4), [0], 0.0, 1, 1)
    with pytest.raises(ValueError):
        orc.sweep(s, 0, (4, 4), [0], 1.0, -1, 1)
    with pytest.raises(ValueError):   # energy change leaves int32
        orc.sweep(np.array([[0, 1, 0, 1]] * 4, np.int32), 0, (4, 4), [-2 ** 31, 2 ** 31 - 1], 1.0, 1, 1)
