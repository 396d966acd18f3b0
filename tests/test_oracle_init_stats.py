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
    # a value outside [0, Q) names no grain: left out of the areas
    a2, ng2, mean2, _ = orc.texture(np.array([[Q, 0, -1, 0]], np.int32), Q)
    assert a2.sum() == 2 and a2[0] == 2 and ng2 == 1 and mean2 == 4.0


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


# ------------------------------------------------------- boundary sites

def _brute_boundary(s, offs, Q):
    """Pure-Python loops over every site and every neighbour offset."""
    shape = s.shape
    n = 0
    for idx in np.ndindex(*shape):
        q = s[idx]
        if not 0 <= q < Q:
            continue
        for o in offs:
            j = tuple((idx[a] + o[a]) % shape[a] for a in range(len(shape)))
            if s[j] != q:
                n += 1
                break
    return n


def test_boundary_sites_closed_forms(orc):
    # uniform lattice: none; 2-colour checkerboard under VN4: every site
    assert orc.boundary_sites(np.zeros((8, 6), np.int32), orc.VN4, (6, 8), 2) == 0
    yy, xx = np.mgrid[0:8, 0:6]
    cb = ((xx + yy) & 1).astype(np.int32)
    assert orc.boundary_sites(cb, orc.VN4, (6, 8), 2) == 48
    assert orc.boundary_sites(cb, orc.MOORE8, (6, 8), 2) == 48
    # a strip of rows across x has two flat interfaces: one row on each side
    # of each is a boundary row, for VN4 and Moore8 alike (4 Lx sites)
    st = np.zeros((16, 10), np.int32)
    st[5:11, :] = 1
    for nbr in (orc.VN4, orc.MOORE8):
        assert orc.boundary_sites(st, nbr, (10, 16), 2) == 4 * 10
    # a slab of planes in 3D: four boundary planes
    sl = np.zeros((8, 6, 4), np.int32)
    sl[2:5] = 1
    for nbr in (orc.VN6, orc.MOORE26):
        assert orc.boundary_sites(sl, nbr, (4, 6, 8), 2) == 4 * 4 * 6
    # values outside [0, Q) are not counted (but still differ from neighbours)
    st2 = st.copy()
    st2[0, 0] = -1
    assert orc.boundary_sites(st2, orc.VN4, (10, 16), 2) == 4 * 10 + 4   # its 4 neighbours join


@pytest.mark.parametrize("nbr,shape", [(0, (6, 8)), (1, (8, 6)), (2, (4, 6, 4)), (3, (4, 4, 6))])
def test_boundary_sites_brute_force(orc, nbr, shape):
    rng = np.random.default_rng(nbr + 10)
    s = rng.integers(0, 3, size=shape).astype(np.int32)
    s[rng.random(shape) < 0.5] = 0
    dims = tuple(reversed(shape))
    offs2 = {0: [(0, 1), (0, -1), (1, 0), (-1, 0)],
             1: [(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1) if (a, b) != (0, 0)]}
    offs3 = {2: [(0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0), (1, 0, 0), (-1, 0, 0)],
             3: [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1) if (a, b, c) != (0, 0, 0)]}
    offs = offs2.get(nbr) or offs3[nbr]
    assert orc.boundary_sites(s, nbr, dims, 3) == _brute_boundary(s, offs, 3)
