"""Pins of the oracle's pair bond energies (Eq. (7)'s J_{q_i,q_n}): the
cubic misorientation angle, the Read-Shockley law, the energy change against
a brute-force Hamiltonian, and reductions to the pinned uniform sweep.

* misorientation: 0 for identical and for cube-symmetric orientations, a
  rotation theta about [001] gives min(theta, 90 - theta), the Sigma-3 twin
  (60 deg about [111]) gives 60 deg, random pairs never exceed the cubic
  maximum 62.80 deg and average Mackenzie's 40.74 deg;
* Read-Shockley: J(0) = 0, J(theta_m) = J_max, J(theta_m / e) = 2 J_max / e,
  increasing with zero slope at theta_m;
* Delta E with pair energies = difference of the full Hamiltonian (every bond
  once) for all four neighbourhoods;
* a table with J_fx off the diagonal is the uniform model (bit-exact sweep);
* relabelling the grains relabels the result (catches swapped indices).
"""
import numpy as np
import pytest

import synth


def _rot(axis, deg):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    t = np.radians(deg)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(t) * K + (1 - np.cos(t)) * K @ K


def _euler(R):
    return synth.matrix_to_bunge(np.asarray(R)[None])[0]


def test_misorientation_special_cases(orc):
    z = [0.0, 0.0, 0.0]
    assert orc.misorientation_deg(z, z) == pytest.approx(0.0, abs=1e-6)
    assert orc.misorientation_deg(z, [np.pi / 2, 0, 0]) == pytest.approx(0.0, abs=1e-6)
    assert orc.misorientation_deg(z, [0, np.pi / 2, 0]) == pytest.approx(0.0, abs=1e-6)
    for th in (5.0, 10.0, 30.0, 44.0, 60.0, 80.0):
        want = min(th, 90.0 - th)
        assert orc.misorientation_deg(z, [np.radians(th), 0, 0]) == pytest.approx(want, abs=1e-6)
    # Sigma-3 twin: 60 deg about [111], from either side, after an arbitrary common rotation
    g0 = _rot([0.3, -0.2, 0.9], 37.0)
    e1 = _euler(g0)
    e2 = _euler(_rot([1, 1, 1], 60.0) @ g0)
    assert orc.misorientation_deg(e1, e2) == pytest.approx(60.0, abs=1e-6)
    assert orc.misorientation_deg(e2, e1) == pytest.approx(60.0, abs=1e-6)


def test_misorientation_distribution_of_random_pairs(orc):
    rng = np.random.default_rng(21)
    n = 20000
    e = synth.matrix_to_bunge(synth.quat_to_matrix(synth.shoemake_quaternions(rng, 2 * n)))
    th = np.array([orc.misorientation_deg(e[2 * k], e[2 * k + 1]) for k in range(n)])
    assert th.max() <= 62.80 + 1e-3          # cubic maximum, Mackenzie (1958)
    assert th.mean() == pytest.approx(40.74, abs=0.35)   # Mackenzie mean for cubic symmetry


def test_read_shockley_closed_forms(orc):
    Jm, tm = 1.0, 15.0
    assert orc.read_shockley(0.0, Jm, tm) == 0.0
    assert orc.read_shockley(tm, Jm, tm) == pytest.approx(Jm, rel=1e-15)
    assert orc.read_shockley(40.0, Jm, tm) == Jm
    assert orc.read_shockley(tm / np.e, Jm, tm) == pytest.approx(2 * Jm / np.e, rel=1e-14)
    xs = np.linspace(0.01, tm, 300)
    J = np.array([orc.read_shockley(x, Jm, tm) for x in xs])
    assert np.all(np.diff(J) > 0)
    h = 1e-4
    assert (Jm - orc.read_shockley(tm - h, Jm, tm)) / h < 1e-3    # zero slope at theta_m


def test_pair_table_properties(orc):
    rng = np.random.default_rng(3)
    e = synth.matrix_to_bunge(synth.quat_to_matrix(synth.shoemake_quaternions(rng, 40)))
    e[7] = e[3]                                  # two grains with one orientation
    e[9] = _euler(_rot([1, 1, 1], 60.0) @ synth.bunge_to_matrix(e[2])[0])   # a twin of grain 2
    Jp = orc.pair_table(e, 1.0, 15.0)
    assert np.array_equal(Jp, Jp.T) and np.all(np.diag(Jp) == 0)
    assert Jp[3, 7] == 0 and Jp[2, 9] == 65536
    assert Jp.min() >= 0 and Jp.max() <= 65536


def _hamiltonian(s, nbr, Jp, B):
    """Every bond once: sum over sites and neighbour offsets, halved."""
    offs = {0: [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0)],
            1: [(a, b, 0) for a in (-1, 0, 1) for b in (-1, 0, 1) if (a, b) != (0, 0)],
            2: [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)],
            3: [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1) if (a, b, c) != (0, 0, 0)]}[nbr]
    s3 = s if s.ndim == 3 else s[None]
    total = 0
    for dx, dy, dz in offs:
        t = np.roll(s3, shift=(-dz, -dy, -dx), axis=(0, 1, 2))
        total += int(Jp[s3, t].astype(np.int64).sum())
    assert total % 2 == 0
    return total // 2 + int(B[s3].astype(np.int64).sum())


@pytest.mark.parametrize("nbr,shape", [(0, (6, 8)), (1, (8, 6)), (2, (4, 6, 4)), (3, (4, 4, 6))])
def test_pair_delta_energy_is_hamiltonian_difference(orc, nbr, shape):
    rng = np.random.default_rng(10 + nbr)
    Q = 5
    s = rng.integers(0, Q, size=shape).astype(np.int32)
    A = rng.integers(0, 50000, size=(Q, Q))
    Jp = np.triu(A, 1)
    Jp = (Jp + Jp.T).astype(np.int32)
    B = rng.integers(-30000, 30000, size=Q).astype(np.int32)
    dims = tuple(reversed(shape))
    H0 = _hamiltonian(s, nbr, Jp, B)
    flat = s.reshape(-1)
    for _ in range(25):
        i = int(rng.integers(0, flat.size))
        qn = int(rng.integers(0, Q))
        t = flat.copy()
        t[i] = qn
        want = _hamiltonian(t.reshape(shape), nbr, Jp, B) - H0
        assert orc.delta_energy_pair(s, nbr, dims, Jp, B, i, qn) == want


@pytest.mark.parametrize("nbr,dims,prop", [(0, (16, 12), 0), (1, (12, 16), 0), (2, (8, 6, 4), 1), (3, (4, 6, 4), 0)])
def test_uniform_table_is_the_uniform_model(orc, nbr, dims, prop):
    rng = np.random.default_rng(nbr)
    Q = 6
    s = rng.integers(0, Q, size=tuple(reversed(dims))).astype(np.int32)
    B = rng.integers(-20000, 20000, size=Q).astype(np.int32)
    Jp = (65536 * (1 - np.eye(Q))).astype(np.int32)
    a = orc.sweep_pair(s, nbr, dims, Jp, B, 0.8, 7, 42, proposal=prop)
    b = orc.sweep(s, nbr, dims, B, 0.8, 7, 42, proposal=prop)
    assert np.array_equal(a, b)


def test_relabelling_grains_relabels_the_result(orc):
    rng = np.random.default_rng(5)
    Q, dims = 7, (16, 16)
    s = rng.integers(0, Q, size=(16, 16)).astype(np.int32)
    A = rng.integers(1000, 90000, size=(Q, Q))
    Jp = np.triu(A, 1)
    Jp = (Jp + Jp.T).astype(np.int32)
    B = rng.integers(-20000, 20000, size=Q).astype(np.int32)
    perm = rng.permutation(Q)            # new label of old grain g is perm[g]
    inv = np.argsort(perm)
    a = orc.sweep_pair(s, 0, dims, Jp, B, 0.9, 9, 3)
    b = orc.sweep_pair(perm[s].astype(np.int32), 0, dims, Jp[np.ix_(inv, inv)], B[inv], 0.9, 9, 3)
    assert np.array_equal(perm[a], b)
    # and a non-uniform table changes the dynamics
    assert not np.array_equal(a, orc.sweep(s, 0, dims, B, 0.9, 9, 3))
