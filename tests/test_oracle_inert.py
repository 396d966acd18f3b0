"""Pin of the oracle's rule for spin values outside [0, Q).

A caller's buffer may hold values that name no grain.  The oracle reads
them as inert: such a site never changes, a neighbour holding one is never
proposed, and its bond is the same before and after a trial (an unlike bond
of energy J under Eq. (7) read as J(1 - delta); no bond at all with a pair
table), so it drops out of the energy change.  The grain statistics leave
inert sites out.

The pin is brute force on tiny lattices: one pure-Python red/black step
whose energy change is the difference of the WHOLE lattice's Hamiltonian
(every bond and every bulk term summed before and after the trial, Eq. (7)),
with the trial spin and acceptance of Sec. 3 and the half-step rule of
Sec. 4, against the oracle's step.  The random words come from the oracle's
Philox (pinned by its published known-answer vectors) and the acceptance
from T(d) (pinned against extended precision).
"""
import itertools

import numpy as np
import pytest

J = 65536


def _offsets(nbr):
    if nbr == 0:     # von Neumann 2D
        return [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0)]
    if nbr == 1:     # Moore 2D
        return [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0)]
    if nbr == 2:     # von Neumann 3D
        return [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    return [(dx, dy, dz) for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3) if (dx, dy, dz) != (0, 0, 0)]


def _colour(nbr, x, y, z):
    if nbr in (0, 2):
        return (x + y + z) & 1
    if nbr == 1:
        return (x & 1) | ((y & 1) << 1)
    return (x & 1) | ((y & 1) << 1) | ((z & 1) << 2)


def _hamiltonian(s, dims, nbr, B, Q, Jp):
    """Eq. (7) summed over every bond once plus the bulk term of every site
    holding a grain; a bond with an inert value is unlike (J) in the uniform
    model and absent with a pair table."""
    Lx, Ly, Lz = dims
    bonds, bulk = 0, 0
    offs = _offsets(nbr)
    for z, y, x in itertools.product(range(Lz), range(Ly), range(Lx)):
        a = s[x + Lx * (y + Ly * z)]
        if 0 <= a < Q:
            bulk += int(B[a])
        for dx, dy, dz in offs:
            j = (x + dx) % Lx + Lx * ((y + dy) % Ly + Ly * ((z + dz) % Lz))
            b = s[j]
            if Jp is None:
                bonds += J * (a != b)
            elif 0 <= a < Q and 0 <= b < Q:
                bonds += int(Jp[a, b])
    assert bonds % 2 == 0   # every bond was visited from both ends
    return bonds // 2 + bulk


def _brute_step(orc, s0, dims, nbr, B, Q, kT, t, seed, Jp=None):
    Lx, Ly, Lz = dims
    offs = _offsets(nbr)
    C = 2 if nbr in (0, 2) else (4 if nbr == 1 else 8)
    s = list(int(v) for v in s0)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for c in range(C):
        before = list(s)
        for z, y, x in itertools.product(range(Lz), range(Ly), range(Lx)):
            if _colour(nbr, x, y, z) != c:
                continue
            i = x + Lx * (y + Ly * z)
            q = before[i]
            r = orc.philox4x32_10([i, t, c, 0], key)[0]
            k = (int(r[0]) * len(offs)) >> 32
            dx, dy, dz = offs[k]
            qn = before[(x + dx) % Lx + Lx * ((y + dy) % Ly + Ly * ((z + dz) % Lz))]
            if not (0 <= q < Q) or not (0 <= qn < Q) or qn == q:
                continue
            trial = list(before)
            trial[i] = qn
            d = _hamiltonian(trial, dims, nbr, B, Q, Jp) - _hamiltonian(before, dims, nbr, B, Q, Jp)
            if d <= 0 or int(r[1]) < orc.threshold(d, kT):
                s[i] = qn
    return np.array(s, dtype=np.int32)


def _lattice(rng, dims, Q):
    n = int(np.prod(dims))
    s = rng.integers(0, Q, size=n).astype(np.int32)
    s[rng.choice(n, size=n // 6, replace=False)] = -1
    s[rng.integers(0, n)] = Q + 7
    s[rng.integers(0, n)] = 1 << 20
    return s


@pytest.mark.parametrize("nbr,dims", [(0, (6, 6, 1)), (1, (4, 6, 1)), (2, (4, 4, 4))])
@pytest.mark.parametrize("pair", [False, True])
def test_inert_values_match_brute_force_step(orc, nbr, dims, pair):
    rng = np.random.default_rng(17 + nbr + 3 * pair)
    Q, kT, seed = 4, 1.3, 0x1234_0000_0007
    s0 = _lattice(rng, dims, Q)
    B = np.array([0, 9000, -7000, 20000], np.int32)
    Jp = None
    if pair:
        A = np.triu(rng.integers(30000, 90000, size=(Q, Q)), 1)
        Jp = (A + A.T).astype(np.int32)
    got = s0.copy()
    want = s0.copy()
    for t in range(3):
        want = _brute_step(orc, want, dims, nbr, B, Q, kT, t, seed, Jp)
    if pair:
        got = orc.sweep_pair(got, nbr, dims[:2] if nbr < 2 else dims, Jp, B, kT, 3, seed)
    else:
        got = orc.sweep(got, nbr, dims[:2] if nbr < 2 else dims, B, kT, 3, seed)
    assert np.array_equal(got, want)
    inert = (s0 < 0) | (s0 >= Q)
    assert np.array_equal(got[inert], s0[inert])
    assert not np.array_equal(got, s0)   # the valid sites did move


def test_inert_values_are_left_out_of_the_statistics(orc):
    rng = np.random.default_rng(3)
    Q = 5
    s = _lattice(rng, (8, 8, 1), Q)
    areas, n, mean, frac = orc.texture(s, Q, np.array([0, 1, -1, 0, 1], np.int32), 2)
    valid = s[(s >= 0) & (s < Q)]
    assert np.array_equal(areas, np.bincount(valid, minlength=Q))
    assert n == int(np.sum(areas > 0)) and mean == pytest.approx(64 / n)
    assert frac[0] == pytest.approx((areas[0] + areas[3]) / 64) and frac[1] == pytest.approx((areas[1] + areas[4]) / 64)
    assert orc.boundary_sites(s, 0, (8, 8), Q) == sum(
        1 for i in range(64) if 0 <= s[i] < Q and any(
            s[(i % 8 + dx) % 8 + 8 * ((i // 8 + dy) % 8)] != s[i] for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1))))


@pytest.mark.parametrize("nbr,dims", [(0, (6, 6, 1)), (1, (4, 6, 1))])
@pytest.mark.parametrize("pair", [False, True])
def test_nfold_weights_with_inert_values_match_brute_force(orc, nbr, dims, pair):
    """The n-fold way's slot weights follow the same rule: zero for an inert
    site and for a slot holding an inert value, else 2^32 min(1, e^{-dE/kT})
    with dE the whole-lattice Hamiltonian difference."""
    rng = np.random.default_rng(5 + nbr + 2 * pair)
    Q, kT = 4, 0.9
    s = _lattice(rng, dims, Q)
    B = np.array([0, 9000, -7000, 20000], np.int32)
    Jp = None
    if pair:
        A = np.triu(rng.integers(30000, 90000, size=(Q, Q)), 1)
        Jp = (A + A.T).astype(np.int32)
    got = orc.nfold_weights(s, nbr, dims[:2], B, kT, Jp=Jp)
    Lx, Ly, _ = dims
    offs = _offsets(nbr)
    H0 = _hamiltonian(list(s), dims, nbr, B, Q, Jp)
    for i in range(Lx * Ly):
        x, y = i % Lx, i // Lx
        for k, (dx, dy, _) in enumerate(offs):
            qn = int(s[(x + dx) % Lx + Lx * ((y + dy) % Ly)])
            if not (0 <= s[i] < Q) or not (0 <= qn < Q) or qn == s[i]:
                assert got[i, k] == 0
                continue
            trial = list(s)
            trial[i] = qn
            d = _hamiltonian(trial, dims, nbr, B, Q, Jp) - H0
            assert int(got[i, k]) == ((1 << 32) if d <= 0 else orc.threshold(d, kT))
