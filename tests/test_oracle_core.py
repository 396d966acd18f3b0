"""Pins of the CPU oracle's building blocks against things other than itself.

- Philox4x32-10 against the published known-answer vectors (Salmon et al.,
  SC'11 / Random123) and basic uniformity.
- T(d) against an extended-precision evaluation of 2^32 exp(-d/(65536 kT)).
- neighbour order and colourings (the Red/Black scheme of Sec. 4 needs that
  sites of one colour share no bond).
- the local energy change against the full Hamiltonian Eq. (7) (read as
  J(1-delta) per bond plus the bulk term) summed over every bond.
"""
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _kat_rows():
    rows = []
    with open(os.path.join(GOLD, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(t, 16) for t in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers(orc):
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = orc.philox4x32_10(ctr, key)[0]
        assert [int(v) for v in got] == want


def test_philox_uniformity(orc):
    n = 1 << 16
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n)
    ctr[:, 1] = 7
    out = orc.philox4x32_10(ctr, [12345, 678])
    for w in range(4):
        u = out[:, w].astype(np.float64) / 2.0 ** 32
        assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
        hist = np.bincount((out[:, w] >> 28).astype(np.int64), minlength=16)
        chi2 = ((hist - n / 16) ** 2 / (n / 16)).sum()
        assert chi2 < 60  # 15 dof, p ~ 1e-7
    # distinct counters / keys give distinct streams
    assert not np.array_equal(out, orc.philox4x32_10(ctr, [12345, 679]))


@pytest.mark.parametrize("kT", [0.3, 0.5, 0.6, 1.0, 1.4, 2.6])
def test_threshold_matches_extended_precision(orc, kT):
    kT32 = float(np.float32(kT))
    ds = np.unique(np.concatenate([np.arange(1, 3000), np.arange(1, 40) * 65536,
                                   np.arange(0, 5) * 65536 + 3015, [65536 * 26 + 7]]))
    prev = 2 ** 32
    for d in ds:
        t = orc.threshold(int(d), kT32)
        exact = np.longdouble(2) ** 32 * np.exp(-np.longdouble(int(d)) / (np.longdouble(65536) * np.longdouble(kT32)))
        # floor() loses < 1; the double exp carries ~1 ulp of 2^32
        assert abs(np.longdouble(t) - exact) <= 1.0 + 2.0 ** 32 * 4e-16
        assert t <= prev  # non-increasing in d
        prev = t
    assert orc.threshold(1, kT32) == min(2 ** 32 - 1, int(np.floor(2.0 ** 32 * np.exp(-1 / (65536 * kT32)))))


def test_threshold_cap_and_floor(orc):
    assert orc.threshold(1, 1e6) == 2 ** 32 - 1         # exp(-tiny) rounds to 1 -> capped
    assert orc.threshold(65536 * 200, 0.5) == 0         # exp(-400) underflows the 2^32 scale


NBR_CASES = [(0, (6, 8)), (1, (6, 8)), (2, (4, 6, 8)), (3, (4, 6, 8))]


@pytest.mark.parametrize("nbr,dims", NBR_CASES)
def test_neighbour_tables(orc, nbr, dims):
    N = int(np.prod(dims))
    M = orc.num_neighbours(nbr)
    table = np.stack([orc.neighbours_of(nbr, dims, i) for i in range(N)])
    assert table.shape == (N, M)
    # distinct neighbours, never the site itself, and the relation is symmetric
    for i in range(N):
        assert len(set(table[i])) == M and i not in table[i]
        for j in table[i]:
            assert i in table[j]
    # same-colour sites share no bond, every colour class is non-empty and equal-sized
    col = np.array([orc.colour_of(nbr, dims, i) for i in range(N)])
    for i in range(N):
        assert all(col[j] != col[i] for j in table[i])
    counts = np.bincount(col, minlength=orc.num_colours(nbr))
    assert len(counts) == orc.num_colours(nbr) and np.all(counts == N // orc.num_colours(nbr))


def test_neighbour_order_explicit(orc):
    # VN4 on 6x8: site (x=2, y=3) -> +x, -x, +y, -y
    dims = (6, 8)
    i = 2 + 6 * 3
    assert list(orc.neighbours_of(0, dims, i)) == [3 + 18, 1 + 18, 2 + 24, 2 + 12]
    # Moore8 adds (+1,+1), (-1,-1), (+1,-1), (-1,+1)
    assert list(orc.neighbours_of(1, dims, i))[4:] == [3 + 24, 1 + 12, 3 + 12, 1 + 24]
    # wrap-around at the origin
    assert list(orc.neighbours_of(0, dims, 0)) == [1, 5, 6, 42]
    # Moore26 starts at (dx,dy,dz) = (-1,-1,-1) and ends at (+1,+1,+1)
    d3 = (4, 6, 8)
    j = 1 + 4 * (2 + 6 * 3)
    nb = list(orc.neighbours_of(3, d3, j))
    assert nb[0] == 0 + 4 * (1 + 6 * 2) and nb[-1] == 2 + 4 * (3 + 6 * 4)
    assert nb[12] == 0 + 4 * (2 + 6 * 3) and nb[13] == 2 + 4 * (2 + 6 * 3)  # (-1,0,0), (+1,0,0)


def _bonds(nbr, dims):
    """Every bond of the periodic lattice once, from an independent offset list."""
    if len(dims) == 2:
        Lx, Ly = dims
        Lz = 1
    else:
        Lx, Ly, Lz = dims
    half = {0: [(1, 0, 0), (0, 1, 0)],
            1: [(1, 0, 0), (0, 1, 0), (1, 1, 0), (1, -1, 0)],
            2: [(1, 0, 0), (0, 1, 0), (0, 0, 1)],
            3: [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                if (dz, dy, dx) > (0, 0, 0)]}[nbr]
    z, y, x = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    a = (x + Lx * (y + Ly * z)).ravel()
    out = []
    for dx, dy, dz in half:
        b = ((x + dx) % Lx + Lx * (((y + dy) % Ly) + Ly * ((z + dz) % Lz))).ravel()
        out.append(np.stack([a, b], 1))
    return np.concatenate(out)


def hamiltonian_fx(spins, bonds, J_fx, B):
    s = np.asarray(spins).ravel()
    return int(J_fx) * int(np.sum(s[bonds[:, 0]] != s[bonds[:, 1]])) + int(np.sum(np.asarray(B, np.int64)[s]))


@pytest.mark.parametrize("nbr,dims", NBR_CASES)
def test_delta_energy_equals_hamiltonian_difference(orc, nbr, dims):
    rng = np.random.default_rng(11 + nbr)
    bonds = _bonds(nbr, dims)
    assert len(bonds) == int(np.prod(dims)) * orc.num_neighbours(nbr) // 2
    for Q, J_fx in [(2, 65536), (3, 65536), (7, 12345)]:
        B = rng.integers(-40000, 40000, size=Q)
        for _ in range(25):
            s = rng.integers(0, Q, size=int(np.prod(dims))).astype(np.int32)
            i = int(rng.integers(0, s.size))
            qn = int(rng.integers(0, Q))
            s2 = s.copy()
            s2[i] = qn
            want = hamiltonian_fx(s2, bonds, J_fx, B) - hamiltonian_fx(s, bonds, J_fx, B)
            assert orc.delta_energy(s, nbr, dims, J_fx, B, i, qn) == want


def test_delta_energy_hand_cases(orc):
    # 4x4 VN4, site (1,1) surrounded by three 2s and one 1; bulk B = [0, 100, 300]
    s = np.zeros((4, 4), dtype=np.int32)
    s[1, 1] = 1
    s[1, 2] = 2; s[1, 0] = 2; s[0, 1] = 2; s[2, 1] = 1
    B = [0, 100, 300]
    i = 1 + 4 * 1
    # 1 -> 2: unlike bonds 3 -> 1, bulk +200
    assert orc.delta_energy(s, 0, (4, 4), 65536, B, i, 2) == 65536 * (1 - 3) + 200
    # 1 -> 0: unlike bonds 3 -> 4, bulk -100
    assert orc.delta_energy(s, 0, (4, 4), 65536, B, i, 0) == 65536 * (4 - 3) - 100
    # 1 -> 1: nothing
    assert orc.delta_energy(s, 0, (4, 4), 65536, B, i, 1) == 0
