"""Exhaustive pins of the oracle's Markov chain on a 4x4 periodic Q=2 lattice.

The Red/Black scheme (Sec. 4) updates one colour class per half step; within
a class the trials are independent, so one half step is the product of the
single-site Metropolis kernels of its sites.  These tests build that product
exactly over all 2^16 states, independently of the oracle's sweep loop:

* symmetric trial mode: the Boltzmann distribution of Eq. (7) with the bulk
  term is invariant under one MC step (up to the 2^-32 quantisation of the
  acceptance threshold);
* both trial modes: the exact distribution after one MC step from a fixed
  start state matches many oracle runs (chi-square), which pins the loop
  order, the colour order, the synchronous half step and the trial-spin draw;
* neighbour-spin trials make the Q uniform states absorbing.
"""
import numpy as np
import pytest
from scipy import stats

L = 4
N = L * L
STATES = np.arange(1 << N, dtype=np.int64)


def _geometry(nbr):
    """Independent neighbour lists and colours for the 4x4 periodic lattice."""
    offs = [(1, 0), (-1, 0), (0, 1), (0, -1)]
    if nbr == 1:
        offs += [(1, 1), (-1, -1), (1, -1), (-1, 1)]
    nb = np.zeros((N, len(offs)), dtype=np.int64)
    col = np.zeros(N, dtype=np.int64)
    for y in range(L):
        for x in range(L):
            i = x + L * y
            nb[i] = [((x + dx) % L) + L * ((y + dy) % L) for dx, dy in offs]
            col[i] = ((x + y) & 1) if nbr == 0 else ((x & 1) | ((y & 1) << 1))
    return nb, col


def _bits(states, i):
    return (states >> i) & 1


def _accept_and_propose(orc, states, i, nb, proposal, B, kT, J_fx):
    """Per state: probability that site i flips during its half step."""
    M = nb.shape[1]
    q = _bits(states, i)
    n_other = np.zeros_like(q)
    for j in nb[i]:
        n_other += (_bits(states, j) != q)
    n_same = M - n_other
    d = J_fx * (n_same - n_other) + np.where(q == 0, B[1] - B[0], B[0] - B[1])
    uniq = np.unique(d[d > 0])
    table = {int(v): orc.threshold(int(v), kT) / 2.0 ** 32 for v in uniq}
    acc = np.ones(len(states))
    pos = d > 0
    acc[pos] = np.array([table[int(v)] for v in d[pos]])
    prop = n_other / M if proposal == 0 else np.ones(len(states))
    return prop * acc


def _apply_half_step(orc, v, colour, nb, col, proposal, B, kT, J_fx):
    """v <- v K_colour over all 2^16 states (sites of one colour commute)."""
    for i in np.nonzero(col == colour)[0]:
        a = _accept_and_propose(orc, STATES, int(i), nb, proposal, B, kT, J_fx)
        partner = STATES ^ (1 << int(i))
        v = v * (1.0 - a) + v[partner] * a[partner]
    return v


def _boltzmann(nb, B, kT, J_fx):
    e = np.zeros(len(STATES))
    for i in range(N):
        for j in nb[i]:   # every bond is seen from both ends: count half each time
            e += 0.5 * J_fx * (_bits(STATES, i) != _bits(STATES, j))
        e += np.where(_bits(STATES, i) == 0, B[0], B[1])
    w = np.exp(-(e - e.min()) / (65536.0 * kT))
    return w / w.sum()


@pytest.mark.parametrize("nbr", [0, 1])
@pytest.mark.parametrize("kT,h", [(1.0, 0), (1.4, 6554), (2.6, -13107)])
def test_boltzmann_invariant_symmetric_trials(orc, nbr, kT, h):
    kT = float(np.float32(kT))
    nb, col = _geometry(nbr)
    B = np.array([0, h])
    pi = _boltzmann(nb, B, kT, 65536)
    v = pi.copy()
    for c in range(int(col.max()) + 1):
        v = _apply_half_step(orc, v, c, nb, col, 1, B, kT, 65536)
    assert np.max(np.abs(v - pi)) / pi.max() < 1e-8
    # the same kernel built with a wrong temperature scale is visibly not invariant
    w = pi.copy()
    for c in range(int(col.max()) + 1):
        w = _apply_half_step(orc, w, c, nb, col, 1, B, 2 * kT, 65536)
    assert np.max(np.abs(w - pi)) / pi.max() > 1e-4


def _exact_one_mcs(orc, start, nbr, proposal, B, kT, J_fx):
    nb, col = _geometry(nbr)
    v = np.zeros(len(STATES))
    v[start] = 1.0
    for c in range(int(col.max()) + 1):
        v = _apply_half_step(orc, v, c, nb, col, proposal, B, kT, J_fx)
    return v


def _chi2_pvalue(counts, probs, K):
    exp = probs * K
    keep = exp >= 5
    o = list(counts[keep]) + [counts[~keep].sum()]
    e = list(exp[keep]) + [exp[~keep].sum()]
    if e[-1] < 5:
        o[-2] += o[-1]; e[-2] += e[-1]
        o, e = o[:-1], e[:-1]
    o, e = np.array(o, float), np.array(e, float)
    stat = ((o - e) ** 2 / e).sum()
    return stats.chi2.sf(stat, len(e) - 1), len(e)


def _to_bits(spins):
    s = np.asarray(spins).ravel()
    return int(np.sum(s.astype(np.int64) << np.arange(N)))


def _from_bits(b):
    return ((b >> np.arange(N)) & 1).astype(np.int32).reshape(L, L)


CASES = [  # nbr, proposal, kT, B, start pattern seed
    (0, 0, 1.4, (0, 0), 5),
    (0, 0, 0.5, (0, 13107), 6),
    (0, 1, 1.0, (0, -6554), 7),
    (1, 0, 1.0, (0, 3277), 8),
    (1, 1, 2.0, (0, 0), 9),
]


@pytest.mark.parametrize("nbr,proposal,kT,B,pat", CASES)
def test_one_step_distribution_matches_oracle(orc, nbr, proposal, kT, B, pat):
    kT = float(np.float32(kT))
    rng = np.random.default_rng(pat)
    start = rng.integers(0, 2, size=(L, L)).astype(np.int32)
    probs = _exact_one_mcs(orc, _to_bits(start), nbr, proposal, np.array(B), kT, 65536)
    assert abs(probs.sum() - 1.0) < 1e-12
    K = 40000
    counts = np.zeros(len(STATES), dtype=np.int64)
    for t in range(K):
        out = orc.sweep(start, nbr, (L, L), B, kT, 1, seed=1000 + pat, mcs0=t, proposal=proposal)
        counts[_to_bits(out)] += 1
    p, ncat = _chi2_pvalue(counts, probs, K)
    assert ncat >= 3
    assert p > 1e-4, (p, ncat)


def test_one_step_distribution_detects_wrong_trial_rule(orc):
    """The same comparison rejects a chain whose trial draw differs
    (symmetric trials simulated, neighbour-spin trials predicted)."""
    kT = float(np.float32(1.4))
    rng = np.random.default_rng(5)
    start = rng.integers(0, 2, size=(L, L)).astype(np.int32)
    probs = _exact_one_mcs(orc, _to_bits(start), 0, 0, np.array([0, 0]), kT, 65536)
    K = 20000
    counts = np.zeros(len(STATES), dtype=np.int64)
    for t in range(K):
        out = orc.sweep(start, 0, (L, L), [0, 0], kT, 1, seed=77, mcs0=t, proposal=1)
        counts[_to_bits(out)] += 1
    p, _ = _chi2_pvalue(counts, probs, K)
    assert p < 1e-6


@pytest.mark.parametrize("nbr,dims", [(0, (8, 6)), (1, (8, 6)), (2, (4, 6, 4)), (3, (4, 4, 6))])
def test_uniform_states_absorbing_with_neighbour_trials(orc, nbr, dims):
    for q in (0, 3):
        s = np.full(tuple(reversed(dims)), q, dtype=np.int32)
        out = orc.sweep(s, nbr, dims, [0, -300000, 5, 400000], 5.0, 20, seed=3)
        assert np.all(out == q)


def test_symmetric_trials_leave_uniform_states(orc):
    s = np.zeros((8, 8), dtype=np.int32)
    out = orc.sweep(s, 0, (8, 8), [0, 0], 5.0, 3, seed=3, proposal=1)
    assert np.any(out != 0)
