"""Pins of the oracle's n-fold way (the rejection-free, continuous-time
counterpart of the Metropolis dynamics that Sec. 1 and Sec. 4 name as the
alternative to red/black updating).

What fixes the answer independently of the oracle:

* the rates: every slot weight equals 2^32 min(1, exp(-dE/kT)) (floored) with
  dE the difference of a brute-force Eq. (7) Hamiltonian, for all four
  neighbourhoods and both trial modes;
* the exponential generator (von Neumann's method) against Exp(1): KS test,
  the geometric law of the integer part and the truncated-exponential law of
  the fraction;
* one event: the first waiting time is Exp(W / (S 2^32)) and the event is
  slot k of site i with probability w_ik / W (Bortz, Kalos, Lebowitz);
* the whole process: on a 3x3 Q=2 lattice the distribution of the state at
  time t equals the row of exp(G t) for the generator G built from the
  brute-force rates (both trial modes, VN4 and Moore8);
* stationarity: with the symmetric trial mode the time average of a long run
  matches the Boltzmann average of Eq. (7) by enumeration of all 2^16 states;
* invariants: a run split into windows equals one run; a single grain has no
  event; relabelling grains relabels the run.
"""
import math

import numpy as np
import pytest
from scipy import linalg, stats

OFFS = {0: [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0)],
        1: [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0)],
        2: [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)],
        3: [(a, b, c) for c in (-1, 0, 1) for b in (-1, 0, 1) for a in (-1, 0, 1) if (a, b, c) != (0, 0, 0)]}


def _energy(s3, nbr, J, B):
    """Eq. (7) read as J(1-delta), every bond once, plus B of each spin."""
    tot = 0
    for dx, dy, dz in OFFS[nbr]:
        t = np.roll(s3, shift=(-dz, -dy, -dx), axis=(0, 1, 2))
        tot += int(np.count_nonzero(s3 != t))
    assert tot % 2 == 0
    return J * (tot // 2) + int(np.asarray(B, dtype=np.int64)[s3].sum())


def _energy_pair(s3, nbr, Jp, B):
    """Eq. (7) with a bond energy per pair of spins, every bond once."""
    tot = 0
    for dx, dy, dz in OFFS[nbr]:
        t = np.roll(s3, shift=(-dz, -dy, -dx), axis=(0, 1, 2))
        tot += int(np.asarray(Jp, dtype=np.int64)[s3, t].sum())
    assert tot % 2 == 0
    return tot // 2 + int(np.asarray(B, dtype=np.int64)[s3].sum())


def _T(d, kT):
    """floor(2^32 exp(-d / (65536 kT))) with kT rounded to float32 first."""
    x = d / (65536.0 * float(np.float32(kT)))
    v = math.ldexp(math.exp(-x), 32)
    return 0xFFFFFFFF if v >= 4294967295.0 else int(math.floor(v))


def _brute_weights(s3, nbr, J, B, kT, proposal, Jp=None):
    """Slot weights from energy differences of the full Hamiltonian."""
    Z, Y, X = s3.shape
    Q = len(B)
    S = len(OFFS[nbr]) if proposal == 0 else Q - 1
    out = np.zeros((s3.size, S), dtype=np.uint64)
    energy = (lambda u: _energy(u, nbr, J, B)) if Jp is None else (lambda u: _energy_pair(u, nbr, Jp, B))
    E0 = energy(s3)
    for z in range(Z):
        for y in range(Y):
            for x in range(X):
                i = x + X * (y + Y * z)
                q = int(s3[z, y, x])
                for k in range(S):
                    if proposal == 0:
                        dx, dy, dz = OFFS[nbr][k]
                        c = int(s3[(z + dz) % Z, (y + dy) % Y, (x + dx) % X])
                        if c == q:
                            continue
                    else:
                        c = (q + 1 + k) % Q
                    t = s3.copy()
                    t[z, y, x] = c
                    d = energy(t) - E0
                    out[i, k] = (1 << 32) if d <= 0 else _T(d, kT)
    return out


@pytest.mark.parametrize("nbr,shape,proposal", [(0, (1, 6, 8), 0), (1, (1, 8, 6), 0), (2, (4, 4, 6), 0),
                                                (3, (4, 4, 4), 0), (0, (1, 6, 6), 1), (2, (4, 4, 4), 1)])
def test_weights_are_metropolis_rates_of_the_hamiltonian(orc, nbr, shape, proposal):
    rng = np.random.default_rng(40 + nbr + 10 * proposal)
    Q = 4
    s3 = rng.integers(0, Q, size=shape).astype(np.int32)
    B = rng.integers(-40000, 40000, size=Q).astype(np.int32)
    J = 65536
    dims = (shape[2], shape[1], shape[0])
    for kT in (0.3, 1.1):
        got = orc.nfold_weights(s3, nbr, dims, B, kT, J_fx=J, proposal=proposal)
        want = _brute_weights(s3, nbr, J, B, kT, proposal)
        assert np.array_equal(got, want)


@pytest.mark.parametrize("nbr,shape", [(0, (1, 8, 8)), (2, (4, 4, 4))])
def test_weights_without_bulk_energy_include_zero_changes(orc, nbr, shape):
    """With B = 0 many trials leave the energy unchanged (d = 0), which the
    rule accepts with certainty: weight 2^32, not the table's 2^32 - 1."""
    rng = np.random.default_rng(60 + nbr)
    s3 = rng.integers(0, 3, size=shape).astype(np.int32)
    B = np.zeros(3, np.int32)
    dims = (shape[2], shape[1], shape[0])
    got = orc.nfold_weights(s3, nbr, dims, B, 0.5)
    want = _brute_weights(s3, nbr, 65536, B, 0.5, 0)
    assert np.array_equal(got, want)
    assert np.count_nonzero(got == (1 << 32)) > 10


@pytest.mark.parametrize("nbr,shape", [(0, (1, 6, 8)), (1, (1, 6, 6)), (2, (4, 4, 4))])
def test_pair_weights_are_rates_of_the_pair_hamiltonian(orc, nbr, shape):
    rng = np.random.default_rng(70 + nbr)
    Q = 5
    s3 = rng.integers(0, Q, size=shape).astype(np.int32)
    A = np.triu(rng.integers(0, 90000, size=(Q, Q)), 1)
    Jp = (A + A.T).astype(np.int32)
    B = rng.integers(-30000, 30000, size=Q).astype(np.int32)
    dims = (shape[2], shape[1], shape[0])
    got = orc.nfold_weights(s3, nbr, dims, B, 0.6, Jp=Jp)
    assert np.array_equal(got, _brute_weights(s3, nbr, 0, B, 0.6, 0, Jp=Jp))


def test_uniform_pair_table_is_the_uniform_run(orc):
    rng = np.random.default_rng(71)
    Q, dims = 6, (12, 10)
    s = rng.integers(0, Q, size=(10, 12)).astype(np.int32)
    B = rng.integers(-20000, 20000, size=Q).astype(np.int32)
    Jp = (65536 * (1 - np.eye(Q))).astype(np.int32)
    a = orc.nfold(s, 0, dims, B, 0.7, seed=4, t_end=2.5)
    b = orc.nfold(s, 0, dims, B, 0.7, seed=4, t_end=2.5, Jp=Jp)
    assert np.array_equal(a[0], b[0]) and a[1:] == b[1:]


def test_selection_is_the_first_cumulative_weight_above_r(orc):
    """Bortz et al.'s choice, at the boundaries of the cumulative sums: entry
    i is taken for sum_{j<i} w_j <= r < sum_{j<=i} w_j; zero weights never."""
    w = np.zeros(300, dtype=np.uint64)
    w[[3, 64, 65, 130, 299]] = [5, 1, 7, 2**40, 9]
    cum = np.cumsum(w.astype(object))
    for i in np.flatnonzero(w):
        lo = int(cum[i] - w[i])
        for r in (lo, lo + int(w[i]) - 1):
            assert orc.nfold_select(w, r) == (int(i), r - lo)
    assert orc.nfold_select(w, int(cum[-1]))[0] == -1
    assert orc.nfold_select(np.zeros(5, np.uint64), 0)[0] == -1


def test_von_neumann_exponential_is_exp1(orc):
    E = orc.nfold_exponentials(seed=7, n0=0, count=200000).astype(np.float64) / 2.0 ** 32
    assert stats.kstest(E, "expon").pvalue > 1e-3
    K = np.floor(E).astype(int)
    frac = E - K
    # integer part: P(K = k) = e^-k (1 - e^-1)
    kmax = 8
    obs = np.array([np.count_nonzero(K == k) for k in range(kmax)] + [np.count_nonzero(K >= kmax)])
    p = np.array([math.exp(-k) * (1 - math.exp(-1)) for k in range(kmax)] + [math.exp(-kmax)])
    assert stats.chisquare(obs, p * len(E)).pvalue > 1e-3
    # fraction: density e^-x / (1 - e^-1) on [0, 1), independent of K
    cdf = lambda x: (1 - np.exp(-x)) / (1 - math.exp(-1))  # noqa: E731
    assert stats.kstest(frac, cdf).pvalue > 1e-3
    assert stats.kstest(frac[K >= 1], cdf).pvalue > 1e-3


def test_one_event_follows_the_rates(orc):
    """First waiting time ~ Exp(W / (S 2^32)); the event is (i, k) with
    probability w_ik / W."""
    s = np.zeros((8, 8), dtype=np.int32)
    s[2, 2] = 1                       # an isolated site of grain 1
    s[5, 4:7] = 2                     # a short bar of grain 2
    B = np.array([0, 20000, -15000], dtype=np.int32)
    kT = 0.7
    w = orc.nfold_weights(s, 0, (8, 8), B, kT).astype(np.float64)
    W = w.sum()
    rate = W / (4 * 2.0 ** 32)
    n = 20000
    times, cells = np.zeros(n), []
    for r in range(n):
        out, t_last, ne, ex = orc.nfold(s, 0, (8, 8), B, kT, seed=1000 + r, t_end=1e9, max_events=1)
        assert ex == 1 and ne == 1
        times[r] = t_last
        (i,) = np.flatnonzero(out.reshape(-1) != s.reshape(-1))
        cells.append((int(i), int(out.reshape(-1)[i])))
    assert stats.kstest(times * rate, "expon").pvalue > 1e-3
    # which site and which new spin: the candidate spin of each slot
    nb = {i: orc.neighbours_of(0, (8, 8), i) for i in range(64)}
    expect = {}
    for i in range(64):
        for k in range(4):
            if w[i, k] > 0:
                key = (i, int(s.reshape(-1)[nb[i][k]]))
                expect[key] = expect.get(key, 0.0) + w[i, k] / W
    keys = sorted(expect)
    obs = np.array([sum(1 for c in cells if c == key) for key in keys], dtype=float)
    assert sum(obs) == n
    exp_counts = np.array([expect[k] for k in keys]) * n
    assert _chisq_p(obs, exp_counts, 5) > 1e-3


def _chisq_p(obs, expc, min_expected):
    """Chi-square p-value with the bins below min_expected merged into one."""
    obs = np.asarray(obs, dtype=float)
    expc = np.asarray(expc, dtype=float)
    big = expc >= min_expected
    o, e = list(obs[big]), list(expc[big])
    if expc[~big].sum() > 0:
        o.append(obs[~big].sum())
        e.append(expc[~big].sum())
    return stats.chisquare(o, e).pvalue


def _generator(nbr, side, J, B, kT, proposal):
    """Continuous-time generator over all 2^(side^2) states of a Q=2 lattice,
    from the brute-force slot weights (rate = w / (S 2^32) per MC step)."""
    n = side * side
    S = len(OFFS[nbr]) if proposal == 0 else 1
    G = np.zeros((1 << n, 1 << n))
    for a in range(1 << n):
        s3 = np.array([(a >> b) & 1 for b in range(n)], dtype=np.int32).reshape(1, side, side)
        w = _brute_weights(s3, nbr, J, B, kT, proposal).astype(np.float64)
        for i in range(n):
            tot = w[i].sum()
            if tot > 0:
                G[a, a ^ (1 << i)] += tot / (S * 2.0 ** 32)   # Q = 2: every slot flips to the other spin
        G[a, a] = -G[a].sum()
    return G


@pytest.mark.parametrize("nbr,proposal,kT,t", [(0, 0, 0.8, 0.6), (1, 0, 1.3, 0.4), (0, 1, 0.9, 0.5)])
def test_state_distribution_matches_the_master_equation(orc, nbr, proposal, kT, t):
    side, J = 3, 65536
    B = np.array([0, 9000], dtype=np.int32)
    G = _generator(nbr, side, J, B, kT, proposal)
    s0 = np.array([[0, 1, 0], [1, 1, 0], [0, 0, 0]], dtype=np.int32)
    a0 = int(sum(int(v) << b for b, v in enumerate(s0.reshape(-1))))
    P = linalg.expm(G * t)[a0]
    n = 20000
    idx = np.zeros(n, dtype=np.int64)
    for r in range(n):
        out = orc.nfold(s0, nbr, (side, side), B, kT, seed=77 + r, t_end=t, proposal=proposal)[0]
        idx[r] = int(sum(int(v) << b for b, v in enumerate(out.reshape(-1))))
    obs = np.bincount(idx, minlength=len(P)).astype(float)
    assert _chisq_p(obs, P * n, 8) > 1e-4
    # the number of grain-1 sites, a coarse statistic with more power per bin
    ones = np.array([bin(a).count("1") for a in range(len(P))])
    o1 = np.bincount(ones[idx], minlength=side * side + 1).astype(float)
    e1 = np.array([P[ones == m].sum() for m in range(side * side + 1)]) * n
    assert _chisq_p(o1, e1, 5) > 1e-4


def test_symmetric_mode_samples_the_boltzmann_distribution(orc):
    """Time average of a long run (snapshots every 0.5 MC step) against the
    exact Boltzmann average of Eq. (7) over all 2^16 states of a 4x4 lattice."""
    side, J, kT = 4, 65536, 1.6
    B = np.array([0, 16000], dtype=np.int32)
    n = side * side
    a = np.arange(1 << n)
    bits = ((a[:, None] >> np.arange(n)[None, :]) & 1).astype(np.int32).reshape(-1, side, side)
    E = J * (np.count_nonzero(bits != np.roll(bits, -1, axis=2), axis=(1, 2)) +
             np.count_nonzero(bits != np.roll(bits, -1, axis=1), axis=(1, 2))) + B[1] * bits.sum(axis=(1, 2))
    beta = 1.0 / (65536.0 * float(np.float32(kT)))
    wB = np.exp(-(E - E.min()) * beta)
    mean_ones = float((wB * bits.sum(axis=(1, 2))).sum() / wB.sum())
    mean_E = float((wB * E).sum() / wB.sum())
    s = np.zeros((side, side), dtype=np.int32)
    t_last, ne = 0.0, 0
    burn, m, dt = 40, 16000, 0.5
    ones, en = np.zeros(m), np.zeros(m)
    for k in range(burn + m):
        s, t_last, ne, _ = orc.nfold(s, 0, (side, side), B, kT, seed=5, t_end=(k + 1) * dt, t_last=t_last,
                                     n_events=ne, proposal=1)
        if k >= burn:
            ones[k - burn] = s.sum()
            en[k - burn] = _energy(s[None], 0, J, B)
    # batch means for the standard error of correlated samples
    nb = 40
    se1 = ones.reshape(nb, -1).mean(axis=1).std(ddof=1) / math.sqrt(nb)
    seE = en.reshape(nb, -1).mean(axis=1).std(ddof=1) / math.sqrt(nb)
    assert abs(ones.mean() - mean_ones) < 4.5 * se1
    assert abs(en.mean() - mean_E) < 4.5 * seE


@pytest.mark.parametrize("nbr,dims", [(0, (16, 16)), (1, (12, 16)), (2, (6, 6, 8)), (3, (6, 6, 6))])
def test_split_run_equals_one_run(orc, nbr, dims):
    rng = np.random.default_rng(8 + nbr)
    Q = 5
    s = rng.integers(0, Q, size=tuple(reversed(dims))).astype(np.int32)
    B = rng.integers(-20000, 20000, size=Q).astype(np.int32)
    one = orc.nfold(s, nbr, dims, B, 0.6, seed=11, t_end=3.0)
    cur, tl, ne = s, 0.0, 0
    for t_end in (0.5, 1.7, 1.7, 3.0):
        cur, tl, ne, _ = orc.nfold(cur, nbr, dims, B, 0.6, seed=11, t_end=t_end, t_last=tl, n_events=ne)
    assert np.array_equal(cur, one[0]) and tl == one[1] and ne == one[2]
    assert one[2] > 20 and one[1] <= 3.0


def test_single_grain_has_no_event(orc):
    s = np.full((8, 8), 3, dtype=np.int32)
    out, tl, ne, ex = orc.nfold(s, 0, (8, 8), np.zeros(5, np.int32), 0.4, seed=1, t_end=100.0, t_last=2.5,
                                n_events=9)
    assert ex == 0 and ne == 9 and tl == 2.5 and np.array_equal(out, s)


def test_relabelling_grains_relabels_the_run(orc):
    rng = np.random.default_rng(12)
    Q, dims = 6, (12, 10)
    s = rng.integers(0, Q, size=(10, 12)).astype(np.int32)
    B = rng.integers(-20000, 20000, size=Q).astype(np.int32)
    perm = rng.permutation(Q)
    inv = np.argsort(perm)
    a = orc.nfold(s, 0, dims, B, 0.7, seed=3, t_end=2.0)
    b = orc.nfold(perm[s].astype(np.int32), 0, dims, B[inv], 0.7, seed=3, t_end=2.0)
    assert np.array_equal(perm[a[0]], b[0]) and a[1] == b[1] and a[2] == b[2]
