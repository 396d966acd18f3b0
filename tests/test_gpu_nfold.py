"""GPU parity of the n-fold way (the rejection-free, continuous-time
counterpart of the Metropolis dynamics named in Sec. 1 and Sec. 4) against
the oracle: the final spins, the time of the last event and the event count
must be identical (integer state: bit-exact; the clock: the same double).

Cases span every neighbourhood and spin type, ragged lattices (N not a
multiple of 64), a lattice with two tree levels run over several launches,
pair bond energies, the symmetric trial mode, runs split between calls,
batches of unequal lattices, a lattice without events, snapshots, a run
after red/black sweeps, the host-side argument checks, and the waiting-time
variates of the event kernel on their own (both paths of the run
measurement).
"""
import numpy as np
import pytest

import oracle
import paper_1007_3509_amd as hmc

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _energies(Q, seed, lo=-30000, hi=30000):
    return np.random.default_rng(seed).integers(lo, hi, size=Q).astype(np.int32)


def _gpu_run(dims, nbr, Q, B, kT, windows, seed, vseed, spin=hmc.HMC_I16, proposal=0, Jp=None):
    say(f"[gpu] nfold dims={dims} nbr={nbr} Q={Q} spin={spin} prop={proposal} pair={Jp is not None} "
        f"kT={kT} windows={windows}")
    with hmc.Lattice(dims, nbr, Q, voronoi_seed=vseed, spin=spin, proposal=proposal) as lat:
        lat.set_grain_energy(B)
        if Jp is not None:
            lat.set_pair_energy(Jp)
        start = lat.spins().astype(np.int32)
        for w in windows:
            lat.nfold(kT, w, seed)
        return start, lat.spins().astype(np.int32), lat.nfold_clock()


def _oracle_run(start, nbr, dims, B, kT, windows, seed, proposal=0, Jp=None):
    t_end = 0.0
    for w in windows:
        t_end = t_end + float(w)
    s, t_last, ne, _ = oracle.nfold(start, nbr, dims, B, kT, seed, t_end, proposal=proposal, Jp=Jp)
    return s, t_end, t_last, ne


CASES = [
    # dims, nbr, Q, spin, kT, mcs
    ((50, 38), hmc.HMC_VN4, 40, hmc.HMC_I16, 0.4, 3.0),
    ((64, 64), hmc.HMC_VN4, 25, hmc.HMC_I32, 0.9, 1.5),
    ((40, 36), hmc.HMC_MOORE8, 30, hmc.HMC_I16, 0.5, 2.0),
    ((12, 10, 14), hmc.HMC_VN6, 30, hmc.HMC_I32, 0.6, 2.0),
    ((16, 12, 10), hmc.HMC_VN6, 40, hmc.HMC_I16, 0.3, 2.5),
    ((8, 10, 8), hmc.HMC_MOORE26, 15, hmc.HMC_I16, 0.7, 1.5),
]


@pytest.mark.parametrize("dims,nbr,Q,spin,kT,mcs", CASES)
def test_nfold_matches_oracle(dims, nbr, Q, spin, kT, mcs):
    B = _energies(Q, Q + nbr)
    start, got, (t_now, t_last, ne) = _gpu_run(dims, nbr, Q, B, kT, [mcs], 77, 5 + nbr, spin=spin)
    want, t_end, w_last, w_ne = _oracle_run(start, nbr, dims, B, kT, [mcs], 77)
    say(f"  events {ne} (oracle {w_ne}), t_last {t_last!r} (oracle {w_last!r})")
    assert w_ne > 50
    assert np.array_equal(got, want)
    assert (ne, t_last, t_now) == (w_ne, w_last, t_end)


def test_nfold_two_levels_and_several_launches():
    """256^2 sites: a two-level tree (1024 runs of 64, 16 sums above) and
    more events than one launch executes."""
    dims, nbr, Q, kT = (256, 256), hmc.HMC_VN4, 300, 1.5
    B = _energies(Q, 9, -8000, 8000)
    start, got, (t_now, t_last, ne) = _gpu_run(dims, nbr, Q, B, kT, [10.0], 5, 31)
    want, t_end, w_last, w_ne = _oracle_run(start, nbr, dims, B, kT, [10.0], 5)
    say(f"  events {ne} (oracle {w_ne})")
    assert w_ne > 1 << 15
    assert np.array_equal(got, want) and (ne, t_last, t_now) == (w_ne, w_last, t_end)


def test_nfold_pair_energies():
    dims, nbr, Q, kT = (48, 40), hmc.HMC_VN4, 20, 0.5
    A = np.triu(np.random.default_rng(3).integers(1000, 80000, size=(Q, Q)), 1)
    Jp = (A + A.T).astype(np.int32)
    B = _energies(Q, 4)
    start, got, (t_now, t_last, ne) = _gpu_run(dims, nbr, Q, B, kT, [2.0], 8, 12, Jp=Jp)
    want, t_end, w_last, w_ne = _oracle_run(start, nbr, dims, B, kT, [2.0], 8, Jp=Jp)
    assert w_ne > 50
    assert np.array_equal(got, want) and (ne, t_last, t_now) == (w_ne, w_last, t_end)


def test_nfold_pair_energies_moore8():
    dims, nbr, Q, kT = (32, 28), hmc.HMC_MOORE8, 12, 0.6
    A = np.triu(np.random.default_rng(5).integers(0, 60000, size=(Q, Q)), 1)
    Jp = (A + A.T).astype(np.int32)
    B = _energies(Q, 6)
    start, got, (t_now, t_last, ne) = _gpu_run(dims, nbr, Q, B, kT, [1.5], 9, 13, Jp=Jp)
    want, t_end, w_last, w_ne = _oracle_run(start, nbr, dims, B, kT, [1.5], 9, Jp=Jp)
    assert np.array_equal(got, want) and (ne, t_last, t_now) == (w_ne, w_last, t_end)


@pytest.mark.parametrize("nbr,dims,Q", [(hmc.HMC_VN4, (20, 18), 5), (hmc.HMC_VN6, (8, 6, 6), 3),
                                        (hmc.HMC_VN4, (16, 16), 65)])
def test_nfold_symmetric_trial_mode(nbr, dims, Q):
    B = _energies(Q, 20 + Q)
    start, got, (t_now, t_last, ne) = _gpu_run(dims, nbr, Q, B, 1.5, [2.0], 3, 2, proposal=1)
    want, t_end, w_last, w_ne = _oracle_run(start, nbr, dims, B, 1.5, [2.0], 3, proposal=1)
    assert w_ne > 50
    assert np.array_equal(got, want) and (ne, t_last, t_now) == (w_ne, w_last, t_end)


def test_nfold_split_run_equals_one_run():
    dims, nbr, Q, kT = (40, 30), hmc.HMC_VN4, 30, 0.5
    B = _energies(Q, 2)
    windows = [0.5, 1.2, 0.0, 0.3, 1.0]
    start, got, (t_now, t_last, ne) = _gpu_run(dims, nbr, Q, B, kT, windows, 21, 4)
    want, t_end, w_last, w_ne = _oracle_run(start, nbr, dims, B, kT, windows, 21)
    assert np.array_equal(got, want) and (ne, t_last, t_now) == (w_ne, w_last, t_end)
    _, one, (t1, l1, n1) = _gpu_run(dims, nbr, Q, B, kT, [t_end], 21, 4)
    assert np.array_equal(one, got) and (n1, l1) == (ne, t_last)


def test_nfold_batch_of_unequal_lattices():
    specs = [((50, 38), 40, 0.4, 101), ((64, 64), 25, 0.8, 102), ((16, 16), 6, 0.5, 103),
             ((128, 96), 150, 0.35, 104), ((4, 4), 3, 1.5, 105), ((30, 24), 1, 0.5, 106)]
    lats, starts, Bs = [], [], []
    try:
        for k, (dims, Q, kT, vs) in enumerate(specs):
            lat = hmc.Lattice(dims, hmc.HMC_VN4, Q, voronoi_seed=vs)
            B = _energies(Q, 200 + k)
            lat.set_grain_energy(B)
            lats.append(lat)
            starts.append(lat.spins().astype(np.int32))
            Bs.append(B)
        kTs = [s[2] for s in specs]
        seeds = [1000 + k for k in range(len(specs))]
        say(f"[gpu] nfold batch of {len(lats)}")
        hmc.hmc_nfold_batch(lats, kTs, 1.5, seeds)
        hmc.hmc_nfold_batch(lats, kTs, 0.5, seeds)
        for k, lat in enumerate(lats):
            want, t_end, w_last, w_ne = _oracle_run(starts[k], hmc.HMC_VN4, specs[k][0], Bs[k], kTs[k], [1.5, 0.5],
                                                    seeds[k])
            t_now, t_last, ne = lat.nfold_clock()
            assert np.array_equal(lat.spins().astype(np.int32), want), k
            assert (ne, t_last, t_now) == (w_ne, w_last, t_end), k
        assert lats[-1].nfold_clock()[2] == 0     # one grain: no event
    finally:
        for lat in lats:
            lat.close()


def test_nfold_single_grain_has_no_event():
    with hmc.Lattice((32, 32), hmc.HMC_VN4, 1, voronoi_seed=1) as lat:
        lat.set_nfold_clock(2.0, 1.5, 9)
        lat.nfold(0.5, 10.0, 3)
        assert lat.nfold_clock() == (12.0, 1.5, 9)
        assert np.all(lat.spins() == 0)


def test_nfold_snapshot_restores_the_clock():
    with hmc.Lattice((40, 40), hmc.HMC_MOORE8, 20, voronoi_seed=6) as lat:
        lat.set_grain_energy(_energies(20, 7))
        lat.nfold(0.6, 0.5, 4)
        hmc.hmc_snapshot(lat.h)
        c0, s0 = lat.nfold_clock(), lat.spins()
        lat.nfold(0.6, 1.0, 4)
        c1, s1 = lat.nfold_clock(), lat.spins()
        hmc.hmc_restore(lat.h)
        assert lat.nfold_clock() == c0 and np.array_equal(lat.spins(), s0)
        lat.nfold(0.6, 1.0, 4)
        assert lat.nfold_clock() == c1 and np.array_equal(lat.spins(), s1)


def test_nfold_after_red_black_sweeps():
    dims, nbr, Q = (48, 32), hmc.HMC_VN4, 30
    B = _energies(Q, 8)
    with hmc.Lattice(dims, nbr, Q, voronoi_seed=9) as lat:
        lat.set_grain_energy(B)
        start = lat.spins().astype(np.int32)
        lat.sweep(0.5, 7, 11)
        lat.nfold(0.5, 1.0, 12)
        mid = oracle.sweep(start, nbr, dims, B, 0.5, 7, 11)
        want, t_last, ne, _ = oracle.nfold(mid, nbr, dims, B, 0.5, 12, 1.0)
        assert np.array_equal(lat.spins().astype(np.int32), want)
        assert lat.nfold_clock() == (1.0, t_last, ne)
        assert lat.mcs == 7


@pytest.mark.parametrize("window", [4, 7, 16, 64])
def test_nfold_waiting_times_match_oracle(window):
    """The event kernel's von Neumann variates, bit for bit: window 64 is the
    event loop's (a decreasing run that ends inside the wave's 64 words is
    measured in one step), the smaller windows send most runs, or all of
    them, down the word-by-word path that a long run takes.  The event
    numbers cross 2^32."""
    seed, n0, count = 0x9E3779B97F4A7C15, (1 << 32) - 3000, 60000
    say(f"[gpu] nfold exponentials window={window} n0={n0} count={count}")
    got = hmc.hmc_nfold_exponentials(seed, n0, count, window)
    want = oracle.nfold_exponentials(seed, n0, count)
    assert np.array_equal(got, want)
    assert len(np.unique(got >> 32)) > 5      # K reaches several integers


def test_nfold_argument_checks():
    with hmc.Lattice((512, 512), hmc.HMC_VN4, 10, voronoi_seed=1) as big:
        with pytest.raises(hmc.HmcError, match="LDS"):
            big.nfold(0.5, 1.0, 1)
    with hmc.Lattice((32, 32), hmc.HMC_VN4, 10, voronoi_seed=1) as a, \
            hmc.Lattice((32, 32), hmc.HMC_MOORE8, 10, voronoi_seed=1) as b, \
            hmc.Lattice((32, 32), hmc.HMC_VN4, 70, voronoi_seed=1, proposal=1) as u:
        with pytest.raises(hmc.HmcError, match="twice"):
            hmc.hmc_nfold_batch([a, a], [0.5, 0.5], 1.0, [1, 2])
        with pytest.raises(hmc.HmcError, match="share"):
            hmc.hmc_nfold_batch([a, b], [0.5, 0.5], 1.0, [1, 2])
        with pytest.raises(hmc.HmcError, match="Q <= 65"):
            u.nfold(0.5, 1.0, 1)
        with pytest.raises(hmc.HmcError, match="mcs"):
            a.nfold(0.5, -1.0, 1)
        with pytest.raises(hmc.HmcError, match="kT"):
            a.nfold(0.0, 1.0, 1)
        with pytest.raises(hmc.HmcError, match="t_last <= t_now"):
            a.set_nfold_clock(1.0, 2.0, 0)
        a.set_site_energy(np.zeros((32, 32), np.int32))
        with pytest.raises(hmc.HmcError, match="per-grain"):
            a.nfold(0.5, 1.0, 1)
        assert a.nfold_clock() == (0.0, 0.0, 0)


def test_nfold_batch_with_many_temperatures():
    """More temperatures in one batch than threshold tables kept between
    calls, twice with other temperatures: every lattice keeps its own table."""
    lats, starts, Bs = [], [], []
    try:
        for k in range(7):
            lat = hmc.Lattice((24, 20 + 2 * k), hmc.HMC_VN4, 10 + k, voronoi_seed=300 + k)
            B = _energies(10 + k, 400 + k)
            lat.set_grain_energy(B)
            lats.append(lat)
            Bs.append(B)
        for rnd, base in enumerate((0.3, 0.55)):
            starts = [lat.spins().astype(np.int32) for lat in lats]
            clocks = [lat.nfold_clock() for lat in lats]
            kTs = [base + 0.05 * k for k in range(7)]
            seeds = [50 + k for k in range(7)]
            say(f"[gpu] nfold batch round {rnd}: kT {kTs}")
            hmc.hmc_nfold_batch(lats, kTs, 1.0, seeds)
            for k, lat in enumerate(lats):
                t_end = clocks[k][0] + 1.0
                want, w_last, w_ne, _ = oracle.nfold(starts[k], hmc.HMC_VN4, lat.dims, Bs[k], kTs[k], seeds[k], t_end,
                                                     t_last=clocks[k][1], n_events=clocks[k][2])
                assert np.array_equal(lat.spins().astype(np.int32), want), (rnd, k)
                assert lat.nfold_clock() == (t_end, w_last, w_ne), (rnd, k)
    finally:
        for lat in lats:
            lat.close()


def test_nfold_driven_flat_strip():
    """A flat strip of a grain with higher bulk energy at low temperature
    (thermally activated kinks): spins set from the host, parity with the
    oracle, and the strip shrinks."""
    s = np.zeros((64, 96), np.int32)
    s[16:48, :] = 1
    B = np.array([0, 19661], np.int32)
    with hmc.Lattice((96, 64), hmc.HMC_VN4, 2) as lat:
        lat.set_spins(s)
        lat.set_grain_energy(B)
        lat.nfold(0.3, 60.0, 17)
        want, t_last, ne, _ = oracle.nfold(s, hmc.HMC_VN4, (96, 64), B, 0.3, 17, 60.0)
        assert np.array_equal(lat.spins().astype(np.int32), want)
        assert lat.nfold_clock() == (60.0, t_last, ne)
        assert ne > 100 and want.sum() < s.sum()
