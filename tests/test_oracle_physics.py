"""Pins of the oracle's sweep against results that hold independently of it.

* Onsager: with symmetric trials, Q=2 and no bulk term, Eq. (7) read as
  J(1-delta) per bond is the square-lattice Ising model with coupling J/2, so
  the equilibrium fraction of unlike bonds has a closed form (Onsager 1944).
* Sec. 4, first validation case: a circular grain shrinks under capillarity
  alone with an area falling linearly in time, and with a bulk driving force
  the sharp-interface law of Sec. 3 (normal speed = mobility x (bulk jump +
  curvature x stiffness), Eqs. (5)-(6)) fits every curve with one pair of
  mobility and stiffness.
* A flat boundary does not drift without a bulk term and moves at a speed
  proportional to, and odd in, the bulk-energy difference (Eqs. (5)-(6)
  with zero curvature; mobility independent of the driving force, Sec. 1).
* Sec. 4, second validation case: the mean grain area of a polycrystal grows
  linearly in time.
* Sec. 5: under the Gaussian bulk energy of Eq. (9), orientations of lower
  bulk energy are favoured.
"""
import numpy as np
import pytest
from scipy import stats
from scipy.optimize import least_squares
from scipy.special import ellipk

import synth

THREADS = 8


def onsager_unlike_fraction(kT, J=1.0):
    K = J / (2.0 * kT)                       # Ising coupling J/2 over kT
    k = 2 * np.sinh(2 * K) / np.cosh(2 * K) ** 2
    u = -1 / np.tanh(2 * K) * (1 + 2 / np.pi * (2 * np.tanh(2 * K) ** 2 - 1) * ellipk(k * k))
    return (1 + u / 2) / 2                   # (1 - <s s'>) / 2 with <s s'> = -u/2


def test_onsager_reference_values():
    assert abs(onsager_unlike_fraction(1.0) - 0.063609) < 2e-6
    assert abs(onsager_unlike_fraction(2.0) - 0.360682) < 2e-6


def _unlike(s):
    return ((s != np.roll(s, 1, 0)).mean() + (s != np.roll(s, 1, 1)).mean()) / 2


@pytest.mark.parametrize("kT,start", [(1.0, "ordered"), (2.0, "random")])
def test_onsager_unlike_bond_fraction(orc, kT, start):
    L = 128
    s = np.zeros((L, L), np.int32) if start == "ordered" else synth.random_spins((L, L), 2, 5)
    s = orc.sweep(s, 0, (L, L), [0, 0], kT, 300, seed=9, proposal=1, threads=THREADS)
    vals = []
    for k in range(80):
        s = orc.sweep(s, 0, (L, L), [0, 0], kT, 10, seed=9, mcs0=300 + 10 * k, proposal=1,
                      threads=THREADS)
        vals.append(_unlike(s))
    batches = np.array(vals).reshape(8, 10).mean(1)
    err = batches.std(ddof=1) / np.sqrt(len(batches))
    assert abs(batches.mean() - onsager_unlike_fraction(kT)) < 4 * err + 2e-4


def _circle_run(orc, L, R0, db, seed, n, step):
    s = synth.circle_grain(L, R0)
    A = [s.sum()]
    for k in range(n // step):
        s = orc.sweep(s, 0, (L, L), [0, int(round(db * 65536))], 1.4, step, seed=seed,
                      mcs0=step * k, threads=THREADS)
        A.append(s.sum())
    return np.arange(len(A)) * step, np.array(A, float)


def test_circle_area_linear_in_time(orc):
    runs = [_circle_run(orc, 128, 40.0, 0.0, s, 1600, 50)[1] for s in (31, 32, 33, 34)]
    t = np.arange(len(runs[0])) * 50.0
    A = np.mean(runs, 0)
    m = (t >= 200) & (A > 0.15 * A[0])
    c = np.polyfit(t[m], A[m], 1)
    r2 = 1 - ((A[m] - np.polyval(c, t[m])) ** 2).sum() / ((A[m] - A[m].mean()) ** 2).sum()
    assert c[0] < 0 and r2 >= 0.99


def test_circle_sharp_interface_fit(orc):
    curves = {db: _circle_run(orc, 256, 80.0, db, 41, 1000, 50) for db in (0.0, 0.05, -0.05, 0.1, -0.1)}

    def model(p, db, t, A0):
        mob, gam = p
        a, out = A0, [A0]
        for k in range(int(t[-1])):
            r = np.sqrt(max(a, 1.0) / np.pi)
            a += 2 * np.pi * mob * (-db * r - gam)      # dA/dt = 2 pi r v_n
            if (k + 1) % 50 == 0:
                out.append(a)
        return np.array(out)

    def res(p):
        return np.concatenate([(model(p, db, t, A[0]) - A) / A[0] for db, (t, A) in curves.items()])

    fit = least_squares(res, [1.0, 0.5])
    mob, gam = fit.x
    assert mob > 0 and gam > 0
    assert np.sqrt(np.mean(fit.fun ** 2)) < 0.03
    assert np.max(np.abs(fit.fun)) < 0.1
    # higher bulk energy inside -> faster shrinkage
    assert curves[0.1][1][-1] < curves[0.05][1][-1] < curves[0.0][1][-1] < curves[-0.05][1][-1]


def _strip_velocity(orc, db, seed, Lx=64, Ly=128, n=600):
    s = synth.flat_strip(Lx, Ly)
    A = [s.sum()]
    for k in range(n // 50):
        s = orc.sweep(s, 0, (Lx, Ly), [0, int(round(db * 65536))], 1.4, 50, seed=seed, mcs0=50 * k,
                      threads=THREADS)
        A.append(s.sum())
    t = np.arange(len(A)) * 50.0
    return -np.polyfit(t, np.array(A, float), 1)[0] / (2 * Lx)


def test_flat_boundary_still_without_bulk_force(orc):
    Lx, Ly = 64, 128
    disp = []
    for s in range(8):
        st = synth.flat_strip(Lx, Ly)
        out = orc.sweep(st, 0, (Lx, Ly), [0, 0], 1.4, 600, seed=60 + s, threads=THREADS)
        disp.append((out.sum() - st.sum()) / (2 * Lx))
    disp = np.array(disp)
    assert abs(disp.mean()) < 3 * disp.std(ddof=1) / np.sqrt(len(disp)) + 0.5


def test_flat_boundary_velocity_linear_and_odd(orc):
    dbs = [-0.2, -0.1, -0.05, 0.05, 0.1, 0.2]
    v = {db: np.mean([_strip_velocity(orc, db, s) for s in (51, 52)]) for db in dbs}
    x = np.array(dbs)
    y = np.array([v[d] for d in dbs])
    c = np.polyfit(x, y, 1)
    r2 = 1 - ((y - np.polyval(c, x)) ** 2).sum() / ((y - y.mean()) ** 2).sum()
    assert c[0] > 0 and r2 >= 0.97
    for d in (0.05, 0.1, 0.2):
        assert abs(v[d] + v[-d]) < 0.3 * abs(v[d])


@pytest.mark.parametrize("kT", [0.5, 1.0])
def test_grain_growth_mean_area_linear(orc, kT):
    L, G = 128, 400
    s = orc.voronoi((L, L), G, 7)
    A = []
    for k in range(16):
        s = orc.sweep(s, 0, (L, L), np.zeros(G, np.int32), kT, 50, seed=8, mcs0=50 * k, threads=THREADS)
        A.append(orc.texture(s, G)[2])
    t = np.arange(1, 17) * 50.0
    A = np.array(A)
    m = t >= 200
    c = np.polyfit(t[m], A[m], 1)
    r2 = 1 - ((A[m] - np.polyval(c, t[m])) ** 2).sum() / ((A[m] - A[m].mean()) ** 2).sum()
    assert c[0] > 0 and r2 >= 0.95


def test_gaussian_bulk_energy_texture(orc):
    L, G = 192, 91 * 12
    b = synth.gaussian_orientation_energy()
    B = synth.quantise(b)
    areas = []
    for seed in (1, 2):
        s = orc.voronoi((L, L), G, 100 + seed) % 91
        s = orc.sweep(s, 0, (L, L), B, 1.0, 1500, seed=seed, threads=THREADS)
        areas.append(orc.texture(s, 91)[0])
    a = np.mean(areas, 0)
    rho, p = stats.spearmanr(b, a)
    assert rho < -0.5 and p < 1e-6
