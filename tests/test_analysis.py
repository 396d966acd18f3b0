"""Host-side analysis layer: the parametric links of Sec. 3 and the fits of
the boundary kinetics and of the texture Gaussian of Sec. 5, checked against
closed forms and exact synthetic data."""
import numpy as np
import pytest

from paper_1007_3509_amd import analysis as an


def test_links_round_trip_and_scaling():
    s = an.Scales(E0=2.5e-3, l0=1.7e-6, t0=4.0, Delta=1.3, J=0.9, tau_mc=1.1)
    g, b, m = 0.71, 0.042, 0.55
    gs, bs, ms = an.si_from_mc(g, b, m, s)
    assert np.allclose(an.mc_from_si(gs, bs, ms, s), (g, b, m), rtol=1e-14)
    # doubling l0: stiffness / 4, bulk density / 8, mobility * 16
    s2 = an.Scales(E0=s.E0, l0=2 * s.l0, t0=s.t0, Delta=s.Delta, J=s.J, tau_mc=s.tau_mc)
    gs2, bs2, ms2 = an.si_from_mc(g, b, m, s2)
    assert gs2 == pytest.approx(gs / 4) and bs2 == pytest.approx(bs / 8) and ms2 == pytest.approx(ms * 16)
    # the time scale that maps m onto a target SI mobility
    target = 3.0e-14
    t0 = an.time_scale(m, target, s)
    s3 = an.Scales(E0=s.E0, l0=s.l0, t0=t0, Delta=s.Delta, J=s.J, tau_mc=s.tau_mc)
    assert an.si_from_mc(g, b, m, s3)[2] == pytest.approx(target, rel=1e-14)


def test_flat_boundary_mobility_exact():
    t = np.arange(0, 1000, 50.0)
    m, db = 0.8, 0.1
    w = 64.0 + 2 * m * (-db) * t           # two boundaries, strip shrinks
    mm, v, r2 = an.flat_boundary_mobility(t, w, db)
    assert mm == pytest.approx(m, rel=1e-12) and v == pytest.approx(-m * db) and r2 == pytest.approx(1.0)
    s = np.zeros((20, 16), np.int32)
    s[5:12] = 1
    assert an.strip_position(s) == 7.0


def _circle_areas(m, gamma, db, r0, t_end, dt=0.01, every=50.0):
    """Exact-in-the-limit RK4 solution of dr/dt = m(-db - gamma/r)."""
    def rate(r):
        return m * (-db - gamma / r)
    r, t, out, ts, nxt = r0, 0.0, [np.pi * r0 ** 2], [0.0], every
    while t < t_end - 1e-9:
        k1 = rate(r); k2 = rate(r + 0.5 * dt * k1); k3 = rate(r + 0.5 * dt * k2); k4 = rate(r + dt * k3)
        r += dt * (k1 + 2 * k2 + 2 * k3 + k4) / 6
        t += dt
        if t >= nxt - 1e-9:
            out.append(np.pi * r * r); ts.append(t); nxt += every
    return np.array(ts), np.array(out)


def test_circle_kinetics_exact():
    m, gamma = 0.9, 0.6
    t, A = _circle_areas(m, gamma, 0.0, 60.0, 1000.0)
    mg, r2 = an.circle_kinetics(t, A)
    assert mg == pytest.approx(m * gamma, rel=1e-6) and r2 > 0.999999
    t, A = _circle_areas(m, gamma, -0.02, 60.0, 1000.0, every=10.0)
    mm, r2 = an.circle_kinetics(t, A, delta_b=-0.02, gamma=gamma)
    assert mm == pytest.approx(m, rel=2e-3) and r2 > 0.999


def test_circle_kinetics_joint_fit_exact():
    m, gamma = 0.7, 0.45
    runs = [(*_circle_areas(m, gamma, db, 60.0, 800.0, every=10.0), db) for db in (0.0, 0.02, -0.02)]
    mm, gg, r2 = an.circle_kinetics_fit(runs)
    assert mm == pytest.approx(m, rel=3e-3) and gg == pytest.approx(gamma, rel=3e-3) and r2 > 0.999


def test_gaussian_width_and_texture_kinetics():
    phi = np.linspace(-45, 45, 91)
    for g in (5.0, 12.0, 30.0):
        assert an.gaussian_width(phi, an.gaussian_density(phi, g)) == pytest.approx(g, rel=1e-7)
    rng = np.random.default_rng(0)
    d = an.gaussian_density(phi, 15.0) * (1 + 0.03 * rng.standard_normal(phi.size))
    assert an.gaussian_width(phi, d) == pytest.approx(15.0, rel=0.03)
    t = np.array([0.0, 100.0, 200.0, 300.0])
    gs = 10.0 + 0.02 * t
    g, k, c, r2 = an.texture_kinetics(t, phi, [an.gaussian_density(phi, x) for x in gs])
    assert np.allclose(g, gs, rtol=1e-7) and k == pytest.approx(0.02, rel=1e-6) and c == pytest.approx(10.0)
