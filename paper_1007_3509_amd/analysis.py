"""Physical units and analysis of sweep outputs (host-side post-processing).

Zhang, Dingreville, Bartel, Lusk, arXiv:1007.3509:

* Sec. 3 (parametric links): the sharp-interface (SI) stiffness, bulk energy
  density and mobility follow from their Monte Carlo counterparts (gamma*,
  b, m) through a characteristic energy E0, length l0 and time t0, the
  lattice spacing Delta, the interaction energy J and the MC time step
  tau_mc:
      gamma*_s = gamma* E0 / (Delta^2 J l0^2)
      b_s      = 2 b E0 / (Delta^3 l0^3)
      m_s      = Delta^4 m l0^4 / (J tau_mc E0 t0)
  ``si_from_mc`` and ``mc_from_si`` evaluate these relations and their
  inverses; ``time_scale`` solves the mobility link for t0, which gives the
  physical duration of one MC step.
* Sec. 3 (SI kinetics, Herring relation): v_n = m_s f_s with
  f_s = [[E_rho]] + kappa gamma*.  In MC units a flat boundary moves at
  v = m f and a circular grain of radius r grows at dr/dt = m (f - gamma*/r),
  so dA/dt = 2 pi m (f r - gamma*), where f is the bulk energy released per
  site swept: f = B[matrix] - B[grain] with energies per grain (the paper's
  Ising-convention "half the bulk energy difference" of Sec. 4 does not
  apply to energies carried by the grains).  ``flat_boundary_mobility`` and
  ``circle_kinetics`` fit m and gamma* to measured widths and areas.
* Sec. 5: texture histograms are fitted to the time-dependent Gaussian
  f(phi, t) = exp(-phi^2 / (2 g(t)^2)) / (g(t) sqrt(2 pi)); ``gaussian_width``
  fits g to one histogram and ``texture_kinetics`` fits the widths of a
  series to a straight line in time (the macroscopic equation of texture
  evolution).

Everything here is numpy on host arrays that the library returns (spins,
grain areas, texture fractions); no step of the sweep runs here.
"""
from dataclasses import dataclass

import numpy as np


# ------------------------------------------------------------ parametric links

@dataclass(frozen=True)
class Scales:
    """Characteristic energy, length and time (E0, l0, t0), lattice spacing
    Delta, interaction energy J and MC time step tau_mc of the links."""
    E0: float
    l0: float
    t0: float
    Delta: float = 1.0
    J: float = 1.0
    tau_mc: float = 1.0


def si_from_mc(gamma_mc, b_mc, m_mc, s: Scales):
    """SI stiffness, bulk energy density and mobility of MC values."""
    gamma_s = gamma_mc * s.E0 / (s.Delta ** 2 * s.J * s.l0 ** 2)
    b_s = 2.0 * b_mc * s.E0 / (s.Delta ** 3 * s.l0 ** 3)
    m_s = s.Delta ** 4 * m_mc * s.l0 ** 4 / (s.J * s.tau_mc * s.E0 * s.t0)
    return gamma_s, b_s, m_s


def mc_from_si(gamma_s, b_s, m_s, s: Scales):
    """Inverse of ``si_from_mc``: the MC values that represent SI ones."""
    gamma_mc = gamma_s * s.Delta ** 2 * s.J * s.l0 ** 2 / s.E0
    b_mc = b_s * s.Delta ** 3 * s.l0 ** 3 / (2.0 * s.E0)
    m_mc = m_s * s.J * s.tau_mc * s.E0 * s.t0 / (s.Delta ** 4 * s.l0 ** 4)
    return gamma_mc, b_mc, m_mc


def time_scale(m_mc, m_s, s: Scales):
    """t0 that makes the MC mobility m_mc represent the SI mobility m_s (the
    mobility link solved for t0); one MC step then lasts tau_mc * t0."""
    return s.Delta ** 4 * m_mc * s.l0 ** 4 / (s.J * s.tau_mc * s.E0 * m_s)


# ----------------------------------------------------------- boundary kinetics

def _line(x, y):
    """Least-squares slope, intercept and R^2 of y on x."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    A = np.stack([x, np.ones_like(x)], axis=1)
    (k, c), *_ = np.linalg.lstsq(A, y, rcond=None)
    res = y - (k * x + c)
    tot = y - y.mean()
    r2 = 1.0 - float(res @ res) / float(tot @ tot) if float(tot @ tot) > 0 else 1.0
    return float(k), float(c), r2


def strip_position(spins, grain=1, axis=0):
    """Mean position of the boundaries of a strip of ``grain`` spanning the
    lattice: the strip's area divided by the lattice's extent across it,
    i.e. its mean width (spins as returned by the library, axis 0 the
    slowest)."""
    s = np.asarray(spins)
    extent = s.size // s.shape[axis]
    return float(np.count_nonzero(s == grain)) / extent


def flat_boundary_mobility(times, widths, delta_b, n_boundaries=2):
    """MC mobility from a flat strip whose grain has bulk energy delta_b
    above the matrix: each of its n boundaries advances into the matrix at
    v = m f with f = -delta_b, so the width changes at n v.  Returns
    (m, v, R^2 of the straight-line fit of the widths)."""
    k, _, r2 = _line(times, widths)
    v = k / n_boundaries
    f = -delta_b
    return (v / f if f != 0 else float("nan")), v, r2


def circle_kinetics(times, areas, delta_b=0.0, gamma=None):
    """Fit a circular grain with bulk energy delta_b above its surroundings
    to dA/dt = 2 pi m (f r - gamma*), f = -delta_b.

    With delta_b = 0 the area is linear in time and only the product
    m gamma* is determined: returns (m * gamma*, R^2).  Otherwise, with
    gamma* given, returns (m, R^2) from the regression of dA/dt on r.
    """
    t = np.asarray(times, dtype=np.float64)
    A = np.asarray(areas, dtype=np.float64)
    f = -delta_b
    if f == 0.0:
        k, _, r2 = _line(t, A)
        return -k / (2.0 * np.pi), r2
    if gamma is None:
        raise ValueError("gamma* is needed to separate m when f != 0")
    dA = np.gradient(A, t)
    r = np.sqrt(A / np.pi)
    # dA/dt = 2 pi m (f r - gamma*): one-parameter fit through the origin
    x = 2.0 * np.pi * (f * r - gamma)
    m = float(x @ dA) / float(x @ x)
    res = dA - m * x
    tot = dA - dA.mean()
    r2 = 1.0 - float(res @ res) / float(tot @ tot) if float(tot @ tot) > 0 else 1.0
    return m, r2


def circle_kinetics_fit(runs):
    """Mobility and stiffness from circular grains at several bulk energies:
    dA/dt = 2 pi m f r - 2 pi (m gamma*) is linear in (m, m gamma*), so the
    rows of every run (times, areas, delta_b) are solved together by least
    squares.  Returns (m, gamma*, R^2)."""
    X, y = [], []
    for times, areas, delta_b in runs:
        t = np.asarray(times, dtype=np.float64)
        A = np.asarray(areas, dtype=np.float64)
        dA = np.gradient(A, t)
        r = np.sqrt(A / np.pi)
        X.append(np.stack([2.0 * np.pi * (-delta_b) * r, -2.0 * np.pi * np.ones_like(r)], axis=1))
        y.append(dA)
    X = np.concatenate(X)
    y = np.concatenate(y)
    (m, mg), *_ = np.linalg.lstsq(X, y, rcond=None)
    res = y - X @ np.array([m, mg])
    tot = y - y.mean()
    r2 = 1.0 - float(res @ res) / float(tot @ tot) if float(tot @ tot) > 0 else 1.0
    return float(m), float(mg / m), r2


# ------------------------------------------------------------- texture kinetics

def gaussian_density(phi, g):
    """The Gaussian texture density of Sec. 5, width g."""
    phi = np.asarray(phi, dtype=np.float64)
    return np.exp(-phi * phi / (2.0 * g * g)) / (g * np.sqrt(2.0 * np.pi))


def gaussian_width(phi, density, lo=None, hi=None, tol=1e-10):
    """Least-squares width g of the Gaussian f(phi) fitted to a histogram
    (bin centres phi, probability densities), by golden-section search on
    [lo, hi] (default: a bracket around the second-moment estimate)."""
    phi = np.asarray(phi, dtype=np.float64)
    d = np.asarray(density, dtype=np.float64)
    w = np.abs(d)
    g2 = float((phi * phi * w).sum() / max(w.sum(), 1e-300))
    g_m = np.sqrt(max(g2, 1e-300))
    lo = 0.05 * g_m if lo is None else lo
    hi = 20.0 * g_m if hi is None else hi

    def cost(g):
        r = d - gaussian_density(phi, g)
        return float(r @ r)

    a, b = lo, hi
    invphi = (np.sqrt(5.0) - 1.0) / 2.0
    c, e = b - invphi * (b - a), a + invphi * (b - a)
    fc, fe = cost(c), cost(e)
    while b - a > tol * max(1.0, abs(b)):
        if fc < fe:
            b, e, fe = e, c, fc
            c = b - invphi * (b - a)
            fc = cost(c)
        else:
            a, c, fc = c, e, fe
            e = a + invphi * (b - a)
            fe = cost(e)
    return 0.5 * (a + b)


def texture_kinetics(times, phi, densities):
    """Gaussian width g(t) of each histogram of a series and the straight
    line through them: returns (g, dg/dt, g(0), R^2)."""
    g = np.array([gaussian_width(phi, d) for d in densities])
    k, c, r2 = _line(times, g)
    return g, k, c, r2
