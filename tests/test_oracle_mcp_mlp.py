"""Pins of the oracle's crystal-plasticity update (Sec. 2, Eqs. (1)-(2),
Table 1, Eq. (4)) and of its double-precision MLP.

* elasticity: a strain state producing uniaxial stress gives that stress
  back, with the closed-form cubic Young's moduli E[100] = 138.52 GPa and
  E[111] = 302.6 GPa (from C11, C12, C44 of Table 1, C12 read for "C22");
* yield: under uniaxial stress, slip starts at sigma = tau0 / m with m the
  FCC {111}<110> Schmid factor of the load axis (computed independently in
  synth); below it the crystal stays elastic and stores 2 tau0^2 / G;
* Eq. (4): E_rho = 2 tau_c^2 / G; Voce hardening monotone in the slip;
* Eq. (2): half-open cumulative intervals;
* higher Schmid factor -> more stored energy under the same load (Sec. 5);
* MLP: analytic gradient vs central differences; closed-form forward cases;
  Adam's first step (Kingma & Ba: -lr g / (|g| + eps)).
"""
import numpy as np
import pytest
from scipy import stats

import synth

C11, C12, C44 = 250800.0, 150000.0, 123500.0


def voigt_stiffness():
    Cv = np.zeros((6, 6))
    Cv[:3, :3] = C12
    for i in range(3):
        Cv[i, i] = C11
        Cv[3 + i, 3 + i] = C44
    return Cv


def strain_for_stress(sig):
    """Tensor strain (3x3) of a stress tensor, by inverting the 6x6 Voigt
    stiffness (engineering shear strains halved)."""
    s6 = np.array([sig[0, 0], sig[1, 1], sig[2, 2], sig[1, 2], sig[0, 2], sig[0, 1]])
    e6 = np.linalg.solve(voigt_stiffness(), s6)
    e = np.diag(e6[:3]).astype(float)
    e[1, 2] = e[2, 1] = e6[3] / 2
    e[0, 2] = e[2, 0] = e6[4] / 2
    e[0, 1] = e[1, 0] = e6[5] / 2
    return e


def six(e):
    return np.array([e[0, 0], e[1, 1], e[2, 2], e[1, 2], e[0, 2], e[0, 1]])


def uniaxial(orc, euler, sigma0, seed=3):
    """Strain (sample frame) that gives uniaxial stress sigma0 along sample z."""
    g = synth.bunge_to_matrix(euler)[0]        # crystal = g . sample
    l = g @ np.array([0.0, 0.0, 1.0])
    sig_c = sigma0 * np.outer(l, l)
    e_c = strain_for_stress(sig_c)
    e_s = g.T @ e_c @ g
    return orc.mcp_one(euler, six(e_s), seed), l, sig_c, e_c


def test_elastic_moduli_closed_form(orc):
    E100 = (C11 - C12) * (C11 + 2 * C12) / (C11 + C12)
    assert E100 == pytest.approx(138524.55, abs=0.01)
    sig = np.diag([10.0, 0.0, 0.0])
    e = strain_for_stress(sig)
    E, tc, gm, K, s_out = orc.mcp_one([0, 0, 0], six(e), 1)
    assert gm == 0.0 and tc == 8.0
    assert np.allclose(s_out, [10, 0, 0, 0, 0, 0], atol=1e-9)
    assert s_out[0] / e[0, 0] == pytest.approx(E100, rel=1e-9)
    assert E == pytest.approx(2 * 8.0 ** 2 / orc.mcp_shear_modulus(), rel=1e-15)
    # [111]: 1/E = S11 - 2 (S11 - S12 - S44/2) / 3
    n = np.ones(3) / np.sqrt(3)
    e111 = strain_for_stress(20.0 * np.outer(n, n))
    _, _, gm, _, s_out = orc.mcp_one([0, 0, 0], six(e111), 1)
    assert gm == 0.0
    assert (20.0 / (n @ e111 @ n)) / 1000 == pytest.approx(302.6, abs=0.1)
    assert np.allclose(s_out, six(20.0 * np.outer(n, n)), atol=1e-9)
    assert orc.mcp_shear_modulus() == pytest.approx((C11 - C12 + 3 * C44) / 5)


@pytest.mark.parametrize("euler", [(0.0, 0.0, 0.0), (0.3, 0.7, 1.1), (2.0, 1.2, 4.0), (np.pi / 8, 0.0, 0.0)])
def test_yield_follows_schmid_law(orc, euler):
    g = synth.bunge_to_matrix(euler)[0]
    l = g @ np.array([0.0, 0.0, 1.0])
    m = synth.schmid_factor(l)[0]
    sy = 8.0 / m
    (E, tc, gm, K, s_out), *_ = uniaxial(orc, euler, 0.98 * sy)
    assert gm == 0.0 and tc == 8.0
    assert E == pytest.approx(2 * 64.0 / orc.mcp_shear_modulus(), rel=1e-15)
    (E2, tc2, gm2, K2, _), *_ = uniaxial(orc, euler, 1.03 * sy)
    assert gm2 > 0.0 and tc2 > 8.0 and E2 > E


def test_paper_orientation_family_yield_values(orc):
    # load along x, rotation theta about z (Sec. 5): 1/sqrt(6) at 0 and 45 deg, 0.4928 at 22.5 deg
    for theta, sy in [(0.0, 19.596), (np.pi / 4, 19.596), (np.pi / 8, 16.234)]:
        m = synth.schmid_factor([np.cos(theta), np.sin(theta), 0.0])[0]
        assert 8.0 / m == pytest.approx(sy, abs=2e-3)


def test_stored_energy_identities(orc):
    rng = np.random.default_rng(5)
    n = 300
    e = synth.matrix_to_bunge(synth.quat_to_matrix(synth.shoemake_quaternions(rng, n)))
    eps = rng.uniform(-2e-3, 2e-3, size=(n, 6))
    E, tc, gm = orc.mcp_solve(e, eps, seed=11, threads=4)
    G = orc.mcp_shear_modulus()
    assert np.allclose(E, 2 * tc ** 2 / G, rtol=1e-14)
    assert np.all(tc >= 8.0) and np.all(tc < 122.0)
    assert np.allclose(tc, [orc.mcp_tau_c(x) for x in gm], rtol=1e-14)
    assert np.all(np.diff([orc.mcp_tau_c(x) for x in np.linspace(0, 0.2, 50)]) > 0)
    assert orc.mcp_tau_c(0.0) == 8.0
    assert orc.mcp_tau_c(1e3) == pytest.approx(122.0)
    # thread count and repetition do not matter; sample index enters the draw
    E1, _, _ = orc.mcp_solve(e, eps, seed=11, threads=1)
    assert np.array_equal(E, E1)
    Ea, _, _ = orc.mcp_solve(e[5:6], eps[5:6], seed=11, sample0=5)
    assert Ea[0] == E[5]


def test_select_half_open_intervals(orc):
    p = [0.25, 0.25, 0.5]
    assert orc.mcp_select(p, 0.0) == 0
    assert orc.mcp_select(p, 0.2499999) == 0
    assert orc.mcp_select(p, 0.25) == 1
    assert orc.mcp_select(p, 0.4999999) == 1
    assert orc.mcp_select(p, 0.5) == 2
    assert orc.mcp_select(p, 0.9999999) == 2
    assert orc.mcp_select([1.0], 0.7) == 0
    assert orc.mcp_select([0.0, 1.0], 0.0) == 1


def test_slip_systems_match_independent_list(orc):
    n, d = orc.mcp_slip_systems()
    assert np.allclose(np.sum(n * d, 1), 0)
    n2, d2 = synth.fcc_slip_systems()

    def canon(v):
        v = np.round(v, 9)
        return tuple(v if v[np.nonzero(v)[0][0]] > 0 else -v)
    assert {canon(a) + canon(b) for a, b in zip(n, d)} == {canon(a) + canon(b) for a, b in zip(n2, d2)}


def test_higher_schmid_factor_stores_more_energy(orc):
    rng = np.random.default_rng(9)
    R = synth.quat_to_matrix(synth.shoemake_quaternions(rng, 400))
    e = synth.matrix_to_bunge(R)
    m, E = [], []
    for k in range(len(e)):
        (Ek, *_), l, _, _ = uniaxial(orc, e[k], 20.0, seed=k)  # the paper's 20 MPa load
        m.append(synth.schmid_factor(l)[0])
        E.append(Ek)
    rho, p = stats.spearmanr(m, E)
    assert rho > 0.8 and p < 1e-20


# ----------------------------------------------------------------- MLP

def _theta(seed, scale=0.3):
    return np.random.default_rng(seed).normal(0, scale, size=64 * 9 + 64 + 64 * 64 + 64 + 64 + 1)


def test_mlp_gradient_matches_central_differences(orc):
    rng = np.random.default_rng(2)
    th = _theta(1)
    X = rng.uniform(-1, 1, size=(7, 9))
    t = rng.normal(size=7)
    loss, g = orc.mlp_loss_grad(th, X, t)
    idx = rng.choice(len(th), size=80, replace=False)
    idx = np.concatenate([idx, [0, 575, 576, 639, 640, 4735, 4736, 4799, 4800, 4863, 4864]])
    h = 1e-6
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (orc.mlp_loss_grad(tp, X, t)[0] - orc.mlp_loss_grad(tm, X, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9
    assert loss == pytest.approx(np.mean((orc.mlp_forward(th, X) - t) ** 2), rel=1e-14)


def test_mlp_forward_closed_forms(orc):
    th = np.zeros(4865)
    th[-1] = 0.75
    X = np.random.default_rng(0).uniform(-1, 1, size=(5, 9))
    assert np.allclose(orc.mlp_forward(th, X), 0.75)
    # one path: W1[0, 2] = a, W2[0, 0] = b, w3[0] = c -> y = c tanh(b tanh(a x2)) + b3
    a, b, c = 0.7, -1.3, 2.0
    th[2] = a
    th[576 + 64 + 0] = b
    th[576 + 64 + 4096 + 64 + 0] = c
    assert np.allclose(orc.mlp_forward(th, X), c * np.tanh(b * np.tanh(a * X[:, 2])) + 0.75, rtol=1e-14)


def test_adam_first_step(orc):
    rng = np.random.default_rng(4)
    th = _theta(3)
    g = rng.normal(size=th.size)
    m, v = np.zeros_like(th), np.zeros_like(th)
    t0 = th.copy()
    orc.adam_step(th, g, m, v, 1, 1e-3)
    assert np.allclose(th, t0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
