"""Pins of the crystal-plasticity oracle beyond yield (Sec. 2, Eqs. (1)-(2),
Table 1), each computed here independently of the oracle: cubic stiffness
and compliance built with numpy from Table 1 (Mandel 6x6 inverse), the FCC
{111}<110> systems enumerated here, Bunge orientations through scipy.

1. Single slip, closed form.  With one active system a the exact
   rate-independent state after a monotone strain path obeys the
   consistency condition
       s * (P_a : C : eps) - gamma * (P_a : C : P_a) = tau_c(gamma)
   (s the sign of the resolved shear stress, tau_c the Voce law), a scalar
   equation solved here by bisection.  The oracle's sub-stepped return
   mapping must converge to it at second order in the sub-step (its only
   error is the linearised hardening of the last sub-step), keep exactly one
   candidate, pick the system predicted here, and leave the stress
   C : (eps - s gamma P_a).
2. Selection, Eq. (1).  In a first plastic sub-step with six candidates the
   frequency of each pick over 10^5 draws of R (Eq. (2)) must match
   exp(-beta E_a) / Z with E_a the elastic energy after the single-slip
   return on a, computed here (chi-square).
3. Planted mistakes -- hardening dropped from the slip increment, the sign
   of beta flipped, the return applied with the wrong sign -- built into
   copies of the oracle compiled here, fail these pins.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.stats import chisquare

C11, C12, C44 = 250800.0, 150000.0, 123500.0     # Table 1, MPa
TAU0, TAUS, H0, BETA = 8.0, 122.0, 440.0, 1000.0
I3 = np.eye(3)
CIJKL = (C12 * np.einsum("ij,kl->ijkl", I3, I3)
         + C44 * (np.einsum("ik,jl->ijkl", I3, I3) + np.einsum("il,jk->ijkl", I3, I3))
         + (C11 - C12 - 2 * C44) * np.einsum("ni,nj,nk,nl->ijkl", I3, I3, I3, I3))
R2 = np.sqrt(2.0)


def _mandel(t):
    return np.array([t[0, 0], t[1, 1], t[2, 2], R2 * t[1, 2], R2 * t[0, 2], R2 * t[0, 1]])


def _from_mandel(v):
    return np.array([[v[0], v[5] / R2, v[4] / R2], [v[5] / R2, v[1], v[3] / R2], [v[4] / R2, v[3] / R2, v[2]]])


CM = np.array([[_mandel(_from_mandel(np.eye(6)[i])) @ _mandel(np.einsum("ijkl,kl->ij", CIJKL, _from_mandel(np.eye(6)[j])))
                for j in range(6)] for i in range(6)])
SM = np.linalg.inv(CM)


def _systems():
    out = []
    for n in ((1, 1, 1), (-1, 1, 1), (1, -1, 1), (1, 1, -1)):
        for d in ((1, -1, 0), (1, 0, -1), (0, 1, -1), (1, 1, 0), (1, 0, 1), (0, 1, 1)):
            if np.dot(n, d) == 0:
                out.append((np.array(n) / np.sqrt(3.0), np.array(d) / np.sqrt(2.0)))
    return out


SYS = _systems()
PS = [0.5 * (np.outer(d, n) + np.outer(n, d)) for n, d in SYS]


def voce(G):
    return TAUS - (TAUS - TAU0) * np.exp(-H0 * G / (TAUS - TAU0))


def voce_slope(G):
    return H0 * np.exp(-H0 * G / (TAUS - TAU0))


def crystal_stress(euler, eps_sample):
    g = Rotation.from_euler("ZXZ", euler).as_matrix().T    # Bunge, passive: sample -> crystal
    eps_c = g @ eps_sample @ g.T
    return eps_c, np.einsum("ijkl,kl->ij", CIJKL, eps_c)


def oracle_index_map(orc):
    """oracle system index -> index into SYS (same plane and direction up to sign)."""
    no, do = orc.mcp_slip_systems()
    out = {}
    for i in range(12):
        for j, (n, d) in enumerate(SYS):
            if min(np.abs(no[i] - n).max(), np.abs(no[i] + n).max()) < 1e-12 and \
                    min(np.abs(do[i] - d).max(), np.abs(do[i] + d).max()) < 1e-12:
                out[i] = j
    assert sorted(out.values()) == list(range(12))
    return out


# --- 1. single slip --------------------------------------------------------

EULER_1 = np.array([1.582, 1.101, 4.243])    # a generic orientation; its second system sits at 0.79 of the first


def single_slip_case():
    unit = np.diag([1.0, -0.5, -0.5])
    _, sig1 = crystal_stress(EULER_1, unit)
    tau1 = np.array([np.sum(sig1 * P) for P in PS])
    a = int(np.argmax(np.abs(tau1)))
    amp = 1.2 * TAU0 / abs(tau1[a])                  # 20 % past the yield strain
    eps = amp * unit
    eps_c, sig = crystal_stress(EULER_1, eps)
    P = PS[a]
    CP = np.einsum("ijkl,kl->ij", CIJKL, P)
    PCP = float(np.sum(P * CP))
    tau = float(np.sum(sig * P))
    s = np.sign(tau)
    lo, hi = 0.0, abs(tau) / PCP                   # residual > 0 at lo, < 0 at hi
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if abs(tau) - mid * PCP - voce(mid) > 0:
            lo = mid
        else:
            hi = mid
    gamma = 0.5 * (lo + hi)
    sig_exact = np.einsum("ijkl,kl->ij", CIJKL, eps_c - s * gamma * P)
    eps6 = np.array([eps[0, 0], eps[1, 1], eps[2, 2], 0.0, 0.0, 0.0])
    return a, eps6, gamma, voce(gamma), sig_exact


def single_slip_problems(orc, dll=None):
    a, eps6, gamma, tc_exact, sig_exact = single_slip_case()
    imap = oracle_index_map(orc)
    out = []
    errs = {}
    for K in (25, 50, 100, 200, 400):
        _, tc, gm, sig6, nc, picks = orc.mcp_run(EULER_1, eps6, 5, K, dll=dll)
        if nc.max() != 1:
            out.append(f"K={K}: {nc.max()} candidates in a sub-step")
        if any(imap[int(p)] != a for p in picks if p >= 0) or not (picks >= 0).any():
            out.append(f"K={K}: picks {sorted(set(picks.tolist()))}, want system {a}")
        errs[K] = abs(tc - tc_exact)
        sig = np.array([[sig6[0], sig6[5], sig6[4]], [sig6[5], sig6[1], sig6[3]], [sig6[4], sig6[3], sig6[2]]])
        # the final stress is the elastic response to the strain less the slip of every sub-step
        P = PS[a]
        eps_c, _ = crystal_stress(EULER_1, np.diag(eps6[:3]))
        s = np.sign(np.sum(sig_exact * P))
        sig_el = np.einsum("ijkl,kl->ij", CIJKL, eps_c - s * gm * P)
        if np.abs(sig - sig_el).max() > 1e-9 * np.abs(sig_el).max():
            out.append(f"K={K}: stress is not C:(eps - s gamma P)")
        if abs(gm - gamma) > 1e-3 * gamma:
            out.append(f"K={K}: slip {gm} vs {gamma}")
    if errs[400] > 1e-11 * tc_exact:
        out.append(f"tau_c error at K=400: {errs[400]:.3g} MPa")
    if not errs[25] > 8.0 * errs[100]:
        out.append(f"not second order: error {errs[25]:.3g} at K=25, {errs[100]:.3g} at K=100")
    return out


def test_single_slip_converges_to_the_consistency_condition(orc):
    a, eps6, gamma, tc_exact, _ = single_slip_case()
    assert gamma > 1e-5 and tc_exact > TAU0 + 1e-3    # the slip hardened the system
    assert single_slip_problems(orc) == []


# --- 2. selection, Eq. (1) --------------------------------------------------

EULER_2 = np.array([0.32332556, 1.39230751, 6.00613659])   # six candidates, probabilities 0.05 .. 0.52
AMP_2 = 2.3296585544e-4


def selection_case():
    eps = AMP_2 * np.diag([1.0, -0.5, -0.5])
    _, sig = crystal_stress(EULER_2, eps)             # K = 1: the trial stress of the first sub-step
    cand, E = [], []
    for j, P in enumerate(PS):
        tau = np.sum(sig * P)
        if abs(tau) <= TAU0:
            continue
        CP = np.einsum("ijkl,kl->ij", CIJKL, P)
        dg = (abs(tau) - TAU0) / (np.sum(P * CP) + voce_slope(0.0))
        sa = sig - np.sign(tau) * dg * CP
        cand.append(j)
        E.append(0.5 * _mandel(sa) @ SM @ _mandel(sa))
    E = np.array(E)
    p = np.exp(-BETA * (E - E.min()))
    eps6 = np.array([eps[0, 0], eps[1, 1], eps[2, 2], 0.0, 0.0, 0.0])
    return eps6, cand, p / p.sum()


def selection_pvalue(orc, dll=None, n=100000):
    eps6, cand, p = selection_case()
    picks, nc = orc.mcp_picks(EULER_2, eps6, 11, n, 1, 1, dll=dll)
    if not np.all(nc == len(cand)):
        return 0.0
    imap = oracle_index_map(orc)
    got = np.array([imap[int(v)] for v in picks])
    counts = np.array([np.sum(got == j) for j in cand])
    if counts.sum() != n:
        return 0.0
    return float(chisquare(counts, n * p).pvalue)


def test_selection_follows_eq1(orc):
    eps6, cand, p = selection_case()
    assert len(cand) == 6 and p.min() > 0.04 and p.max() > 0.5
    assert selection_pvalue(orc) > 1e-3


# --- 3. frame invariance on multi-slip paths --------------------------------
# Turning the sample frame by any rotation R turns the orientation into
# g R^T and the strain into R eps R^T; the crystal-frame strain, and with it
# every sub-step of the solve (candidates, Eq. (1) probabilities, Eq. (2)
# picks with the same random stream, the Voce hardening and Eq. (4)), is
# unchanged.  This holds at any path length, so it checks the long paths
# where several systems compete, which have no closed form.

def _rotated(euler, eps, R):
    M = Rotation.from_euler("ZXZ", euler).as_matrix()          # g = M^T
    return Rotation.from_matrix(R @ M).as_euler("ZXZ"), R @ eps @ R.T


def _eps6(t):
    return np.array([t[0, 0], t[1, 1], t[2, 2], t[1, 2], t[0, 2], t[0, 1]])


def frame_problems(orc, dll=None, n=24, K=60):
    rng = np.random.default_rng(2024)
    out, multi = [], 0
    for i in range(n):
        euler = rng.uniform([0.0, 0.0, 0.0], [2 * np.pi, np.pi, 2 * np.pi])
        A = rng.normal(size=(3, 3))
        eps = 1.5e-3 * (A + A.T) / np.linalg.norm(A + A.T)      # several times the yield strain
        E0, tc0, gm0, _, nc0, p0 = orc.mcp_run(euler, _eps6(eps), 7, K, sample=i, dll=dll)
        multi += int(nc0.max() >= 2)
        for _ in range(2):
            R = Rotation.from_quat(rng.normal(size=4)).as_matrix()
            euler_r, eps_r = _rotated(euler, eps, R)
            E1, tc1, gm1, _, nc1, p1 = orc.mcp_run(euler_r, _eps6(eps_r), 7, K, sample=i, dll=dll)
            if not (np.array_equal(p0, p1) and np.array_equal(nc0, nc1)):
                out.append(f"crystal {i}: other candidates or picks in a turned sample frame")
            elif not (abs(E1 - E0) <= 1e-9 * abs(E0) and abs(tc1 - tc0) <= 1e-9 * tc0
                      and abs(gm1 - gm0) <= 1e-9 * max(gm0, 1e-30)):
                out.append(f"crystal {i}: E {E0} vs {E1}, tau_c {tc0} vs {tc1}")
    if multi < n // 2:
        out.append(f"only {multi} of {n} paths had several candidates in a sub-step")
    return out


def test_stored_energy_is_frame_invariant_on_multislip_paths(orc):
    assert frame_problems(orc) == []


# --- 3. planted mistakes ----------------------------------------------------

PLANTS = {
    "hardening dropped from the slip increment": ("dg[k] = (fabs(tau) - tc) / (PCP[cand[k]] + h);",
                                                   "dg[k] = (fabs(tau) - tc) / (PCP[cand[k]]);"),
    "beta sign flipped": ("p[k] = exp(-MCP_BETA * (E[k] - Emin));", "p[k] = exp(MCP_BETA * (E[k] - Emin));"),
    "return with the wrong sign": ("sig[i][j] = str[i][j] - sgn * dg[pick] * CP[cand[pick]][i][j];",
                                   "sig[i][j] = str[i][j] + sgn * dg[pick] * CP[cand[pick]][i][j];"),
    "crystal-frame strain transposed": ("acc += g[i][p] * es[p][q] * g[j][q];",
                                        "acc += g[p][i] * es[p][q] * g[q][j];"),
}


@pytest.fixture(scope="module")
def planted(tmp_path_factory):
    import oracle
    src = os.path.dirname(oracle.__file__)
    out = {}
    for name, (old, new) in PLANTS.items():
        d = tmp_path_factory.mktemp("plant")
        for f in ("oracle.c", "mcp_mlp.c"):
            shutil.copy(os.path.join(src, f), d / f)
        text = (d / "mcp_mlp.c").read_text()
        assert text.count(old) == 1, name
        (d / "mcp_mlp.c").write_text(text.replace(old, new))
        lib = d / "libplant.so"
        subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", "-o", str(lib),
                        str(d / "oracle.c"), str(d / "mcp_mlp.c"), "-lm"], check=True)
        out[name] = ctypes.CDLL(str(lib))
    return out


@pytest.mark.parametrize("name", sorted(PLANTS))
def test_planted_mcp_mistakes_fail_the_pins(orc, planted, name):
    dll = planted[name]
    caught = bool(single_slip_problems(orc, dll=dll)) or selection_pvalue(orc, dll=dll) < 1e-3 \
        or bool(frame_problems(orc, dll=dll))
    assert caught, f"planted mistake not caught: {name}"
