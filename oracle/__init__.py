"""CPU oracle for the red/black Potts sweep with a per-grain bulk energy.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library (``paper_1007_3509_amd``) never imports it, and it never imports the
product library: the two share nothing but the seeded input generators in
``synth``.

The arithmetic lives in ``oracle.c`` (plain C, double precision where the
method uses floating point); this module only marshals numpy arrays.
Each wrapper names the passage of Zhang, Dingreville, Bartel & Lusk,
"Hybrid Monte Carlo simulation of stress-induced texture evolution with
inelastic effects", that it follows.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

VN4, MOORE8, VN6, MOORE26 = 0, 1, 2, 3
PROP_NEIGHBOUR, PROP_UNIFORM = 0, 1

_lib = None


def lib():
    global _lib
    if _lib is None:
        # ORACLE_LIB: another build of this library (the sanitizer build)
        path = os.environ.get("ORACLE_LIB") or _build.ensure_built()
        L = C.CDLL(path)
        P = C.POINTER
        u32p, i32p, i64p, f64p = P(C.c_uint32), P(C.c_int32), P(C.c_int64), P(C.c_double)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox_many.argtypes = [u32p, C.c_int64, u32p, u32p]
        L.orc_threshold.argtypes = [C.c_int64, C.c_float]
        L.orc_threshold.restype = C.c_uint32
        L.orc_num_neighbours.argtypes = [C.c_int]
        L.orc_num_colours.argtypes = [C.c_int]
        L.orc_neighbours_of.argtypes = [C.c_int, i32p, C.c_int64, i64p]
        L.orc_colour_of.argtypes = [C.c_int, i32p, C.c_int64]
        L.orc_delta_energy.argtypes = [i32p, C.c_int, i32p, C.c_int32, i32p, C.c_int64, C.c_int32]
        L.orc_delta_energy.restype = C.c_int64
        L.orc_sweep.argtypes = [i32p, C.c_int, C.c_int, i32p, C.c_int32, i32p, C.c_int32, C.c_float,
                                C.c_uint64, C.c_int32, C.c_uint64, C.c_int]
        L.orc_voronoi_points.argtypes = [C.c_int, i32p, C.c_int32, C.c_uint64, i64p]
        L.orc_voronoi_brute.argtypes = [C.c_int, i32p, C.c_int32, C.c_uint64, i32p]
        L.orc_voronoi_grid.argtypes = [C.c_int, i32p, C.c_int32, C.c_uint64, i32p, C.c_int]
        L.orc_texture.argtypes = [i32p, C.c_int64, C.c_int32, i32p, C.c_int32, i64p, i32p, f64p, f64p]
        L.orc_mcp_one.argtypes = [f64p, f64p, C.c_uint64, C.c_uint64, f64p, f64p, C.POINTER(C.c_int), f64p]
        L.orc_mcp_one.restype = C.c_double
        L.orc_mcp_solve.argtypes = [f64p, f64p, C.c_int64, C.c_uint64, C.c_uint64, f64p, f64p, f64p, C.c_int]
        L.orc_mcp_select.argtypes = [f64p, C.c_int, C.c_double]
        L.orc_mcp_tau_c.argtypes = [C.c_double]
        L.orc_mcp_tau_c.restype = C.c_double
        L.orc_mcp_shear_modulus.restype = C.c_double
        L.orc_mcp_slip_systems.argtypes = [f64p, f64p]
        L.orc_mlp_forward.argtypes = [f64p, f64p, C.c_int64, f64p]
        L.orc_mlp_loss_grad.argtypes = [f64p, f64p, f64p, C.c_int64, f64p]
        L.orc_mlp_loss_grad.restype = C.c_double
        L.orc_adam_step.argtypes = [f64p, f64p, f64p, f64p, C.c_int64, C.c_double, C.c_double, C.c_double,
                                    C.c_double]
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _dims3(dims):
    d = list(dims) + [1] * (3 - len(dims))
    return np.asarray(d, dtype=np.int32)


def num_neighbours(nbr):
    return lib().orc_num_neighbours(nbr)


def num_colours(nbr):
    return lib().orc_num_colours(nbr)


def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon et al., SC'11) of one or many 4-word counters."""
    ctr = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(-1, 4))
    key = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(2))
    out = np.empty_like(ctr)
    lib().orc_philox_many(_ptr(ctr, C.c_uint32), ctr.shape[0], _ptr(key, C.c_uint32),
                          _ptr(out, C.c_uint32))
    return out


def threshold(d, kT):
    """T(d) = min(2^32-1, floor(2^32 exp(-d/(65536 kT)))) -- the Metropolis
    acceptance probability of Sec. 3 / Sec. 4 in uint32 fixed point."""
    return int(lib().orc_threshold(int(d), float(kT)))


def threshold_many(d, kT):
    """T(d) of an array of d (uint32; d <= 0 gives 2^32 - 1)."""
    d = np.ascontiguousarray(np.asarray(d, dtype=np.int64).reshape(-1))
    out = np.empty(d.size, dtype=np.uint32)
    f = lib().orc_threshold_many
    f.argtypes = [C.POINTER(C.c_int64), C.c_int64, C.c_float, C.POINTER(C.c_uint32)]
    f(_ptr(d, C.c_int64), d.size, float(kT), _ptr(out, C.c_uint32))
    return out


def neighbours_of(nbr, dims, i):
    out = np.empty(26, dtype=np.int64)
    d = _dims3(dims)
    m = lib().orc_neighbours_of(nbr, _ptr(d, C.c_int32), int(i), _ptr(out, C.c_int64))
    return out[:m].copy()


def colour_of(nbr, dims, i):
    d = _dims3(dims)
    return lib().orc_colour_of(nbr, _ptr(d, C.c_int32), int(i))


def delta_energy(spins, nbr, dims, J_fx, B, i, q_new):
    """Change of Eq. (7) (bond term J(1-delta), bulk term b(q)) in 2^-16 units."""
    s = np.ascontiguousarray(np.asarray(spins, dtype=np.int32).reshape(-1))
    b = np.ascontiguousarray(np.asarray(B, dtype=np.int32))
    d = _dims3(dims)
    return int(lib().orc_delta_energy(_ptr(s, C.c_int32), nbr, _ptr(d, C.c_int32), int(J_fx),
                                      _ptr(b, C.c_int32), int(i), int(q_new)))


def sweep(spins, nbr, dims, B, kT, n_mcs, seed, mcs0=0, J_fx=65536,
          proposal=PROP_NEIGHBOUR, threads=1):
    """n_mcs red/black Metropolis steps (Sec. 4) of Eq. (7); returns new spins
    with the input's shape and dtype."""
    src = np.asarray(spins)
    s = np.ascontiguousarray(src.astype(np.int32).reshape(-1))
    b = np.ascontiguousarray(np.asarray(B, dtype=np.int32))
    d = _dims3(dims)
    rc = lib().orc_sweep(_ptr(s, C.c_int32), int(nbr), int(proposal), _ptr(d, C.c_int32),
                         int(J_fx), _ptr(b, C.c_int32), int(len(b)), float(kT), int(mcs0),
                         int(n_mcs), int(seed), int(threads))
    if rc != 0:
        raise ValueError(f"orc_sweep failed with {rc}")
    return s.reshape(src.shape).astype(src.dtype)


def voronoi_points(ndim, dims, G, vseed):
    d = _dims3(dims)
    pts = np.empty((G, 3), dtype=np.int64)
    lib().orc_voronoi_points(ndim, _ptr(d, C.c_int32), int(G), int(vseed), _ptr(pts, C.c_int64))
    return pts[:, :ndim].copy()


def voronoi(dims, G, vseed, method="grid", threads=1):
    """Initial microstructure: nearest seed point, ties to the lower index."""
    ndim = len(dims)
    d = _dims3(dims)
    N = int(np.prod(dims))
    out = np.empty(N, dtype=np.int32)
    if method == "brute":
        rc = lib().orc_voronoi_brute(ndim, _ptr(d, C.c_int32), int(G), int(vseed), _ptr(out, C.c_int32))
    else:
        rc = lib().orc_voronoi_grid(ndim, _ptr(d, C.c_int32), int(G), int(vseed), _ptr(out, C.c_int32),
                                    int(threads))
    if rc != 0:
        raise ValueError(f"voronoi failed with {rc}")
    return out.reshape(tuple(reversed(dims)))


def sweep_pair(spins, nbr, dims, Jp, B, kT, n_mcs, seed, mcs0=0, proposal=PROP_NEIGHBOUR, threads=1):
    """As sweep with a bond energy per pair of spins (Eq. (7)'s J_{q_i,q_n}):
    Jp int32[Q, Q], symmetric, zero diagonal, 2^-16 units."""
    src = np.asarray(spins)
    s = np.ascontiguousarray(src.astype(np.int32).reshape(-1))
    b = np.ascontiguousarray(np.asarray(B, dtype=np.int32))
    jp = np.ascontiguousarray(np.asarray(Jp, dtype=np.int32))
    Q = len(b)
    assert jp.shape == (Q, Q)
    d = _dims3(dims)
    f = lib().orc_sweep_pair
    f.argtypes = [C.POINTER(C.c_int32), C.c_int, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                  C.POINTER(C.c_int32), C.c_int32, C.c_float, C.c_uint64, C.c_int32, C.c_uint64, C.c_int]
    rc = f(_ptr(s, C.c_int32), int(nbr), int(proposal), _ptr(d, C.c_int32), _ptr(jp, C.c_int32),
           _ptr(b, C.c_int32), int(Q), float(kT), int(mcs0), int(n_mcs), int(seed), int(threads))
    if rc != 0:
        raise ValueError(f"orc_sweep_pair failed with {rc}")
    return s.reshape(src.shape).astype(src.dtype)


FIELD_CARRY, FIELD_RECRYSTALLISE = 0, 1


def sweep_field(spins, field, rule, nbr, dims, B, kT, n_mcs, seed, mcs0=0, J_fx=65536, threads=1):
    """As sweep with a per-site bulk field (Eq. (7)'s b_i inside grains,
    2^-16 units) added to the grain energies B; a swept site takes the field
    of the neighbour whose spin it adopts (FIELD_CARRY) or zero
    (FIELD_RECRYSTALLISE).  Returns (spins, field)."""
    src = np.asarray(spins)
    s = np.ascontiguousarray(src.astype(np.int32).reshape(-1))
    e = np.ascontiguousarray(np.asarray(field, dtype=np.int32).reshape(-1).copy())
    b = np.ascontiguousarray(np.asarray(B, dtype=np.int32))
    d = _dims3(dims)
    f = lib().orc_sweep_field
    f.argtypes = [C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int, C.c_int, C.POINTER(C.c_int32), C.c_int32,
                  C.POINTER(C.c_int32), C.c_int32, C.c_float, C.c_uint64, C.c_int32, C.c_uint64, C.c_int]
    rc = f(_ptr(s, C.c_int32), _ptr(e, C.c_int32), int(rule), int(nbr), _ptr(d, C.c_int32), int(J_fx),
           _ptr(b, C.c_int32), len(b), float(kT), int(mcs0), int(n_mcs), int(seed), int(threads))
    if rc != 0:
        raise ValueError(f"orc_sweep_field failed with {rc}")
    return s.reshape(src.shape).astype(src.dtype), e.reshape(src.shape)


def nfold(spins, nbr, dims, B, kT, seed, t_end, t_last=0.0, n_events=0, J_fx=65536,
          proposal=PROP_NEIGHBOUR, max_events=-1, Jp=None):
    """The n-fold way (rejection-free, continuous-time) counterpart of the
    Metropolis dynamics of Sec. 3, named in Sec. 1 and Sec. 4 as the
    alternative to red/black updating: run until t_end (MC steps) from the
    clock (t_last, n_events).  Jp: optional Q x Q bond energies (Eq. (7)'s
    J_{q_i,q_n}).  Returns (spins, t_last, n_events, executed)."""
    src = np.asarray(spins)
    s = np.ascontiguousarray(src.astype(np.int32).reshape(-1))
    b = np.ascontiguousarray(np.asarray(B, dtype=np.int32))
    d = _dims3(dims)
    tl = C.c_double(float(t_last))
    ne = C.c_uint64(int(n_events))
    i32p = C.POINTER(C.c_int32)
    tail = [C.c_int32, C.c_float, C.c_uint64, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_uint64), C.c_int64]
    if Jp is None:
        f = lib().orc_nfold
        f.argtypes = [i32p, C.c_int, C.c_int, i32p, C.c_int32, i32p] + tail
        bond = int(J_fx)
    else:
        jp = np.ascontiguousarray(np.asarray(Jp, dtype=np.int32))
        f = lib().orc_nfold_pair
        f.argtypes = [i32p, C.c_int, C.c_int, i32p, i32p, i32p] + tail
        bond = _ptr(jp, C.c_int32)
    f.restype = C.c_int64
    rc = f(_ptr(s, C.c_int32), int(nbr), int(proposal), _ptr(d, C.c_int32), bond, _ptr(b, C.c_int32),
           len(b), float(kT), int(seed), float(t_end), C.byref(tl), C.byref(ne), int(max_events))
    if rc < 0:
        raise ValueError(f"orc_nfold failed with {rc}")
    return s.reshape(src.shape).astype(src.dtype), tl.value, ne.value, int(rc)


def nfold_exponentials(seed, n0, count):
    """Exp(1) variates of the n-fold way's event streams n0 .. n0+count-1,
    32.32 fixed point (von Neumann's comparison method)."""
    out = np.zeros(int(count), dtype=np.uint64)
    f = lib().orc_nfold_exponentials
    f.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, C.POINTER(C.c_uint64)]
    f(int(seed), int(n0), int(count), _ptr(out, C.c_uint64))
    return out


def nfold_select(w, r):
    """Index of the entry whose cumulative weight first exceeds r, and the
    rest of r (the n-fold way's choice of site and slot); (-1, r) if r is
    not below the total."""
    a = np.ascontiguousarray(np.asarray(w, dtype=np.uint64))
    rest = C.c_uint64(0)
    f = lib().orc_nfold_select
    f.argtypes = [C.POINTER(C.c_uint64), C.c_int64, C.c_uint64, C.POINTER(C.c_uint64)]
    f.restype = C.c_int64
    i = int(f(_ptr(a, C.c_uint64), a.size, int(r), C.byref(rest)))
    return i, (rest.value if i >= 0 else int(r))


def nfold_weights(spins, nbr, dims, B, kT, J_fx=65536, proposal=PROP_NEIGHBOUR, Jp=None):
    """Integer rate weights w_ik of every slot of every site (N x S)."""
    s = np.ascontiguousarray(np.asarray(spins, dtype=np.int32).reshape(-1))
    b = np.ascontiguousarray(np.asarray(B, dtype=np.int32))
    d = _dims3(dims)
    S = num_neighbours(nbr) if proposal == PROP_NEIGHBOUR else len(b) - 1
    out = np.zeros((s.size, S), dtype=np.uint64)
    jp = None if Jp is None else np.ascontiguousarray(np.asarray(Jp, dtype=np.int32))
    f = lib().orc_nfold_weights
    f.argtypes = [C.POINTER(C.c_int32), C.c_int, C.c_int, C.POINTER(C.c_int32), C.c_int32,
                  C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int32, C.c_float, C.POINTER(C.c_uint64)]
    rc = f(_ptr(s, C.c_int32), int(nbr), int(proposal), _ptr(d, C.c_int32), int(J_fx),
           None if jp is None else _ptr(jp, C.c_int32), _ptr(b, C.c_int32), len(b), float(kT),
           _ptr(out, C.c_uint64))
    if rc < 0:
        raise ValueError("orc_nfold_weights failed")
    return out


def delta_energy_pair(spins, nbr, dims, Jp, B, i, q_new):
    s = np.ascontiguousarray(np.asarray(spins, dtype=np.int32).reshape(-1))
    b = np.ascontiguousarray(np.asarray(B, dtype=np.int32))
    jp = np.ascontiguousarray(np.asarray(Jp, dtype=np.int32))
    d = _dims3(dims)
    f = lib().orc_delta_energy_pair
    f.argtypes = [C.POINTER(C.c_int32), C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int32,
                  C.POINTER(C.c_int32), C.c_int64, C.c_int32]
    f.restype = C.c_int64
    return int(f(_ptr(s, C.c_int32), int(nbr), _ptr(d, C.c_int32), _ptr(jp, C.c_int32), len(b),
                 _ptr(b, C.c_int32), int(i), int(q_new)))


def misorientation_deg(e1, e2):
    """Cubic misorientation angle (degrees) of two Bunge orientations."""
    f = lib().orc_misorientation_deg
    f.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double)]
    f.restype = C.c_double
    a = np.ascontiguousarray(np.asarray(e1, dtype=np.float64))
    b = np.ascontiguousarray(np.asarray(e2, dtype=np.float64))
    return float(f(_ptr(a, C.c_double), _ptr(b, C.c_double)))


def read_shockley(theta_deg, J_max, theta_m_deg):
    f = lib().orc_read_shockley
    f.argtypes = [C.c_double, C.c_double, C.c_double]
    f.restype = C.c_double
    return float(f(float(theta_deg), float(J_max), float(theta_m_deg)))


def pair_table(euler, J_max, theta_m_deg):
    """Q x Q Read-Shockley bond energies (2^-16 units) of Q orientations."""
    e = np.ascontiguousarray(np.asarray(euler, dtype=np.float64).reshape(-1, 3))
    Q = e.shape[0]
    out = np.empty((Q, Q), dtype=np.int32)
    f = lib().orc_pair_table
    f.argtypes = [C.POINTER(C.c_double), C.c_int32, C.c_double, C.c_double, C.POINTER(C.c_int32)]
    f(_ptr(e, C.c_double), Q, float(J_max), float(theta_m_deg), _ptr(out, C.c_int32))
    return out


def boundary_sites(spins, nbr, dims, Q):
    """Sites with a spin in [0, Q) and at least one unlike neighbour: the
    only sites whose trial can change the state (Sec. 3)."""
    s = np.ascontiguousarray(np.asarray(spins).astype(np.int32).reshape(-1))
    d = _dims3(dims)
    f = lib().orc_boundary_sites
    f.argtypes = [C.POINTER(C.c_int32), C.c_int, C.POINTER(C.c_int32), C.c_int32]
    f.restype = C.c_int64
    return int(f(_ptr(s, C.c_int32), int(nbr), _ptr(d, C.c_int32), int(Q)))


def texture(spins, Q, grain_bin=None, n_bins=0):
    """(areas[Q], n_grains, mean_area, frac[n_bins]) of a spin field."""
    s = np.ascontiguousarray(np.asarray(spins).astype(np.int32).reshape(-1))
    areas = np.empty(Q, dtype=np.int64)
    frac = np.zeros(max(n_bins, 1), dtype=np.float64)
    ng = C.c_int32(0)
    mean = C.c_double(0.0)
    if grain_bin is None:
        gb = np.full(Q, -1, dtype=np.int32)
    else:
        gb = np.ascontiguousarray(np.asarray(grain_bin, dtype=np.int32))
    rc = lib().orc_texture(_ptr(s, C.c_int32), s.size, int(Q), _ptr(gb, C.c_int32), int(n_bins),
                           _ptr(areas, C.c_int64), C.byref(ng), C.byref(mean), _ptr(frac, C.c_double))
    if rc != 0:
        raise ValueError("texture: spin out of range")
    return areas, int(ng.value), float(mean.value), frac[:n_bins].copy()


# ------------------------------------------------ crystal plasticity (Sec. 2)

MCP_TAU0, MCP_TAUS, MCP_H0, MCP_BETA = 8.0, 122.0, 440.0, 1000.0
MLP_PARAMS = 64 * 9 + 64 + 64 * 64 + 64 + 64 + 1


def _f64(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a if n is None else a.reshape(n)


def mcp_one(euler, eps6, seed, sample=0):
    """One crystal: (E_rho [MPa], tau_c, accumulated slip, sub-steps, crystal-frame stress[6])."""
    e, s = _f64(euler, 3), _f64(eps6, 6)
    tc, gm, sig = C.c_double(), C.c_double(), np.zeros(6)
    K = C.c_int()
    E = lib().orc_mcp_one(_ptr(e, C.c_double), _ptr(s, C.c_double), int(seed), int(sample), C.byref(tc),
                          C.byref(gm), C.byref(K), _ptr(sig, C.c_double))
    return E, tc.value, gm.value, K.value, sig


def mcp_run(euler, eps6, seed, K, sample=0, dll=None):
    """One crystal in an explicit number K of sub-steps: (E_rho, tau_c,
    accumulated slip, crystal-frame stress[6], candidates per sub-step[K],
    system picked per sub-step[K], -1 when elastic).  dll: another build of
    this library (the tests' planted-mistake copies), default this one."""
    e, s = _f64(euler, 3), _f64(eps6, 6)
    tc, gm, sig = C.c_double(), C.c_double(), np.zeros(6)
    nc, picks = np.zeros(K, np.int32), np.zeros(K, np.int32)
    f = (dll or lib()).orc_mcp_run
    f.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_uint64, C.c_uint64, C.c_int,
                  C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int32),
                  C.POINTER(C.c_int32)]
    f.restype = C.c_double
    E = f(_ptr(e, C.c_double), _ptr(s, C.c_double), int(seed), int(sample), int(K), C.byref(tc), C.byref(gm),
          _ptr(sig, C.c_double), _ptr(nc, C.c_int32), _ptr(picks, C.c_int32))
    return E, tc.value, gm.value, sig, nc, picks


def mcp_picks(euler, eps6, seed, n, K, step, sample0=0, dll=None):
    """(system picked at sub-step `step` of K, candidates at that sub-step)
    for n sample indices of one crystal."""
    e, s = _f64(euler, 3), _f64(eps6, 6)
    picks, nc = np.full(n, -2, np.int32), np.zeros(n, np.int32)
    f = (dll or lib()).orc_mcp_picks
    f.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_uint64, C.c_uint64, C.c_int64, C.c_int,
                  C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    f(_ptr(e, C.c_double), _ptr(s, C.c_double), int(seed), int(sample0), int(n), int(K), int(step),
      _ptr(picks, C.c_int32), _ptr(nc, C.c_int32))
    return picks, nc


def mcp_solve(euler, eps6, seed, sample0=0, threads=1):
    """Many crystals: (E_rho, tau_c, accumulated slip) arrays."""
    e = _f64(euler).reshape(-1, 3)
    s = _f64(eps6).reshape(-1, 6)
    n = e.shape[0]
    E, tc, gm = np.empty(n), np.empty(n), np.empty(n)
    lib().orc_mcp_solve(_ptr(e, C.c_double), _ptr(s, C.c_double), n, int(seed), int(sample0),
                        _ptr(E, C.c_double), _ptr(tc, C.c_double), _ptr(gm, C.c_double), int(threads))
    return E, tc, gm


def mcp_select(p, R):
    """Eq. (2): the slip system chosen by R from probabilities p."""
    pa = _f64(p)
    return lib().orc_mcp_select(_ptr(pa, C.c_double), len(pa), float(R))


def mcp_tau_c(gamma):
    return lib().orc_mcp_tau_c(float(gamma))


def mcp_shear_modulus():
    return lib().orc_mcp_shear_modulus()


def mcp_slip_systems():
    n, d = np.zeros((12, 3)), np.zeros((12, 3))
    lib().orc_mcp_slip_systems(_ptr(n, C.c_double), _ptr(d, C.c_double))
    return n, d


def mlp_forward(theta, X):
    th, x = _f64(theta), _f64(X).reshape(-1, 9)
    y = np.empty(x.shape[0])
    lib().orc_mlp_forward(_ptr(th, C.c_double), _ptr(x, C.c_double), x.shape[0], _ptr(y, C.c_double))
    return y


def mlp_loss_grad(theta, X, t):
    th, x, tt = _f64(theta), _f64(X).reshape(-1, 9), _f64(t)
    g = np.empty(MLP_PARAMS)
    loss = lib().orc_mlp_loss_grad(_ptr(th, C.c_double), _ptr(x, C.c_double), _ptr(tt, C.c_double), x.shape[0],
                                   _ptr(g, C.c_double))
    return loss, g


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """In place on theta, m, v (float64 arrays)."""
    lib().orc_adam_step(_ptr(theta, C.c_double), _ptr(_f64(g), C.c_double), _ptr(m, C.c_double),
                        _ptr(v, C.c_double), int(t), float(lr), float(b1), float(b2), float(eps))


def available_threads():
    return max(1, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
