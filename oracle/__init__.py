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
        path = _build.ensure_built()
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


def available_threads():
    return max(1, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
