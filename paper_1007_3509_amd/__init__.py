"""Python binding of libhmc (include/hmc.h): argument marshalling only.

Every function here has the name of the C entry point it calls and does no
arithmetic of the method; all of it runs in the HIP library.  If the library
is not built the import still works but the first call raises, loudly --
there is no CPU fallback.

The method is the red/black Q-state Potts sweep with a per-grain bulk energy
of Zhang, Dingreville, Bartel & Lusk (arXiv:1007.3509), Sec. 3 Eq. (7) and
Sec. 4.
"""
import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhmc.so")

HMC_OK, HMC_E_INVAL, HMC_E_NOMEM, HMC_E_DEVICE, HMC_E_RANGE, HMC_E_STATE, HMC_E_INTERNAL = 0, -1, -2, -3, -4, -5, -6
HMC_VN4, HMC_MOORE8, HMC_VN6, HMC_MOORE26 = 0, 1, 2, 3
HMC_I16, HMC_I32 = 0, 1
HMC_PROP_NEIGHBOUR, HMC_PROP_UNIFORM = 0, 1

NDIM = {HMC_VN4: 2, HMC_MOORE8: 2, HMC_VN6: 3, HMC_MOORE26: 3}
COLOURS = {HMC_VN4: 2, HMC_MOORE8: 4, HMC_VN6: 2, HMC_MOORE26: 8}

_STATUS = {0: "HMC_OK", -1: "HMC_E_INVAL", -2: "HMC_E_NOMEM", -3: "HMC_E_DEVICE", -4: "HMC_E_RANGE",
           -5: "HMC_E_STATE", -6: "HMC_E_INTERNAL"}


class HmcError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class hmc_lattice_desc(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("dims", C.c_int32 * 3), ("nbr", C.c_int32), ("spin", C.c_int32),
                ("proposal", C.c_int32), ("J_fx", C.c_int32)]


_lib = None

# (name, restype, argtypes)
_SIGS = [
    ("hmc_abi_version", C.c_int32, []),
    ("hmc_last_error", C.c_char_p, []),
    ("hmc_device_count", C.c_int32, []),
    ("hmc_lattice_create", C.c_int32, [C.POINTER(hmc_lattice_desc), C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    ("hmc_lattice_init", C.c_int32, [C.POINTER(hmc_lattice_desc), C.c_int32, C.c_uint64, C.c_void_p,
                                     C.POINTER(C.c_void_p)]),
    ("hmc_lattice_wrap", C.c_int32, [C.POINTER(hmc_lattice_desc), C.c_void_p, C.c_int32, C.c_void_p,
                                     C.POINTER(C.c_void_p)]),
    ("hmc_lattice_free", C.c_int32, [C.c_void_p]),
    ("hmc_set_grain_energy", C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32]),
    ("hmc_set_pair_energy", C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32]),
    ("hmc_set_site_energy", C.c_int32, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_int32, C.c_int32]),
    ("hmc_get_site_energy", C.c_int32, [C.c_void_p, C.c_void_p, C.c_uint64]),
    ("hmc_misorientation_energy", C.c_int32, [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                              C.c_void_p]),
    ("hmc_sweep", C.c_int32, [C.c_void_p, C.c_float, C.c_int32, C.c_uint64]),
    ("hmc_texture_stats", C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                                      C.POINTER(C.c_double), C.c_void_p]),
    ("hmc_grain_areas", C.c_int32, [C.c_void_p, C.c_void_p]),
    ("hmc_texture_stats_static", C.c_int32, [C.c_void_p, C.c_int32, C.c_uint64, C.c_int32, C.c_void_p, C.c_int32,
                                             C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.c_void_p]),
    ("hmc_get_spins", C.c_int32, [C.c_void_p, C.c_void_p, C.c_uint64]),
    ("hmc_set_spins", C.c_int32, [C.c_void_p, C.c_void_p, C.c_uint64]),
    ("hmc_snapshot", C.c_int32, [C.c_void_p]),
    ("hmc_restore", C.c_int32, [C.c_void_p]),
    ("hmc_get_mcs", C.c_int32, [C.c_void_p, C.POINTER(C.c_uint64)]),
    ("hmc_set_mcs", C.c_int32, [C.c_void_p, C.c_uint64]),
    ("hmc_set_tiling", C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    ("hmc_get_tiling", C.c_int32, [C.c_void_p, C.c_void_p]),
    ("hmc_set_sweep_kernel", C.c_int32, [C.c_void_p, C.c_int32]),
    ("hmc_get_sweep_kernel", C.c_int32, [C.c_void_p, C.POINTER(C.c_int32)]),
    ("hmc_profile", C.c_int32, [C.c_void_p, C.c_int32]),
    ("hmc_profile_read", C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int64)]),
    ("hmc_profile_trials", C.c_int32, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("hmc_boundary_sites", C.c_int32, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("hmc_synchronize", C.c_int32, [C.c_void_p]),
    ("hmc_threshold_table_host", C.c_int32, [C.c_float, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                             C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64]),
    ("hmc_threshold_table", C.c_int32, [C.c_void_p, C.c_float, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p,
                                        C.c_uint64]),
    ("hmc_ensemble_create", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)]),
    ("hmc_ensemble_set_tiling", C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    ("hmc_ensemble_get_tiling", C.c_int32, [C.c_void_p, C.c_void_p]),
    ("hmc_ensemble_sweep", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    ("hmc_ensemble_synchronize", C.c_int32, [C.c_void_p]),
    ("hmc_ensemble_autotune", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    ("hmc_ensemble_free", C.c_int32, [C.c_void_p]),
    ("hmc_ensemble_profile", C.c_int32, [C.c_void_p, C.c_int32]),
    ("hmc_ensemble_profile_read", C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                              C.POINTER(C.c_int64)]),
    ("hmc_nfold", C.c_int32, [C.c_void_p, C.c_float, C.c_double, C.c_uint64]),
    ("hmc_nfold_batch", C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_double, C.c_void_p]),
    ("hmc_nfold_clock", C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.POINTER(C.c_uint64)]),
    ("hmc_nfold_set_clock", C.c_int32, [C.c_void_p, C.c_double, C.c_double, C.c_uint64]),
    ("hmc_nfold_exponentials", C.c_int32, [C.c_uint64, C.c_uint64, C.c_int64, C.c_int32, C.c_void_p]),
    ("hmc_autotune", C.c_int32, [C.POINTER(hmc_lattice_desc), C.c_int32, C.c_float, C.c_int32, C.c_char_p,
                                 C.c_void_p, C.POINTER(C.c_double)]),
    ("hmc_tuning_load", C.c_int32, [C.c_char_p, C.POINTER(C.c_int32)]),
    ("hmc_mcp_solve", C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_uint64, C.c_uint64, C.c_int32,
                                  C.c_void_p, C.c_void_p]),
    ("hmc_mlp_create", C.c_int32, [C.c_uint64, C.POINTER(C.c_void_p)]),
    ("hmc_mlp_free", C.c_int32, [C.c_void_p]),
    ("hmc_mlp_get_params", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hmc_mlp_set_params", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hmc_mlp_train", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32,
                                  C.c_int32, C.c_float, C.c_uint64, C.POINTER(C.c_float)]),
    ("hmc_mlp_predict", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]),
    ("hmc_mlp_infer", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    ("hmc_mlp_forward", C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    ("hmc_mlp_loss_grad", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_float),
                                      C.c_void_p]),
    ("hmc_mlp_adam_step", C.c_int32, [C.c_void_p, C.c_void_p, C.c_float]),
    ("hmc_surrogate_update", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                                         C.c_int32, C.c_double, C.c_uint64, C.POINTER(C.c_int32),
                                         C.POINTER(C.c_double), C.c_void_p]),
]


def lib():
    """The loaded libhmc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # HMC_LIBRARY: another build of this same library (e.g. the host-sanitizer build)
        path = os.environ.get("HMC_LIBRARY") or LIB_PATH
        if not os.path.exists(path):
            raise ImportError(f"libhmc.so is not built ({path}); run __graft_entry__.build()")
        L = C.CDLL(path)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_names():
    return [s[0] for s in _SIGS]


def _check(status):
    if status != HMC_OK:
        raise HmcError(status, lib().hmc_last_error().decode())


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def make_desc(dims, nbr, spin=HMC_I16, proposal=HMC_PROP_NEIGHBOUR, J_fx=65536):
    d = hmc_lattice_desc()
    d.ndim = len(dims)
    for a in range(3):
        d.dims[a] = int(dims[a]) if a < len(dims) else 1
    d.nbr, d.spin, d.proposal, d.J_fx = int(nbr), int(spin), int(proposal), int(J_fx)
    return d


# ----------------------------------------------------------- C entry points

def hmc_abi_version():
    return lib().hmc_abi_version()


def hmc_device_count():
    return lib().hmc_device_count()


def hmc_lattice_create(desc, n_grains, stream=None):
    h = C.c_void_p()
    _check(lib().hmc_lattice_create(C.byref(desc), int(n_grains), stream, C.byref(h)))
    return h


def hmc_lattice_init(desc, n_grains, voronoi_seed, stream=None):
    h = C.c_void_p()
    _check(lib().hmc_lattice_init(C.byref(desc), int(n_grains), int(voronoi_seed), stream, C.byref(h)))
    return h


def hmc_lattice_wrap(desc, dev_ptr, n_grains, stream=None):
    """Lattice over a caller-owned device buffer (an integer device address,
    e.g. a torch tensor's data_ptr()); the buffer must outlive the handle."""
    h = C.c_void_p()
    _check(lib().hmc_lattice_wrap(C.byref(desc), C.c_void_p(int(dev_ptr)), int(n_grains), stream, C.byref(h)))
    return h.value


def hmc_lattice_free(h):
    _check(lib().hmc_lattice_free(h))


def hmc_set_grain_energy(h, B_fx):
    b = np.ascontiguousarray(np.asarray(B_fx, dtype=np.int32))
    _check(lib().hmc_set_grain_energy(h, _ptr(b), int(b.size), 0))


def hmc_set_pair_energy(h, Jp):
    """Pair bond energies int32[Q, Q] (2^-16 units), or None for the uniform J_fx."""
    if Jp is None:
        _check(lib().hmc_set_pair_energy(h, None, 0, 0))
        return
    j = np.ascontiguousarray(np.asarray(Jp, dtype=np.int32))
    _check(lib().hmc_set_pair_energy(h, _ptr(j), j.shape[0], 0))


HMC_FIELD_CARRY, HMC_FIELD_RECRYSTALLISE = 0, 1


def hmc_set_site_energy(h, E_site, rule=HMC_FIELD_CARRY):
    """Per-site bulk field int32[N] (2^-16 units), or None to remove it."""
    if E_site is None:
        _check(lib().hmc_set_site_energy(h, None, 0, 0, 0))
        return
    e = np.ascontiguousarray(np.asarray(E_site, dtype=np.int32))
    _check(lib().hmc_set_site_energy(h, _ptr(e), e.size, 0, int(rule)))


def hmc_get_site_energy(h, shape):
    out = np.empty(shape, dtype=np.int32)
    _check(lib().hmc_get_site_energy(h, _ptr(out), out.size))
    return out


def hmc_misorientation_energy(euler, J_max, theta_m_deg):
    e = np.ascontiguousarray(np.asarray(euler, dtype=np.float64).reshape(-1, 3))
    out = np.empty((e.shape[0], e.shape[0]), dtype=np.int32)
    _check(lib().hmc_misorientation_energy(_ptr(e), e.shape[0], float(J_max), float(theta_m_deg), 0, _ptr(out)))
    return out


def hmc_sweep(h, kT, n_mcs, seed):
    _check(lib().hmc_sweep(h, float(kT), int(n_mcs), int(seed)))


def hmc_texture_stats(h, grain_bin=None, n_bins=0):
    ng = C.c_int32()
    mean = C.c_double()
    frac = np.zeros(max(int(n_bins), 1), dtype=np.float64)
    gb = None if grain_bin is None else np.ascontiguousarray(np.asarray(grain_bin, dtype=np.int32))
    _check(lib().hmc_texture_stats(h, None if gb is None else _ptr(gb), int(n_bins), C.byref(ng), C.byref(mean),
                                   _ptr(frac)))
    return int(ng.value), float(mean.value), frac[:int(n_bins)].copy()


HMC_STATIC_MAX_GRAINS, HMC_STATIC_MAX_BINS = 65536, 1024


def hmc_texture_stats_static(dev_spins, spin, n_sites, n_grains, grain_bin=None, n_bins=0, stream=None):
    """Grain statistics of n_sites spins in device memory at address
    dev_spins, without any allocation: (n_grains present, mean area, frac)."""
    ng = C.c_int32()
    mean = C.c_double()
    frac = np.zeros(max(int(n_bins), 1), dtype=np.float64)
    gb = None if grain_bin is None else np.ascontiguousarray(np.asarray(grain_bin, dtype=np.int32))
    _check(lib().hmc_texture_stats_static(C.c_void_p(int(dev_spins) if dev_spins else None), int(spin), int(n_sites),
                                          int(n_grains), None if gb is None else _ptr(gb), int(n_bins),
                                          None if stream is None else C.c_void_p(int(stream)), C.byref(ng),
                                          C.byref(mean), _ptr(frac)))
    return int(ng.value), float(mean.value), frac[:int(n_bins)].copy()


def hmc_grain_areas(h, n_grains):
    out = np.empty(int(n_grains), dtype=np.int64)
    _check(lib().hmc_grain_areas(h, _ptr(out)))
    return out


def hmc_get_spins(h, shape, dtype):
    out = np.empty(shape, dtype=dtype)
    _check(lib().hmc_get_spins(h, _ptr(out), out.nbytes))
    return out


def hmc_set_spins(h, spins):
    s = np.ascontiguousarray(spins)
    _check(lib().hmc_set_spins(h, _ptr(s), s.nbytes))


def hmc_snapshot(h):
    _check(lib().hmc_snapshot(h))


def hmc_restore(h):
    _check(lib().hmc_restore(h))


def hmc_get_mcs(h):
    v = C.c_uint64()
    _check(lib().hmc_get_mcs(h, C.byref(v)))
    return int(v.value)


def hmc_set_mcs(h, mcs):
    _check(lib().hmc_set_mcs(h, int(mcs)))


def hmc_set_tiling(h, tx=0, ty=0, tz=0, mcs_per_launch=0):
    _check(lib().hmc_set_tiling(h, int(tx), int(ty), int(tz), int(mcs_per_launch)))


HMC_KERNEL_AUTO, HMC_KERNEL_GENERIC, HMC_KERNEL_COMPILED = 0, 1, 2


def hmc_set_sweep_kernel(h, which):
    _check(lib().hmc_set_sweep_kernel(h, int(which)))


def hmc_get_sweep_kernel(h):
    w = C.c_int32()
    _check(lib().hmc_get_sweep_kernel(h, C.byref(w)))
    return int(w.value)


def hmc_get_tiling(h):
    out = np.zeros(4, dtype=np.int32)
    _check(lib().hmc_get_tiling(h, _ptr(out)))
    return tuple(int(v) for v in out)


def hmc_profile(h, enable=True):
    _check(lib().hmc_profile(h, int(bool(enable))))


def hmc_profile_read(h):
    ms = C.c_double()
    n = C.c_int64()
    su = C.c_int64()
    _check(lib().hmc_profile_read(h, C.byref(ms), C.byref(n), C.byref(su)))
    return float(ms.value), int(n.value), int(su.value)


def hmc_profile_trials(h):
    n = C.c_int64()
    _check(lib().hmc_profile_trials(h, C.byref(n)))
    return n.value


def hmc_boundary_sites(h):
    n = C.c_int64()
    _check(lib().hmc_boundary_sites(h, C.byref(n)))
    return n.value


def hmc_synchronize(h):
    _check(lib().hmc_synchronize(h))


def hmc_threshold_table_host(kT, M, J_fx, Bmin, Bmax):
    """(layout dict, table uint32[rows*TW], bounds uint32[2*rows*nb]) as the
    host builds them, no device needed."""
    lay = np.zeros(6, np.int32)
    _check(lib().hmc_threshold_table_host(float(kT), int(M), int(J_fx), int(Bmin), int(Bmax), _ptr(lay), None, 0,
                                          None, 0))
    dn_lo, rows, R, TW, nb, bw = (int(v) for v in lay)
    table = np.zeros(rows * TW, np.uint32)
    bounds = np.zeros(2 * rows * nb, np.uint32)
    _check(lib().hmc_threshold_table_host(float(kT), int(M), int(J_fx), int(Bmin), int(Bmax), _ptr(lay), _ptr(table),
                                          table.size, _ptr(bounds), bounds.size))
    return dict(kind=0, dn_lo=dn_lo, rows=rows, R=R, TW=TW, nb=nb, bw=bw, Dmax=-1), table, bounds


def hmc_threshold_table(h, kT):
    """(layout dict, table, bounds) that a sweep of the lattice at kT reads,
    copied back from device memory."""
    lay = np.zeros(8, np.int32)
    _check(lib().hmc_threshold_table(h, float(kT), _ptr(lay), None, 0, None, 0))
    kind, dn_lo, rows, R, TW, nb, bw, Dmax = (int(v) for v in lay)
    table = np.zeros(rows * TW, np.uint32)
    bounds = np.zeros(2 * rows * nb, np.uint32)
    _check(lib().hmc_threshold_table(h, float(kT), _ptr(lay), _ptr(table), table.size, _ptr(bounds) if bounds.size else None,
                                     bounds.size))
    return dict(kind=kind, dn_lo=dn_lo, rows=rows, R=R, TW=TW, nb=nb, bw=bw, Dmax=Dmax), table, bounds


def _handles(lats):
    hs = [l.h if isinstance(l, Lattice) else l for l in lats]
    arr = (C.c_void_p * len(hs))(*[h.value if isinstance(h, C.c_void_p) else h for h in hs])
    return arr, len(hs)


def hmc_ensemble_create(lats):
    arr, n = _handles(lats)
    h = C.c_void_p()
    _check(lib().hmc_ensemble_create(arr, n, C.byref(h)))
    return h


def hmc_ensemble_set_tiling(E, tx=0, ty=0, tz=0, mcs_per_launch=0):
    _check(lib().hmc_ensemble_set_tiling(E, int(tx), int(ty), int(tz), int(mcs_per_launch)))


def hmc_ensemble_get_tiling(E):
    out = np.zeros(4, dtype=np.int32)
    _check(lib().hmc_ensemble_get_tiling(E, _ptr(out)))
    return tuple(int(v) for v in out)


def hmc_ensemble_sweep(E, kT, seed, n_mcs):
    k = np.ascontiguousarray(np.asarray(kT, dtype=np.float32))
    s = np.ascontiguousarray(np.asarray(seed, dtype=np.uint64))
    _check(lib().hmc_ensemble_sweep(E, _ptr(k), _ptr(s), int(n_mcs)))


def hmc_ensemble_synchronize(E):
    _check(lib().hmc_ensemble_synchronize(E))


def hmc_ensemble_profile(E, enable):
    _check(lib().hmc_ensemble_profile(E, int(bool(enable))))


def hmc_ensemble_profile_read(E):
    ms, n, su = C.c_double(), C.c_int64(), C.c_int64()
    _check(lib().hmc_ensemble_profile_read(E, C.byref(ms), C.byref(n), C.byref(su)))
    return ms.value, n.value, su.value


def hmc_ensemble_autotune(E, kT, seed, n_mcs):
    k = np.ascontiguousarray(np.asarray(kT, dtype=np.float32))
    s = np.ascontiguousarray(np.asarray(seed, dtype=np.uint64))
    out = np.zeros(4, dtype=np.int32)
    _check(lib().hmc_ensemble_autotune(E, _ptr(k), _ptr(s), int(n_mcs), _ptr(out)))
    return tuple(int(v) for v in out)


def hmc_ensemble_free(E):
    _check(lib().hmc_ensemble_free(E))


def hmc_nfold(h, kT, mcs, seed):
    _check(lib().hmc_nfold(h, float(kT), float(mcs), int(seed)))


def hmc_nfold_batch(lats, kT, mcs, seed):
    arr, n = _handles(lats)
    k = np.ascontiguousarray(np.asarray(kT, dtype=np.float32).reshape(-1))
    s = np.ascontiguousarray(np.asarray(seed, dtype=np.uint64).reshape(-1))
    if k.size != n or s.size != n:
        raise ValueError("one kT and one seed per lattice")
    _check(lib().hmc_nfold_batch(arr, n, _ptr(k), float(mcs), _ptr(s)))


def hmc_nfold_clock(h):
    t_now, t_last, ne = C.c_double(), C.c_double(), C.c_uint64()
    _check(lib().hmc_nfold_clock(h, C.byref(t_now), C.byref(t_last), C.byref(ne)))
    return t_now.value, t_last.value, ne.value


def hmc_nfold_set_clock(h, t_now, t_last, n_events):
    _check(lib().hmc_nfold_set_clock(h, float(t_now), float(t_last), int(n_events)))


def hmc_nfold_exponentials(seed, n0, count, window=64):
    out = np.zeros(int(count), dtype=np.uint64)
    _check(lib().hmc_nfold_exponentials(int(seed), int(n0), int(count), int(window), _ptr(out)))
    return out


def hmc_autotune(desc, n_grains, kT, n_mcs, cache_path=None):
    out = np.zeros(4, dtype=np.int32)
    us = C.c_double()
    path = None if cache_path is None else str(cache_path).encode()
    _check(lib().hmc_autotune(C.byref(desc), int(n_grains), float(kT), int(n_mcs), path, _ptr(out), C.byref(us)))
    return tuple(int(v) for v in out), float(us.value)


def hmc_tuning_load(cache_path):
    n = C.c_int32()
    _check(lib().hmc_tuning_load(str(cache_path).encode(), C.byref(n)))
    return int(n.value)


MLP_PARAMS = 4865


def _f64(a, cols=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a if cols is None else a.reshape(-1, cols)


def hmc_mcp_solve(euler, eps, seed, sample0=0, with_tauc=False):
    e, p = _f64(euler, 3), _f64(eps, 6)
    n = e.shape[0]
    E = np.empty(n)
    tc = np.empty(n) if with_tauc else None
    _check(lib().hmc_mcp_solve(_ptr(e), _ptr(p), n, int(seed), int(sample0), 0, _ptr(E),
                               None if tc is None else _ptr(tc)))
    return (E, tc) if with_tauc else E


def hmc_mlp_create(seed=0):
    h = C.c_void_p()
    _check(lib().hmc_mlp_create(int(seed), C.byref(h)))
    return h


def hmc_mlp_free(M):
    _check(lib().hmc_mlp_free(M))


def hmc_mlp_get_params(M):
    th = np.empty(MLP_PARAMS, dtype=np.float32)
    norm = np.empty(2)
    _check(lib().hmc_mlp_get_params(M, _ptr(th), _ptr(norm)))
    return th, norm


def hmc_mlp_set_params(M, theta, norm=None):
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float32))
    nm = None if norm is None else np.ascontiguousarray(np.asarray(norm, dtype=np.float64))
    _check(lib().hmc_mlp_set_params(M, _ptr(th), None if nm is None else _ptr(nm)))


def hmc_mlp_train(M, euler, eps, E, epochs, batch, lr, seed):
    e, p, y = _f64(euler, 3), _f64(eps, 6), _f64(E)
    loss = C.c_float()
    _check(lib().hmc_mlp_train(M, _ptr(e), _ptr(p), _ptr(y), e.shape[0], 0, int(epochs), int(batch), float(lr),
                               int(seed), C.byref(loss)))
    return float(loss.value)


def hmc_mlp_predict(M, euler, eps):
    e, p = _f64(euler, 3), _f64(eps, 6)
    out = np.empty(e.shape[0])
    _check(lib().hmc_mlp_predict(M, _ptr(e), _ptr(p), e.shape[0], 0, _ptr(out)))
    return out


def hmc_mlp_infer(M, X_dev_ptr, y_dev_ptr, n, stream=None):
    """Device addresses in and out (scaled features n x 9 float32 -> n
    standardised float32 outputs); asynchronous on `stream`."""
    _check(lib().hmc_mlp_infer(M, C.c_void_p(int(X_dev_ptr)), C.c_void_p(int(y_dev_ptr)), int(n), stream))


def hmc_mlp_forward(M, X):
    x = np.ascontiguousarray(np.asarray(X, dtype=np.float32).reshape(-1, 9))
    y = np.empty(x.shape[0], dtype=np.float32)
    _check(lib().hmc_mlp_forward(M, _ptr(x), x.shape[0], _ptr(y)))
    return y


def hmc_mlp_loss_grad(M, X, t):
    x = np.ascontiguousarray(np.asarray(X, dtype=np.float32).reshape(-1, 9))
    tt = np.ascontiguousarray(np.asarray(t, dtype=np.float32))
    g = np.empty(MLP_PARAMS, dtype=np.float32)
    loss = C.c_float()
    _check(lib().hmc_mlp_loss_grad(M, _ptr(x), _ptr(tt), x.shape[0], C.byref(loss), _ptr(g)))
    return float(loss.value), g


def hmc_mlp_adam_step(M, grad, lr):
    g = np.ascontiguousarray(np.asarray(grad, dtype=np.float32))
    _check(lib().hmc_mlp_adam_step(M, _ptr(g), float(lr)))


def hmc_surrogate_update(L, M, euler, eps6, E_scale, mode=0, n_audit=64, audit_tol=0.05, seed=0):
    h = L.h if isinstance(L, Lattice) else L
    e = _f64(euler, 3)
    p = _f64(eps6)
    used = C.c_int32()
    err = C.c_double()
    B = np.empty(e.shape[0], dtype=np.int32)
    _check(lib().hmc_surrogate_update(h, M, _ptr(e), _ptr(p), float(E_scale), int(mode), int(n_audit),
                                      float(audit_tol), int(seed), C.byref(used), C.byref(err), _ptr(B)))
    return B, bool(used.value), float(err.value)


# --------------------------------------------------------- convenience class

class Lattice:
    """Owns one hmc_lattice handle (same calls, numpy in and out)."""

    def __init__(self, dims, nbr, n_grains, voronoi_seed=None, spin=HMC_I16, proposal=HMC_PROP_NEIGHBOUR,
                 J_fx=65536, stream=None, dev_ptr=None):
        self.dims = tuple(int(d) for d in dims)
        self.nbr, self.spin, self.n_grains = int(nbr), int(spin), int(n_grains)
        self.dtype = np.int16 if spin == HMC_I16 else np.int32
        desc = make_desc(self.dims, nbr, spin, proposal, J_fx)
        if dev_ptr is not None:
            self.h = hmc_lattice_wrap(desc, dev_ptr, n_grains, stream)
        elif voronoi_seed is None:
            self.h = hmc_lattice_create(desc, n_grains, stream)
        else:
            self.h = hmc_lattice_init(desc, n_grains, voronoi_seed, stream)

    @property
    def shape(self):
        return tuple(reversed(self.dims))

    def set_grain_energy(self, B_fx):
        hmc_set_grain_energy(self.h, B_fx)

    def set_pair_energy(self, Jp):
        hmc_set_pair_energy(self.h, Jp)

    def set_site_energy(self, E_site, rule=HMC_FIELD_CARRY):
        hmc_set_site_energy(self.h, E_site, rule)

    def site_energy(self):
        return hmc_get_site_energy(self.h, self.shape)

    def sweep(self, kT, n_mcs, seed):
        hmc_sweep(self.h, kT, n_mcs, seed)

    def nfold(self, kT, mcs, seed):
        """Advance by mcs MC steps of continuous time with the n-fold way."""
        hmc_nfold(self.h, kT, mcs, seed)

    def nfold_clock(self):
        """(t_now, t_last, n_events) of the n-fold way."""
        return hmc_nfold_clock(self.h)

    def set_nfold_clock(self, t_now, t_last, n_events):
        hmc_nfold_set_clock(self.h, t_now, t_last, n_events)

    def spins(self):
        return hmc_get_spins(self.h, self.shape, self.dtype)

    def set_spins(self, s):
        hmc_set_spins(self.h, np.asarray(s, dtype=self.dtype).reshape(self.shape))

    def texture_stats(self, grain_bin=None, n_bins=0):
        return hmc_texture_stats(self.h, grain_bin, n_bins)

    def grain_areas(self):
        return hmc_grain_areas(self.h, self.n_grains)

    @property
    def mcs(self):
        return hmc_get_mcs(self.h)

    @mcs.setter
    def mcs(self, v):
        hmc_set_mcs(self.h, v)

    def set_tiling(self, tx=0, ty=0, tz=0, mcs_per_launch=0):
        hmc_set_tiling(self.h, tx, ty, tz, mcs_per_launch)

    def tiling(self):
        return hmc_get_tiling(self.h)

    def boundary_sites(self):
        return hmc_boundary_sites(self.h)

    def synchronize(self):
        hmc_synchronize(self.h)

    def close(self):
        if getattr(self, "h", None):
            hmc_lattice_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
