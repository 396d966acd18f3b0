"""Seeded synthetic inputs shared by the HIP path, the oracle, tests and bench.

This module holds none of the sweep's arithmetic: it only draws the per-grain
quantities that the workloads are defined by (Schmid factors, bulk energies,
temperatures, lattice sizes, seeds) with numpy's PCG64, and quantises the
energies to the 2^-16 fixed point both paths consume.  The random numbers the
method itself draws (Voronoi seed points, Metropolis trials) come from each
side's own Philox implementation, keyed by the seeds given here.

Workloads (all synthetic, shaped after the paper's experiments: square and
cubic periodic lattices, Voronoi polycrystals, per-orientation bulk energies):

  voronoi_2d_64      64x64 VN4, int32, 40 grains, zero bulk energy, kT 0.5,
                     100 MCS, seeds 1.
  schmid_2d_1024     1024x1024 VN4, int16, 2000 grains, m_g ~ U[0.27,0.5]
                     (PCG64 2002), E_g = 0.2 m_g, kT 0.5, 1000 MCS, seeds 2.
  schmid_3d_256      256^3 VN6, int16, 20000 grains, Schmid factor of a
                     uniform SO(3) orientation (Shoemake, PCG64 3003) under a
                     [001] load, E_g = 0.15 m_g, kT 0.6, 500 MCS, seeds 3.
  ensemble_moore8    64 Moore-8 lattices, sides in {128,...,1024}, 50..2000
                     grains, kT ~ U[0.3,1.0], energies as schmid_2d_1024,
                     1000 MCS (PCG64 4004), seeds 40000+j / 4000+j.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

VN4, MOORE8, VN6, MOORE26 = 0, 1, 2, 3
I16, I32 = 0, 1

FIXED_ONE = 65536  # 2^16: energies are stored as int32 multiples of 2^-16


def quantise(E):
    """Energy -> int32 in 2^-16 units, rounding half to even."""
    return np.rint(np.asarray(E, dtype=np.float64) * FIXED_ONE).astype(np.int32)


# ---------------------------------------------------------------- Schmid

def fcc_slip_systems():
    """The 12 FCC {111}<110> slip systems as unit (normal, direction) pairs."""
    normals = [(1, 1, 1), (-1, 1, 1), (1, -1, 1), (1, 1, -1)]
    dirs = [(1, -1, 0), (1, 0, -1), (0, 1, -1), (1, 1, 0), (1, 0, 1), (0, 1, 1)]
    n_out, d_out = [], []
    for n in normals:
        n = np.asarray(n, dtype=np.float64)
        for d in dirs:
            d = np.asarray(d, dtype=np.float64)
            if abs(float(n @ d)) < 1e-12:
                n_out.append(n / np.linalg.norm(n))
                d_out.append(d / np.linalg.norm(d))
    return np.asarray(n_out), np.asarray(d_out)


def schmid_factor(load_axes):
    """max over the 12 systems of |l.n||l.d| for unit load axes l (crystal frame)."""
    l = np.atleast_2d(np.asarray(load_axes, dtype=np.float64))
    l = l / np.linalg.norm(l, axis=1, keepdims=True)
    n, d = fcc_slip_systems()
    return np.max(np.abs(l @ n.T) * np.abs(l @ d.T), axis=1)


def shoemake_quaternions(rng, count):
    """Uniform random unit quaternions (w, x, y, z), Shoemake's method."""
    u1, u2, u3 = rng.random(count), rng.random(count), rng.random(count)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    x, y = a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2)
    z, w = b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)
    return np.stack([w, x, y, z], axis=1)


def quat_to_matrix(q):
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z); R[:, 0, 1] = 2 * (x * y - z * w); R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w); R[:, 1, 1] = 1 - 2 * (x * x + z * z); R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w); R[:, 2, 1] = 2 * (y * z + x * w); R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def matrix_to_bunge(R):
    """Bunge ZXZ Euler angles (phi1, Phi, phi2) of passive rotation matrices."""
    Phi = np.arccos(np.clip(R[:, 2, 2], -1.0, 1.0))
    phi1 = np.arctan2(R[:, 2, 0], -R[:, 2, 1])
    phi2 = np.arctan2(R[:, 0, 2], R[:, 1, 2])
    small = np.abs(np.sin(Phi)) < 1e-9
    phi1 = np.where(small, np.arctan2(R[:, 0, 1], R[:, 0, 0]), phi1)
    phi2 = np.where(small, 0.0, phi2)
    return np.stack([np.mod(phi1, 2 * np.pi), Phi, np.mod(phi2, 2 * np.pi)], axis=1)


def bunge_to_matrix(e):
    """Passive (sample -> crystal) rotation from Bunge ZXZ angles."""
    e = np.atleast_2d(np.asarray(e, dtype=np.float64))
    c1, s1 = np.cos(e[:, 0]), np.sin(e[:, 0])
    c, s = np.cos(e[:, 1]), np.sin(e[:, 1])
    c2, s2 = np.cos(e[:, 2]), np.sin(e[:, 2])
    g = np.empty((e.shape[0], 3, 3))
    g[:, 0, 0] = c1 * c2 - s1 * s2 * c; g[:, 0, 1] = s1 * c2 + c1 * s2 * c; g[:, 0, 2] = s2 * s
    g[:, 1, 0] = -c1 * s2 - s1 * c2 * c; g[:, 1, 1] = -s1 * s2 + c1 * c2 * c; g[:, 1, 2] = c2 * s
    g[:, 2, 0] = s1 * s; g[:, 2, 1] = -c1 * s; g[:, 2, 2] = c
    return g


def schmid_bins(m, lo=0.27, width=0.01, n_bins=23):
    """Grain -> Schmid-factor bin (23 bins of 0.01 on [0.27, 0.50])."""
    b = np.floor((np.asarray(m) - lo) / width).astype(np.int64)
    return np.clip(b, 0, n_bins - 1).astype(np.int32)


# -------------------------------------------------------------- workloads

@dataclass
class Workload:
    name: str
    dims: tuple               # (Lx, Ly) or (Lx, Ly, Lz), x fastest
    nbr: int
    spin: int
    n_grains: int
    kT: float
    n_mcs: int
    voronoi_seed: int
    sweep_seed: int
    B: np.ndarray             # int32[n_grains], 2^-16 units
    m: Optional[np.ndarray] = None      # Schmid factor per grain
    euler: Optional[np.ndarray] = None  # Bunge angles per grain
    n_bins: int = 23
    J_fx: int = FIXED_ONE
    extra: dict = field(default_factory=dict)

    @property
    def ndim(self):
        return len(self.dims)

    @property
    def n_sites(self):
        return int(np.prod(self.dims))

    @property
    def spin_dtype(self):
        return np.int16 if self.spin == I16 else np.int32

    @property
    def grain_bin(self):
        if self.m is None:
            return np.full(self.n_grains, -1, dtype=np.int32)
        return schmid_bins(self.m, n_bins=self.n_bins)

    @property
    def colours(self):
        return {VN4: 2, MOORE8: 4, VN6: 2, MOORE26: 8}[self.nbr]


def voronoi_2d_64():
    G = 40
    return Workload("voronoi_2d_64", (64, 64), VN4, I32, G, 0.5, 100, 1, 1,
                    np.zeros(G, dtype=np.int32), n_bins=0)


def schmid_2d(side=1024, G=2000, seed=2002, n_mcs=1000, vseed=2, sseed=2, kT=0.5, name=None):
    rng = np.random.Generator(np.random.PCG64(seed))
    m = 0.27 + 0.23 * rng.random(G)
    return Workload(name or f"schmid_2d_{side}", (side, side), VN4, I16, G, kT, n_mcs, vseed, sseed,
                    quantise(0.2 * m), m=m)


def schmid_2d_1024():
    return schmid_2d(name="schmid_2d_1024")


def schmid_3d(side=256, G=20000, seed=3003, n_mcs=500, vseed=3, sseed=3, kT=0.6, name=None, spin=None):
    rng = np.random.Generator(np.random.PCG64(seed))
    g = quat_to_matrix(shoemake_quaternions(rng, G))   # passive: crystal = g . sample
    load = g @ np.array([0.0, 0.0, 1.0])        # [001] load axis in the crystal frame
    m = schmid_factor(load)
    return Workload(name or f"schmid_3d_{side}", (side, side, side), VN6, spin if spin is not None else I16, G, kT,
                    n_mcs, vseed,
                    sseed, quantise(0.15 * m), m=m, euler=matrix_to_bunge(g))


def schmid_3d_256():
    return schmid_3d(name="schmid_3d_256")


def stress_2d_16384():
    """16384^2 VN4 int16 (512 MiB per buffer, beyond the 256 MiB Infinity
    Cache), 32000 grains with energies as schmid_2d_1024, kT 0.5, 100 MCS."""
    return schmid_2d(side=16384, G=32000, seed=2003, n_mcs=100, vseed=7, sseed=7, name="stress_2d_16384")


def misorientation_2d_1024():
    """schmid_2d_1024 with a bond energy per pair of grains: Read-Shockley
    (J_max 1, theta_m 15 deg) of Shoemake-uniform orientations (PCG64 2004)."""
    w = schmid_2d(name="misorientation_2d_1024")
    rng = np.random.Generator(np.random.PCG64(2004))
    w.euler = matrix_to_bunge(quat_to_matrix(shoemake_quaternions(rng, w.n_grains)))
    w.extra["pair"] = (1.0, 15.0)
    return w


def moore26_3d_128():
    """128^3 Moore 26-neighbour (8-colour) int16, 2500 grains (mean volume as
    schmid_3d_256 / 1.0), energies as schmid_3d_256, kT 0.6, 100 MCS."""
    w = schmid_3d(side=128, G=2500, seed=3007, n_mcs=100, vseed=13, sseed=13, name="moore26_3d_128")
    w.nbr = MOORE26
    return w


def heterogeneous_field(spins, B, amplitude=0.25, period=64.0):
    """Per-site bulk field varying inside every grain (a stand-in for the
    stored energy a continuum solve would give): B[q_i] modulated by
    1 + amplitude * prod_k sin(2 pi x_k / period), rounded to integers
    (2^-16 units)."""
    s = np.asarray(spins)
    grids = np.meshgrid(*[np.arange(n) for n in s.shape], indexing="ij")
    mod = np.ones(s.shape)
    for gk in grids:
        mod = mod * np.sin(2 * np.pi * gk / period)
    return np.rint(np.asarray(B, dtype=np.float64)[s] * (1.0 + amplitude * mod)).astype(np.int32)


def field_2d_1024(rule=0):
    """schmid_2d_1024 with a per-site field inside the grains (the grain
    energies modulated by +-25 % with period 64); rule 0 carries the field
    with the boundary, rule 1 recrystallises swept sites."""
    w = schmid_2d(name="field_2d_1024" if rule == 0 else "recrystallise_2d_1024")
    w.extra["field_rule"] = rule
    return w


def stress_3d_512():
    """512^3 VN6 int32 (512 MiB per buffer), 160000 grains (mean volume as
    schmid_3d_256) with energies as schmid_3d_256, kT 0.6, 50 MCS."""
    return schmid_3d(side=512, G=160000, seed=3005, n_mcs=50, vseed=9, sseed=9, name="stress_3d_512", spin=I32)


def nfold_ensemble_128(count=1024, seed=6006, n_mcs=20):
    """A batch for the n-fold way at low temperature: `count` VN4 128^2
    lattices (int16), 200 Voronoi grains each, grain energies as
    schmid_2d_1024 (E = 0.2 m, m in [0.27, 0.5]), kT 0.25, n_mcs MC steps of
    continuous time; Voronoi seed 60000+j, event seed 6000+j."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out: List[Workload] = []
    for j in range(count):
        m = 0.27 + 0.23 * rng.random(200)
        out.append(Workload(f"nfold_ensemble_128[{j}]", (128, 128), VN4, I16, 200, 0.25, n_mcs, 60000 + j,
                            6000 + j, quantise(0.2 * m), m=m))
    return out


def nfold_strip_128(count=1024, n_mcs=100):
    """The regime the rejection-free method is for: `count` VN4 128^2
    lattices (int16), each a flat strip of grain 1 (rows 32..95) in grain 0
    with a bulk energy 0.3 J higher, at kT 0.3.  The flat boundaries move
    only through thermally activated kinks (a few events per MC step per
    lattice) while a sweep still tries every boundary site each step.  Event
    seed 7000+j."""
    B = quantise(np.array([0.0, 0.3]))
    out: List[Workload] = []
    for j in range(count):
        w = Workload(f"nfold_strip_128[{j}]", (128, 128), VN4, I16, 2, 0.3, n_mcs, 0, 7000 + j, B)
        w.extra["spins"] = flat_strip(128, 128)
        out.append(w)
    return out


def ensemble_moore8(count=64, seed=4004, n_mcs=1000):
    rng = np.random.Generator(np.random.PCG64(seed))
    sides = rng.choice(np.array([128, 256, 512, 1024]), size=count)
    Gs = rng.integers(50, 2001, size=count)
    kTs = rng.uniform(0.3, 1.0, size=count).astype(np.float32)
    out: List[Workload] = []
    for j in range(count):
        m = 0.27 + 0.23 * rng.random(int(Gs[j]))
        side = int(sides[j])
        out.append(Workload(f"ensemble_moore8[{j}]", (side, side), MOORE8, I16, int(Gs[j]),
                            float(kTs[j]), n_mcs, 40000 + j, 4000 + j, quantise(0.2 * m), m=m))
    return out


# ------------------------------------------------- paper-shaped test inputs

def circle_grain(side=256, radius=80.0):
    """Q=2 bicrystal: a disc of spin 1 centred in a periodic square of spin 0
    (Sec. 4, first validation case, scaled down)."""
    y, x = np.mgrid[0:side, 0:side]
    c = (side - 1) / 2.0
    return ((x - c) ** 2 + (y - c) ** 2 <= radius ** 2).astype(np.int32)


def flat_strip(Lx=128, Ly=256):
    """Q=2 periodic strip with two flat (10) boundaries at y = Ly/4, 3Ly/4."""
    s = np.zeros((Ly, Lx), dtype=np.int32)
    s[Ly // 4: 3 * Ly // 4, :] = 1
    return s


def gaussian_orientation_energy(n_orient=91, width=46.0):
    """Eq. (9): b(n) = (32 pi)^-1/2 exp(-(n-46)^2 / (2 width^2)), n = 1..91."""
    n = np.arange(1, n_orient + 1, dtype=np.float64)
    return (32 * np.pi) ** -0.5 * np.exp(-((n - 46.0) ** 2) / (2 * width ** 2))


def random_spins(dims, Q, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, Q, size=tuple(reversed(dims))).astype(np.int32)


# ------------------------------------------------- learned driving force

STRAIN_BOX = 2e-3


def crystal_inputs(n, seed=5005, strain_box=STRAIN_BOX):
    """Training inputs of the stored-energy surrogate: uniform SO(3)
    orientations as Bunge angles (Shoemake quaternions, PCG64) and strain
    components uniform in +-strain_box, (e11, e22, e33, e23, e13, e12)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    euler = matrix_to_bunge(quat_to_matrix(shoemake_quaternions(rng, n)))
    eps = rng.uniform(-strain_box, strain_box, size=(n, 6))
    return euler, eps


def uniaxial_strain(k, n_queries=50, strain_box=STRAIN_BOX):
    """Query k of a monotonic uniaxial path along x with lateral contraction,
    diag(e, -e/2, -e/2) with e = (k / n_queries) * strain_box (the loading of
    the paper's single-crystal test, Sec. 2, scaled to the training box)."""
    e = (k / n_queries) * strain_box
    return np.array([e, -e / 2, -e / 2, 0.0, 0.0, 0.0])


# Training recipe of the stored-energy network for the learned 256^3
# workload: sizes, seeds and optimiser settings (inputs of the run, shared by
# the benchmark and the tests).
LEARNED = dict(n_train=1000000, n_test=20000, data_seed=5005, solver_seed=50, init_seed=7, train_seed=1,
               epochs=200, batch=4096, lr=1e-2, every=10, n_audit=64, audit_tol=0.25)
