"""Pins of the seeded input generators (no sweep arithmetic lives there).

Schmid factors of the FCC {111}<110> family against closed forms: a load in
the (001) plane at angle theta from [100] gives 1/sqrt(6) at 0 and 45 degrees
and a maximum near 22.5 degrees, symmetric about 22.5 degrees (Sec. 5), and
the global FCC range is [sqrt(6)/9, 1/2]."""
import numpy as np
import pytest

import synth


def _m(theta_deg):
    t = np.radians(np.atleast_1d(theta_deg))
    return synth.schmid_factor(np.stack([np.cos(t), np.sin(t), 0 * t], 1))


def test_schmid_closed_forms():
    assert _m(0)[0] == pytest.approx(1 / np.sqrt(6), abs=1e-12)
    assert _m(45)[0] == pytest.approx(1 / np.sqrt(6), abs=1e-12)
    assert _m(90)[0] == pytest.approx(1 / np.sqrt(6), abs=1e-12)
    th = np.linspace(0, 45, 4501)
    m = _m(th)
    assert th[np.argmax(m)] == pytest.approx(22.5, abs=0.01)
    assert m.max() == pytest.approx(0.4928, abs=1e-4)
    assert np.allclose(_m(th), _m(45 - th), atol=1e-12)
    assert _m(10)[0] == pytest.approx(0.46575, abs=1e-5)
    assert synth.schmid_factor([1, 1, 1])[0] == pytest.approx(np.sqrt(6) / 9, abs=1e-12)
    assert synth.schmid_factor([0, 1, 1])[0] == pytest.approx(np.sqrt(6) / 6, abs=1e-12)
    assert synth.schmid_factor([1, 2, 3])[0] <= 0.5 + 1e-12


def test_slip_systems():
    n, d = synth.fcc_slip_systems()
    assert n.shape == (12, 3) and d.shape == (12, 3)
    assert np.allclose(np.sum(n * d, 1), 0)
    assert np.allclose(np.linalg.norm(n, axis=1), 1) and np.allclose(np.linalg.norm(d, axis=1), 1)
    def canon(v):   # direction up to sign
        v = np.round(v, 6)
        return tuple(v if v[np.nonzero(v)[0][0]] > 0 else -v)
    assert len({canon(x) for x in d}) == 6
    assert len({canon(x) for x in n}) == 4
    assert len({canon(a) + canon(b) for a, b in zip(n, d)}) == 12


def test_uniform_orientations_and_euler_roundtrip():
    q = synth.shoemake_quaternions(np.random.default_rng(0), 20000)
    R = synth.quat_to_matrix(q)
    assert np.allclose(np.einsum("nij,nkj->nik", R, R), np.eye(3), atol=1e-12)
    assert np.allclose(np.linalg.det(R), 1)
    # Haar measure: the rotated z axis is uniform on the sphere -> cos uniform on [-1,1]
    z = R[:, 2, 2]
    assert abs(z.mean()) < 0.02 and abs((z ** 2).mean() - 1 / 3) < 0.01
    e = synth.matrix_to_bunge(R[:200])
    assert np.allclose(synth.bunge_to_matrix(e), R[:200], atol=1e-10)


def test_workload_energies():
    w = synth.schmid_2d_1024()
    assert w.B.dtype == np.int32 and w.B.shape == (2000,)
    assert w.B.min() >= int(np.rint(0.2 * 0.27 * 65536)) and w.B.max() <= int(np.rint(0.2 * 0.5 * 65536))
    w3 = synth.schmid_3d_256()
    assert w3.m.min() >= np.sqrt(6) / 9 - 1e-12 and w3.m.max() <= 0.5 + 1e-12
    assert np.array_equal(w3.B, np.rint(0.15 * w3.m * 65536).astype(np.int32))
    assert np.array_equal(synth.quantise([0.5 / 65536, 1.5 / 65536, 2.5 / 65536]), [0, 2, 2])
    ens = synth.ensemble_moore8()
    assert len(ens) == 64
    assert {w.dims[0] for w in ens} <= {128, 256, 512, 1024}
    assert all(50 <= w.n_grains <= 2000 and 0.3 <= w.kT <= 1.0 for w in ens)


def test_gaussian_energy_eq9():
    b = synth.gaussian_orientation_energy()
    assert len(b) == 91 and np.argmax(b) == 45
    assert b.max() == pytest.approx((32 * np.pi) ** -0.5)
    assert b[0] == pytest.approx((32 * np.pi) ** -0.5 * np.exp(-45 ** 2 / (2 * 46 ** 2)))
