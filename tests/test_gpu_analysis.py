"""GPU runs of the paper's calibration cases (Sec. 4: a circular grain and
flat boundaries in a Q=2 lattice at the paper's effective temperature 1.4)
through the analysis layer: the circle's area falls linearly without bulk
energy, one (mobility, stiffness) pair describes it at several bulk energies,
and flat boundaries move at a speed linear in the bulk energy with the same
sign convention; the mobility then fixes the physical time of one MC step
through the parametric links."""
import numpy as np
import pytest

import paper_1007_3509_amd as hmc
import synth
from paper_1007_3509_amd import analysis as an

pytestmark = pytest.mark.gpu

KT = 1.4


def say(*a):
    print(*a, flush=True)


def _circle(db, seed, n=12, every=100):
    s = synth.circle_grain(256, 80.0).astype(np.int16)
    with hmc.Lattice((256, 256), hmc.HMC_VN4, 2) as lat:
        lat.set_spins(s)
        lat.set_grain_energy(synth.quantise(np.array([0.0, db])))
        t, A = [0.0], [float(lat.grain_areas()[1])]
        for k in range(n):
            lat.sweep(KT, every, seed)
            t.append((k + 1.0) * every)
            A.append(float(lat.grain_areas()[1]))
    return np.array(t), np.array(A)


def _strip(db, seed, n=10, every=100):
    s = synth.flat_strip(128, 256).astype(np.int16)
    with hmc.Lattice((128, 256), hmc.HMC_VN4, 2) as lat:
        lat.set_spins(s)
        lat.set_grain_energy(synth.quantise(np.array([0.0, db])))
        t, w = [0.0], [an.strip_position(s)]
        for k in range(n):
            lat.sweep(KT, every, seed)
            t.append((k + 1.0) * every)
            w.append(an.strip_position(lat.spins()))
    return np.array(t), np.array(w)


def test_circle_calibration_on_gpu():
    say("[gpu] circles")

    def mean_circle(db, seeds=(7, 8, 9, 10)):
        curves = [_circle(db, s) for s in seeds]
        return curves[0][0], np.mean([c[1] for c in curves], axis=0)

    t, A = mean_circle(0.0)
    mg, r2 = an.circle_kinetics(t[2:], A[2:])
    say(f"[gpu] circle m*gamma*={mg:.3f} R^2={r2:.4f}")
    assert mg > 0 and r2 >= 0.99
    runs = [(t, A, 0.0)] + [(*mean_circle(db), db) for db in (0.03, -0.03)]
    m, gamma, r2 = an.circle_kinetics_fit([(tt[2:], aa[2:], db) for tt, aa, db in runs])
    say(f"[gpu] circle fit m={m:.3f} gamma*={gamma:.3f} R^2={r2:.3f}")
    assert m > 0 and gamma > 0 and r2 > 0.8
    # more bulk energy inside: faster shrinkage
    assert runs[1][1][-1] < runs[0][1][-1] < runs[2][1][-1]


def test_flat_boundary_calibration_on_gpu():
    say("[gpu] strips")
    mob = {}
    for db in (0.05, -0.05, 0.1, -0.1):
        t, w = _strip(db, 11)
        m, v, r2 = an.flat_boundary_mobility(t, w, db)
        mob[db] = (m, v)
        say(f"[gpu] strip db={db} m={m:.3f} v={v:.4f} R^2={r2:.3f}")
        assert np.sign(v) == -np.sign(db) and m > 0
    ms = np.array([x[0] for x in mob.values()])
    assert ms.max() < 1.6 * ms.min()          # speed linear in the driving force
    # physical time of one MC step for a literature-scale SI mobility
    s = an.Scales(E0=1.0, l0=1.0, t0=1.0)
    t0 = an.time_scale(float(ms.mean()), 2.0 * float(ms.mean()), s)
    assert t0 == pytest.approx(0.5)
