"""The uint32 threshold table of the Metropolis rule (Sec. 3), built on the
host by the library, against the oracle's T(d) for every (dn, dB) a trial can
reach, on every workload's (kT, M, range of B).

The library keeps T in rows dn = dn_lo..M and columns dB = -R..R and, per
bucket of columns, the two bounds the kernel decides most trials with (a
trial reads the table only when r1 lies between them).  Checked here, with
no GPU (the host builder is exported without device work):

* every entry whose d = J dn + dB is positive equals the oracle's T(d);
* no reachable positive d lies outside the rows (the row below dn_lo has no
  positive d);
* each bucket's lower bound is T at its largest d and its upper bound T at
  its smallest positive d, so every entry of the bucket lies between them;
* the kernel's bucket index, a multiply-high by floor(2^32/bw) + 1, equals
  col // bw for every column whenever the library selects it (TW * bw < 2^32);
* planted mistakes -- one entry off by one, one bound off by one, one row
  too few -- are caught by the same checks.
"""
import numpy as np
import pytest

import synth

J = 65536


def table_problems(orc, kT, M, J_fx, Bmin, Bmax, lay, table, bounds):
    """Every way the table differs from the oracle's T(d) (empty: none)."""
    out = []
    R = Bmax - Bmin
    dn_lo, rows, TW, nb, bw = lay["dn_lo"], lay["rows"], lay["TW"], lay["nb"], lay["bw"]
    if lay["R"] != R or TW != 2 * R + 1:
        out.append(f"columns: R {lay['R']} TW {TW}, want R {R}")
        return out
    if rows != M - dn_lo + 1 or table.size != rows * TW or bounds.size != 2 * rows * nb:
        out.append("sizes")
        return out
    if dn_lo > -M and J_fx * (dn_lo - 1) + R > 0:
        out.append(f"row dn = {dn_lo - 1} has positive d but is missing")
    dn = dn_lo + np.arange(rows, dtype=np.int64)[:, None]
    dB = np.arange(TW, dtype=np.int64)[None, :] - R
    d = J_fx * dn + dB
    T = orc.threshold_many(d, kT).reshape(rows, TW)
    tab = table.reshape(rows, TW)
    bad = (d > 0) & (tab != T)
    if bad.any():
        r, c = np.argwhere(bad)[0]
        out.append(f"{int(bad.sum())} entries differ, first (dn {dn_lo + r}, dB {c - R}): {tab[r, c]} vs {T[r, c]}")
    if nb * bw < TW:
        out.append(f"buckets {nb} x {bw} do not cover {TW} columns")
    bd = bounds.reshape(rows, nb, 2)
    for r in range(rows):
        for b in range(nb):
            c0, c1 = b * bw, min(TW, (b + 1) * bw) - 1
            dd = d[r, c0:c1 + 1]
            pos = dd > 0
            if not pos.any():
                continue
            lo, hi = int(bd[r, b, 0]), int(bd[r, b, 1])
            if lo != int(T[r, c1]) or hi != int(T[r, c0:c1 + 1][pos][0]):
                out.append(f"bounds of (dn {dn_lo + r}, bucket {b}): ({lo}, {hi})")
            vals = T[r, c0:c1 + 1][pos].astype(np.int64)
            if vals.min() < lo or vals.max() > hi:
                out.append(f"bucket (dn {dn_lo + r}, {b}) has entries outside its bounds")
    if bw >= 2 and TW * bw < (1 << 32):
        m = (1 << 32) // bw + 1
        cols = np.arange(TW, dtype=np.uint64)
        if not np.array_equal((cols * np.uint64(m)) >> np.uint64(32), cols // np.uint64(bw)):
            out.append("multiply-high bucket index differs from col // bw")
    return out


def _cases():
    """(name, kT, M, Bmin, Bmax) of every workload's lattices."""
    cases = []
    w = synth.voronoi_2d_64()
    cases.append((w.name, w.kT, 4, int(w.B.min()), int(w.B.max())))
    for f, M in ((synth.schmid_2d_1024, 4), (synth.schmid_3d_256, 6), (synth.moore26_3d_128, 26),
                 (synth.stress_2d_16384, 4), (synth.stress_3d_512, 6)):
        w = f()
        cases.append((w.name, w.kT, M, int(w.B.min()), int(w.B.max())))
    for j, w in enumerate(synth.ensemble_moore8()):
        cases.append((f"ensemble_moore8[{j}]", w.kT, 8, int(w.B.min()), int(w.B.max())))
    # temperatures and ranges off the workloads: high and low kT, a single
    # column (uniform B), negative energies
    for kT, M, lo, hi in ((0.05, 4, 0, 0), (5.0, 8, -30000, 30000), (0.3, 6, -100, 7000), (1.0, 26, 5, 6)):
        cases.append((f"kT{kT}_M{M}", kT, M, lo, hi))
    return cases


@pytest.fixture(scope="module")
def hmc():
    import paper_1007_3509_amd as h
    try:
        h.lib()
    except Exception as e:   # noqa: BLE001
        pytest.fail(f"libhmc.so not built: {e}")
    return h


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_host_table_equals_oracle(orc, hmc, case):
    name, kT, M, lo, hi = case
    lay, table, bounds = hmc.hmc_threshold_table_host(kT, M, J, lo, hi)
    assert table_problems(orc, kT, M, J, lo, hi, lay, table, bounds) == []


def test_planted_table_mistakes_are_caught(orc, hmc):
    w = synth.schmid_2d_1024()
    kT, M, lo, hi = w.kT, 4, int(w.B.min()), int(w.B.max())
    lay, table, bounds = hmc.hmc_threshold_table_host(kT, M, J, lo, hi)
    assert table_problems(orc, kT, M, J, lo, hi, lay, table, bounds) == []
    R, TW = lay["R"], lay["TW"]
    # one entry with d > 0 off by one
    t2 = table.copy()
    r = lay["rows"] - 1
    t2[r * TW + TW // 2] += 1
    assert table_problems(orc, kT, M, J, lo, hi, lay, t2, bounds)
    # one bound off by one
    b2 = bounds.copy()
    b2[2 * (lay["nb"] * r + 1) + 1] -= 1
    assert table_problems(orc, kT, M, J, lo, hi, lay, table, b2)
    # a row too few (dn_lo raised by one, first row dropped)
    lay2 = dict(lay, dn_lo=lay["dn_lo"] + 1, rows=lay["rows"] - 1)
    assert table_problems(orc, kT, M, J, lo, hi, lay2, table[TW:], bounds[2 * lay["nb"]:])
    # a table built for another temperature
    lay3, t3, b3 = hmc.hmc_threshold_table_host(kT * 1.0001, M, J, lo, hi)
    assert table_problems(orc, kT, M, J, lo, hi, lay3, t3, b3)
    assert R == hi - lo


def test_host_table_rejects_bad_arguments(hmc):
    for args in ((0.0, 4, J, 0, 10), (float("nan"), 4, J, 0, 10), (0.5, 5, J, 0, 10), (0.5, 4, 0, 0, 10),
                 (0.5, 4, J, 10, 0)):
        with pytest.raises(hmc.HmcError):
            hmc.hmc_threshold_table_host(*args)
    with pytest.raises(hmc.HmcError) as e:
        hmc.hmc_threshold_table_host(0.5, 26, 1 << 24, -(1 << 29), 1 << 29)
    assert e.value.status == hmc.HMC_E_RANGE
