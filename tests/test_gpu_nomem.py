"""GPU: the HMC_MAX_BYTES cap on the library's device memory.  Run in a
child process (the cap is read once per process): a lattice whose buffers
exceed the cap fails with HMC_E_NOMEM before any kernel runs, and one that
fits works until an allocation beyond the cap (a snapshot) is refused with
HMC_E_NOMEM while the lattice stays usable."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import paper_1007_3509_amd as hmc
try:
    hmc.Lattice((256, 256), hmc.HMC_VN4, 40, voronoi_seed=1)      # 2 x 128 KiB of spins: over the cap
    print("BIG-CREATED")
except hmc.HmcError as e:
    print("BIG", e.status)
lat = hmc.Lattice((64, 64), hmc.HMC_VN4, 40, voronoi_seed=1)        # 2 x 8 KiB + small tables: fits
lat.set_grain_energy(np.zeros(40, np.int32))
lat.sweep(0.5, 3, 1)
print("SMALL-OK", lat.mcs)
lat2 = hmc.Lattice((64, 64), hmc.HMC_VN4, 40, voronoi_seed=2)
keep = []
try:
    for _ in range(8):                                              # keep allocating until the cap refuses
        keep.append(hmc.Lattice((64, 64), hmc.HMC_VN4, 40, voronoi_seed=3))
    print("NO-REFUSAL")
except hmc.HmcError as e:
    print("MORE", e.status)
lat.sweep(0.5, 2, 1)
print("STILL-OK", lat.mcs)
"""


def test_byte_cap_gives_nomem():
    env = dict(os.environ, HMC_MAX_BYTES=str(120 * 1024))
    print("[gpu] HMC_MAX_BYTES child", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], env=env, capture_output=True, text=True, timeout=120)
    out = r.stdout
    assert r.returncode == 0, r.stdout + r.stderr
    assert "BIG -2" in out, out            # HMC_E_NOMEM
    assert "SMALL-OK 3" in out, out
    assert "MORE -2" in out, out
    assert "STILL-OK 5" in out, out
