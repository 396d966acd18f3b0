"""The benchmark's host-side contract, without a GPU: more than one GPU is
refused with a message before any device work, and the committed rocprofv3
summaries carry the machine-readable figures the benchmark reads (and are
ignored for a tiling other than the one they were taken with)."""
import json
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

SWEEP = {"schmid_2d_1024", "schmid_3d_256", "stress_2d_16384", "stress_3d_512", "misorientation_2d_1024",
         "moore26_3d_128", "field_2d_1024", "recrystallise_2d_1024"}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "error" in line and line["n_gpus"] == 2


def _fields(path):
    out = {}
    for line in open(path):
        m = re.match(r"^(\w+): (\S+)(\s.*)?$", line)
        if m:
            out[m.group(1)] = m.group(2)
    return out


@pytest.mark.parametrize("workload", sorted(SWEEP))
def test_sweep_profiles_are_machine_readable(workload):
    kernel = {"stress_2d_16384": "lat2d_kernel", "moore26_3d_128": "lat26_kernel"}.get(workload, "sweep_tile_kernel")
    f = _fields(os.path.join(ROOT, "profiles", f"{kernel}_{workload}.md"))
    assert re.fullmatch(r"[0-9a-f]{64}", f["kernel_source_sha256"])
    assert float(f["traffic_bytes_per_launch"]) > 0 and float(f["valu_wave_instructions_per_launch"]) > 0
    tiling = tuple(int(v) for v in f["tiling"].split(","))
    assert len(tiling) == 4
    # a tiling other than the measured one never borrows its figures
    other = (tiling[0], tiling[1], tiling[2], tiling[3] + 1)
    assert bench.measured_profile(workload, other, kernel=kernel) == {}


def test_ensemble_and_nfold_profiles_are_machine_readable():
    f = _fields(os.path.join(ROOT, "profiles", "ens2d_kernel_ensemble_moore8.md"))
    assert float(f["traffic_bytes_per_launch"]) > 0 and float(f["valu_wave_instructions_per_launch"]) > 0
    assert bench.measured_profile("ensemble_moore8", (1, 1, 1, 1), kernel="ens2d_kernel") == {}
    assert bench.measured_profile("ensemble_moore8", (128, 128, 1, 3), kernel="ens2d_kernel")
    g = _fields(os.path.join(ROOT, "profiles", "nfold_kernel_nfold_ensemble_128.md"))
    assert re.fullmatch(r"[0-9a-f]{64}", g["kernel_source_sha256"])
    assert float(g["traffic_bytes_per_launch"]) > 0 and float(g["valu_wave_instructions_per_launch"]) > 0


def test_every_profile_names_the_command_that_made_it():
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        text = open(os.path.join(ROOT, "profiles", name)).read()
        assert "rocprofv3 --kernel-trace --stats" in text, name
        assert "bench.py" in text, name


def test_cpu_baseline_reports_host_and_checks_single_thread(orc):
    """The CPU leg on a small job: every MC step of the job within the
    budget, the host's CPUs named, and the single-thread prefix equal to the
    threaded run's state after the same steps; a check that returns the
    oracle's own spins is reported bit-exact, any other is not."""
    import synth

    w = synth.voronoi_2d_64()
    start = orc.voronoi(w.dims, w.n_grains, w.voronoi_seed)
    want = orc.sweep(start, w.nbr, w.dims, w.B, w.kT, w.n_mcs, w.sweep_seed)
    calls = []

    def gpu_check(sample, Jp=None):
        calls.append(sample)
        return orc.sweep(start, w.nbr, w.dims, w.B, w.kT, sample, w.sweep_seed)

    out = bench.cpu_baseline(w, start, w.n_mcs, 30.0, gpu_check)
    assert calls == [w.n_mcs] and np.array_equal(gpu_check(w.n_mcs), want)
    assert out["gpu_bit_exact_on_sample"] is True
    assert out["single_core"]["same_as_threaded"] is True
    assert 1 <= out["single_core"]["sample_mcs"] <= w.n_mcs
    assert out["cores"] >= 1 and out["host_cpus"] >= out["affinity_cpus"] >= 1
    assert f"first {w.n_mcs} of {w.n_mcs}" in out["sample"]

    def wrong(sample, Jp=None):
        s = gpu_check(sample).copy()
        s[0] = (s[0] + 1) % w.n_grains
        return s

    assert bench.cpu_baseline(w, start, w.n_mcs, 30.0, wrong)["gpu_bit_exact_on_sample"] is False
