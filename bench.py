"""Throughput of the red/black Potts sweep with per-grain bulk energy on one GPU.

One step = one whole job of the workload: restore the initial Voronoi
polycrystal (device-to-device copy), run n_mcs red/black MC steps, and read
the grain statistics (grain count, mean area, Schmid-bin area fractions).
Inputs are resident in HBM before timing starts.

Printed: one JSON line with site-updates/s (the metric, from the
uninstrumented timed loop), the roofline entry of the sweep kernel (its
average launch duration from HIP events bound to every sweep dispatch on the
lattice's stream, taken on a replay of the same steps right after the timed
loop, against MI355X peak HBM bandwidth, with the algorithmic bytes per site
update stated below) and the CPU oracle timed on the host cores on a bounded
sample of the same job.

Other workloads (--workload): the 256^3 and 16384^2 lattices print the same
line; ensemble_moore8 compares one ensemble call with the same lattices swept
one by one; learned_3d_256 compares the trained stored-energy network with
the crystal-plasticity solver in the loop.

Algorithmic bytes per site update: (C + 1) * s -- one half step reads every
spin and writes the 1/C of them whose colour it updates (s = bytes per spin,
C = colours).  The kernel fuses several half steps per launch, so its real
DRAM traffic is lower; the measured traffic is reported separately.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

PEAK_HBM_GBPS = 8000.0
VALU_ISSUE_PER_S = 256 * 2.4e9      # wave64 VALU instructions per second, whole chip
WORKLOADS = {
    "voronoi_2d_64": synth.voronoi_2d_64,
    "schmid_2d_1024": synth.schmid_2d_1024,
    "schmid_3d_256": synth.schmid_3d_256,
    "stress_2d_16384": synth.stress_2d_16384,
    "stress_3d_512": synth.stress_3d_512,
    "misorientation_2d_1024": synth.misorientation_2d_1024,
    "moore26_3d_128": synth.moore26_3d_128,
    "field_2d_1024": lambda: synth.field_2d_1024(0),
    "recrystallise_2d_1024": lambda: synth.field_2d_1024(1),
}
SPECIAL = ("ensemble_moore8", "learned_3d_256", "nfold_ensemble_128", "nfold_strip_128")
NBR_NAME = {0: "VN4", 1: "Moore8", 2: "VN6", 3: "Moore26"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="schmid_3d_256", choices=sorted(WORKLOADS) + list(SPECIAL))
    ap.add_argument("--mcs", type=int, default=0, help="override MC steps per job")
    ap.add_argument("--tiling", default="", help="tx,ty,tz,k (default: library choice)")
    ap.add_argument("--kernel", default="auto", choices=("auto", "generic"),
                    help="sweep kernel: auto (the compiled-tile kernel where it applies) or the general one")
    ap.add_argument("--cpu-seconds", type=float, default=30.0, help="budget of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def source_sha(kernel_file):
    """sha256 of a kernel's source file followed by the header it inlines
    (random numbers, acceptance helpers): what a profile was taken on."""
    import hashlib

    csrc = os.path.join(ROOT, "paper_1007_3509_amd", "csrc")
    h = hashlib.sha256()
    for f in (kernel_file, "common.hpp"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_profile(workload, tiling, kernel="sweep_tile_kernel"):
    """Per-launch figures of the sweep (or ensemble) kernel from the committed
    rocprofv3 summary (scaled HBM bytes, VALU wave instructions), or {} when
    the kernel source or the tiling changed since they were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.md")
    if not os.path.exists(path):
        return {}
    keys = ("traffic_bytes_per_launch", "valu_wave_instructions_per_launch", "kernel_source_sha256", "tiling")
    fields = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in keys:
            k, v = line.split(":", 1)
            fields[k.strip()] = (v.split() or [""])[0]
    sha = source_sha("sweep_vn6.hip" if kernel == "vn6_tile_kernel" else "sweep.hip")
    if fields.get("kernel_source_sha256") != sha or fields.get("tiling") != ",".join(str(v) for v in tiling):
        return {}
    return {k: float(fields[k]) for k in keys[:2] if k in fields}


def host_threads():
    """Threads the oracle may use (the CPUs this process may run on, capped by
    OMP_NUM_THREADS when that is set) and a description of the host."""
    affinity = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS", "")
    threads = min(affinity, int(omp)) if omp.isdigit() and int(omp) > 0 else affinity
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return threads, {"host_cpus": os.cpu_count(), "affinity_cpus": affinity, "cpu_model": model}


def cpu_baseline(w, start, n_mcs, budget_s, gpu_check, field=None):
    """The oracle, as it stands, on the same job from the same initial state:
    as many MC steps of the job as the budget allows on every host thread, and
    the first steps of that run again on one thread (reference semantics),
    which must give the same spins."""
    import oracle

    threads, host = host_threads()
    pair = w.extra.get("pair")
    extra = {}
    if pair:
        # the oracle's own table; the GPU run of the check takes the same table
        Jp = oracle.pair_table(w.euler, *pair)
        extra["pair_table_max_abs_diff_gpu_vs_oracle"] = int(np.max(np.abs(gpu_check.table().astype(np.int64) - Jp)))

        def run(state, n, th, mcs0):
            return oracle.sweep_pair(state, w.nbr, w.dims, Jp, w.B, w.kT, n, w.sweep_seed, mcs0=mcs0, threads=th)
        spins_of = lambda state: state  # noqa: E731
        state0 = start
    elif field is not None:
        Jp = None
        zeros = np.zeros(w.n_grains, np.int32)

        def run(state, n, th, mcs0):
            return oracle.sweep_field(state[0], state[1], w.extra["field_rule"], w.nbr, w.dims, zeros, w.kT, n,
                                      w.sweep_seed, mcs0=mcs0, threads=th)
        spins_of = lambda state: state[0]  # noqa: E731
        state0 = (start, field)
    else:
        Jp = None

        def run(state, n, th, mcs0):
            return oracle.sweep(state, w.nbr, w.dims, w.B, w.kT, n, w.sweep_seed, mcs0=mcs0, threads=th)
        spins_of = lambda state: state  # noqa: E731
        state0 = start
    run(state0, 1, threads, 0)          # warm the thread pool and caches
    t0 = time.perf_counter()
    run(state0, 2, threads, 0)
    per_mcs = (time.perf_counter() - t0) / 2
    t0 = time.perf_counter()
    run(state0, 1, 1, 0)
    per1 = time.perf_counter() - t0
    sample = int(max(1, min(n_mcs, budget_s / max(per_mcs, 1e-9))))
    # the single-thread leg repeats the first s1 steps (about a third of the budget)
    s1 = int(max(1, min(sample, budget_s / 3 / max(per1, 1e-9))))
    t0 = time.perf_counter()
    mid = run(state0, s1, threads, 0)
    out = run(mid, sample - s1, threads, s1) if sample > s1 else mid
    dt = time.perf_counter() - t0
    exact = bool(np.array_equal(gpu_check(sample, Jp), spins_of(out)))
    t0 = time.perf_counter()
    one = run(state0, s1, 1, 0)
    dt1 = time.perf_counter() - t0
    same_1t = bool(np.array_equal(spins_of(one), spins_of(mid)))
    return {
        "value": w.n_sites * sample / dt,
        "unit": "site-updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{w.name}: first {sample} of {n_mcs} MC steps from the same initial grains "
                  f"({w.n_sites * sample:.3g} site updates, {dt:.1f} s on {threads} threads)",
        **host,
        "gpu_bit_exact_on_sample": exact,
        "single_core": {"value": w.n_sites * s1 / dt1, "sample_mcs": s1,
                        "same_as_threaded": same_1t,
                        "note": "the first sample_mcs steps on one thread against the threaded run's state "
                                "after the same steps"},
        **extra,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; runs on several GPUs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import paper_1007_3509_amd as hmc

    if hmc.hmc_device_count() < 1:
        print(json.dumps({"error": "no HIP device visible"}))
        sys.exit(1)
    if args.workload == "ensemble_moore8":
        return bench_ensemble(args, hmc)
    if args.workload == "learned_3d_256":
        return bench_learned(args, hmc)
    if args.workload in ("nfold_ensemble_128", "nfold_strip_128"):
        return bench_nfold(args, hmc)
    w = WORKLOADS[args.workload]()
    n_mcs = args.mcs or w.n_mcs
    lat = hmc.Lattice(w.dims, w.nbr, w.n_grains, voronoi_seed=w.voronoi_seed, spin=w.spin)
    lat.set_grain_energy(w.B)
    pair = w.extra.get("pair")
    gpu_table = None
    if pair:   # bond energy per pair of grains, built on the GPU from the orientations
        gpu_table = hmc.hmc_misorientation_energy(w.euler, *pair)
        lat.set_pair_energy(gpu_table)
    if args.tiling:
        lat.set_tiling(*[int(v) for v in args.tiling.split(",")])
    if args.kernel == "generic":
        hmc.hmc_set_sweep_kernel(lat.h, hmc.HMC_KERNEL_GENERIC)
    start = lat.spins()
    rule = w.extra.get("field_rule")
    field = None
    if rule is not None:   # bulk energy per site: the grain energies modulated inside every grain
        field = synth.heterogeneous_field(start, w.B, 0.25, 64.0)
        lat.set_grain_energy(np.zeros(w.n_grains, np.int32))
        lat.set_site_energy(field, rule)
    fb_start = lat.boundary_sites() / w.n_sites
    hmc.hmc_snapshot(lat.h)
    gbin = w.grain_bin if w.n_bins else None

    def step():
        hmc.hmc_restore(lat.h)
        lat.sweep(w.kT, n_mcs, w.sweep_seed)
        return lat.texture_stats(gbin, w.n_bins)

    for _ in range(args.warmup):
        step()
    lat.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats = step()
    lat.synchronize()
    t1 = time.perf_counter()
    # The same steps replayed with HIP events bound to every sweep dispatch
    # (hipExtLaunchKernel) on the lattice's stream: the kernel's own duration
    # per launch.  Kept out of the timed loop above, where the per-dispatch
    # events would add several microseconds to every launch.
    hmc.hmc_profile(lat.h, True)
    hmc.hmc_profile_read(lat.h)          # reset counters
    hmc.hmc_profile_trials(lat.h)
    for _ in range(args.steps):
        step()
    lat.synchronize()
    kernel_ms, launches, su = hmc.hmc_profile_read(lat.h)
    trials = hmc.hmc_profile_trials(lat.h)
    hmc.hmc_profile(lat.h, False)
    fb_end = lat.boundary_sites() / w.n_sites

    total_su = w.n_sites * n_mcs * args.steps
    elapsed = t1 - t0
    value = total_su / elapsed
    s_bytes = np.dtype(w.spin_dtype).itemsize
    C = w.colours
    # spins (and the per-site field, int32) read for every pass, written for the updated colour
    bytes_per_su = (C + 1) * (s_bytes + (4 if field is not None else 0))
    avg_launch_s = kernel_ms / 1e3 / max(launches, 1)
    su_per_launch = su / max(launches, 1)
    achieved = su_per_launch * bytes_per_su / avg_launch_s / 1e9
    tiling = lat.tiling()
    if hmc.hmc_get_sweep_kernel(lat.h) == hmc.HMC_KERNEL_COMPILED:
        kname = "lat26_kernel" if w.nbr == hmc.HMC_MOORE26 else ("vn6_tile_kernel" if len(w.dims) == 3 else "lat2d_kernel")
    else:
        kname = "sweep_tile_kernel"
    prof = measured_profile(w.name, tiling, kernel=kname)
    traffic = prof.get("traffic_bytes_per_launch")
    valu = prof.get("valu_wave_instructions_per_launch")

    out = {
        "metric": "Potts site-updates/s (HBM GB/s vs peak in roofline), 1 MI355X, bit-exact vs oracle",
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int16" if s_bytes == 2 else "int32",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "lattice": "x".join(str(d) for d in w.dims),
            "neighbourhood": NBR_NAME[w.nbr],
            "spins": "int16" if s_bytes == 2 else "int32",
            "grains": w.n_grains,
            "kT": w.kT,
            "mcs_per_step": n_mcs,
            "tiling": ({"tile": list(tiling[:3]), "mcs_per_launch": tiling[3]} if tiling[3] > 0
                       else {"tile": list(tiling[:3]), "colour_passes_per_launch": -tiling[3]}),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBPS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBPS,
            "traffic": traffic,
            "traffic_note": "scaled FETCH_SIZE+WRITE_SIZE bytes per launch from profiles/ (null if the kernel changed)",
            "kernel": kname,
            "avg_launch_us": avg_launch_s * 1e6,
            "launch_timing": "HIP events bound to each sweep dispatch, replay of the timed steps",
            "launches": launches,
            "bytes_per_site_update": bytes_per_su,
            "site_updates_per_launch": su_per_launch,
            "philox_calls_per_site_update": trials / max(su, 1),
            "boundary_site_fraction": {"start": fb_start, "end": fb_end},
            "work_note": "Philox calls = queued trials including the redundant halo work of fused steps; "
                         "boundary fraction = sites with an unlike neighbour / N",
            "traffic_gbps": traffic / avg_launch_s / 1e9 if traffic else None,
            "valu": {
                "wave_instructions_per_launch": valu,
                "per_site_update": valu / su_per_launch if valu else None,
                "issue_frac": valu / (avg_launch_s * VALU_ISSUE_PER_S) if valu else None,
                "note": "SQ_INSTS_VALU from profiles/ (null if the kernel changed) against 256 CUs x 2.4 GHz x "
                        "1 VALU wave instruction per CU per cycle: the resource that binds this kernel",
            },
        },
        "final_grains": stats[0],
        "final_mean_area": stats[1],
    }
    if not args.no_cpu_baseline:
        def gpu_check(sample, Jp=None):  # noqa: E306
            if Jp is not None:
                lat.set_pair_energy(Jp)
            hmc.hmc_restore(lat.h)
            lat.sweep(w.kT, sample, w.sweep_seed)
            return lat.spins().astype(np.int32)
        gpu_check.table = lambda: gpu_table
        out["cpu_baseline"] = cpu_baseline(w, start.astype(np.int32), n_mcs, args.cpu_seconds, gpu_check, field)
    lat.close()
    print(json.dumps(out), flush=True)


def _line(metric, value, args, ms, config, **extra):
    out = {"metric": metric, "value": value, "unit": "site-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int16", "data": "synthetic", "config": config}
    out.update(extra)
    print(json.dumps(out), flush=True)


def bench_ensemble(args, hmc):
    """64 Moore-8 lattices of uneven size, temperature and seed: one ensemble
    call (persistent kernel, HIP-graph replay) against the same lattices swept
    one after another with hmc_sweep; the ensemble kernel against the HBM
    roofline; the oracle on the smallest members as the CPU baseline."""
    members = synth.ensemble_moore8()
    n_mcs = args.mcs or members[0].n_mcs
    lats = []
    for w in members:
        lat = hmc.Lattice(w.dims, w.nbr, w.n_grains, voronoi_seed=w.voronoi_seed, spin=w.spin)
        lat.set_grain_energy(w.B)
        hmc.hmc_snapshot(lat.h)
        lats.append(lat)
    starts = [lat.spins().astype(np.int32) for lat in lats]
    kT = np.array([w.kT for w in members], np.float32)
    seeds = np.array([w.sweep_seed for w in members], np.uint64)
    E = hmc.hmc_ensemble_create(lats)
    tiling = hmc.hmc_ensemble_get_tiling(E)
    total_sites = sum(w.n_sites for w in members)

    def restore():
        # every member's initial state, restored outside the timed region
        for lat in lats:
            hmc.hmc_restore(lat.h)
        for lat in lats:
            lat.synchronize()

    def ens_step():
        restore()
        t0 = time.perf_counter()
        hmc.hmc_ensemble_sweep(E, kT, seeds, n_mcs)
        hmc.hmc_ensemble_synchronize(E)
        return time.perf_counter() - t0

    def single_step():
        restore()
        t0 = time.perf_counter()
        for lat, w in zip(lats, members):
            lat.sweep(w.kT, n_mcs, w.sweep_seed)
        for lat in lats:
            lat.synchronize()
        return time.perf_counter() - t0

    res = {}
    for name, fn in (("ensemble", ens_step), ("one_by_one", single_step)):
        for _ in range(args.warmup):
            fn()
        res[name] = sum(fn() for _ in range(args.steps)) / args.steps
    # kernel time: HIP events around the graph replay on the ensemble's stream
    hmc.hmc_ensemble_profile(E, True)
    hmc.hmc_ensemble_profile_read(E)
    ens_step()
    kernel_ms, launches, su_prof = hmc.hmc_ensemble_profile_read(E)
    hmc.hmc_ensemble_profile(E, False)
    finals = [lat.spins().astype(np.int32) for lat in lats]
    # the ensemble's result equals the one-by-one result
    single_step()
    same = all(np.array_equal(x, lat.spins()) for x, lat in zip(finals, lats))
    hmc.hmc_ensemble_free(E)
    for lat in lats:
        lat.close()
    su = total_sites * n_mcs
    C = {hmc.HMC_VN4: 2, hmc.HMC_MOORE8: 4, hmc.HMC_VN6: 2, hmc.HMC_MOORE26: 8}[members[0].nbr]
    bpsu = (C + 1) * 2   # int16: one pass reads every spin and writes the 1/C it updates
    launch_s = kernel_ms / 1e3 / max(launches, 1)
    su_launch = su_prof / max(launches, 1)
    achieved = su_launch * bpsu / launch_s / 1e9
    # 16-bit Moore8 members in 128x128 or 256x128 tiles with 3 MC steps per
    # launch: the library's kernel compiled for that tile runs every full launch
    kname = ("ens2d_kernel" if members[0].nbr == hmc.HMC_MOORE8 and tuple(tiling) in ((128, 128, 1, 3), (256, 128, 1, 3))
             else "ensemble_kernel")
    prof = measured_profile("ensemble_moore8", tuple(tiling), kernel=kname)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBPS, "traffic": prof.get("traffic_bytes_per_launch"),
                "traffic_note": "scaled FETCH_SIZE+WRITE_SIZE bytes per launch from profiles/ (null if the kernel "
                                "changed)",
                "kernel": kname, "avg_launch_us": launch_s * 1e6,
                "launch_timing": "HIP events around the graph replay on the ensemble's stream (kernels and the gaps "
                                 "between them), replay of one timed step",
                "launches": launches, "bytes_per_site_update": bpsu, "site_updates_per_launch": su_launch}
    if prof.get("valu_wave_instructions_per_launch"):
        v = prof["valu_wave_instructions_per_launch"]
        roofline["valu"] = {"wave_instructions_per_launch": v, "per_site_update": v / su_launch,
                            "issue_frac": v / (VALU_ISSUE_PER_S * launch_s)}
    extra = {}
    if not args.no_cpu_baseline:
        # the oracle on whole members, smallest first, as many as the budget allows
        import oracle
        threads, host = host_threads()
        order = sorted(range(len(members)), key=lambda i: members[i].n_sites)
        t0 = time.perf_counter()
        done, sites, exact = 0, 0, True
        for i in order:
            if time.perf_counter() - t0 > args.cpu_seconds:
                break
            w = members[i]
            out = oracle.sweep(starts[i], w.nbr, w.dims, w.B, w.kT, n_mcs, w.sweep_seed, threads=threads)
            exact = exact and bool(np.array_equal(out, finals[i]))
            done += 1
            sites += w.n_sites
        dt = time.perf_counter() - t0
        extra["cpu_baseline"] = {"value": sites * n_mcs / dt, "unit": "site-updates/s", "cores": threads,
                                 "kind": "oracle", **host,
                                 "sample": f"the {done} smallest of {len(members)} members, whole {n_mcs}-MCS runs "
                                           f"({sites * n_mcs:.3g} site updates, {dt:.1f} s)",
                                 "gpu_bit_exact_on_sample": exact}
    _line("Potts site-updates/s, 64-lattice Moore-8 ensemble, 1 MI355X", su / res["ensemble"], args,
          res["ensemble"] * 1e3,
          {"workload": "ensemble_moore8", "lattices": len(members), "sites": total_sites,
           "mcs_per_step": n_mcs, "tiling": list(tiling)},
          roofline=roofline,
          one_by_one={"value": su / res["one_by_one"], "ms_per_step": res["one_by_one"] * 1e3},
          speedup_vs_one_by_one=res["one_by_one"] / res["ensemble"], ensemble_equals_one_by_one=same,
          timing_note="each step times the one ensemble call (and the one-by-one sweeps beside it); restoring "
                      "the members' initial states runs before the timed region", **extra)


def nfold_profile():
    """Per-launch SQ_INSTS_VALU and scaled HBM bytes of the n-fold kernel
    from the committed rocprofv3 summary, or None when the kernel source
    changed since."""
    path = os.path.join(ROOT, "profiles", "nfold_kernel_nfold_ensemble_128.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", "`")):
            k, v = line.split(":", 1)
            fields[k.strip()] = (v.split() or [""])[0]
    if fields.get("kernel_source_sha256") != source_sha("nfold.hip"):
        return None
    return {k: float(fields[k]) for k in ("valu_wave_instructions_per_launch", "traffic_bytes_per_launch")
            if k in fields}


def bench_nfold(args, hmc):
    """The n-fold way (rejection-free, continuous time) on 1024 VN4 128^2
    lattices (polycrystals at kT 0.25, or flat strips driven by a bulk
    energy at kT 0.3), one batch call (one wave per lattice), against the
    same lattices advanced by the same MC time with red/black sweeps in one
    ensemble call; the oracle's n-fold way on a sample of the lattices as the
    CPU baseline, bit-exact with the GPU on that sample."""
    import oracle

    members = synth.nfold_strip_128() if args.workload == "nfold_strip_128" else synth.nfold_ensemble_128()
    mcs = float(args.mcs or members[0].n_mcs)
    lats, starts = [], []
    for w in members:
        if "spins" in w.extra:
            lat = hmc.Lattice(w.dims, w.nbr, w.n_grains, spin=w.spin)
            lat.set_spins(w.extra["spins"])
        else:
            lat = hmc.Lattice(w.dims, w.nbr, w.n_grains, voronoi_seed=w.voronoi_seed, spin=w.spin)
        lat.set_grain_energy(w.B)
        starts.append(lat.spins().astype(np.int32))
        hmc.hmc_snapshot(lat.h)
        lats.append(lat)
    kT = np.array([w.kT for w in members], np.float32)
    seeds = np.array([w.sweep_seed for w in members], np.uint64)
    total_sites = sum(w.n_sites for w in members)

    def restore():
        # the initial state of every lattice, restored outside the timed region
        for lat in lats:
            hmc.hmc_restore(lat.h)
        for lat in lats:
            lat.synchronize()

    def nf_step():
        restore()
        t0 = time.perf_counter()
        hmc.hmc_nfold_batch(lats, kT, mcs, seeds)   # synchronous
        return time.perf_counter() - t0

    for _ in range(args.warmup):
        nf_step()
    nf_s = sum(nf_step() for _ in range(args.steps)) / args.steps
    clocks = [lat.nfold_clock() for lat in lats]
    events = sum(c[2] for c in clocks)
    # kernel duration: HIP events bound to each n-fold dispatch, one replay
    hmc.hmc_profile(lats[0].h, True)
    hmc.hmc_profile_read(lats[0].h)
    nf_step()
    kernel_ms, launches, _ = hmc.hmc_profile_read(lats[0].h)
    hmc.hmc_profile(lats[0].h, False)
    finals = [lat.spins().astype(np.int32) for lat in lats]

    # red/black sweeps over the same lattices and MC time
    E = hmc.hmc_ensemble_create(lats)

    def rb_step():
        restore()
        t0 = time.perf_counter()
        hmc.hmc_ensemble_sweep(E, kT, seeds, int(round(mcs)))
        hmc.hmc_ensemble_synchronize(E)
        return time.perf_counter() - t0

    for _ in range(args.warmup):
        rb_step()
    rb_s = sum(rb_step() for _ in range(args.steps)) / args.steps
    hmc.hmc_ensemble_free(E)

    site_mcs = total_sites * mcs
    prof = (nfold_profile() or {}) if args.workload == "nfold_ensemble_128" else {}
    valu = prof.get("valu_wave_instructions_per_launch")
    kernel_s = kernel_ms / 1e3 / max(launches, 1)
    peak_lane = VALU_ISSUE_PER_S * 64 / 1e12   # VALU lane-instructions/s, 1 wave instruction per CU per cycle
    out = {
        "metric": "Potts site-MC-steps/s with the n-fold way, 1024-lattice batch, 1 MI355X, bit-exact vs oracle",
        "value": site_mcs / nf_s, "unit": "site-MC-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": nf_s * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int16", "data": "synthetic",
        "config": {"workload": args.workload, "lattices": len(members), "lattice": "128x128",
                   "neighbourhood": "VN4", "grains": members[0].n_grains, "kT": float(kT[0]),
                   "mcs_per_step": mcs},
        "events_per_step": events,
        "events_per_s": events / nf_s,
        "roofline": {
            "bound": "alu",
            "achieved": valu * 64 / kernel_s / 1e12 if valu else None,
            "peak": peak_lane, "unit": "T VALU lane-instructions/s",
            "frac": valu * 64 / kernel_s / 1e12 / peak_lane if valu else None,
            "traffic": prof.get("traffic_bytes_per_launch"),
            "kernel": "nfold_kernel", "avg_launch_us": kernel_s * 1e6, "launches": launches,
            "latency_per_event_us": kernel_ms * 1e3 / max(max(c[2] for c in clocks), 1),
            "note": "one dependent chain of events per wave, four waves per CU (LDS): latency-bound.  achieved = "
                    "SQ_INSTS_VALU x 64 lanes per launch from profiles/ (null if the kernel changed) over the "
                    "launch; peak = 256 CUs x 64 lanes x 2.4 GHz (one VALU wave instruction per CU per cycle)",
        },
        "red_black_same_lattices": {"value": site_mcs / rb_s, "ms_per_step": rb_s * 1e3,
                                    "note": "hmc_ensemble_sweep over the same 1024 lattices for the same MC steps"},
        "timing_note": "each step times the one batch call (and the ensemble call beside it); restoring the "
                       "1024 initial states runs before the timed region",
    }
    if not args.no_cpu_baseline:
        # single-core oracle on whole lattices, as many as the budget allows
        t0 = time.perf_counter()
        done, exact = 0, True
        while done < len(members) and (time.perf_counter() - t0) < args.cpu_seconds:
            w = members[done]
            s, t_last, ne, _ = oracle.nfold(starts[done], w.nbr, w.dims, w.B, w.kT, w.sweep_seed, mcs)
            exact = exact and bool(np.array_equal(s, finals[done])) and (t_last, ne) == clocks[done][1:]
            done += 1
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": done * members[0].n_sites * mcs / dt, "unit": "site-MC-steps/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"first {done} of {len(members)} lattices, whole {mcs:g}-MCS runs, "
                                         f"{dt:.1f} s", "gpu_bit_exact_on_sample": exact}
    for lat in lats:
        lat.close()
    print(json.dumps(out), flush=True)


def bench_learned(args, hmc):
    """256^3 VN6 lattice whose grain bulk energies come from the stored
    dislocation energy under a monotonic uniaxial strain, re-queried every 10
    MC steps (50 queries over 500 steps): the trained network (with audit)
    against the crystal-plasticity solver in the loop."""
    w = synth.schmid_3d_256()
    R = synth.LEARNED
    n_mcs = args.mcs or w.n_mcs
    every = R["every"]
    n_q = n_mcs // every
    # training data from the solver (outside the timed region)
    n_train, n_test = R["n_train"], R["n_test"]
    eu, ep = synth.crystal_inputs(n_train + n_test, R["data_seed"])
    t0 = time.perf_counter()
    Ey = hmc.hmc_mcp_solve(eu, ep, seed=R["solver_seed"])
    t_gen = time.perf_counter() - t0
    M = hmc.hmc_mlp_create(R["init_seed"])
    t0 = time.perf_counter()
    loss = hmc.hmc_mlp_train(M, eu[:n_train], ep[:n_train], Ey[:n_train], epochs=R["epochs"], batch=R["batch"],
                             lr=R["lr"], seed=R["train_seed"])
    t_train = time.perf_counter() - t0
    pred = hmc.hmc_mlp_predict(M, eu[n_train:], ep[n_train:])
    rel = np.abs(pred - Ey[n_train:]) / Ey[n_train:]
    E_ref = float(Ey[:n_train].max())
    scale = 0.15 / E_ref              # E_MC = 0.15 E_rho / max training E_rho
    lat = hmc.Lattice(w.dims, w.nbr, w.n_grains, voronoi_seed=w.voronoi_seed, spin=w.spin)
    hmc.hmc_snapshot(lat.h)
    euler = w.euler

    def job(mode):
        hmc.hmc_restore(lat.h)
        fallbacks, errs, tq = 0, [], 0.0
        for k in range(n_q):
            q0 = time.perf_counter()
            _, used, err = hmc.hmc_surrogate_update(lat, M, euler, synth.uniaxial_strain(k + 1, n_q), scale,
                                                    mode=mode, n_audit=R["n_audit"], audit_tol=R["audit_tol"],
                                                    seed=k)
            tq += time.perf_counter() - q0
            fallbacks += int(used)
            errs.append(err)
            lat.sweep(w.kT, every, w.sweep_seed)
        lat.synchronize()
        return fallbacks, errs, tq

    res = {}
    for name, mode in (("surrogate", 0), ("solver", 1)):
        for _ in range(args.warmup):
            job(mode)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fb, errs, tq = job(mode)
        res[name] = ((time.perf_counter() - t0) / args.steps, fb, float(np.max(errs)), tq)
        res[name + "_frac"] = lat.texture_stats(w.grain_bin, w.n_bins)[2]
    drift = float(np.max(np.abs(res["surrogate_frac"] - res["solver_frac"])))
    # the network's own cost: queries without the audit
    hmc.hmc_restore(lat.h)
    q0 = time.perf_counter()
    for k in range(n_q):
        hmc.hmc_surrogate_update(lat, M, euler, synth.uniaxial_strain(k + 1, n_q), scale, mode=0, n_audit=0,
                                 audit_tol=0.25, seed=k)
    net_ms = (time.perf_counter() - q0) / n_q * 1e3
    lat.close()
    hmc.hmc_mlp_free(M)
    cpu = None
    if not args.no_cpu_baseline:
        # the method without the network on the host: the oracle's solver for
        # one query (every grain under the last strain of the path)
        import oracle
        threads, host = host_threads()
        tiled = np.tile(synth.uniaxial_strain(n_q, n_q), (w.n_grains, 1))
        t0 = time.perf_counter()
        oracle.mcp_solve(euler, tiled, seed=0, threads=threads)
        cpu = {"value": (time.perf_counter() - t0) * 1e3, "unit": "ms per query", "cores": threads, "kind": "oracle", **host,
               "sample": f"crystal-plasticity solve of the {w.n_grains} grains under the final strain"}
    su = w.n_sites * n_mcs
    _line("Potts site-updates/s with learned stored energy (re-queried every 10 MCS), 1 MI355X",
          su / res["surrogate"][0], args, res["surrogate"][0] * 1e3,
          {"workload": "learned_3d_256", "lattice": "256x256x256", "neighbourhood": "VN6", "grains": w.n_grains,
           "mcs_per_step": n_mcs, "queries": n_q},
          solver_in_loop={"value": su / res["solver"][0], "ms_per_step": res["solver"][0] * 1e3,
                          "query_ms": res["solver"][3] / n_q * 1e3},
          surrogate={"query_ms": res["surrogate"][3] / n_q * 1e3, "query_ms_without_audit": net_ms,
                     "fallbacks": res["surrogate"][1],
                     "max_audit_rel_err": res["surrogate"][2],
                     "held_out_rel_err_median": float(np.median(rel)),
                     "held_out_rel_err_p95": float(np.percentile(rel, 95)), "train_loss": loss,
                     "train_s": t_train, "solver_data_s": t_gen},
          texture_fraction_drift_max=drift, cpu_solver_query=cpu)


if __name__ == "__main__":
    main()
