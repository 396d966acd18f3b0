"""GPU: whole jobs of the graded workloads against the oracle, bit-exact
(Sec. 3 Metropolis trials, Sec. 4 Red/Black half steps, Sec. 6 grain energy).

* 256^3 VN6 int16 (20 000 grains, Schmid energies, kT 0.6): the whole
  500-step job, and on to 1000 steps, spins and grain statistics equal;
* the 64-lattice Moore8 ensemble (sides 128..1024, kT 0.3..1.0, one HIP-graph
  call): every member after its whole 1000 steps equals the oracle;
* the learned 256^3 run: a network trained on the workload's 10^6 solver
  samples drives the grain energies, re-queried every 10 steps for 500
  steps; the spins equal the oracle's fed the same integer energies, and
  the network's held-out error and the texture drift against the solver in
  the loop over four seeds are reported (as warnings, so that they show in
  the run's summary) and bounded.
"""
import os
import warnings
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import paper_1007_3509_amd as hmc
import synth

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, len(os.sched_getaffinity(0))))


def say(*a):
    print(*a, flush=True)


def test_schmid_3d_256_whole_job_500_and_1000_mcs():
    w = synth.schmid_3d_256()
    say(f"[gpu] {w.name}: whole {w.n_mcs}-step job and on to 1000")
    with hmc.Lattice(w.dims, w.nbr, w.n_grains, voronoi_seed=w.voronoi_seed, spin=w.spin) as lat:
        lat.set_grain_energy(w.B)
        start = lat.spins().astype(np.int32)
        lat.sweep(w.kT, w.n_mcs, w.sweep_seed)
        got500 = lat.spins().astype(np.int32)
        ng, mean, frac = lat.texture_stats(w.grain_bin, w.n_bins)
        lat.sweep(w.kT, 1000 - w.n_mcs, w.sweep_seed)
        got1000 = lat.spins().astype(np.int32)
        assert lat.mcs == 1000
    want = oracle.sweep(start, w.nbr, w.dims, w.B, w.kT, w.n_mcs, w.sweep_seed, threads=THREADS)
    assert np.array_equal(got500, want), f"{int(np.sum(got500 != want))} sites differ after {w.n_mcs} steps"
    _, ng_o, mean_o, frac_o = oracle.texture(want, w.n_grains, w.grain_bin, w.n_bins)
    assert ng == ng_o and mean == mean_o and np.array_equal(frac, frac_o)
    want = oracle.sweep(want, w.nbr, w.dims, w.B, w.kT, 1000 - w.n_mcs, w.sweep_seed, mcs0=w.n_mcs,
                        threads=THREADS)
    assert np.array_equal(got1000, want), f"{int(np.sum(got1000 != want))} sites differ after 1000 steps"


def test_ensemble_moore8_every_member_whole_1000_mcs():
    members = synth.ensemble_moore8()
    say(f"[gpu] ensemble_moore8: {len(members)} members, {members[0].n_mcs} steps in one call")
    lats = []
    try:
        for w in members:
            lat = hmc.Lattice(w.dims, w.nbr, w.n_grains, voronoi_seed=w.voronoi_seed, spin=w.spin)
            lat.set_grain_energy(w.B)
            lats.append(lat)
        starts = [lat.spins().astype(np.int32) for lat in lats]
        E = hmc.hmc_ensemble_create(lats)
        try:
            kT = np.array([w.kT for w in members], np.float32)
            seeds = np.array([w.sweep_seed for w in members], np.uint64)
            hmc.hmc_ensemble_sweep(E, kT, seeds, members[0].n_mcs)
            hmc.hmc_ensemble_synchronize(E)
        finally:
            hmc.hmc_ensemble_free(E)
        finals = [lat.spins().astype(np.int32) for lat in lats]
        assert all(lat.mcs == members[0].n_mcs for lat in lats)
    finally:
        for lat in lats:
            lat.close()
    say("[cpu] oracle on every member")
    per = max(1, THREADS // 4)

    def one(i):
        w = members[i]
        return oracle.sweep(starts[i], w.nbr, w.dims, w.B, w.kT, w.n_mcs, w.sweep_seed, threads=per)

    order = sorted(range(len(members)), key=lambda i: -members[i].n_sites)
    with ThreadPoolExecutor(max_workers=4) as pool:
        wants = dict(zip(order, pool.map(one, order)))
    bad = [i for i in range(len(members)) if not np.array_equal(finals[i], wants[i])]
    assert not bad, f"members differing from the oracle: {bad}"


def _train_network():
    R = synth.LEARNED
    n_train, n_test = R["n_train"], R["n_test"]
    eu, ep = synth.crystal_inputs(n_train + n_test, R["data_seed"])
    Ey = hmc.hmc_mcp_solve(eu, ep, seed=R["solver_seed"])
    M = hmc.hmc_mlp_create(R["init_seed"])
    loss = hmc.hmc_mlp_train(M, eu[:n_train], ep[:n_train], Ey[:n_train], epochs=R["epochs"], batch=R["batch"],
                             lr=R["lr"], seed=R["train_seed"])
    pred = hmc.hmc_mlp_predict(M, eu[n_train:], ep[n_train:])
    rel = np.abs(pred - Ey[n_train:]) / Ey[n_train:]
    return M, loss, rel, float(Ey[:n_train].max())


def test_learned_3d_256_whole_run_bit_exact_with_error_and_drift():
    w = synth.schmid_3d_256()
    R = synth.LEARNED
    n_q = w.n_mcs // R["every"]
    say(f"[gpu] learned_3d_256: train on {R['n_train']} solver samples, {R['epochs']} epochs")
    M, loss, rel, E_ref = _train_network()
    scale = 0.15 / E_ref
    try:
        fracs = {}
        logged = None
        start = None
        fallbacks = 0
        for sseed in (w.sweep_seed, w.sweep_seed + 1, w.sweep_seed + 2, w.sweep_seed + 3):
            for mode in (0, 1):     # 0: network with audit and fallback, 1: solver in the loop
                say(f"[gpu] 500 steps, sweep seed {sseed}, mode {mode}")
                with hmc.Lattice(w.dims, w.nbr, w.n_grains, voronoi_seed=w.voronoi_seed, spin=w.spin) as lat:
                    if start is None:
                        start = lat.spins().astype(np.int32)
                    Bs = []
                    for k in range(n_q):
                        B, used, _ = hmc.hmc_surrogate_update(lat, M, w.euler, synth.uniaxial_strain(k + 1, n_q),
                                                              scale, mode=mode, n_audit=R["n_audit"],
                                                              audit_tol=R["audit_tol"], seed=k)
                        fallbacks += int(used) if mode == 0 else 0
                        Bs.append(B)
                        lat.sweep(w.kT, R["every"], sseed)
                    fracs[(sseed, mode)] = lat.texture_stats(w.grain_bin, w.n_bins)[2]
                    if logged is None:
                        logged = (Bs, lat.spins().astype(np.int32), sseed)
    finally:
        hmc.hmc_mlp_free(M)
    # the network-driven run against the oracle fed the same integer energies
    Bs, got, sseed = logged
    say("[cpu] oracle replay of the network-driven run")
    s = start
    for k, B in enumerate(Bs):
        s = oracle.sweep(s, w.nbr, w.dims, B, w.kT, R["every"], sseed, mcs0=R["every"] * k, threads=THREADS)
    assert np.array_equal(got, s), f"{int(np.sum(got != s))} sites differ from the oracle"
    drift = max(float(np.max(np.abs(fracs[(sd, 0)] - fracs[(sd, 1)]))) for sd in {k[0] for k in fracs})
    med, p95 = float(np.median(rel)), float(np.percentile(rel, 95))
    warnings.warn(f"learned_3d_256: held-out relative energy error median {med:.4f}, p95 {p95:.4f} "
                  f"({R['n_test']} samples); max texture-fraction drift vs the solver in the loop at "
                  f"{w.n_mcs} steps over 4 seeds {drift:.2e}; {fallbacks} of {4 * n_q} queries fell back; "
                  f"train loss {loss:.3g}")
    # the training recipe gives median 0.019, p95 0.056 with the orientation
    # as its cubic fundamental-zone Rodrigues vector (raw Euler angles
    # stopped at p95 0.141-0.147); the target is a p95 of at most 0.10
    assert med < 0.03 and p95 < 0.10
    assert drift < 5e-3
