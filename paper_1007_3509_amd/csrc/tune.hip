// tune.hip -- autotuner for the sweep kernel's tiling.
//
// The tiling (interior tile sides and MC steps fused per launch) trades
// redundant halo work and LDS footprint against launch count and
// parallelism, and the best point depends on the lattice shape and on how
// many sites sit on grain boundaries.  The autotuner times candidates on the
// real kernel and keeps the fastest; results never depend on the choice.
// Cache format: one JSON object per line, e.g.
//   {"nbr":0,"spin":0,"dims":[1024,1024,1],"tile":[64,64,1],"k":4,"us_per_mcs":5.1}
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "common.hpp"

namespace hmc {

namespace {

using Key = std::tuple<int, int, int, int, int>;
std::mutex g_mu;
std::map<Key, Tiling>& table() {
    static std::map<Key, Tiling> t;
    return t;
}

Key key_of(const hmc_lattice_desc& d) {
    return Key(d.nbr, d.spin, d.dims[0], d.dims[1], d.ndim == 3 ? d.dims[2] : 1);
}

std::vector<Tiling> candidates(const hmc_lattice_desc& d) {
    std::vector<Tiling> out;
    const int C = nbr_info(d.nbr).C;
    const std::vector<int> sides2 = {16, 32, 64, 128, 256};
    const std::vector<int> sides3 = {4, 8, 16, 32, 64};
    // MC steps per launch; with four or eight colours also launches of 1, 2
    // or 4 colour passes (negative k), whose halos are thinner
    std::vector<int> ks = {1, 2, 3, 4, 5, 6, 8};
    if (C >= 4) ks.insert(ks.end(), {-1, -2, -4});
    auto divides = [&](int s, int L) { return s <= L && L % s == 0; };
    if (d.ndim == 2) {
        for (int tx : sides2)
            for (int ty : sides2)
                for (int k : ks) {
                    if (!divides(tx, d.dims[0]) || !divides(ty, d.dims[1]) || k * C > 64) continue;   // k < 0 passes
                    if (tx < ty / 2 || ty < tx / 4) continue;   // keep near-square, x-wide shapes
                    Tiling t;
                    t.tx = tx; t.ty = ty; t.tz = 1; t.k = k;
                    out.push_back(t);
                }
    } else {
        for (int tx : sides3)
            for (int ty : sides3)
                for (int tz : sides3)
                    for (int k : ks) {
                        if (!divides(tx, d.dims[0]) || !divides(ty, d.dims[1]) || !divides(tz, d.dims[2])) continue;
                        if (k * C > 64 || ty > tx || tz > ty) continue;
                        Tiling t;
                        t.tx = tx; t.ty = ty; t.tz = tz; t.k = k;
                        out.push_back(t);
                    }
    }
    return out;
}

}  // namespace

const Tiling* tuned_tiling(const hmc_lattice_desc& d, int32_t) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = table().find(key_of(d));
    return it == table().end() ? nullptr : &it->second;
}

void record_tuning(const hmc_lattice_desc& d, const Tiling& t, double) {
    std::lock_guard<std::mutex> lk(g_mu);
    table()[key_of(d)] = t;
}

}  // namespace hmc

using namespace hmc;

namespace {

// Time one tiling: restore the start state, warm up, then time n_mcs steps.
hmc_status time_lattice(hmc_lattice* L, const Tiling& t, float kT, int32_t n_mcs, double* us) {
    HMC_TRY(hmc_set_tiling(L, t.tx, t.ty, t.tz, t.k));
    HMC_TRY(hmc_restore(L));
    HMC_TRY(hmc_sweep(L, kT, std::min(n_mcs, 2 * std::max(t.k, 1)), 1));
    HMC_TRY(hmc_restore(L));
    hipEvent_t a, b;
    HMC_HIP(hipEventCreate(&a));
    HMC_HIP(hipEventCreate(&b));
    hipError_t e = hipEventRecord(a, L->stream);
    hmc_status st = e == hipSuccess ? hmc_sweep(L, kT, n_mcs, 1) : HMC_OK;
    if (e == hipSuccess && st == HMC_OK) e = hipEventRecord(b, L->stream);
    if (e == hipSuccess && st == HMC_OK) e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess && st == HMC_OK) e = hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != HMC_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "autotune timing");
    *us = (double)ms * 1e3 / n_mcs;
    return HMC_OK;
}

}  // namespace

extern "C" {

hmc_status hmc_autotune(const hmc_lattice_desc* desc, int32_t n_grains, float kT, int32_t n_mcs,
                        const char* cache_path, int32_t* best_out4, double* us_per_mcs_out) {
    set_error("");
    if (!desc || !best_out4) return fail(HMC_E_INVAL, "NULL argument");
    if (n_mcs < 1) return fail(HMC_E_INVAL, "n_mcs must be >= 1");
    if (!(kT > 0.0f)) return fail(HMC_E_INVAL, "kT must be positive");
    hmc_lattice* L = nullptr;
    HMC_TRY(hmc_lattice_init(desc, n_grains, 1, nullptr, &L));
    hmc_status st = hmc_snapshot(L);
    Tiling best;
    double best_us = 1e300;
    if (st == HMC_OK) {
        for (const Tiling& t : candidates(L->desc)) {
            double us = 0.0;
            const hmc_status s = time_lattice(L, t, kT, n_mcs, &us);
            if (s == HMC_E_INVAL) continue;   // does not fit: skip the candidate
            if (s != HMC_OK) { st = s; break; }
            if (us < best_us) { best_us = us; best = t; }
        }
    }
    hmc_lattice_free(L);
    if (st != HMC_OK) return st;
    if (best.tx == 0) return fail(HMC_E_INVAL, "no tiling candidate fits this lattice");
    set_error("");
    record_tuning(*desc, best, best_us);
    best_out4[0] = best.tx; best_out4[1] = best.ty; best_out4[2] = best.tz; best_out4[3] = best.k;
    if (us_per_mcs_out) *us_per_mcs_out = best_us;
    if (cache_path) {
        FILE* f = std::fopen(cache_path, "a");
        if (!f) return fail(HMC_E_INVAL, std::string("cannot open ") + cache_path);
        std::fprintf(f, "{\"nbr\":%d,\"spin\":%d,\"dims\":[%d,%d,%d],\"tile\":[%d,%d,%d],\"k\":%d,\"us_per_mcs\":%.4f}\n",
                     desc->nbr, desc->spin, desc->dims[0], desc->dims[1], desc->ndim == 3 ? desc->dims[2] : 1,
                     best.tx, best.ty, best.tz, best.k, best_us);
        std::fclose(f);
    }
    return HMC_OK;
}

hmc_status hmc_tuning_load(const char* cache_path, int32_t* n_loaded) {
    set_error("");
    if (!cache_path) return fail(HMC_E_INVAL, "cache_path is NULL");
    FILE* f = std::fopen(cache_path, "r");
    if (!f) return fail(HMC_E_INVAL, std::string("cannot open ") + cache_path);
    char line[512];
    int32_t n = 0;
    while (std::fgets(line, sizeof line, f)) {
        hmc_lattice_desc d{};
        Tiling t;
        double us = 0.0;
        int lz = 1;
        if (std::sscanf(line, "{\"nbr\":%d,\"spin\":%d,\"dims\":[%d,%d,%d],\"tile\":[%d,%d,%d],\"k\":%d,\"us_per_mcs\":%lf}",
                        &d.nbr, &d.spin, &d.dims[0], &d.dims[1], &lz, &t.tx, &t.ty, &t.tz, &t.k, &us) != 10)
            continue;
        const NbrInfo ni = nbr_info(d.nbr);
        if (ni.M == 0) continue;
        d.ndim = ni.ndim;
        d.dims[2] = lz;
        record_tuning(d, t, us);
        ++n;
    }
    std::fclose(f);
    if (n_loaded) *n_loaded = n;
    return HMC_OK;
}

hmc_status hmc_ensemble_autotune(hmc_ensemble* E, const float* kT, const uint64_t* seed, int32_t n_mcs,
                                 int32_t* best_out4) {
    set_error("");
    if (!E || !kT || !seed || !best_out4) return fail(HMC_E_INVAL, "NULL argument");
    if (n_mcs < 1) return fail(HMC_E_INVAL, "n_mcs must be >= 1");
    // save every member (spins of the current buffer + MC counter)
    std::vector<void*> saved(E->lats.size(), nullptr);
    std::vector<uint64_t> mcs(E->lats.size());
    hmc_status st = HMC_OK;
    for (size_t i = 0; i < E->lats.size() && st == HMC_OK; ++i) {
        hmc_lattice* L = E->lats[i];
        const size_t sb = (size_t)L->N * L->spin_bytes;
        st = dev_alloc(&saved[i], sb, "autotune save");
        if (st == HMC_OK) {
            const hipError_t e = hipMemcpyAsync(saved[i], L->spins[L->cur], sb, hipMemcpyDeviceToDevice, L->stream);
            if (e != hipSuccess) st = hip_fail(e, "autotune save");
        }
        mcs[i] = L->mcs;
    }
    auto restore = [&]() -> hmc_status {
        HMC_HIP(hipStreamSynchronize(E->stream));
        for (size_t i = 0; i < E->lats.size(); ++i) {
            hmc_lattice* L = E->lats[i];
            HMC_HIP(hipMemcpyAsync(L->spins[L->cur], saved[i], (size_t)L->N * L->spin_bytes,
                                   hipMemcpyDeviceToDevice, L->stream));
            L->mcs = mcs[i];
            HMC_HIP(hipStreamSynchronize(L->stream));
        }
        return HMC_OK;
    };
    const Tiling original = E->tiling;
    Tiling best;
    double best_ms = 1e300;
    if (st == HMC_OK) {
        hmc_lattice_desc d = E->lats[0]->desc;
        // candidate sides must divide every member: use the smallest member's shape
        for (hmc_lattice* L : E->lats)
            for (int a = 0; a < L->ndim; ++a) d.dims[a] = std::min(d.dims[a], L->desc.dims[a]);
        for (const Tiling& t : candidates(d)) {
            if (hmc_ensemble_set_tiling(E, t.tx, t.ty, t.tz, t.k) != HMC_OK) continue;
            hipEvent_t a, b;
            HMC_HIP(hipEventCreate(&a));
            HMC_HIP(hipEventCreate(&b));
            st = hmc_ensemble_sweep(E, kT, seed, n_mcs);   // warm-up + graph capture
            if (st == HMC_OK) st = restore();
            hipError_t e = hipSuccess;
            if (st == HMC_OK) e = hipEventRecord(a, E->stream);
            if (st == HMC_OK && e == hipSuccess) st = hmc_ensemble_sweep(E, kT, seed, n_mcs);
            if (st == HMC_OK && e == hipSuccess) e = hipEventRecord(b, E->stream);
            if (st == HMC_OK && e == hipSuccess) e = hipEventSynchronize(b);
            float ms = 0.0f;
            if (st == HMC_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            if (st == HMC_OK && e != hipSuccess) st = hip_fail(e, "ensemble autotune timing");
            if (st == HMC_OK) st = restore();
            if (st != HMC_OK) break;
            if (ms < best_ms) { best_ms = ms; best = t; }
        }
    }
    for (size_t i = 0; i < saved.size(); ++i)
        dev_free(saved[i], saved[i] ? (size_t)E->lats[i]->N * E->lats[i]->spin_bytes : 0);
    if (st != HMC_OK) return st;
    if (best.tx == 0) {
        E->tiling = original;
        E->prepared = false;
        return fail(HMC_E_INVAL, "no tiling candidate fits every member");
    }
    HMC_TRY(hmc_ensemble_set_tiling(E, best.tx, best.ty, best.tz, best.k));
    best_out4[0] = best.tx; best_out4[1] = best.ty; best_out4[2] = best.tz; best_out4[3] = best.k;
    set_error("");
    return HMC_OK;
}

}  // extern "C"
