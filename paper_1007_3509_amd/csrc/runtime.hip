// runtime.hip -- host runtime and C ABI of libhmc.
//
// Validation happens here, on the host, before any device work: invalid
// arguments return HMC_E_INVAL without touching the GPU.  The threshold
// table T(d) = min(2^32-1, floor(2^32 exp(-d/(65536 kT)))) of the Metropolis
// rule (Sec. 3-4 of the paper) is evaluated here in double precision with the
// C library exp and uploaded; kernels only compare integers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "common.hpp"

namespace hmc {

namespace {
thread_local std::string g_error;
std::atomic<uint64_t> g_bytes{0};

uint64_t byte_cap() {
    static uint64_t cap = [] {
        const char* s = std::getenv("HMC_MAX_BYTES");
        if (!s || !*s) return std::numeric_limits<uint64_t>::max();
        return (uint64_t)std::strtoull(s, nullptr, 10);
    }();
    return cap;
}

// Keep libm's exp out of reach of any compile-time rewriting.
double (*volatile g_exp)(double) = &std::exp;
}  // namespace

void set_error(const std::string& msg) { g_error = msg; }

hmc_status fail(hmc_status code, const std::string& msg) {
    g_error = msg;
    return code;
}

hmc_status hip_fail(hipError_t e, const char* what) {
    g_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? HMC_E_NOMEM : HMC_E_DEVICE;
}

hmc_status dev_alloc(void** p, size_t bytes, const char* what) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    const uint64_t now = g_bytes.fetch_add(bytes) + bytes;
    if (now > byte_cap()) {
        g_bytes.fetch_sub(bytes);
        return fail(HMC_E_NOMEM, std::string(what) + ": HMC_MAX_BYTES cap exceeded");
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        g_bytes.fetch_sub(bytes);
        *p = nullptr;
        return hip_fail(e, what);
    }
    return HMC_OK;
}

void dev_free(void* p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    g_bytes.fetch_sub(bytes == 0 ? 16 : bytes);
}

NbrInfo nbr_info(int nbr) {
    switch (nbr) {
    case HMC_VN4: return {4, 2, 2};
    case HMC_MOORE8: return {8, 4, 2};
    case HMC_VN6: return {6, 2, 3};
    case HMC_MOORE26: return {26, 8, 3};
    default: return {0, 0, 0};
    }
}

uint32_t threshold_value(int64_t d, float kT) {
    const double x = (double)d / (65536.0 * (double)kT);
    const double v = std::ldexp(g_exp(-x), 32);
    if (v >= 4294967295.0) return 0xFFFFFFFFu;
    return (uint32_t)std::floor(v);
}

namespace {
constexpr size_t kTableCapBytes = 256ull << 20;
}

hmc_status table_host(float kT, int M, int32_t J_fx, int32_t Bmin, int32_t Bmax, TableLayout& lay,
                      std::vector<uint32_t>& host) {
    const int64_t R = (int64_t)Bmax - Bmin;
    if (R < 0) return fail(HMC_E_INVAL, "Bmax < Bmin");
    int64_t dn_lo = -M;
    while (dn_lo <= M && (int64_t)J_fx * dn_lo + R <= 0) ++dn_lo;
    if (dn_lo > M) dn_lo = M;   // no positive d possible; keep one row
    const int64_t rows = M - dn_lo + 1;
    const int64_t TW = 2 * R + 1;
    const size_t entries = (size_t)(rows * TW);
    // at least two columns per bucket unless the row has a single column
    const int64_t nb = TW == 1 ? 1 : std::max<int64_t>(1, std::min<int64_t>(TW / 2, kBoundPairs / std::max<int64_t>(rows, 1)));
    const int64_t bw = (TW + nb - 1) / nb;
    const size_t nbound = 2 * (size_t)(rows * nb);
    const size_t bytes = (entries + nbound) * sizeof(uint32_t);
    if (bytes > kTableCapBytes)
        return fail(HMC_E_RANGE, "threshold table would need " + std::to_string(bytes) + " bytes");
    host.assign(entries + nbound, 0xFFFFFFFFu);
    for (int64_t r = 0; r < rows; ++r) {
        const int64_t dn = dn_lo + r;
        for (int64_t j = 0; j < TW; ++j) {
            const int64_t d = (int64_t)J_fx * dn + (j - R);
            if (d > 0) host[(size_t)(r * TW + j)] = threshold_value(d, kT);
        }
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t c0 = b * bw, c1 = std::min<int64_t>(TW, (b + 1) * bw) - 1;
            const int64_t dmax = (int64_t)J_fx * dn + (c1 - R);
            const int64_t dmin = std::max<int64_t>(1, (int64_t)J_fx * dn + (c0 - R));
            uint32_t* bd = &host[entries + 2 * (size_t)(r * nb + b)];
            if (c0 <= c1 && dmax > 0) {
                bd[0] = threshold_value(dmax, kT);
                bd[1] = threshold_value(dmin, kT);
            }
        }
    }
    lay.dn_lo = (int32_t)dn_lo;
    lay.rows = (int32_t)rows;
    lay.R = (int32_t)R;
    lay.TW = (int32_t)TW;
    lay.nb = (int32_t)nb;
    lay.bw = (int32_t)bw;
    return HMC_OK;
}

hmc_status build_table(Table& tab, float kT, int M, int32_t J_fx, int32_t Bmin, int32_t Bmax, hipStream_t stream) {
    uint32_t bits;
    std::memcpy(&bits, &kT, sizeof bits);
    if (tab.valid && tab.kT_bits == bits && tab.Bmin == Bmin && tab.Bmax == Bmax) return HMC_OK;
    TableLayout lay;
    std::vector<uint32_t> host;
    HMC_TRY(table_host(kT, M, J_fx, Bmin, Bmax, lay, host));
    const size_t entries = (size_t)lay.rows * (size_t)lay.TW;
    const size_t bytes = host.size() * sizeof(uint32_t);
    // the slot the sweeps queued since the last build do not read; the
    // sweeps that read it were queued before that build, earlier in the stream
    const int s = tab.valid ? tab.slot ^ 1 : tab.slot;
    if (!tab.uploaded[s]) HMC_HIP(hipEventCreateWithFlags(&tab.uploaded[s], hipEventDisableTiming));
    HMC_HIP(hipEventSynchronize(tab.uploaded[s]));   // the last upload from this slot's staging
    if (tab.slot_bytes[s] < bytes) {
        HMC_HIP(hipStreamSynchronize(stream));   // growing: nothing queued may still read the old slot
        dev_free(tab.slot_dev[s], tab.slot_bytes[s]);
        tab.slot_dev[s] = nullptr;
        tab.slot_bytes[s] = 0;
        void* p = nullptr;
        HMC_TRY(dev_alloc(&p, bytes, "threshold table"));
        tab.slot_dev[s] = static_cast<uint32_t*>(p);
        tab.slot_bytes[s] = bytes;
    }
    if (tab.pin_bytes[s] < bytes) {
        if (tab.pin[s]) (void)hipHostFree(tab.pin[s]);
        tab.pin[s] = nullptr;
        tab.pin_bytes[s] = 0;
        void* p = nullptr;
        HMC_HIP(hipHostMalloc(&p, bytes, hipHostMallocDefault));
        tab.pin[s] = static_cast<uint32_t*>(p);
        tab.pin_bytes[s] = bytes;
    }
    std::memcpy(tab.pin[s], host.data(), bytes);
    HMC_HIP(hipMemcpyAsync(tab.slot_dev[s], tab.pin[s], bytes, hipMemcpyHostToDevice, stream));
    HMC_HIP(hipEventRecord(tab.uploaded[s], stream));
    tab.slot = s;
    tab.dev = tab.slot_dev[s];
    tab.bytes = tab.slot_bytes[s];
    tab.bounds = tab.dev + entries;
    tab.nb = lay.nb;
    tab.bw = lay.bw;
    tab.dn_lo = lay.dn_lo;
    tab.rows = lay.rows;
    tab.R = lay.R;
    tab.TW = lay.TW;
    tab.kT_bits = bits;
    tab.Bmin = Bmin;
    tab.Bmax = Bmax;
    tab.valid = true;
    return HMC_OK;
}

hmc_status build_direct_table(hmc_lattice* L, float kT) {
    uint32_t bits;
    std::memcpy(&bits, &kT, sizeof bits);
    // largest possible d: every bond of the new spin at the largest energy,
    // none of the old, plus the spreads of the grain energies and the field
    const int64_t bond = L->pair ? L->Jp_max : L->desc.J_fx;
    const int64_t Dmax = (int64_t)L->M * bond + ((int64_t)L->Bmax - L->Bmin) +
                         (L->field ? (int64_t)L->Fmax - L->Fmin : 0);
    if (L->d_Tg && L->Tg_kT_bits == bits && L->Tg_Dmax == Dmax) return HMC_OK;
    const size_t bytes = (size_t)(Dmax + 1) * sizeof(uint32_t);
    if (bytes > kTableCapBytes) return fail(HMC_E_RANGE, "threshold table would need " + std::to_string(bytes) + " bytes");
    std::vector<uint32_t> host((size_t)Dmax + 1);
    host[0] = 0xFFFFFFFFu;   // d <= 0 is accepted before the table is read
    for (int64_t d = 1; d <= Dmax; ++d) host[(size_t)d] = threshold_value(d, kT);
    if (L->Tg_bytes != bytes) {
        dev_free(L->d_Tg, L->Tg_bytes);
        L->d_Tg = nullptr;
        L->Tg_bytes = 0;
        HMC_TRY(dev_alloc(reinterpret_cast<void**>(&L->d_Tg), bytes, "threshold table"));
        L->Tg_bytes = bytes;
    }
    HMC_HIP(hipMemcpyAsync(L->d_Tg, host.data(), bytes, hipMemcpyHostToDevice, L->stream));
    HMC_HIP(hipStreamSynchronize(L->stream));
    L->Tg_kT_bits = bits;
    L->Tg_Dmax = (int32_t)Dmax;
    return HMC_OK;
}

void free_table(Table& tab) {
    for (int s = 0; s < 2; ++s) {
        if (tab.uploaded[s]) {
            (void)hipEventSynchronize(tab.uploaded[s]);
            (void)hipEventDestroy(tab.uploaded[s]);
        }
        dev_free(tab.slot_dev[s], tab.slot_bytes[s]);
        if (tab.pin[s]) (void)hipHostFree(tab.pin[s]);
    }
    tab = Table{};
}

namespace {

hmc_status validate_desc(const hmc_lattice_desc* d, int32_t n_grains) {
    if (!d) return fail(HMC_E_INVAL, "desc is NULL");
    const NbrInfo ni = nbr_info(d->nbr);
    if (ni.M == 0) return fail(HMC_E_INVAL, "unknown neighbourhood " + std::to_string(d->nbr));
    if (d->ndim != ni.ndim)
        return fail(HMC_E_INVAL, "neighbourhood " + std::to_string(d->nbr) + " needs ndim " + std::to_string(ni.ndim));
    uint64_t N = 1;
    for (int a = 0; a < d->ndim; ++a) {
        if (d->dims[a] < 4 || d->dims[a] % 2 != 0 || d->dims[a] > (1 << 22))
            return fail(HMC_E_INVAL, "lattice side " + std::to_string(d->dims[a]) + " must be even and in [4, 2^22]");
        N *= (uint64_t)d->dims[a];
    }
    if (N >= (1ull << 32)) return fail(HMC_E_INVAL, "lattice must have fewer than 2^32 sites");
    if (d->spin != HMC_I16 && d->spin != HMC_I32) return fail(HMC_E_INVAL, "spin type must be HMC_I16 or HMC_I32");
    if (d->proposal != HMC_PROP_NEIGHBOUR && d->proposal != HMC_PROP_UNIFORM)
        return fail(HMC_E_INVAL, "unknown trial mode");
    if (d->J_fx < 1 || d->J_fx > (1 << 24)) return fail(HMC_E_INVAL, "J_fx must be in [1, 2^24]");
    if (n_grains < 1) return fail(HMC_E_INVAL, "n_grains must be >= 1");
    if (d->spin == HMC_I16 && n_grains > 32767) return fail(HMC_E_INVAL, "n_grains > 32767 needs int32 spins");
    if ((int64_t)d->J_fx * ni.M >= (1ll << 31)) return fail(HMC_E_RANGE, "J_fx * M overflows int32");
    return HMC_OK;
}

hmc_status check_energy_range(const hmc_lattice* L, int32_t Bmin, int32_t Bmax, int32_t Jbond, int32_t Fmin = 0,
                              int32_t Fmax = 0) {
    const int64_t maxabs = std::max<int64_t>(std::llabs((int64_t)Bmin), std::llabs((int64_t)Bmax));
    const int64_t fabs_max = std::max<int64_t>(std::llabs((int64_t)Fmin), std::llabs((int64_t)Fmax));
    if ((int64_t)Jbond * L->M + 2 * maxabs + 2 * fabs_max >= (1ll << 31))
        return fail(HMC_E_RANGE, "(largest bond energy)*M + 2 max|B| + 2 max|field| must stay below 2^31");
    return HMC_OK;
}

int32_t bond_max(const hmc_lattice* L) { return L->pair ? L->Jp_max : L->desc.J_fx; }

void destroy(hmc_lattice* L) {
    if (!L) return;
    if (L->stream) (void)hipStreamSynchronize(L->stream);
    const size_t sb = (size_t)L->N * L->spin_bytes;
    if (!L->borrowed) dev_free(L->spins[0], sb);
    dev_free(L->spins[1], sb);
    dev_free(L->snap, sb);
    dev_free(L->dB, (size_t)L->Q * 4);
    if (L->hB_uploaded) (void)hipEventSynchronize(L->hB_uploaded);
    if (L->hB_pinned) (void)hipHostFree(L->hB_pinned);
    if (L->hB_uploaded) (void)hipEventDestroy(L->hB_uploaded);
    dev_free(L->d_areas, (size_t)L->Q * 4);
    dev_free(L->d_stats, (size_t)(1 + L->stats_bins_cap) * 8);
    dev_free(L->d_gbin, (size_t)L->Q * 4);
    dev_free(L->d_trials, kTrialSlots * sizeof(unsigned long long));
    dev_free(L->d_count, sizeof(unsigned long long));
    dev_free(L->d_Jp, (size_t)L->Q * (size_t)L->Q * 4);
    dev_free(L->d_field[0], (size_t)L->N * 4);
    dev_free(L->d_field[1], (size_t)L->N * 4);
    dev_free(L->field_snap, (size_t)L->N * 4);
    dev_free(L->d_Tg, L->Tg_bytes);
    free_table(L->table);
    for (auto& e : L->events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    if (L->own_stream && L->stream) (void)hipStreamDestroy(L->stream);
    delete L;
}

hmc_status create(const hmc_lattice_desc* d, int32_t n_grains, void* stream, hmc_lattice** out,
                  void* borrowed_spins = nullptr) {
    if (!out) return fail(HMC_E_INVAL, "out is NULL");
    *out = nullptr;
    HMC_TRY(validate_desc(d, n_grains));
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(HMC_E_DEVICE, "no HIP device available");
    hmc_lattice* L = new hmc_lattice();
    L->desc = *d;
    if (d->ndim == 2) L->desc.dims[2] = 1;
    L->Q = n_grains;
    const NbrInfo ni = nbr_info(d->nbr);
    L->M = ni.M;
    L->C = ni.C;
    L->ndim = ni.ndim;
    L->N = (int64_t)L->desc.dims[0] * L->desc.dims[1] * L->desc.dims[2];
    L->spin_bytes = d->spin == HMC_I16 ? 2 : 4;
    (void)hipGetDevice(&L->device);
    hmc_status st = HMC_OK;
    hipError_t e;
    if (stream) {
        L->stream = static_cast<hipStream_t>(stream);
    } else {
        e = hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking);
        if (e != hipSuccess) { st = hip_fail(e, "hipStreamCreate"); L->stream = nullptr; }
        L->own_stream = true;
    }
    const size_t sb = (size_t)L->N * L->spin_bytes;
    if (borrowed_spins) {
        L->spins[0] = borrowed_spins;
        L->borrowed = true;
    } else if (st == HMC_OK) {
        st = dev_alloc(&L->spins[0], sb, "spins");
    }
    if (st == HMC_OK) st = dev_alloc(&L->spins[1], sb, "spins (second buffer)");
    if (st == HMC_OK) st = dev_alloc(reinterpret_cast<void**>(&L->dB), (size_t)L->Q * 4, "grain energies");
    if (st == HMC_OK) st = dev_alloc(reinterpret_cast<void**>(&L->d_areas), (size_t)L->Q * 4, "grain areas");
    if (st == HMC_OK) st = dev_alloc(reinterpret_cast<void**>(&L->d_gbin), (size_t)L->Q * 4, "grain bins");
    if (st == HMC_OK) {
        L->stats_bins_cap = 64;
        st = dev_alloc(reinterpret_cast<void**>(&L->d_stats), (size_t)(1 + L->stats_bins_cap) * 8, "stats");
    }
    if (st == HMC_OK) {
        e = L->borrowed ? hipSuccess : hipMemsetAsync(L->spins[0], 0, sb, L->stream);
        if (e == hipSuccess) e = hipMemsetAsync(L->dB, 0, (size_t)L->Q * 4, L->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
        if (e != hipSuccess) st = hip_fail(e, "lattice set-up");
    }
    if (st != HMC_OK) {
        destroy(L);
        return st;
    }
    L->hB.assign((size_t)L->Q, 0);
    L->Bmin = L->Bmax = 0;
    *out = L;
    return HMC_OK;
}

}  // namespace
}  // namespace hmc

using namespace hmc;

extern "C" {

int32_t hmc_abi_version(void) { return 6; }

const char* hmc_last_error(void) { return g_error.c_str(); }

int32_t hmc_device_count(void) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return 0;
    return n;
}

hmc_status hmc_lattice_create(const hmc_lattice_desc* desc, int32_t n_grains, void* stream, hmc_lattice** out) {
    g_error.clear();
    return create(desc, n_grains, stream, out);
}

hmc_status hmc_lattice_init(const hmc_lattice_desc* desc, int32_t n_grains, uint64_t voronoi_seed, void* stream,
                            hmc_lattice** out) {
    g_error.clear();
    hmc_lattice* L = nullptr;
    HMC_TRY(create(desc, n_grains, stream, &L));
    const hmc_status st = launch_voronoi(L, voronoi_seed);
    if (st != HMC_OK) {
        destroy(L);
        *out = nullptr;
        return st;
    }
    *out = L;
    return HMC_OK;
}

hmc_status hmc_lattice_wrap(const hmc_lattice_desc* desc, void* dev_spins, int32_t n_grains, void* stream,
                            hmc_lattice** out) {
    g_error.clear();
    if (!dev_spins) {
        if (out) *out = nullptr;
        return fail(HMC_E_INVAL, "dev_spins is NULL");
    }
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, dev_spins) != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        if (out) *out = nullptr;
        return fail(HMC_E_INVAL, "dev_spins is not device memory");
    }
    if (desc && desc->dims[0] > 0 && desc->dims[1] > 0) {
        // the allocation holding dev_spins must cover the whole lattice
        const uint64_t n = (uint64_t)desc->dims[0] * desc->dims[1] * (desc->ndim == 3 ? (uint64_t)desc->dims[2] : 1u);
        const uint64_t bytes = n * (desc->spin == HMC_I16 ? 2u : 4u);
        const uint64_t align = desc->spin == HMC_I16 ? 2u : 4u;
        hipDeviceptr_t base = nullptr;
        size_t size = 0;
        if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)dev_spins) == hipSuccess) {
            const uint64_t off = (uint64_t)((char*)dev_spins - (char*)base);
            if (off + bytes > size) {
                if (out) *out = nullptr;
                return fail(HMC_E_INVAL, "dev_spins allocation is smaller than the lattice");
            }
        } else {
            (void)hipGetLastError();
        }
        if ((uintptr_t)dev_spins % align) {
            if (out) *out = nullptr;
            return fail(HMC_E_INVAL, "dev_spins is not aligned to the spin size");
        }
    }
    return create(desc, n_grains, stream, out, dev_spins);
}

hmc_status hmc_lattice_free(hmc_lattice* L) {
    g_error.clear();
    destroy(L);
    return HMC_OK;
}

hmc_status hmc_set_grain_energy(hmc_lattice* L, const int32_t* B_fx, int32_t n_grains, int32_t on_device) {
    g_error.clear();
    if (!L || !B_fx) return fail(HMC_E_INVAL, "NULL argument");
    if (n_grains != L->Q)
        return fail(HMC_E_INVAL, "n_grains " + std::to_string(n_grains) + " != lattice Q " + std::to_string(L->Q));
    std::vector<int32_t> h((size_t)n_grains);
    if (on_device) {
        HMC_HIP(hipMemcpyAsync(h.data(), B_fx, (size_t)n_grains * 4, hipMemcpyDeviceToHost, L->stream));
        HMC_HIP(hipStreamSynchronize(L->stream));
    } else {
        std::memcpy(h.data(), B_fx, (size_t)n_grains * 4);
    }
    int32_t lo = h[0], hi = h[0];
    for (int32_t v : h) {
        lo = std::min(lo, v);
        hi = std::max(hi, v);
    }
    HMC_TRY(check_energy_range(L, lo, hi, bond_max(L), L->Fmin, L->Fmax));
    // Staged through pinned memory: the copy runs in stream order after the
    // sweeps already queued (which read the old energies) and the host does
    // not wait for them; only the previous upload from the staging buffer
    // must have finished before it is overwritten.
    if (!L->hB_pinned) {
        void* p = nullptr;
        HMC_HIP(hipHostMalloc(&p, (size_t)L->Q * 4, hipHostMallocDefault));
        L->hB_pinned = static_cast<int32_t*>(p);
        const hipError_t e = hipEventCreateWithFlags(&L->hB_uploaded, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipHostFree(L->hB_pinned);
            L->hB_pinned = nullptr;
            return hip_fail(e, "hipEventCreateWithFlags");
        }
    } else {
        HMC_HIP(hipEventSynchronize(L->hB_uploaded));
    }
    std::memcpy(L->hB_pinned, h.data(), (size_t)n_grains * 4);
    HMC_HIP(hipMemcpyAsync(L->dB, L->hB_pinned, (size_t)n_grains * 4, hipMemcpyHostToDevice, L->stream));
    HMC_HIP(hipEventRecord(L->hB_uploaded, L->stream));
    L->hB.swap(h);
    L->Bmin = lo;
    L->Bmax = hi;
    return HMC_OK;
}

hmc_status hmc_set_pair_energy(hmc_lattice* L, const int32_t* Jp, int32_t n_grains, int32_t on_device) {
    g_error.clear();
    if (!L) return fail(HMC_E_INVAL, "lattice is NULL");
    const size_t QQ = (size_t)L->Q * (size_t)L->Q;
    if (!Jp) {   // back to the uniform J_fx
        dev_free(L->d_Jp, QQ * 4);
        L->d_Jp = nullptr;
        L->pair = false;
        L->Jp_max = 0;
        return HMC_OK;
    }
    if (n_grains != L->Q) return fail(HMC_E_INVAL, "n_grains must equal the lattice's Q");
    if (QQ * 4 > ((size_t)1 << 33)) return fail(HMC_E_INVAL, "pair table larger than 8 GiB");
    std::vector<int32_t> h(QQ);
    if (on_device) {
        HMC_HIP(hipMemcpyAsync(h.data(), Jp, QQ * 4, hipMemcpyDeviceToHost, L->stream));
        HMC_HIP(hipStreamSynchronize(L->stream));
    } else {
        std::memcpy(h.data(), Jp, QQ * 4);
    }
    int32_t jmax = 0;
    const size_t Q = (size_t)L->Q;
    for (size_t a = 0; a < Q; ++a) {
        if (h[a * Q + a] != 0) return fail(HMC_E_INVAL, "pair table diagonal must be zero");
        for (size_t b = a + 1; b < Q; ++b) {
            const int32_t v = h[a * Q + b];
            if (v != h[b * Q + a]) return fail(HMC_E_INVAL, "pair table must be symmetric");
            if (v < 0 || v > (1 << 24)) return fail(HMC_E_INVAL, "pair energies must lie in [0, 2^24]");
            jmax = std::max(jmax, v);
        }
    }
    if (L->field) return fail(HMC_E_INVAL, "pair bond energies and a per-site field are not combined");
    HMC_TRY(check_energy_range(L, L->Bmin, L->Bmax, jmax));
    if (!L->d_Jp) HMC_TRY(dev_alloc(reinterpret_cast<void**>(&L->d_Jp), QQ * 4, "pair energies"));
    HMC_HIP(hipMemcpyAsync(L->d_Jp, h.data(), QQ * 4, hipMemcpyHostToDevice, L->stream));
    HMC_HIP(hipStreamSynchronize(L->stream));
    L->pair = true;
    L->Jp_max = jmax;
    return HMC_OK;
}

hmc_status hmc_set_site_energy(hmc_lattice* L, const int32_t* E_site, uint64_t n_sites, int32_t on_device,
                               int32_t rule) {
    g_error.clear();
    if (!L) return fail(HMC_E_INVAL, "lattice is NULL");
    const size_t bytes = (size_t)L->N * 4;
    if (!E_site) {   // back to grain energies only
        dev_free(L->d_field[0], bytes);
        dev_free(L->d_field[1], bytes);
        dev_free(L->field_snap, bytes);
        L->d_field[0] = L->d_field[1] = L->field_snap = nullptr;
        L->field = false;
        L->Fmin = L->Fmax = 0;
        return HMC_OK;
    }
    if (n_sites != (uint64_t)L->N) return fail(HMC_E_INVAL, "n_sites must equal the lattice's N");
    if (rule != HMC_FIELD_CARRY && rule != HMC_FIELD_RECRYSTALLISE) return fail(HMC_E_INVAL, "unknown field rule");
    if (L->desc.proposal != HMC_PROP_NEIGHBOUR)
        return fail(HMC_E_INVAL, "a per-site field needs neighbour trials (the swept site takes a neighbour's value)");
    if (L->pair) return fail(HMC_E_INVAL, "pair bond energies and a per-site field are not combined");
    std::vector<int32_t> h((size_t)L->N);
    if (on_device) {
        HMC_HIP(hipMemcpyAsync(h.data(), E_site, bytes, hipMemcpyDeviceToHost, L->stream));
        HMC_HIP(hipStreamSynchronize(L->stream));
    } else {
        std::memcpy(h.data(), E_site, bytes);
    }
    int32_t lo = h[0], hi = h[0];
    for (int32_t v : h) {
        lo = std::min(lo, v);
        hi = std::max(hi, v);
    }
    if (lo < -(1 << 24) || hi > (1 << 24)) return fail(HMC_E_INVAL, "field values must lie in [-2^24, 2^24]");
    if (rule == HMC_FIELD_RECRYSTALLISE) {   // swept sites hold zero
        lo = std::min(lo, 0);
        hi = std::max(hi, 0);
    }
    HMC_TRY(check_energy_range(L, L->Bmin, L->Bmax, L->desc.J_fx, lo, hi));
    for (int b = 0; b < 2; ++b)
        if (!L->d_field[b]) HMC_TRY(dev_alloc(reinterpret_cast<void**>(&L->d_field[b]), bytes, "site field"));
    HMC_HIP(hipMemcpyAsync(L->d_field[L->cur], h.data(), bytes, hipMemcpyHostToDevice, L->stream));
    HMC_HIP(hipStreamSynchronize(L->stream));
    L->field = true;
    L->Fmin = lo;
    L->Fmax = hi;
    L->frule = (uint32_t)rule;
    L->Tg_Dmax = -1;   // rebuild the threshold table
    return HMC_OK;
}

hmc_status hmc_get_site_energy(hmc_lattice* L, int32_t* out, uint64_t n_sites) {
    g_error.clear();
    if (!L || !out) return fail(HMC_E_INVAL, "NULL argument");
    if (!L->field) return fail(HMC_E_STATE, "no per-site field set");
    if (n_sites != (uint64_t)L->N) return fail(HMC_E_INVAL, "n_sites must equal the lattice's N");
    HMC_HIP(hipMemcpyAsync(out, L->d_field[L->cur], (size_t)L->N * 4, hipMemcpyDeviceToHost, L->stream));
    HMC_HIP(hipStreamSynchronize(L->stream));
    return HMC_OK;
}

hmc_status hmc_sweep(hmc_lattice* L, float kT, int32_t n_mcs, uint64_t seed) {
    g_error.clear();
    if (!L) return fail(HMC_E_INVAL, "lattice is NULL");
    if (!(kT > 0.0f) || !std::isfinite(kT)) return fail(HMC_E_INVAL, "kT must be positive and finite");
    if (n_mcs < 0) return fail(HMC_E_INVAL, "n_mcs must be >= 0");
    return launch_sweep(L, kT, n_mcs, seed);
}

hmc_status hmc_grain_areas(hmc_lattice* L, int64_t* areas_out) {
    g_error.clear();
    if (!L || !areas_out) return fail(HMC_E_INVAL, "NULL argument");
    HMC_TRY(launch_histogram(L));
    std::vector<uint32_t> a((size_t)L->Q);
    HMC_HIP(hipMemcpyAsync(a.data(), L->d_areas, a.size() * 4, hipMemcpyDeviceToHost, L->stream));
    HMC_HIP(hipStreamSynchronize(L->stream));
    for (size_t q = 0; q < a.size(); ++q) areas_out[q] = (int64_t)a[q];
    return HMC_OK;
}

hmc_status hmc_texture_stats(hmc_lattice* L, const int32_t* grain_bin, int32_t n_bins, int32_t* n_grains_out,
                             double* mean_area_out, double* frac_out) {
    g_error.clear();
    if (!L || !n_grains_out || !mean_area_out) return fail(HMC_E_INVAL, "NULL argument");
    if (n_bins < 0 || n_bins > (1 << 20)) return fail(HMC_E_INVAL, "n_bins must be in [0, 2^20]");
    if (n_bins > 0 && (!grain_bin || !frac_out)) return fail(HMC_E_INVAL, "grain_bin / frac_out is NULL");
    if (grain_bin && n_bins > 0)
        for (int32_t q = 0; q < L->Q; ++q)
            if (grain_bin[q] < -1 || grain_bin[q] >= n_bins)
                return fail(HMC_E_INVAL, "grain_bin[" + std::to_string(q) + "] outside [-1, n_bins)");
    if (n_bins > L->stats_bins_cap) {
        dev_free(L->d_stats, (size_t)(1 + L->stats_bins_cap) * 8);
        L->d_stats = nullptr;
        L->stats_bins_cap = 0;
        HMC_TRY(dev_alloc(reinterpret_cast<void**>(&L->d_stats), (size_t)(1 + n_bins) * 8, "stats"));
        L->stats_bins_cap = n_bins;
    }
    const int32_t* dgb = nullptr;
    if (grain_bin && n_bins > 0) {
        HMC_HIP(hipMemcpyAsync(L->d_gbin, grain_bin, (size_t)L->Q * 4, hipMemcpyHostToDevice, L->stream));
        dgb = L->d_gbin;
    }
    HMC_TRY(launch_histogram(L));
    HMC_TRY(launch_bin_stats(L, dgb, n_bins));
    std::vector<unsigned long long> h((size_t)(1 + n_bins));
    HMC_HIP(hipMemcpyAsync(h.data(), L->d_stats, h.size() * 8, hipMemcpyDeviceToHost, L->stream));
    HMC_HIP(hipStreamSynchronize(L->stream));
    const int64_t ng = (int64_t)h[0];
    *n_grains_out = (int32_t)ng;
    *mean_area_out = ng > 0 ? (double)L->N / (double)ng : 0.0;
    for (int32_t b = 0; b < n_bins; ++b) frac_out[b] = (double)h[1 + b] / (double)L->N;
    return HMC_OK;
}

hmc_status hmc_get_spins(hmc_lattice* L, void* host_dst, uint64_t bytes) {
    g_error.clear();
    if (!L || !host_dst) return fail(HMC_E_INVAL, "NULL argument");
    if (bytes != (uint64_t)L->N * L->spin_bytes) return fail(HMC_E_INVAL, "bytes must equal N * spin size");
    HMC_HIP(hipMemcpyAsync(host_dst, L->spins[L->cur], bytes, hipMemcpyDeviceToHost, L->stream));
    HMC_HIP(hipStreamSynchronize(L->stream));
    return HMC_OK;
}

hmc_status hmc_set_spins(hmc_lattice* L, const void* host_src, uint64_t bytes) {
    g_error.clear();
    if (!L || !host_src) return fail(HMC_E_INVAL, "NULL argument");
    if (bytes != (uint64_t)L->N * L->spin_bytes) return fail(HMC_E_INVAL, "bytes must equal N * spin size");
    for (int64_t i = 0; i < L->N; ++i) {
        const int64_t v = L->spin_bytes == 2 ? (int64_t) static_cast<const int16_t*>(host_src)[i]
                                             : (int64_t) static_cast<const int32_t*>(host_src)[i];
        if (v < 0 || v >= L->Q)
            return fail(HMC_E_INVAL, "spin " + std::to_string(v) + " at site " + std::to_string(i) + " outside [0, Q)");
    }
    HMC_HIP(hipMemcpyAsync(L->spins[L->cur], host_src, bytes, hipMemcpyHostToDevice, L->stream));
    HMC_HIP(hipStreamSynchronize(L->stream));
    return HMC_OK;
}

hmc_status hmc_snapshot(hmc_lattice* L) {
    g_error.clear();
    if (!L) return fail(HMC_E_INVAL, "lattice is NULL");
    const size_t sb = (size_t)L->N * L->spin_bytes;
    if (!L->snap) HMC_TRY(dev_alloc(&L->snap, sb, "snapshot"));
    HMC_HIP(hipMemcpyAsync(L->snap, L->spins[L->cur], sb, hipMemcpyDeviceToDevice, L->stream));
    if (L->field) {
        if (!L->field_snap)
            HMC_TRY(dev_alloc(reinterpret_cast<void**>(&L->field_snap), (size_t)L->N * 4, "field snapshot"));
        HMC_HIP(hipMemcpyAsync(L->field_snap, L->d_field[L->cur], (size_t)L->N * 4, hipMemcpyDeviceToDevice,
                               L->stream));
    }
    L->snap_mcs = L->mcs;
    L->snap_nf_t_now = L->nf_t_now;
    L->snap_nf_t_last = L->nf_t_last;
    L->snap_nf_events = L->nf_events;
    L->has_snap = true;
    return HMC_OK;
}

hmc_status hmc_restore(hmc_lattice* L) {
    g_error.clear();
    if (!L) return fail(HMC_E_INVAL, "lattice is NULL");
    if (!L->has_snap) return fail(HMC_E_STATE, "no snapshot taken");
    const size_t sb = (size_t)L->N * L->spin_bytes;
    HMC_HIP(hipMemcpyAsync(L->spins[L->cur], L->snap, sb, hipMemcpyDeviceToDevice, L->stream));
    if (L->field && L->field_snap)
        HMC_HIP(hipMemcpyAsync(L->d_field[L->cur], L->field_snap, (size_t)L->N * 4, hipMemcpyDeviceToDevice,
                               L->stream));
    L->mcs = L->snap_mcs;
    L->nf_t_now = L->snap_nf_t_now;
    L->nf_t_last = L->snap_nf_t_last;
    L->nf_events = L->snap_nf_events;
    return HMC_OK;
}

hmc_status hmc_get_mcs(const hmc_lattice* L, uint64_t* mcs) {
    g_error.clear();
    if (!L || !mcs) return fail(HMC_E_INVAL, "NULL argument");
    *mcs = L->mcs;
    return HMC_OK;
}

hmc_status hmc_set_mcs(hmc_lattice* L, uint64_t mcs) {
    g_error.clear();
    if (!L) return fail(HMC_E_INVAL, "lattice is NULL");
    L->mcs = mcs;
    return HMC_OK;
}

hmc_status hmc_set_tiling(hmc_lattice* L, int32_t tx, int32_t ty, int32_t tz, int32_t mcs_per_launch) {
    g_error.clear();
    if (!L) return fail(HMC_E_INVAL, "lattice is NULL");
    if (tx < 0 || ty < 0 || tz < 0) return fail(HMC_E_INVAL, "tile sides must be >= 0");
    Tiling t;
    t.tx = tx;
    t.ty = ty;
    t.tz = L->ndim == 3 ? tz : 1;
    t.k = mcs_per_launch;   // < 0: -mcs_per_launch colour passes per launch
    HMC_TRY(choose_tiling(L, t, true));
    L->tiling = t;
    L->tiling_explicit = true;
    return HMC_OK;
}

hmc_status hmc_set_sweep_kernel(hmc_lattice* L, int32_t which) {
    g_error.clear();
    if (!L) return fail(HMC_E_INVAL, "lattice is NULL");
    if (which != HMC_KERNEL_AUTO && which != HMC_KERNEL_GENERIC) return fail(HMC_E_INVAL, "unknown sweep kernel");
    L->sweep_kernel = which;
    return HMC_OK;
}

hmc_status hmc_get_sweep_kernel(const hmc_lattice* L, int32_t* which) {
    g_error.clear();
    if (!L || !which) return fail(HMC_E_INVAL, "NULL argument");
    Tiling t = L->tiling;
    HMC_TRY(choose_tiling(L, t, L->tiling_explicit));
    const void* fn = nullptr;
    size_t bytes = 0;
    int per_cu = 1;
    *which = (compiled_vn6(L, t, &fn, &bytes, &per_cu) || compiled2d(L, t, &fn, &bytes)) ? HMC_KERNEL_COMPILED
                                                                                           : HMC_KERNEL_GENERIC;
    return HMC_OK;
}

hmc_status hmc_get_tiling(const hmc_lattice* L, int32_t* out4) {
    g_error.clear();
    if (!L || !out4) return fail(HMC_E_INVAL, "NULL argument");
    Tiling t = L->tiling;
    HMC_TRY(choose_tiling(L, t, L->tiling_explicit));
    out4[0] = t.tx;
    out4[1] = t.ty;
    out4[2] = t.tz;
    out4[3] = t.k;
    return HMC_OK;
}

hmc_status hmc_profile(hmc_lattice* L, int32_t enable) {
    g_error.clear();
    if (!L) return fail(HMC_E_INVAL, "lattice is NULL");
    if (enable && !L->d_trials) {
        HMC_TRY(dev_alloc(reinterpret_cast<void**>(&L->d_trials), kTrialSlots * sizeof(unsigned long long),
                          "trial counters"));
        HMC_HIP(hipMemsetAsync(L->d_trials, 0, kTrialSlots * sizeof(unsigned long long), L->stream));
    }
    L->profiling = enable != 0;
    return HMC_OK;
}

hmc_status hmc_profile_trials(hmc_lattice* L, int64_t* trials) {
    g_error.clear();
    if (!L || !trials) return fail(HMC_E_INVAL, "NULL argument");
    *trials = 0;
    if (!L->d_trials) return HMC_OK;
    std::vector<unsigned long long> h(kTrialSlots);
    HMC_HIP(hipMemcpyAsync(h.data(), L->d_trials, kTrialSlots * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           L->stream));
    HMC_HIP(hipMemsetAsync(L->d_trials, 0, kTrialSlots * sizeof(unsigned long long), L->stream));
    HMC_HIP(hipStreamSynchronize(L->stream));
    unsigned long long total = 0;
    for (unsigned long long v : h) total += v;
    *trials = (int64_t)total;
    return HMC_OK;
}

hmc_status hmc_boundary_sites(hmc_lattice* L, int64_t* n_out) {
    g_error.clear();
    if (!L || !n_out) return fail(HMC_E_INVAL, "NULL argument");
    if (!L->d_count)
        HMC_TRY(dev_alloc(reinterpret_cast<void**>(&L->d_count), sizeof(unsigned long long), "boundary count"));
    HMC_TRY(launch_boundary_count(L));
    unsigned long long h = 0;
    HMC_HIP(hipMemcpyAsync(&h, L->d_count, sizeof(h), hipMemcpyDeviceToHost, L->stream));
    HMC_HIP(hipStreamSynchronize(L->stream));
    *n_out = (int64_t)h;
    return HMC_OK;
}

hmc_status hmc_profile_read(hmc_lattice* L, double* kernel_ms, int64_t* launches, int64_t* site_updates) {
    g_error.clear();
    if (!L || !kernel_ms || !launches || !site_updates) return fail(HMC_E_INVAL, "NULL argument");
    HMC_HIP(hipStreamSynchronize(L->stream));
    double total = 0.0;
    for (size_t i = 0; i < L->events_used; ++i) {
        float ms = 0.0f;
        HMC_HIP(hipEventElapsedTime(&ms, L->events[i].first, L->events[i].second));
        total += ms;
    }
    *kernel_ms = total;
    *launches = L->prof_launches;
    *site_updates = L->prof_su;
    L->events_used = 0;
    L->prof_launches = 0;
    L->prof_su = 0;
    return HMC_OK;
}

hmc_status hmc_synchronize(hmc_lattice* L) {
    g_error.clear();
    if (!L) return fail(HMC_E_INVAL, "lattice is NULL");
    HMC_HIP(hipStreamSynchronize(L->stream));
    return HMC_OK;
}

hmc_status hmc_threshold_table_host(float kT, int32_t M, int32_t J_fx, int32_t Bmin, int32_t Bmax, int32_t* layout6,
                                    uint32_t* table, uint64_t table_cap, uint32_t* bounds, uint64_t bounds_cap) {
    g_error.clear();
    if (!layout6) return fail(HMC_E_INVAL, "layout is NULL");
    if (!(kT > 0.0f) || !std::isfinite(kT)) return fail(HMC_E_INVAL, "kT must be positive and finite");
    if (M != 4 && M != 6 && M != 8 && M != 26) return fail(HMC_E_INVAL, "M must be 4, 6, 8 or 26");
    if (J_fx < 1 || J_fx > (1 << 24)) return fail(HMC_E_INVAL, "J_fx must be in [1, 2^24]");
    if (Bmin > Bmax) return fail(HMC_E_INVAL, "Bmin > Bmax");
    if ((int64_t)J_fx * M + 2 * std::max(std::llabs((int64_t)Bmin), std::llabs((int64_t)Bmax)) >= (1ll << 31))
        return fail(HMC_E_RANGE, "J_fx * M + 2 max|B| must stay below 2^31");
    TableLayout lay;
    std::vector<uint32_t> host;
    HMC_TRY(table_host(kT, M, J_fx, Bmin, Bmax, lay, host));
    const int32_t v[6] = {lay.dn_lo, lay.rows, lay.R, lay.TW, lay.nb, lay.bw};
    std::memcpy(layout6, v, sizeof v);
    const size_t entries = (size_t)lay.rows * (size_t)lay.TW, nbound = 2 * (size_t)lay.rows * (size_t)lay.nb;
    if (table) {
        if (table_cap < entries) return fail(HMC_E_INVAL, "table buffer smaller than rows * TW");
        std::memcpy(table, host.data(), entries * 4);
    }
    if (bounds) {
        if (bounds_cap < nbound) return fail(HMC_E_INVAL, "bounds buffer smaller than 2 * rows * nb");
        std::memcpy(bounds, host.data() + entries, nbound * 4);
    }
    return HMC_OK;
}

hmc_status hmc_threshold_table(hmc_lattice* L, float kT, int32_t* layout8, uint32_t* table, uint64_t table_cap,
                               uint32_t* bounds, uint64_t bounds_cap) {
    g_error.clear();
    if (!L || !layout8) return fail(HMC_E_INVAL, "NULL argument");
    if (!(kT > 0.0f) || !std::isfinite(kT)) return fail(HMC_E_INVAL, "kT must be positive and finite");
    if (L->pair || L->field) {
        HMC_TRY(build_direct_table(L, kT));
        const int32_t v[8] = {1, 0, 1, 0, L->Tg_Dmax + 1, 0, 0, L->Tg_Dmax};
        std::memcpy(layout8, v, sizeof v);
        const size_t entries = (size_t)L->Tg_Dmax + 1;
        if (table) {
            if (table_cap < entries) return fail(HMC_E_INVAL, "table buffer smaller than Dmax + 1");
            HMC_HIP(hipMemcpyAsync(table, L->d_Tg, entries * 4, hipMemcpyDeviceToHost, L->stream));
        }
        HMC_HIP(hipStreamSynchronize(L->stream));
        return HMC_OK;
    }
    HMC_TRY(build_table(L->table, kT, L->M, L->desc.J_fx, L->Bmin, L->Bmax, L->stream));
    const Table& t = L->table;
    const int32_t v[8] = {0, t.dn_lo, t.rows, t.R, t.TW, t.nb, t.bw, -1};
    std::memcpy(layout8, v, sizeof v);
    const size_t entries = (size_t)t.rows * (size_t)t.TW, nbound = 2 * (size_t)t.rows * (size_t)t.nb;
    if (table) {
        if (table_cap < entries) return fail(HMC_E_INVAL, "table buffer smaller than rows * TW");
        HMC_HIP(hipMemcpyAsync(table, t.dev, entries * 4, hipMemcpyDeviceToHost, L->stream));
    }
    if (bounds) {
        if (bounds_cap < nbound) return fail(HMC_E_INVAL, "bounds buffer smaller than 2 * rows * nb");
        HMC_HIP(hipMemcpyAsync(bounds, t.bounds, nbound * 4, hipMemcpyDeviceToHost, L->stream));
    }
    HMC_HIP(hipStreamSynchronize(L->stream));
    return HMC_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ ensembles

extern "C" {

hmc_status hmc_ensemble_create(hmc_lattice* const* lats, int32_t n, hmc_ensemble** out) {
    g_error.clear();
    if (!out) return fail(HMC_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!lats || n < 1) return fail(HMC_E_INVAL, "need at least one lattice");
    for (int32_t i = 0; i < n; ++i) {
        if (!lats[i]) return fail(HMC_E_INVAL, "lattice " + std::to_string(i) + " is NULL");
        const hmc_lattice* a = lats[i];
        const hmc_lattice* b = lats[0];
        if (a->desc.nbr != b->desc.nbr || a->desc.spin != b->desc.spin || a->desc.proposal != b->desc.proposal)
            return fail(HMC_E_INVAL, "ensemble members must share neighbourhood, spin type and trial mode");
        for (int32_t j = 0; j < i; ++j)
            if (lats[j] == lats[i]) return fail(HMC_E_INVAL, "lattice " + std::to_string(i) + " appears twice");
        if (lats[i]->pair || lats[i]->field)
            return fail(HMC_E_INVAL, "ensembles take lattices with uniform bonds and grain energies only");
    }
    hmc_ensemble* E = new hmc_ensemble();
    E->lats.assign(lats, lats + n);
    hipError_t e = hipStreamCreateWithFlags(&E->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&E->ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (E->stream) (void)hipStreamDestroy(E->stream);
        delete E;
        return hip_fail(e, "ensemble stream");
    }
    *out = E;
    return HMC_OK;
}

hmc_status hmc_ensemble_set_tiling(hmc_ensemble* E, int32_t tx, int32_t ty, int32_t tz, int32_t mcs_per_launch) {
    g_error.clear();
    if (!E) return fail(HMC_E_INVAL, "ensemble is NULL");
    if (tx < 0 || ty < 0 || tz < 0 || mcs_per_launch < 0) return fail(HMC_E_INVAL, "tiling values must be >= 0");
    Tiling t;
    t.tx = tx;
    t.ty = ty;
    t.tz = E->lats[0]->ndim == 3 ? tz : 1;
    t.k = mcs_per_launch;
    const Tiling old = E->tiling;
    E->tiling = t;
    E->prepared = false;
    const hmc_status st = ensemble_prepare(E);
    if (st != HMC_OK) {
        E->tiling = old;
        E->prepared = false;
        return st;
    }
    return HMC_OK;
}

hmc_status hmc_ensemble_get_tiling(hmc_ensemble* E, int32_t* out4) {
    g_error.clear();
    if (!E || !out4) return fail(HMC_E_INVAL, "NULL argument");
    if (!E->prepared) HMC_TRY(ensemble_prepare(E));
    out4[0] = E->tiling.tx;
    out4[1] = E->tiling.ty;
    out4[2] = E->tiling.tz;
    out4[3] = E->tiling.k;
    return HMC_OK;
}

hmc_status hmc_nfold_batch(hmc_lattice* const* lats, int32_t n, const float* kT, double mcs, const uint64_t* seed) {
    g_error.clear();
    if (!lats || !kT || !seed) return fail(HMC_E_INVAL, "NULL argument");
    if (n < 1) return fail(HMC_E_INVAL, "n must be >= 1");
    if (!(mcs >= 0.0) || !std::isfinite(mcs)) return fail(HMC_E_INVAL, "mcs must be finite and >= 0");
    const hmc_lattice* L0 = lats[0];
    if (!L0) return fail(HMC_E_INVAL, "lattice 0 is NULL");
    const int limit = lds_limit_bytes();
    for (int32_t b = 0; b < n; ++b) {
        const hmc_lattice* L = lats[b];
        const std::string who = "lattice " + std::to_string(b);
        if (!L) return fail(HMC_E_INVAL, who + " is NULL");
        for (int32_t c = 0; c < b; ++c)
            if (lats[c] == L) return fail(HMC_E_INVAL, who + " appears twice in the batch");
        if (L->device != L0->device) return fail(HMC_E_INVAL, who + " is on another device");
        if (L->desc.nbr != L0->desc.nbr || L->desc.spin != L0->desc.spin || L->desc.proposal != L0->desc.proposal ||
            L->pair != L0->pair)
            return fail(HMC_E_INVAL, who + ": a batch shares neighbourhood, spin type, trial mode and bond model");
        if (L->field) return fail(HMC_E_STATE, who + ": the n-fold way takes per-grain bulk energies only");
        if (L->desc.proposal == HMC_PROP_UNIFORM && (L->pair || L->Q > 65))
            return fail(HMC_E_INVAL, who + ": the symmetric trial mode of the n-fold way needs uniform bonds and Q <= 65");
        if (!(kT[b] > 0.0f) || !std::isfinite(kT[b]))
            return fail(HMC_E_INVAL, "kT[" + std::to_string(b) + "] must be positive and finite");
        if (!std::isfinite(L->nf_t_now + mcs)) return fail(HMC_E_INVAL, who + ": clock would overflow");
        const size_t need = nfold_lds_bytes(L->N, L->spin_bytes, L->Q);
        if (need > (size_t)limit)
            return fail(HMC_E_RANGE, who + ": the n-fold way keeps a lattice and its grain energies in LDS; " +
                                         std::to_string(L->N) + " sites and " + std::to_string(L->Q) +
                                         " grains need " + std::to_string(need) + " bytes, the device has " +
                                         std::to_string(limit));
        // coordinates by multiply-high are exact while j * Lx and j * Ly stay below 2^32
        if ((uint64_t)L->N * (uint64_t)L->desc.dims[0] >= (1ull << 32) ||
            (uint64_t)L->N * (uint64_t)L->desc.dims[1] >= (1ull << 32))
            return fail(HMC_E_RANGE, who + ": lattice too large for the n-fold way");
    }
    return launch_nfold(lats, n, kT, mcs, seed);
}

hmc_status hmc_nfold(hmc_lattice* L, float kT, double mcs, uint64_t seed) {
    return hmc_nfold_batch(&L, 1, &kT, mcs, &seed);
}

hmc_status hmc_nfold_exponentials(uint64_t seed, uint64_t n0, int64_t count, int32_t window, uint64_t* out) {
    g_error.clear();
    return nfold_exponentials(seed, n0, count, window, out);
}

hmc_status hmc_nfold_clock(const hmc_lattice* L, double* t_now, double* t_last, uint64_t* n_events) {
    g_error.clear();
    if (!L || !t_now || !t_last || !n_events) return fail(HMC_E_INVAL, "NULL argument");
    *t_now = L->nf_t_now;
    *t_last = L->nf_t_last;
    *n_events = L->nf_events;
    return HMC_OK;
}

hmc_status hmc_nfold_set_clock(hmc_lattice* L, double t_now, double t_last, uint64_t n_events) {
    g_error.clear();
    if (!L) return fail(HMC_E_INVAL, "lattice is NULL");
    if (!std::isfinite(t_now) || !std::isfinite(t_last) || t_last > t_now)
        return fail(HMC_E_INVAL, "the clock needs finite times with t_last <= t_now");
    L->nf_t_now = t_now;
    L->nf_t_last = t_last;
    L->nf_events = n_events;
    return HMC_OK;
}

hmc_status hmc_ensemble_sweep(hmc_ensemble* E, const float* kT, const uint64_t* seed, int32_t n_mcs) {
    g_error.clear();
    if (!E || !kT || !seed) return fail(HMC_E_INVAL, "NULL argument");
    if (n_mcs < 0) return fail(HMC_E_INVAL, "n_mcs must be >= 0");
    for (size_t i = 0; i < E->lats.size(); ++i)
        if (!(kT[i] > 0.0f) || !std::isfinite(kT[i]))
            return fail(HMC_E_INVAL, "kT[" + std::to_string(i) + "] must be positive and finite");
    return launch_ensemble(E, kT, seed, n_mcs);
}

hmc_status hmc_ensemble_synchronize(hmc_ensemble* E) {
    g_error.clear();
    if (!E) return fail(HMC_E_INVAL, "ensemble is NULL");
    HMC_HIP(hipStreamSynchronize(E->stream));
    return HMC_OK;
}

hmc_status hmc_ensemble_profile(hmc_ensemble* E, int32_t enable) {
    g_error.clear();
    if (!E) return fail(HMC_E_INVAL, "ensemble is NULL");
    E->profiling = enable != 0;
    return HMC_OK;
}

hmc_status hmc_ensemble_profile_read(hmc_ensemble* E, double* kernel_ms, int64_t* launches, int64_t* site_updates) {
    g_error.clear();
    if (!E || !kernel_ms || !launches || !site_updates) return fail(HMC_E_INVAL, "NULL argument");
    HMC_HIP(hipStreamSynchronize(E->stream));
    double total = 0.0;
    for (size_t i = 0; i < E->events_used; ++i) {
        float ms = 0.0f;
        HMC_HIP(hipEventElapsedTime(&ms, E->events[i].first, E->events[i].second));
        total += ms;
    }
    *kernel_ms = total;
    *launches = E->prof_launches;
    *site_updates = E->prof_su;
    E->events_used = 0;
    E->prof_launches = 0;
    E->prof_su = 0;
    return HMC_OK;
}

hmc_status hmc_ensemble_free(hmc_ensemble* E) {
    g_error.clear();
    if (!E) return HMC_OK;
    (void)hipStreamSynchronize(E->stream);
    for (auto& e : E->events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    for (auto& kv : E->graphs) (void)hipGraphExecDestroy(kv.second);
    dev_free(E->d_tiles, E->tiles_bytes);
    dev_free(E->d_lats, E->lats_bytes);
    for (int i = 0; i < 2; ++i) {
        if (E->h_stage[i]) (void)hipHostFree(E->h_stage[i]);
        if (E->stage_ev[i]) (void)hipEventDestroy(E->stage_ev[i]);
    }
    (void)hipEventDestroy(E->ev);
    (void)hipStreamDestroy(E->stream);
    delete E;
    return HMC_OK;
}

}  // extern "C"
