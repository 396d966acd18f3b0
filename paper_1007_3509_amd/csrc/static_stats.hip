// static_stats.hip -- grain statistics of a caller's device buffer without
// any allocation.
//
// The same counts as hmc_texture_stats (per-spin areas, present-grain count,
// per-bin areas; the orientation-class area fractions the paper follows over
// time, Sec. 5), for callers that may not allocate device memory (code
// under graph capture, tight serving loops).  The per-grain areas, the
// grain-to-bin map and the bin sums live in one file-scope device array,
// `scratch`, of fixed size; each device holds its own copy until the
// process ends, and host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.  Calls on one device
// share that array: calls that overlap in time on one device race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace hmc {
namespace {
constexpr int32_t kStaticMaxGrains = HMC_STATIC_MAX_GRAINS;
constexpr int32_t kStaticMaxBins = HMC_STATIC_MAX_BINS;
// [bin sums uint64[1 + max bins], padded | areas uint32[max grains] | bins int32[max grains]]
constexpr size_t kStatsOff = 0;
constexpr size_t kAreasOff = ((size_t)(1 + kStaticMaxBins) * 8 + 255) / 256 * 256;
constexpr size_t kBinsOff = kAreasOff + (size_t)kStaticMaxGrains * 4;
constexpr size_t kScratchBytes = kBinsOff + (size_t)kStaticMaxGrains * 4;
}  // namespace
}  // namespace hmc

// The working memory (about 0.5 MiB per device).  Host code never uses this
// name as an address: on the host it is only a handle for
// hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[hmc::kScratchBytes];

namespace hmc {
namespace {

std::mutex g_scratch_mu;
std::vector<unsigned char*> g_scratch_addr;   // per device; null until first use

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
hmc_status scratch_address(unsigned char** out) {
    int dev = 0;
    HMC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((size_t)dev >= g_scratch_addr.size()) g_scratch_addr.resize((size_t)dev + 1, nullptr);
    if (!g_scratch_addr[(size_t)dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
        g_scratch_addr[(size_t)dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch_addr[(size_t)dev];
    return HMC_OK;
}

}  // namespace
}  // namespace hmc

using namespace hmc;

extern "C" hmc_status hmc_texture_stats_static(const void* dev_spins, int32_t spin, uint64_t n_sites,
                                               int32_t n_grains, const int32_t* grain_bin, int32_t n_bins,
                                               void* stream, int32_t* n_grains_out, double* mean_area_out,
                                               double* frac_out) {
    set_error("");
    // host-side validation, before any device work
    if (!dev_spins || !n_grains_out || !mean_area_out) return fail(HMC_E_INVAL, "NULL argument");
    if (spin != HMC_I16 && spin != HMC_I32) return fail(HMC_E_INVAL, "spin type must be HMC_I16 or HMC_I32");
    if (n_sites == 0 || n_sites >= (1ull << 32)) return fail(HMC_E_INVAL, "n_sites must be in [1, 2^32)");
    if (n_grains < 1 || n_grains > kStaticMaxGrains)
        return fail(HMC_E_INVAL, "n_grains must be in [1, " + std::to_string(kStaticMaxGrains) +
                                     "] (the fixed scratch of the allocation-free statistics)");
    if (n_bins < 0 || n_bins > kStaticMaxBins)
        return fail(HMC_E_INVAL, "n_bins must be in [0, " + std::to_string(kStaticMaxBins) +
                                     "] (the fixed scratch of the allocation-free statistics)");
    if (n_bins > 0 && (!grain_bin || !frac_out)) return fail(HMC_E_INVAL, "grain_bin / frac_out is NULL");
    if (n_bins > 0)
        for (int32_t q = 0; q < n_grains; ++q)
            if (grain_bin[q] < -1 || grain_bin[q] >= n_bins)
                return fail(HMC_E_INVAL, "grain_bin[" + std::to_string(q) + "] outside [-1, n_bins)");
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, dev_spins) != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return fail(HMC_E_INVAL, "dev_spins is not device memory");
    }
    if ((uintptr_t)dev_spins % (spin == HMC_I16 ? 2u : 4u))
        return fail(HMC_E_INVAL, "dev_spins is not aligned to the spin size");

    unsigned char* base = nullptr;
    HMC_TRY(scratch_address(&base));
    auto* d_stats = reinterpret_cast<unsigned long long*>(base + kStatsOff);
    auto* d_areas = reinterpret_cast<uint32_t*>(base + kAreasOff);
    auto* d_bins = reinterpret_cast<int32_t*>(base + kBinsOff);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (n_bins > 0)
        HMC_HIP(hipMemcpyAsync(d_bins, grain_bin, (size_t)n_grains * 4, hipMemcpyHostToDevice, s));
    HMC_TRY(launch_areas(dev_spins, spin == HMC_I16, n_sites, (uint32_t)n_grains, d_areas, s));
    HMC_TRY(launch_bins(d_areas, n_grains, n_bins > 0 ? d_bins : nullptr, n_bins, d_stats, s));
    unsigned long long h[1 + kStaticMaxBins];
    HMC_HIP(hipMemcpyAsync(h, d_stats, (size_t)(1 + n_bins) * 8, hipMemcpyDeviceToHost, s));
    HMC_HIP(hipStreamSynchronize(s));
    const int64_t ng = (int64_t)h[0];
    *n_grains_out = (int32_t)ng;
    *mean_area_out = ng > 0 ? (double)n_sites / (double)ng : 0.0;
    for (int32_t b = 0; b < n_bins; ++b) frac_out[b] = (double)h[1 + b] / (double)n_sites;
    return HMC_OK;
}
