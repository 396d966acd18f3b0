// init_stats.hip -- initial microstructure and grain statistics.
//
// Voronoi labelling: the paper does not state its initial polycrystal; the
// library uses a seeded Voronoi tessellation (point g from Philox with
// counter (g, 0, 0, 0x564F524E), fixed-point coordinates in 1/256 site,
// periodic squared distance in integers, ties to the lower index).  Points
// are generated on the host and staged through LDS; each thread labels one
// site by exact brute force.
//
// Grain statistics: the orientation distribution the paper follows over time
// (Sec. 5) is the area fraction of grains grouped by orientation class.
// A histogram kernel counts sites per spin value with run-length
// aggregation inside each wavefront (neighbouring sites of a row mostly share
// a grain, so one atomic per run instead of one per site); a second kernel
// reduces per-grain areas into the present-grain count (wavefront ballot +
// popcount) and per-bin areas (LDS-privatised bins).
#include <hip/hip_runtime.h>

#include <vector>

#include "common.hpp"

namespace hmc {

namespace {

constexpr int kVorThreads = 256;

// Nearest seed point of every site by expanding rings of a uniform cell grid.
// The grid has nc_k cells along axis k; a coordinate X (fixed point, 256 per
// site) lies in cell floor(X nc_k / (256 L_k)), so every cell is at least
// w_k = floor(256 L_k / nc_k) wide.  After the rings 0..r around the site's
// cell are searched, any point not yet seen lies at least r cells away along
// some axis, hence at periodic distance >= r w_min; the search stops once the
// best squared distance is below (r w_min)^2, which also settles ties (an
// unseen point cannot be as close).  Ties between seen points go to the lower
// index, as in a scan in index order.
template <typename Dist, typename Spin, int D>
__global__ void __launch_bounds__(kVorThreads)
voronoi_kernel(Spin* __restrict__ out, const int4* __restrict__ pts, const int32_t* __restrict__ cell_start, int ncx,
               int ncy, int ncz, uint32_t wmin, uint32_t Lx, uint32_t Ly, uint32_t Lz, uint64_t N) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint32_t x = (uint32_t)(i % Lx), y = (uint32_t)((i / Lx) % Ly), z = (uint32_t)(i / ((uint64_t)Lx * Ly));
    const int32_t px = (int32_t)(256u * x), py = (int32_t)(256u * y), pz = (int32_t)(256u * z);
    const int32_t spx = (int32_t)(256u * Lx), spy = (int32_t)(256u * Ly), spz = (int32_t)(256u * Lz);
    const int cx = (int)((uint64_t)x * (uint64_t)ncx / Lx), cy = (int)((uint64_t)y * (uint64_t)ncy / Ly);
    const int cz = D == 3 ? (int)((uint64_t)z * (uint64_t)ncz / Lz) : 0;
    Dist best = ~(Dist)0;
    int32_t bg = 0x7FFFFFFF;
    auto scan_cell = [&](int ax, int ay, int az) __attribute__((always_inline)) {
        const int cell = ax + ncx * (ay + ncy * az);
        const int p1 = cell_start[cell + 1];
        for (int p = cell_start[cell]; p < p1; ++p) {
            const int4 q = pts[p];
            int32_t dx = q.x - px;
            dx = dx < 0 ? -dx : dx;
            dx = min(dx, spx - dx);
            int32_t dy = q.y - py;
            dy = dy < 0 ? -dy : dy;
            dy = min(dy, spy - dy);
            Dist d2 = (Dist)dx * (Dist)dx + (Dist)dy * (Dist)dy;
            if (D == 3) {
                int32_t dz = q.z - pz;
                dz = dz < 0 ? -dz : dz;
                dz = min(dz, spz - dz);
                d2 += (Dist)dz * (Dist)dz;
            }
            if (d2 < best || (d2 == best && q.w < bg)) {
                best = d2;
                bg = q.w;
            }
        }
    };
    auto wrap = [](int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); };
    for (int r = 0;; ++r) {
        // offsets along each axis, each cyclic cell at most once
        const int lox = -min(r, (ncx - 1) / 2), hix = min(r, ncx / 2);
        const int loy = -min(r, (ncy - 1) / 2), hiy = min(r, ncy / 2);
        const int loz = D == 3 ? -min(r, (ncz - 1) / 2) : 0, hiz = D == 3 ? min(r, ncz / 2) : 0;
        bool any = false;
        for (int dz = loz; dz <= hiz; ++dz) {
            const int az = wrap(cz + dz, ncz);
            for (int dy = loy; dy <= hiy; ++dy) {
                const int ay = wrap(cy + dy, ncy);
                const bool shell_yz = max(abs(dy), abs(dz)) == r;
                if (shell_yz) {
                    for (int dx = lox; dx <= hix; ++dx) scan_cell(wrap(cx + dx, ncx), ay, az);
                    any = true;
                } else {   // only the two x ends of this row belong to ring r
                    if (lox == -r) { scan_cell(wrap(cx - r, ncx), ay, az); any = true; }
                    if (hix == r && r > 0) { scan_cell(wrap(cx + r, ncx), ay, az); any = true; }
                }
            }
        }
        if (!any) break;   // every cell has been searched
        const uint64_t reach = (uint64_t)r * wmin;
        if ((uint64_t)best < reach * reach) break;
    }
    out[i] = (Spin)bg;
}

constexpr int kHistThreads = 256;

template <typename Spin>
__global__ void __launch_bounds__(kHistThreads)
histogram_kernel(const Spin* __restrict__ s, uint64_t N, uint32_t Q, uint32_t* __restrict__ areas) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // uniform trip count per wave so that the wave-level votes see all lanes
    const uint64_t wave_base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u);
    for (uint64_t b = wave_base; b < N; b += stride) {
        const uint64_t i = b + lane;
        const bool ok = i < N;
        const int32_t q = ok ? (int32_t)s[i] : -1;
        const int32_t prev = __shfl_up(q, 1);
        const bool head = ok && (lane == 0 || prev != q);
        const uint64_t heads = __ballot(head);
        const uint64_t valid = __ballot(ok);
        if (head && (uint32_t)q < Q) {   // values outside [0, Q) are not counted
            // run ends at the next head or at the last valid lane
            const uint64_t later = heads & ~((2ull << lane) - 1ull);
            const uint32_t end = later ? (uint32_t)__ffsll((long long)later) - 1u
                                       : 64u - (uint32_t)__clzll((long long)valid);
            atomicAdd(&areas[q], end - lane);
        }
    }
}

// Sites (with a spin in [0, Q)) that have at least one neighbour holding
// another value: the grain-boundary sites, the only ones whose trial can
// change anything (Sec. 3).
template <int NBR, typename Spin>
__global__ void __launch_bounds__(kHistThreads)
boundary_kernel(const Spin* __restrict__ s, uint32_t Lx, uint32_t Ly, uint32_t Lz, uint32_t Q,
                unsigned long long* __restrict__ count) {
    constexpr int M = NBR == HMC_VN4 ? 4 : NBR == HMC_MOORE8 ? 8 : NBR == HMC_VN6 ? 6 : 26;
    const uint64_t N = (uint64_t)Lx * Ly * Lz;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t wave_base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u);
    for (uint64_t b = wave_base; b < N; b += stride) {
        const uint64_t i = b + (threadIdx.x & 63u);
        bool hit = false;
        if (i < N) {
            // 32-bit coordinates: a lattice has fewer than 2^32 sites
            const uint32_t ii = (uint32_t)i, yz = ii / Lx;
            const uint32_t x = ii - yz * Lx, z = yz / Ly, y = yz - z * Ly;
            const int32_t q = (int32_t)s[ii];
            // one step along an axis, periodic
            auto step = [](uint32_t c, int d, uint32_t L) -> uint32_t {
                return d > 0 ? (c + 1 == L ? 0u : c + 1) : (d < 0 ? (c == 0 ? L - 1 : c - 1) : c);
            };
            if ((uint32_t)q < Q) {
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    const uint32_t xn = step(x, nbr_dx(NBR, k), Lx);
                    const uint32_t yn = step(y, nbr_dy(NBR, k), Ly);
                    const uint32_t zn = step(z, nbr_dz(NBR, k), Lz);
                    hit |= (int32_t)s[xn + Lx * (yn + Ly * zn)] != q;
                }
            }
        }
        const uint64_t mask = __ballot(hit);
        if ((threadIdx.x & 63u) == 0 && mask) atomicAdd(count, (unsigned long long)__popcll(mask));
    }
}

constexpr int kBinThreads = 256;
constexpr int kMaxLdsBins = 4096;

__global__ void __launch_bounds__(kBinThreads)
bin_stats_kernel(const uint32_t* __restrict__ areas, int32_t Q, const int32_t* __restrict__ gbin, int32_t n_bins,
                 unsigned long long* __restrict__ out /* 1 + n_bins */) {
    __shared__ unsigned long long bins[kMaxLdsBins];
    const bool lds_bins = n_bins <= kMaxLdsBins;
    if (lds_bins)
        for (int b = threadIdx.x; b < n_bins; b += blockDim.x) bins[b] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t wave_base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
    const uint32_t lane = threadIdx.x & 63u;
    for (int64_t b0 = wave_base; b0 < Q; b0 += stride) {
        const int64_t q = b0 + lane;
        const uint32_t a = q < Q ? areas[q] : 0u;
        const uint64_t present = __ballot(a > 0);
        if (lane == 0 && present) atomicAdd(&out[0], (unsigned long long)__popcll(present));
        if (a > 0 && gbin != nullptr) {
            const int32_t bin = gbin[q];
            if (bin >= 0 && bin < n_bins) {
                if (lds_bins) atomicAdd(&bins[bin], (unsigned long long)a);
                else atomicAdd(&out[1 + bin], (unsigned long long)a);
            }
        }
    }
    __syncthreads();
    if (lds_bins)
        for (int b = threadIdx.x; b < n_bins; b += blockDim.x)
            if (bins[b]) atomicAdd(&out[1 + b], bins[b]);
}

// Zero n 32-bit words (a kernel rather than a memset node, so that the
// statistics stay correct inside a caller's captured graph).
__global__ void __launch_bounds__(256) clear_kernel(uint32_t* __restrict__ p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

int grid_for(uint64_t n, int threads, int cap) {
    uint64_t g = (n + threads - 1) / threads;
    if (g > (uint64_t)cap) g = cap;
    return g < 1 ? 1 : (int)g;
}

}  // namespace

hmc_status launch_voronoi(hmc_lattice* L, uint64_t vseed) {
    const int32_t G = L->Q;
    const int ndim = L->ndim;
    const uint32_t Lx = (uint32_t)L->desc.dims[0], Ly = (uint32_t)L->desc.dims[1];
    const uint32_t Lz = ndim == 3 ? (uint32_t)L->desc.dims[2] : 1u;
    const uint32_t Ls[3] = {Lx, Ly, Lz};
    const uint64_t N = (uint64_t)L->N;
    // seed points (fixed point, 256 per site) from Philox
    std::vector<int32_t> pts((size_t)G * 3, 0);
    const uint32_t k0 = (uint32_t)(vseed & 0xFFFFFFFFu), k1 = (uint32_t)(vseed >> 32);
    for (int32_t g = 0; g < G; ++g) {
        uint32_t r[4];
        philox4x32_10((uint32_t)g, 0u, 0u, 0x564F524Eu, k0, k1, r);
        for (int a = 0; a < ndim; ++a)
            pts[(size_t)g * 3 + a] = (int32_t)(((uint64_t)r[a] * ((uint64_t)Ls[a] * 256u)) >> 32);
    }
    // cell grid with about two points per cell
    int nc[3] = {1, 1, 1};
    const double per_axis = std::pow((double)G / (2.0 * (double)N), 1.0 / ndim);
    uint32_t wmin = 0xFFFFFFFFu;
    for (int a = 0; a < ndim; ++a) {
        nc[a] = (int)std::max(1.0, std::min((double)Ls[a], std::floor(Ls[a] * per_axis)));
        wmin = std::min(wmin, (uint32_t)((256ull * Ls[a]) / (uint64_t)nc[a]));
    }
    const size_t ncells = (size_t)nc[0] * nc[1] * nc[2];
    std::vector<int32_t> cell_of((size_t)G), start(ncells + 1, 0);
    for (int32_t g = 0; g < G; ++g) {
        size_t c = 0, mul = 1;
        for (int a = 0; a < ndim; ++a) {
            const uint64_t ca = (uint64_t)pts[(size_t)g * 3 + a] * (uint64_t)nc[a] / (256ull * Ls[a]);
            c += (size_t)ca * mul;
            mul *= (size_t)nc[a];
        }
        cell_of[g] = (int32_t)c;
        ++start[c + 1];
    }
    for (size_t c = 0; c < ncells; ++c) start[c + 1] += start[c];
    std::vector<int4> sorted((size_t)G);
    {
        std::vector<int32_t> fill(start.begin(), start.end() - 1);
        for (int32_t g = 0; g < G; ++g) {
            const size_t at = (size_t)fill[cell_of[g]]++;
            sorted[at] = make_int4(pts[(size_t)g * 3], pts[(size_t)g * 3 + 1], pts[(size_t)g * 3 + 2], g);
        }
    }
    void *dpts = nullptr, *dstart = nullptr;
    const size_t bp = sorted.size() * sizeof(int4), bs = start.size() * sizeof(int32_t);
    HMC_TRY(dev_alloc(&dpts, bp, "voronoi points"));
    hmc_status st = dev_alloc(&dstart, bs, "voronoi cells");
    if (st != HMC_OK) {
        dev_free(dpts, bp);
        return st;
    }
    hipError_t e = hipMemcpyAsync(dpts, sorted.data(), bp, hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dstart, start.data(), bs, hipMemcpyHostToDevice, L->stream);
    // 32-bit distances suffice while ndim * (128 * L_max)^2 < 2^32
    const uint64_t half = 128ull * std::max(Lx, std::max(Ly, Lz));
    const bool d32 = (uint64_t)ndim * half * half < (1ull << 32);
    const dim3 grid((unsigned)((N + kVorThreads - 1) / kVorThreads));
    const int4* P = static_cast<const int4*>(dpts);
    const int32_t* S = static_cast<const int32_t*>(dstart);
    if (e == hipSuccess) {
        void* out = L->spins[L->cur];
#define HMC_VORONOI(DIST, SPIN, DIM)                                                                               \
    voronoi_kernel<DIST, SPIN, DIM><<<grid, kVorThreads, 0, L->stream>>>((SPIN*)out, P, S, nc[0], nc[1], nc[2], wmin, \
                                                                         Lx, Ly, Lz, N)
        if (L->desc.spin == HMC_I16) {
            if (ndim == 2) {
                if (d32) HMC_VORONOI(uint32_t, int16_t, 2); else HMC_VORONOI(uint64_t, int16_t, 2);
            } else {
                if (d32) HMC_VORONOI(uint32_t, int16_t, 3); else HMC_VORONOI(uint64_t, int16_t, 3);
            }
        } else {
            if (ndim == 2) {
                if (d32) HMC_VORONOI(uint32_t, int32_t, 2); else HMC_VORONOI(uint64_t, int32_t, 2);
            } else {
                if (d32) HMC_VORONOI(uint32_t, int32_t, 3); else HMC_VORONOI(uint64_t, int32_t, 3);
            }
        }
#undef HMC_VORONOI
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    dev_free(dpts, bp);
    dev_free(dstart, bs);
    if (e != hipSuccess) return hip_fail(e, "voronoi");
    return HMC_OK;
}

hmc_status launch_areas(const void* spins, bool i16, uint64_t N, uint32_t Q, uint32_t* d_areas, hipStream_t stream) {
    clear_kernel<<<grid_for(Q, 256, 256), 256, 0, stream>>>(d_areas, Q);
    const int grid = grid_for(N, kHistThreads, 4096);
    if (i16)
        histogram_kernel<int16_t><<<grid, kHistThreads, 0, stream>>>((const int16_t*)spins, N, Q, d_areas);
    else
        histogram_kernel<int32_t><<<grid, kHistThreads, 0, stream>>>((const int32_t*)spins, N, Q, d_areas);
    HMC_HIP(hipGetLastError());
    return HMC_OK;
}

hmc_status launch_bins(const uint32_t* d_areas, int32_t Q, const int32_t* d_gbin, int32_t n_bins,
                       unsigned long long* d_stats, hipStream_t stream) {
    const uint64_t words = (uint64_t)(1 + n_bins) * 2;
    clear_kernel<<<grid_for(words, 256, 64), 256, 0, stream>>>(reinterpret_cast<uint32_t*>(d_stats), words);
    const int grid = grid_for((uint64_t)Q, kBinThreads, 1024);
    bin_stats_kernel<<<grid, kBinThreads, 0, stream>>>(d_areas, Q, d_gbin, n_bins, d_stats);
    HMC_HIP(hipGetLastError());
    return HMC_OK;
}

hmc_status launch_histogram(hmc_lattice* L) {
    return launch_areas(L->spins[L->cur], L->desc.spin == HMC_I16, (uint64_t)L->N, (uint32_t)L->Q, L->d_areas,
                        L->stream);
}

hmc_status launch_boundary_count(hmc_lattice* L) {
    HMC_HIP(hipMemsetAsync(L->d_count, 0, sizeof(unsigned long long), L->stream));
    const uint32_t Lx = (uint32_t)L->desc.dims[0], Ly = (uint32_t)L->desc.dims[1];
    const uint32_t Lz = L->ndim == 3 ? (uint32_t)L->desc.dims[2] : 1u;
    const int grid = grid_for((uint64_t)L->N, kHistThreads, 4096);
    const void* sp = L->spins[L->cur];
    const uint32_t Q = (uint32_t)L->Q;
    const bool i16 = L->desc.spin == HMC_I16;
#define HMC_BOUNDARY(NB)                                                                                         \
    if (i16)                                                                                                     \
        boundary_kernel<NB, int16_t><<<grid, kHistThreads, 0, L->stream>>>((const int16_t*)sp, Lx, Ly, Lz, Q,     \
                                                                            L->d_count);                          \
    else                                                                                                         \
        boundary_kernel<NB, int32_t><<<grid, kHistThreads, 0, L->stream>>>((const int32_t*)sp, Lx, Ly, Lz, Q,     \
                                                                            L->d_count);
    switch (L->desc.nbr) {
        case HMC_VN4: HMC_BOUNDARY(HMC_VN4) break;
        case HMC_MOORE8: HMC_BOUNDARY(HMC_MOORE8) break;
        case HMC_VN6: HMC_BOUNDARY(HMC_VN6) break;
        default: HMC_BOUNDARY(HMC_MOORE26) break;
    }
#undef HMC_BOUNDARY
    HMC_HIP(hipGetLastError());
    return HMC_OK;
}

hmc_status launch_bin_stats(hmc_lattice* L, const int32_t* d_gbin, int32_t n_bins) {
    return launch_bins(L->d_areas, L->Q, d_gbin, n_bins, L->d_stats, L->stream);
}

}  // namespace hmc
