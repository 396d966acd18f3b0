// sweep.hip -- red/black Potts Metropolis sweep for gfx950.
//
// Method (Zhang, Dingreville, Bartel, Lusk, arXiv:1007.3509):
//   Eq. (7), Sec. 3: bond energy J between unlike neighbours plus a bulk
//     energy b(q) of the grain a site belongs to (Sec. 6);
//   Sec. 3: trial flips accepted by the Metropolis rule on the change of H;
//   Sec. 4: Red/Black updating -- one colour class per half step, every trial
//     of a half step sees the state at its start.
//
// Kernel design (one workgroup per tile, temporally blocked):
//   * A workgroup owns an interior tile of TX x TY (x TZ) sites and stages
//     the tile plus a halo of H = P sites per side into LDS with coalesced
//     row loads (periodic wrap through per-box coordinate tables).
//   * It then runs P consecutive colour passes (k MC steps, P = k*C) in LDS.
//     After pass p only sites at least p+1 rings inside the box are still
//     exact, so the halo is consumed one ring per pass and the interior is
//     exact after P passes; halo work is recomputed redundantly, which keeps
//     the result bit-identical to one launch per pass because every trial's
//     random numbers depend only on (site, step, colour).
//   * Reads come from one spin buffer and the interior goes to the other
//     (ping-pong), so tiles never see each other's partial updates.
//   * Each pass has two phases.  Phase 1 walks the colour class (enumerated
//     directly, no wasted lanes) and appends to an LDS queue every site with
//     a neighbour of another spin (with neighbour-spin trials a site whose
//     neighbours all equal its own spin can only propose itself: a no-op,
//     and skipping its draw is exact because the generator is counter-based).
//     Wave-level ballot + one LDS atomic per wave build the queue.  Phase 2
//     runs Philox, the trial and the integer acceptance only for queued
//     sites, so SIMD lanes are not wasted on interior sites.
//   * Acceptance is integer: d = J_fx*(c(q)-c(q')) + B[q'] - B[q], accept iff
//     d <= 0 or r1 < T(d) from the host-built uint32 table.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>

#include "common.hpp"

namespace hmc {

namespace {

constexpr int kThreads = 1024;
constexpr int kWave = 64;
constexpr int kMaxRows = 64;        // threshold rows: at most 2M+1 = 53
constexpr int kMaxPasses = 64;      // colour passes fused in one launch
constexpr int kLdsGrainLimit = 4096; // grain energies staged in LDS up to this Q
constexpr int kStaticLds = 8 + 8 * kMaxRows + 64;   // qcount + tbound + slack

struct SweepParams {
    const void* src;
    void* dst;
    const int32_t* B;
    const uint32_t* T;
    const uint32_t* Tb;       // per-row (lower, upper) bounds of T
    uint32_t Lx, Ly, Lz;
    uint32_t TX, TY, TZ;
    uint32_t ntx, nty, ntz;
    uint32_t BX, BY, BZ;      // LDS box (BZ = 1 in 2D)
    uint32_t H;               // halo per side (= passes of this launch)
    uint32_t P;               // passes in this launch
    uint32_t t0;              // MC step index of the first pass
    uint32_t k0, k1;          // Philox key
    int32_t J_fx;
    int32_t Q;
    int32_t dn_lo, TW, R, rows;   // threshold-table layout
    uint32_t uniform;         // 1: symmetric trial spins
    uint32_t xcd_group;       // tiles per XCD (0: identity mapping)
    uint32_t queue_off, coord_off, grain_off;   // byte offsets in dynamic LDS
    uint32_t m_bx, m_by, m_tx, m_ty;            // reciprocals (see magic())
    uint32_t m_pass[kMaxPasses][2];             // per pass: per-row and rows reciprocals
};

template <int NBR>
struct Traits;
template <>
struct Traits<HMC_VN4> {
    static constexpr int M = 4, C = 2, D = 2;
};
template <>
struct Traits<HMC_MOORE8> {
    static constexpr int M = 8, C = 4, D = 2;
};
template <>
struct Traits<HMC_VN6> {
    static constexpr int M = 6, C = 2, D = 3;
};
template <>
struct Traits<HMC_MOORE26> {
    static constexpr int M = 26, C = 8, D = 3;
};

__device__ __forceinline__ uint32_t wrap_coord(int64_t a, uint32_t L) {
    int64_t r = a % (int64_t)L;
    return (uint32_t)(r < 0 ? r + L : r);
}

// floor(f / d) = umulhi(f, m) with m = floor(2^32 / d) + 1, exact whenever
// f * d < 2^32 (all box indices here are < 2^16 and d < 2^10); d = 1 is
// encoded as m = 0.  The reciprocals are computed on the host.
__host__ __device__ inline uint32_t magic(uint32_t d) { return d > 1 ? (uint32_t)(0x100000000ull / d) + 1u : 0u; }
__device__ __forceinline__ uint32_t fdiv(uint32_t f, uint32_t m) { return m ? __umulhi(f, m) : f; }

template <int NBR, typename Spin, bool kGrainsInLds>
__global__ void __launch_bounds__(kThreads) sweep_tile_kernel(SweepParams p) {
    using Tr = Traits<NBR>;
    constexpr int M = Tr::M, C = Tr::C, D = Tr::D;
    constexpr bool kCheckerboard = (NBR == HMC_VN4 || NBR == HMC_VN6);
    constexpr int kUnroll = 4;

    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t qcount[2];
    __shared__ uint32_t tbound[2 * kMaxRows];
    Spin* box = reinterpret_cast<Spin*>(smem);
    uint32_t* queue = reinterpret_cast<uint32_t*>(smem + p.queue_off);
    uint32_t* gxs = reinterpret_cast<uint32_t*>(smem + p.coord_off);
    uint32_t* gys = gxs + p.BX;
    uint32_t* gzs = gys + p.BY;
    int32_t* sB = reinterpret_cast<int32_t*>(smem + p.grain_off);
    const int32_t* __restrict__ Bq = kGrainsInLds ? sB : p.B;

    const Spin* __restrict__ src = static_cast<const Spin*>(p.src);
    Spin* __restrict__ dst = static_cast<Spin*>(p.dst);

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = tid / kWave;
    const uint32_t nthr = blockDim.x;

    // Tile of this workgroup.  Consecutive workgroups are spread over the 8
    // XCDs round-robin; regroup so that each XCD gets a contiguous run of
    // tiles and the halos it reads stay in its own L2.
    uint32_t b = blockIdx.x;
    if (p.xcd_group) b = (b & 7u) * p.xcd_group + (b >> 3);
    const uint32_t tx = b % p.ntx;
    const uint32_t ty = (b / p.ntx) % p.nty;
    const uint32_t tz = b / (p.ntx * p.nty);
    const uint32_t H = p.H;
    const uint32_t Hz = (D == 3) ? H : 0u;
    const int64_t x0 = (int64_t)tx * p.TX - (int64_t)H;
    const int64_t y0 = (int64_t)ty * p.TY - (int64_t)H;
    const int64_t z0 = (int64_t)tz * p.TZ - (int64_t)Hz;

    for (uint32_t u = tid; u < p.BX; u += nthr) gxs[u] = wrap_coord(x0 + u, p.Lx);
    for (uint32_t v = tid; v < p.BY; v += nthr) gys[v] = wrap_coord(y0 + v, p.Ly);
    for (uint32_t w = tid; w < p.BZ; w += nthr) gzs[w] = (D == 3) ? wrap_coord(z0 + w, p.Lz) : 0u;
    for (uint32_t r = tid; r < 2u * (uint32_t)p.rows; r += nthr) tbound[r] = p.Tb[r];
    if (kGrainsInLds)
        for (uint32_t q = tid; q < (uint32_t)p.Q; q += nthr) sB[q] = p.B[q];
    if (tid < 2) qcount[tid] = 0;
    __syncthreads();

    // Stage tile + halo: flat box index, consecutive threads on consecutive x
    // (coalesced), kUnroll independent loads in flight per thread.
    const uint32_t box_n = p.BX * p.BY * p.BZ;
    for (uint32_t e0 = tid; e0 < box_n; e0 += kUnroll * nthr) {
        int32_t v[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const uint32_t e = e0 + j * nthr;
            const uint32_t ec = e < box_n ? e : 0u;
            const uint32_t r = fdiv(ec, p.m_bx);
            const uint32_t u = ec - __umul24(r, p.BX);
            const uint32_t w = (D == 3) ? fdiv(r, p.m_by) : 0u;
            const uint32_t vv = r - __umul24(w, p.BY);
            const uint32_t g = gxs[u] + p.Lx * (gys[vv] + p.Ly * gzs[w]);
            v[j] = (int32_t)src[g];
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const uint32_t e = e0 + j * nthr;
            if (e < box_n) box[e] = (Spin)v[j];
        }
    }
    __syncthreads();

    int off[M];
#pragma unroll
    for (int k = 0; k < M; ++k)
        off[k] = nbr_dx(NBR, k) + nbr_dy(NBR, k) * (int)p.BX + nbr_dz(NBR, k) * (int)(p.BX * p.BY);

    // parities of box coordinate 0 along each axis (global coordinate parity)
    const uint32_t px = (uint32_t)(x0 & 1), py = (uint32_t)(y0 & 1), pz = (uint32_t)(z0 & 1);

    for (uint32_t pass = 0; pass < p.P; ++pass) {
        const uint32_t c = pass % C;
        const uint32_t t = p.t0 + pass / C;
        const uint32_t lo = pass + 1;
        const uint32_t loz = (D == 3) ? lo : 0;
        const uint32_t Wx = p.BX - 2 * lo;
        const uint32_t Wy = p.BY - 2 * lo;
        const uint32_t Wz = (D == 3) ? p.BZ - 2 * lo : 1;
        // colour-class enumeration: sites per row, rows per plane, planes
        const uint32_t per_row = Wx / 2;
        const uint32_t rows = kCheckerboard ? Wy : Wy / 2;
        const uint32_t planes = (kCheckerboard || D == 2) ? Wz : Wz / 2;
        const uint32_t total = per_row * rows * planes;
        const uint32_t m_row = p.m_pass[pass][0], m_rows = p.m_pass[pass][1];
        uint32_t* qc = &qcount[pass & 1];
        const uint32_t cx = c & 1u, cy = (c >> 1) & 1u, cz = (c >> 2) & 1u;

        // ---- phase 1: queue the sites of colour c that can change
        for (uint32_t f0 = wave * kWave; f0 < total; f0 += 2 * nthr) {
            bool push[2];
            uint32_t packed[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const uint32_t f = f0 + j * nthr + lane;
                push[j] = false;
                packed[j] = 0;
                if (f < total) {
                    const uint32_t rr = fdiv(f, m_row);
                    const uint32_t jj = f - __umul24(rr, per_row);
                    const uint32_t pl = (D == 3) ? fdiv(rr, m_rows) : 0u;
                    const uint32_t ri = rr - __umul24(pl, rows);
                    uint32_t u, v, w;
                    if (kCheckerboard) {
                        v = lo + ri;
                        w = loz + pl;
                        const uint32_t a = (lo + v + w + px + py + pz) & 1u;
                        u = lo + 2 * jj + ((c ^ a) & 1u);
                    } else {
                        u = lo + 2 * jj + ((cx ^ (lo + px)) & 1u);
                        v = lo + 2 * ri + ((cy ^ (lo + py)) & 1u);
                        w = (D == 3) ? lo + 2 * pl + ((cz ^ (lo + pz)) & 1u) : 0u;
                    }
                    const uint32_t idx = u + __umul24(p.BX, v + __umul24(p.BY, w));
                    const Spin s = box[idx];
                    bool diff = p.uniform != 0;
#pragma unroll
                    for (int k = 0; k < M; ++k) diff |= (box[(int)idx + off[k]] != s);
                    push[j] = diff;
                    packed[j] = u | (v << 10) | (w << 20);
                }
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const uint64_t mask = __ballot(push[j]);
                if (mask) {
                    uint32_t base = 0;
                    if (lane == 0) base = atomicAdd(qc, (uint32_t)__popcll(mask));
                    base = __shfl(base, 0);
                    if (push[j]) queue[base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull))] = packed[j];
                }
            }
        }
        __syncthreads();

        // ---- phase 2: Metropolis trial for every queued site
        const uint32_t count = *qc;
        if (tid == 0) qcount[(pass + 1) & 1] = 0;
        for (uint32_t e0 = tid; e0 < count; e0 += 2 * nthr) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const uint32_t e = e0 + j * nthr;
                if (e >= count) continue;
                const uint32_t packed = queue[e];
                const uint32_t u = packed & 1023u, v = (packed >> 10) & 1023u, w = packed >> 20;
                const int idx = (int)(u + __umul24(p.BX, v + __umul24(p.BY, w)));
                const int32_t q = (int32_t)box[idx];
                if ((uint32_t)q >= (uint32_t)p.Q) continue;
                const int32_t bq = Bq[q];
                const uint32_t site = gxs[u] + p.Lx * (gys[v] + p.Ly * gzs[w]);
                const Philox2 r = philox_r01(site, t, c, 0u, p.k0, p.k1);
                int32_t qn;
                if (!p.uniform) {
                    const uint32_t k = __umulhi(r.r0, (uint32_t)M);
                    int o = off[0];
#pragma unroll
                    for (int kk = 1; kk < M; ++kk) o = (k == (uint32_t)kk) ? off[kk] : o;
                    qn = (int32_t)box[idx + o];
                } else {
                    qn = q + 1 + (int32_t)__umulhi(r.r0, (uint32_t)(p.Q - 1));
                    if (qn >= p.Q) qn -= p.Q;
                }
                if (qn == q || (uint32_t)qn >= (uint32_t)p.Q) continue;
                int cq = 0, cn = 0;
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    const int32_t s = (int32_t)box[idx + off[k]];
                    cq += (s == q);
                    cn += (s == qn);
                }
                const int32_t dn = cq - cn;
                const int32_t dB = Bq[qn] - bq;
                const int32_t d = p.J_fx * dn + dB;
                bool accept = d <= 0;
                if (!accept) {
                    // T is non-increasing in d: the row's bounds decide most trials
                    const int row = dn - p.dn_lo;
                    if (r.r1 < tbound[2 * row]) accept = true;
                    else if (r.r1 < tbound[2 * row + 1]) accept = r.r1 < p.T[row * p.TW + dB + p.R];
                }
                if (accept) box[idx] = (Spin)qn;
            }
        }
        __syncthreads();
    }

    // Interior back to global memory: flat over the tile, coalesced rows.
    const uint32_t tile_n = p.TX * p.TY * p.TZ;
    const uint32_t gx0 = gxs[H];
    for (uint32_t e = tid; e < tile_n; e += nthr) {
        const uint32_t r = fdiv(e, p.m_tx);
        const uint32_t u = e - __umul24(r, p.TX);
        const uint32_t w = (D == 3) ? fdiv(r, p.m_ty) : 0u;
        const uint32_t vv = r - __umul24(w, p.TY);
        const Spin val = box[(H + u) + __umul24(p.BX, (H + vv) + __umul24(p.BY, Hz + w))];
        dst[gx0 + u + p.Lx * (gys[H + vv] + p.Ly * gzs[Hz + w])] = val;
    }
}

template <int NBR>
const void* kernel_for(int spin, bool grains_in_lds) {
    if (spin == HMC_I16)
        return grains_in_lds ? reinterpret_cast<const void*>(&sweep_tile_kernel<NBR, int16_t, true>)
                             : reinterpret_cast<const void*>(&sweep_tile_kernel<NBR, int16_t, false>);
    return grains_in_lds ? reinterpret_cast<const void*>(&sweep_tile_kernel<NBR, int32_t, true>)
                         : reinterpret_cast<const void*>(&sweep_tile_kernel<NBR, int32_t, false>);
}

const void* kernel_ptr(int nbr, int spin, bool grains_in_lds) {
    switch (nbr) {
    case HMC_VN4: return kernel_for<HMC_VN4>(spin, grains_in_lds);
    case HMC_MOORE8: return kernel_for<HMC_MOORE8>(spin, grains_in_lds);
    case HMC_VN6: return kernel_for<HMC_VN6>(spin, grains_in_lds);
    default: return kernel_for<HMC_MOORE26>(spin, grains_in_lds);
    }
}

struct Layout {
    uint32_t BX, BY, BZ, H;
    size_t queue_off, coord_off, grain_off, bytes;
    bool grains_in_lds;
};

Layout box_layout(const hmc_lattice* L, const Tiling& t, int passes) {
    Layout o{};
    o.H = (uint32_t)passes;
    o.BX = (uint32_t)(t.tx + 2 * passes);
    o.BY = (uint32_t)(t.ty + 2 * passes);
    o.BZ = L->ndim == 3 ? (uint32_t)(t.tz + 2 * passes) : 1u;
    const size_t elems = (size_t)o.BX * o.BY * o.BZ;
    size_t qcap;
    switch (L->desc.nbr) {
    case HMC_VN4: case HMC_VN6: qcap = elems / 2 + 1; break;
    case HMC_MOORE8: qcap = elems / 4 + 1; break;
    default: qcap = elems / 8 + 1; break;
    }
    o.queue_off = (elems * L->spin_bytes + 15) / 16 * 16;
    o.coord_off = o.queue_off + (qcap * 4 + 15) / 16 * 16;
    o.grain_off = (o.coord_off + (size_t)(o.BX + o.BY + o.BZ) * 4 + 15) / 16 * 16;
    o.bytes = o.grain_off;
    o.grains_in_lds = false;
    const size_t with_grains = o.grain_off + (size_t)L->Q * 4;
    if (L->Q <= kLdsGrainLimit && (int64_t)with_grains + kStaticLds <= lds_limit_bytes()) {
        o.grains_in_lds = true;
        o.bytes = with_grains;
    }
    return o;
}

int largest_even_divisor_at_most(int L, int target) {
    for (int d = std::min(L, target) & ~1; d >= 2; d -= 2)
        if (L % d == 0) return d;
    return 2;
}

}  // namespace

int lds_limit_bytes() {
    static int cached = -1;
    if (cached < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            cached = std::min(v, 65536);
        else
            cached = 65536;
    }
    return cached;
}

hmc_status choose_tiling(const hmc_lattice* L, Tiling& t, bool explicit_request) {
    const int* dims = L->desc.dims;
    Tiling r = t;
    if (!explicit_request || r.tx == 0 || r.ty == 0 || (L->ndim == 3 && r.tz == 0) || r.k == 0) {
        int tile2 = 64, tile3 = 16, k = 1;
        switch (L->desc.nbr) {
        case HMC_VN4: tile2 = 64; k = 4; break;
        case HMC_MOORE8: tile2 = 64; k = 2; break;
        case HMC_VN6: tile3 = 16; k = 1; break;
        default: tile3 = 8; k = 1; break;
        }
        if (r.tx == 0) r.tx = largest_even_divisor_at_most(dims[0], L->ndim == 2 ? tile2 : tile3);
        if (r.ty == 0) r.ty = largest_even_divisor_at_most(dims[1], L->ndim == 2 ? tile2 : tile3);
        if (L->ndim == 3 && r.tz == 0) r.tz = largest_even_divisor_at_most(dims[2], tile3);
        if (r.k == 0) r.k = k;
    }
    if (L->ndim == 2) r.tz = 1;
    const int sides[3] = {r.tx, r.ty, r.tz};
    for (int a = 0; a < L->ndim; ++a) {
        if (sides[a] < 2 || sides[a] % 2 != 0 || dims[a] % sides[a] != 0)
            return fail(HMC_E_INVAL, "tile side " + std::to_string(sides[a]) +
                                         " must be an even divisor of the lattice side " + std::to_string(dims[a]));
    }
    if (r.k < 1 || r.k * L->C > kMaxPasses)
        return fail(HMC_E_INVAL, "mcs_per_launch * colours must be in [1, " + std::to_string(kMaxPasses) + "]");
    const int passes = r.k * L->C;
    const Layout lay = box_layout(L, r, passes);
    if (lay.BX > 1023 || lay.BY > 1023 || lay.BZ > 1023)
        return fail(HMC_E_INVAL, "tile + halo exceeds 1023 sites along an axis");
    if ((int64_t)lay.bytes + kStaticLds > lds_limit_bytes())
        return fail(HMC_E_INVAL, "tile + halo needs " + std::to_string(lay.bytes) + " B of LDS, limit " +
                                     std::to_string(lds_limit_bytes()));
    t = r;
    return HMC_OK;
}

hmc_status launch_sweep(hmc_lattice* L, float kT, int32_t n_mcs, uint64_t seed) {
    if (n_mcs == 0) return HMC_OK;
    HMC_TRY(build_table(L->table, kT, L->M, L->desc.J_fx, L->Bmin, L->Bmax, L->stream));
    if (L->table.rows > kMaxRows) return fail(HMC_E_INTERNAL, "threshold table has too many rows");
    Tiling t = L->tiling;
    HMC_TRY(choose_tiling(L, t, L->tiling_explicit));
    L->tiling = t;

    const int* dims = L->desc.dims;
    SweepParams p{};
    p.B = L->dB;
    p.T = L->table.dev;
    p.Tb = L->table.bounds;
    p.rows = L->table.rows;
    p.Lx = (uint32_t)dims[0];
    p.Ly = (uint32_t)dims[1];
    p.Lz = L->ndim == 3 ? (uint32_t)dims[2] : 1u;
    p.TX = (uint32_t)t.tx;
    p.TY = (uint32_t)t.ty;
    p.TZ = L->ndim == 3 ? (uint32_t)t.tz : 1u;
    p.ntx = p.Lx / p.TX;
    p.nty = p.Ly / p.TY;
    p.ntz = p.Lz / p.TZ;
    p.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
    p.k1 = (uint32_t)(seed >> 32);
    p.J_fx = L->desc.J_fx;
    p.Q = L->Q;
    p.dn_lo = L->table.dn_lo;
    p.TW = L->table.TW;
    p.R = L->table.R;
    p.uniform = L->desc.proposal == HMC_PROP_UNIFORM ? 1u : 0u;
    const uint32_t ntiles = p.ntx * p.nty * p.ntz;
    p.xcd_group = (ntiles % 8 == 0) ? ntiles / 8 : 0u;

    int32_t remaining = n_mcs;
    uint64_t t_next = L->mcs;
    while (remaining > 0) {
        const int k = std::min<int32_t>(t.k, remaining);
        const int passes = k * L->C;
        const Layout lay = box_layout(L, t, passes);
        p.BX = lay.BX; p.BY = lay.BY; p.BZ = lay.BZ;
        p.H = lay.H;
        p.P = (uint32_t)passes;
        p.t0 = (uint32_t)t_next;
        p.queue_off = (uint32_t)lay.queue_off;
        p.coord_off = (uint32_t)lay.coord_off;
        p.grain_off = (uint32_t)lay.grain_off;
        p.m_bx = magic(lay.BX);
        p.m_by = magic(lay.BY);
        p.m_tx = magic(p.TX);
        p.m_ty = magic(p.TY);
        for (int ps = 0; ps < passes; ++ps) {
            const uint32_t lo = (uint32_t)ps + 1;
            const uint32_t Wx = lay.BX - 2 * lo, Wy = lay.BY - 2 * lo;
            const bool cb = L->desc.nbr == HMC_VN4 || L->desc.nbr == HMC_VN6;
            p.m_pass[ps][0] = magic(Wx / 2);
            p.m_pass[ps][1] = magic(cb ? Wy : Wy / 2);
        }
        const void* kfn = kernel_ptr(L->desc.nbr, L->desc.spin, lay.grains_in_lds);
        p.src = L->spins[L->cur];
        p.dst = L->spins[L->cur ^ 1];
        void* args[] = {&p};
        if (L->profiling) {
            // Events bound to the dispatch itself: they time the kernel, not
            // the queue around it.
            if (L->events_used == L->events.size()) {
                hipEvent_t a, b;
                HMC_HIP(hipEventCreate(&a));
                HMC_HIP(hipEventCreate(&b));
                L->events.emplace_back(a, b);
            }
            const auto& ev = L->events[L->events_used++];
            HMC_HIP(hipExtLaunchKernel(kfn, dim3(ntiles), dim3(kThreads), args, lay.bytes, L->stream, ev.first,
                                       ev.second, 0));
            L->prof_launches += 1;
            L->prof_su += (int64_t)k * L->N;
        } else {
            HMC_HIP(hipLaunchKernel(kfn, dim3(ntiles), dim3(kThreads), args, lay.bytes, L->stream));
        }
        L->cur ^= 1;
        t_next += (uint64_t)k;
        remaining -= k;
    }
    L->mcs += (uint64_t)n_mcs;
    return HMC_OK;
}

}  // namespace hmc
