// sweep_vn6.hip -- the red/black Metropolis sweep of Sec. 3-4 specialised
// for the three-dimensional six-neighbour lattice with 16-bit spins,
// neighbour-spin trials, one bond energy J and per-grain bulk energies
// (Eq. (7) read as J(1 - delta) plus b(q); Sec. 6: the energy belongs to the
// grain).  Same method, random numbers and integer acceptance as the generic
// tile kernel in sweep.hip, so the two give identical spins; this one fixes
// the tile and its box at compile time, which turns every index computation
// into constants and shifts:
//
//   * the box of a TX x TY x TZ tile adds 2 sites of halo along y and z and
//     4 along x (rows of whole 8-byte words), enough for the two colour
//     passes (one MC step) a launch runs;
//   * persistent workgroups walk their share of the tiles.  Tiles whose
//     LDS fits twice in a CU run two workgroups per CU (eight waves per
//     SIMD, 64 registers a lane): while one waits at a barrier the other
//     issues.  Larger tiles run one workgroup per CU, and while it runs the
//     passes of one tile the next tile's box is already on its way from
//     global memory into registers (its barriers wait for LDS traffic only,
//     so those loads stay in flight) and goes to LDS once the current tile
//     is stored;
//   * per pass, phase 1 walks the 4-site words of the pass region with a
//     fixed word column per thread (so the column's bounds and the colour
//     pattern are loop invariant) and queues the sites of the pass colour
//     that have a neighbour of another spin; phase 2 runs Philox and the
//     trial on the queued sites only;
//   * queue entries carry the box index and the box row, and per-row global
//     offsets live in LDS, so a trial finds its site number with two LDS
//     reads and no multiplication.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.hpp"

namespace hmc {

namespace {

constexpr int kVThreads = 1024;
constexpr size_t kCuLdsBytes = 160 * 1024;   // LDS of one CU on this chip
constexpr int kVWave = 64;

constexpr size_t align16(size_t b) { return (b + 15) / 16 * 16; }

template <int TX, int TY, int TZ>
struct VGeom {
    static constexpr int H = 2, HX = 4;   // halo: two passes; x rounded up to whole words
    static constexpr int BX = TX + 2 * HX, BY = TY + 2 * H, BZ = TZ + 2 * H;
    static constexpr int BXY = BX * BY, NBOX = BXY * BZ;
    static constexpr int NW = BX / 4, NROWS = BY * BZ, NWORDS = NW * NROWS;
    // the largest pass region (one ring in, x from the padded edge) holds
    // exactly half of its sites in each colour
    static constexpr int QCAP = (BX - 2 * (1 + HX - H)) * (BY - 2) * (BZ - 2) / 2 + 1;
    static constexpr size_t kBoundOff = 0;                                       // uint32[2 * kBoundPairs]
    static constexpr size_t kCountOff = kBoundOff + 8 * kBoundPairs;             // uint32[2]
    static constexpr size_t kOffsetOff = kCountOff + 16;                         // int32[8]: neighbour offsets
    // two sets of tables (the tile in the box and the next one)
    static constexpr size_t kGxStride = align16(4 * (size_t)BX) / 4, kRowStride = align16(4 * (size_t)NROWS) / 4;
    static constexpr size_t kGxOff = kOffsetOff + 32;                            // uint32[2][BX]
    static constexpr size_t kRowOff = kGxOff + 8 * kGxStride;                    // uint32[2][NROWS]
    static constexpr size_t kBoxOff = kRowOff + 8 * kRowStride;                  // int16[NBOX]
    static constexpr size_t kQueueOff = kBoxOff + align16(2 * (size_t)NBOX);     // uint32[QCAP]
    static constexpr size_t kGrainOff = kQueueOff + align16(4 * (size_t)QCAP);   // int32[Q] (grains in LDS)
    static_assert(TX % 4 == 0 && TY % 2 == 0 && TZ % 2 == 0, "tile sides");
    static_assert(NBOX < 65536 && NROWS < 65536, "queue entries pack the box index and row in 16 bits each");
};

__device__ __forceinline__ uint32_t vwrap(int32_t a, uint32_t L) {
    while (a < 0) a += (int32_t)L;
    while (a >= (int32_t)L) a -= (int32_t)L;
    return (uint32_t)a;
}

// Grain energies: kGrainGlobal read from global memory (L2-resident),
// kGrainLds32 staged in LDS (few grains).  (20 000 grains as 16-bit offsets
// in LDS, staged once per workgroup, measured slower -- 75.8 against 71.4 us
// per 256^3 step -- the random reads of the offsets conflict in the banks.)
enum { kGrainGlobal = 0, kGrainLds32 = 1 };

// Workgroup barrier for LDS traffic only: waits for this wave's LDS
// operations, not for its global loads, so a prefetch of the next tile stays
// in flight across the passes (all communication inside a pass is in LDS).
// s_waitcnt operand that waits for vector memory operations only (vmcnt 0,
// export and LDS/scalar counters left at their maxima)
constexpr int kWaitVmcnt0 = 0x0F70;

__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// kPerCU: resident workgroups per CU the kernel is built for (1 or 2); with
// one, the next tile's box is prefetched into registers during the passes.
template <int TX, int TY, int TZ, int kGrains, int kPerCU>
__global__ void __launch_bounds__(kVThreads) __attribute__((amdgpu_waves_per_eu(4 * kPerCU)))
vn6_tile_kernel(Vn6Args a) {
    using G = VGeom<TX, TY, TZ>;
    constexpr bool kPrefetch = kPerCU == 1;
    constexpr int BX = G::BX, BY = G::BY, BZ = G::BZ, BXY = G::BXY, NW = G::NW, H = G::H, HX = G::HX;
    constexpr int PRE = (G::NWORDS + kVThreads - 1) / kVThreads;   // box words per thread
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* tbound = reinterpret_cast<uint32_t*>(smem + G::kBoundOff);
    uint32_t* qcount = reinterpret_cast<uint32_t*>(smem + G::kCountOff);
    // table set 0 or 1
    auto gxs = [&](int set) __attribute__((always_inline)) {
        return reinterpret_cast<uint32_t*>(smem + G::kGxOff) + set * G::kGxStride;
    };
    auto rows = [&](int set) __attribute__((always_inline)) {
        return reinterpret_cast<uint32_t*>(smem + G::kRowOff) + set * G::kRowStride;
    };
    int16_t* box = reinterpret_cast<int16_t*>(smem + G::kBoxOff);
    uint64_t* boxw = reinterpret_cast<uint64_t*>(smem + G::kBoxOff);
    uint32_t* queue = reinterpret_cast<uint32_t*>(smem + G::kQueueOff);
    int32_t* sB = reinterpret_cast<int32_t*>(smem + G::kGrainOff);
    int32_t* noff = reinterpret_cast<int32_t*>(smem + G::kOffsetOff);
    // energy of grain q (q in [0, Q))
    auto energy = [&](int32_t q) __attribute__((always_inline)) -> int32_t {
        if constexpr (kGrains == kGrainLds32) return sB[q];
        else return a.B[q];
    };

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kVWave - 1);
    const uint64_t lanes_below = (1ull << lane) - 1ull;

    // This workgroup's tiles.  Consecutive workgroups are dispatched to the 8
    // XCDs in turn; with xcd_blocks each XCD's workgroups share one
    // contiguous block of tiles (halos shared in its own L2), taken in turn.
    uint32_t first = blockIdx.x, stride = gridDim.x, end = a.ntiles;
    if (a.xcd_blocks) {
        const uint32_t per_xcd = (a.ntiles + 7u) / 8u, xcd = blockIdx.x & 7u;
        first = xcd * per_xcd + (blockIdx.x >> 3);
        stride = gridDim.x >> 3;
        end = min(a.ntiles, (xcd + 1u) * per_xcd);
    }
    auto origin = [&](uint32_t tile, int32_t& x0, int32_t& y0, int32_t& z0) __attribute__((always_inline)) {
        const uint32_t tx = tile % a.ntx, ty = (tile / a.ntx) % a.nty, tz = tile / (a.ntx * a.nty);
        x0 = (int32_t)(tx * TX) - HX;
        y0 = (int32_t)(ty * TY) - H;
        z0 = (int32_t)(tz * TZ) - H;
    };
    // per-box-column x and per-box-row offset y Lx + z Lx Ly of the global site
    auto make_tables = [&](uint32_t tile, int set) __attribute__((always_inline)) {
        int32_t x0, y0, z0;
        origin(tile, x0, y0, z0);
        for (uint32_t u = tid; u < (uint32_t)BX; u += kVThreads) gxs(set)[u] = vwrap(x0 + (int32_t)u, a.Lx);
        for (uint32_t r = tid; r < (uint32_t)G::NROWS; r += kVThreads) {
            const uint32_t v = r % BY, w = r / BY;
            rows(set)[r] = a.Lx * (vwrap(y0 + (int32_t)v, a.Ly) + a.Ly * vwrap(z0 + (int32_t)w, a.Lz));
        }
    };
    // Box words (four spins each) of a tile into registers, and from there to
    // LDS.  Rows start at a global x that is a multiple of 4 and Lx is a
    // multiple of 4, so a word never wraps.
    uint64_t pre[PRE];
    auto prefetch = [&](int set) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < PRE; ++j) {
            const uint32_t e = tid + (uint32_t)j * kVThreads;
            const uint32_t ec = e < (uint32_t)G::NWORDS ? e : 0u;
            const uint32_t r = ec / NW, u4 = ec - r * NW;
            const uint32_t site = gxs(set)[4 * u4] + rows(set)[r];   // < 2^32 sites
            pre[j] = *reinterpret_cast<const uint64_t*>(a.src + site);
        }
    };
    auto commit = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < PRE; ++j) {
            const uint32_t e = tid + (uint32_t)j * kVThreads;
            if (e < (uint32_t)G::NWORDS) boxw[e] = pre[j];
        }
    };

    for (uint32_t r = tid; r < 2u * (uint32_t)a.nbound; r += kVThreads) tbound[r] = a.Tb[r];
    if constexpr (kGrains == kGrainLds32)
        for (uint32_t q = tid; q < (uint32_t)a.Q; q += kVThreads) sB[q] = a.B[q];
    if (tid < 6) {   // box offset of neighbour k in the trial order +x -x +y -y +z -z
        const int32_t st = tid < 2 ? 1 : (tid < 4 ? BX : BXY);
        noff[tid] = (tid & 1) ? -st : st;
    }
    if (tid < 2) qcount[tid] = 0;
    if (first < end) make_tables(first, 0);
    if (first + stride < end) make_tables(first + stride, 1);
    lds_barrier();
    if (first < end) {
        prefetch(0);
        commit();
    }
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);   // every lane's words, committed or not, have landed
    lds_barrier();

    unsigned long long drawn = 0;
    int S = 0;   // table set of the tile in the box
    for (uint32_t tile = first; tile < end; tile += stride, S ^= 1) {
        const uint32_t nxt = tile + stride;
        const bool has_next = nxt < end;
        if constexpr (kPrefetch)
            if (has_next) prefetch(S ^ 1);   // in flight during the passes
        const uint32_t* gx = gxs(S);
        const uint32_t* rowL = rows(S);
        int32_t x0, y0, z0;
        origin(tile, x0, y0, z0);
        const uint32_t org = (uint32_t)(x0 + y0 + z0) & 1u;   // colour parity of box site (0, 0, 0)

        // One colour pass over ring R of the box (R = 1: first of two passes,
        // R = 2: the tile itself), colour c, MC step t; queue counter slot qs.
        auto pass = [&](auto ring, uint32_t c, uint32_t t, uint32_t qs) __attribute__((always_inline)) {
            constexpr int R = decltype(ring)::value;
            constexpr int LOX = R + (HX - H);
            constexpr int S_LO = LOX >> 2, S_HI = (BX - LOX - 1) >> 2, NSEG = S_HI - S_LO + 1;
            constexpr int WY = BY - 2 * R, WZ = BZ - 2 * R, ROWS = WY * WZ;
            constexpr int RPI = kVThreads / NSEG, ACT = RPI * NSEG, ITER = (ROWS + RPI - 1) / RPI;
            constexpr int DV = RPI % WY, DW = RPI / WY;
            uint32_t* qc = &qcount[qs];

            // Phase 1: thread -> fixed word column sg, rows rr0, rr0 + RPI, ...
            const uint32_t sg = S_LO + tid % NSEG;
            const uint32_t rr0 = tid / NSEG;
            const bool tact = tid < (uint32_t)ACT;
            uint32_t okmask = 0;   // fields of the word inside the pass region
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t uu = 4 * sg + j;
                okmask |= (uu >= (uint32_t)LOX && uu < (uint32_t)(BX - LOX)) ? (1u << j) : 0u;
            }
            uint32_t v = R + rr0 % WY, w = R + rr0 / WY;
#pragma unroll 2
            for (int it = 0; it < ITER; ++it) {
                bool pa = false, pb = false;
                uint32_t ea = 0, eb = 0;
                if (tact && rr0 + (uint32_t)it * RPI < (uint32_t)ROWS) {
                    const uint32_t row = v + BY * w;
                    const uint32_t wi = row * NW + sg;
                    const uint64_t S = boxw[wi];
                    const uint64_t U = boxw[wi + NW], D = boxw[wi - NW];
                    const uint64_t F = boxw[wi + NW * BY], K = boxw[wi - NW * BY];
                    const uint32_t k = (c + v + w + org) & 1u;   // first field of colour c
                    // the one x neighbour outside the word that a colour-c field
                    // has: the site before the word (k = 0) or after it (k = 1)
                    const uint32_t e = (uint16_t)box[k ? 4 * wi + 4 : 4 * wi - 1];
                    // the word shifted by one site towards +x and towards -x, as
                    // 32-bit halves (funnel shifts instead of 64-bit shifts)
                    const uint32_t lo = (uint32_t)S, hi = (uint32_t)(S >> 32);
                    const uint32_t mid = __builtin_amdgcn_alignbit(hi, lo, 16);   // sites 1, 2
                    const uint32_t xl = (lo ^ ((lo << 16) | e)) | (lo ^ mid) | (lo ^ (uint32_t)U) |
                                        (lo ^ (uint32_t)D) | (lo ^ (uint32_t)F) | (lo ^ (uint32_t)K);
                    const uint32_t xh = (hi ^ mid) | (hi ^ __builtin_amdgcn_alignbit(e, hi, 16)) |
                                        (hi ^ (uint32_t)(U >> 32)) | (hi ^ (uint32_t)(D >> 32)) |
                                        (hi ^ (uint32_t)(F >> 32)) | (hi ^ (uint32_t)(K >> 32));
                    const uint32_t fa = __builtin_amdgcn_ubfe(xl, 16 * k, 16);
                    const uint32_t fb = __builtin_amdgcn_ubfe(xh, 16 * k, 16);
                    pa = fa != 0 && ((okmask >> k) & 1u);
                    pb = fb != 0 && ((okmask >> (k + 2)) & 1u);
                    const uint32_t ia = 4 * wi + k;
                    ea = ia | (row << 16);
                    eb = (ia + 2) | (row << 16);
                }
                const uint64_t ma = __ballot(pa), mb = __ballot(pb);
                const uint32_t na = (uint32_t)__popcll(ma);
                const uint32_t n = na + (uint32_t)__popcll(mb);
                if (n) {
                    uint32_t base = 0;
                    if (lane == 0) base = atomicAdd(qc, n);
                    base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
                    if (pa) queue[base + (uint32_t)__popcll(ma & lanes_below)] = ea;
                    if (pb) queue[base + na + (uint32_t)__popcll(mb & lanes_below)] = eb;
                }
                v += DV;
                w += DW;
                if (v >= (uint32_t)(R + WY)) {
                    v -= WY;
                    w += 1;
                }
            }
            lds_barrier();
            const uint32_t count = *qc;
            if (tid == 0) {
                qcount[qs ^ 1u] = 0;
                drawn += count;
            }

            // Phase 2: the Metropolis trial of every queued site.  Reads that do
            // not depend on the random numbers are issued before Philox.
            auto trial = [&](uint32_t e) __attribute__((always_inline)) {
                const uint32_t idx = e & 0xFFFFu, row = e >> 16;
                const uint32_t u = idx - row * BX;
                const int32_t q = box[idx];
                int32_t nb[6];
                nb[0] = box[idx + 1];
                nb[1] = box[idx - 1];
                nb[2] = box[idx + BX];
                nb[3] = box[idx - BX];
                nb[4] = box[idx + BXY];
                nb[5] = box[idx - BXY];
                const uint32_t site = gx[u] + rowL[row];
                const bool q_ok = (uint32_t)q < (uint32_t)a.Q;   // a value outside [0, Q) never moves
                const int32_t bq = energy(q_ok ? q : 0);
                const Philox2 rn = philox_r01(site, t, c, 0u, a.k0, a.k1);
                const uint32_t kk = __umulhi(rn.r0, 6u);
                const int32_t qn = box[(int32_t)idx + noff[kk]];
                if (!q_ok || qn == q || (uint32_t)qn >= (uint32_t)a.Q) return;
                const int32_t dn = like_difference16<6>(nb, q, qn);
                const int32_t dB = energy(qn) - bq;
                const int32_t d = __mul24(a.J_fx, dn) + dB;   // J_fx < 2^23 (checked on the host)
                bool accept = d <= 0;
                if (!accept) {
                    // T is non-increasing in d: the bucket's bounds decide almost every trial
                    const int rowT = dn - a.dn_lo;
                    const uint32_t col = (uint32_t)(dB + a.R);
                    const uint32_t bucket = a.m_bw ? __umulhi(col, a.m_bw) : col / a.bw;
                    const uint32_t bk = (uint32_t)rowT * (uint32_t)a.nb + bucket;
                    if (rn.r1 < tbound[2 * bk]) accept = true;
                    else if (rn.r1 < tbound[2 * bk + 1]) accept = rn.r1 < a.T[rowT * a.TW + (int)col];
                }
                if (accept) box[idx] = (int16_t)qn;
            };
            for (uint32_t e0 = tid; e0 < count; e0 += 2 * kVThreads) {
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const uint32_t e = e0 + j * kVThreads;
                    if (e < count) trial(queue[e]);
                }
            }
            lds_barrier();
        };

        for (uint32_t p = 0; p < a.npass; ++p) {
            const uint32_t gp = a.c0 + p;   // pass counted from colour 0 of MC step t0
            const uint32_t c = gp & 1u, t = a.t0 + (gp >> 1);
            if (a.npass == 2 && p == 0) pass(std::integral_constant<int, 1>{}, c, t, p & 1u);
            else pass(std::integral_constant<int, 2>{}, c, t, p & 1u);
        }

        // Every vector load of this workgroup has arrived by now (with one
        // workgroup per CU that includes the next box, issued before the
        // passes): wait for them here, before the stores, so that nothing
        // later (the commit, the next box loaded into the same registers) has
        // to wait for the stores themselves to complete.
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        // The tile back to global memory, 8-byte words.
        constexpr int TW4 = TX / 4;
        const uint32_t gx0 = (uint32_t)(x0 + HX);
        for (uint32_t e = tid; e < (uint32_t)(TW4 * TY * TZ); e += kVThreads) {
            const uint32_t u4 = e % TW4, rr = e / TW4;
            const uint32_t vv = rr % TY, ww = rr / TY;
            const uint32_t brow = (H + vv) + BY * (H + ww);
            const uint64_t val = boxw[brow * NW + HX / 4 + u4];
            *reinterpret_cast<uint64_t*>(a.dst + gx0 + 4 * u4 + rowL[brow]) = val;
        }
        lds_barrier();   // the box, the queue and this tile's tables are free
        if (tid == 0) {
            qcount[0] = 0;
            qcount[1] = 0;
        }
        if (has_next) {
            if constexpr (!kPrefetch) prefetch(S ^ 1);
            commit();
            if (nxt + stride < end) make_tables(nxt + stride, S);
        }
        lds_barrier();
    }

    if (a.trials && tid == 0) atomicAdd(&a.trials[blockIdx.x & (kTrialSlots - 1)], drawn);
}

template <int TX, int TY, int TZ>
bool pick(const Tiling& t, int32_t Q, bool& fits, const void*& fn, size_t& bytes, int& per_cu) {
    if (t.tx != TX || t.ty != TY || t.tz != TZ) return false;
    using G = VGeom<TX, TY, TZ>;
    const int64_t limit = lds_limit_bytes();
    const bool lds_grains = Q <= 4096 && (int64_t)(G::kGrainOff + 4 * (size_t)Q) <= limit;
    bytes = G::kGrainOff + (lds_grains ? 4 * (size_t)Q : 0);
    fn = lds_grains ? reinterpret_cast<const void*>(&vn6_tile_kernel<TX, TY, TZ, kGrainLds32, 1>)
                    : reinterpret_cast<const void*>(&vn6_tile_kernel<TX, TY, TZ, kGrainGlobal, 1>);
    per_cu = 1;
    // two workgroups per CU when the LDS holds two (a CU's LDS equals the
    // per-workgroup limit); only tiles whose bare box can pair are built so
    if constexpr (2 * G::kGrainOff <= kCuLdsBytes) {
        if (2 * (int64_t)bytes <= limit) {
            per_cu = 2;
            fn = lds_grains ? reinterpret_cast<const void*>(&vn6_tile_kernel<TX, TY, TZ, kGrainLds32, 2>)
                            : reinterpret_cast<const void*>(&vn6_tile_kernel<TX, TY, TZ, kGrainGlobal, 2>);
        }
    }
    fits = (int64_t)bytes <= limit;
    return true;
}

}  // namespace

bool vn6_kernel_for(const Tiling& t, int32_t Q, const void** fn, size_t* lds_bytes, int* per_cu) {
    bool fits = false;
    const void* f = nullptr;
    size_t bytes = 0;
    int pc = 1;
    const bool known = pick<64, 16, 16>(t, Q, fits, f, bytes, pc) || pick<32, 32, 16>(t, Q, fits, f, bytes, pc) ||
                       pick<32, 16, 16>(t, Q, fits, f, bytes, pc) || pick<16, 16, 16>(t, Q, fits, f, bytes, pc) ||
                       pick<64, 16, 8>(t, Q, fits, f, bytes, pc);
    if (!known || !fits) return false;
    *fn = f;
    *lds_bytes = bytes;
    *per_cu = pc;
    return true;
}

}  // namespace hmc
