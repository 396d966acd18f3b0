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
//
// Ensemble mode (many independent lattices of uneven size, temperature and
// seed): the same per-tile routine runs from a persistent kernel that walks
// a ragged tile table covering every lattice; each launch advances every
// lattice by k MC steps, and the launch sequence of a call is captured once
// into a HIP graph and replayed.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <numeric>

#include "common.hpp"

namespace hmc {

namespace {

constexpr int kThreads = 1024;
constexpr int kWave = 64;
constexpr int kMaxRows = 64;         // threshold rows: at most 2M+1 = 53
constexpr int kMaxPasses = 64;       // colour passes fused in one launch
constexpr int kLdsGrainLimit = 4096; // grain energies staged in LDS up to this Q
constexpr int kHeaderBytes = 8 * kBoundPairs + 16;   // threshold bucket bounds + queue counters

// Per-lattice arguments (uniform over a workgroup).
struct LatArgs {
    const void* src;
    void* dst;
    const int32_t* B;
    const uint32_t* T;
    const uint32_t* Tb;       // per-row (lower, upper) bounds of T
    uint32_t Lx, Ly, Lz;
    uint32_t TX, TY, TZ;
    uint32_t ntx, nty;
    uint32_t t0;              // MC step index of the first pass
    uint32_t c0;              // colour of the first pass (launches may start inside an MC step)
    uint32_t k0, k1;          // Philox key
    int32_t J_fx;
    int32_t Q;
    int32_t dn_lo, TW, R, rows;   // threshold-table layout
    int32_t nb, nbound;       // buckets per row, bound pairs in total
    uint32_t bw, m_bw;        // bucket width and its reciprocal (m_bw = 0: divide)
    uint32_t uniform;         // 1: symmetric trial spins
    unsigned long long* trials;   // when not null: kTrialSlots counters of Philox draws (queued trials)
    const int32_t* Jp;        // pair bond energies int32[Q*Q] (pair mode)
    const uint32_t* Tg;       // pair and field modes: T(d) for d = 0..Dmax
    int32_t Dmax;
    const int32_t* fsrc;      // field mode: per-site bulk energy, read
    int32_t* fdst;            //   and written (ping-pong with the spins)
    uint32_t frule;           //   0: a swept site takes the proposing neighbour's field, 1: zero
};

// Per-launch arguments: the LDS box and its precomputed reciprocals.
struct RunArgs {
    uint32_t BX, BY, BZ;      // LDS box (BZ = 1 in 2D)
    uint32_t H;               // halo per side (= passes of this launch) along y and z
    uint32_t HX;              // halo along x: H, or H rounded up to 4 for 8-byte row access
    uint32_t vec;             // 1: stage and store 16-bit spins four at a time (8-byte aligned)
    uint32_t P;               // passes in this launch
    uint32_t box_off, queue_off, coord_off, grain_off;   // byte offsets in dynamic LDS
    uint32_t m_bx, m_by, m_tx, m_ty;
    uint32_t m_bx4, m_tx4;    // reciprocals of BX / 4 and TX / 4 (vec)
    uint32_t field_off;       // byte offset of the per-site field box in LDS (field mode)
    uint32_t m_pass[kMaxPasses][2];   // per pass: per-row and rows reciprocals
};

// Ensemble member as the device sees it.
struct EnsLat {
    LatArgs a;                // src/dst/t0 filled in by the kernel
    void* buf[2];
    uint32_t cur;             // buffer holding the state at the call's start
    uint32_t t_base;          // MC step of the call's first step
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

// a mod L for a box coordinate: a lies within a few periods of [0, L) (the
// halo is at most a few sides), so a 32-bit add or subtract settles it.
__device__ __forceinline__ uint32_t wrap_coord(int64_t a, uint32_t L) {
    int32_t r = (int32_t)a;
    while (r < 0) r += (int32_t)L;
    while (r >= (int32_t)L) r -= (int32_t)L;
    return (uint32_t)r;
}

// floor(f / d) = umulhi(f, m) with m = floor(2^32 / d) + 1, exact whenever
// f * d < 2^32 (all box indices here are < 2^16 and d < 2^10); d = 1 is
// encoded as m = 0.  The reciprocals are computed on the host.
__host__ __device__ inline uint32_t magic(uint32_t d) { return d > 1 ? (uint32_t)(0x100000000ull / d) + 1u : 0u; }
__device__ __forceinline__ uint32_t fdiv(uint32_t f, uint32_t m) { return m ? __umulhi(f, m) : f; }

// Box offset of neighbour k (k from the trial draw, so not a constant),
// computed from the neighbour order without an indexed table.
template <int NBR>
__device__ __forceinline__ int nbr_offset(uint32_t k, int BX, int BXY) {
    if (NBR == HMC_MOORE26) {
        const int m = (int)k + (k >= 13 ? 1 : 0);
        const int dz = m / 9, rem = m - 9 * dz;
        const int dy = rem / 3, dx = rem - 3 * dy;
        return (dx - 1) + (dy - 1) * BX + (dz - 1) * BXY;
    }
    const int sgn = 1 - 2 * (int)(k & 1u);
    if (NBR == HMC_MOORE8 && k >= 4) {
        const int dy = (k < 6) ? sgn : -sgn;   // (+1,+1) (-1,-1) (+1,-1) (-1,+1)
        return sgn + dy * BX;
    }
    const uint32_t axis = k >> 1;           // +x -x +y -y (+z -z)
    const int stride = axis == 0 ? 1 : (axis == 1 ? BX : BXY);
    return sgn * stride;
}

// One tile: stage tile + halo, run g.P colour passes in LDS, write the interior.
// Ends with every thread past its last LDS access of the tile (callers that
// process another tile put a barrier before reusing LDS).
template <int NBR, typename Spin, bool kGrainsInLds, bool kSwar, bool kPair = false, bool kField = false>
__device__ __forceinline__ void process_tile(const LatArgs& a, const RunArgs& g, uint32_t tx, uint32_t ty,
                                             uint32_t tz, unsigned char* smem) {
    using Tr = Traits<NBR>;
    constexpr int M = Tr::M, C = Tr::C, D = Tr::D;
    constexpr bool kCheckerboard = (NBR == HMC_VN4 || NBR == HMC_VN6);
    constexpr int kUnroll = 4;

    uint32_t* tbound = reinterpret_cast<uint32_t*>(smem);
    uint32_t* qcount = reinterpret_cast<uint32_t*>(smem + kHeaderBytes - 16);
    Spin* box = reinterpret_cast<Spin*>(smem + g.box_off);
    int32_t* fbox = reinterpret_cast<int32_t*>(smem + g.field_off);   // field mode only
    uint32_t* queue = reinterpret_cast<uint32_t*>(smem + g.queue_off);
    uint32_t* gxs = reinterpret_cast<uint32_t*>(smem + g.coord_off);
    uint32_t* gys = gxs + g.BX;
    uint32_t* gzs = gys + g.BY;
    int32_t* sB = reinterpret_cast<int32_t*>(smem + g.grain_off);
    const int32_t* __restrict__ Bq = kGrainsInLds ? sB : a.B;

    const Spin* __restrict__ src = static_cast<const Spin*>(a.src);
    Spin* __restrict__ dst = static_cast<Spin*>(a.dst);

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = tid / kWave;
    const uint32_t nthr = blockDim.x;

    const uint32_t H = g.H;
    const uint32_t Hz = (D == 3) ? H : 0u;
    const uint32_t HX = g.HX;
    const int64_t x0 = (int64_t)tx * a.TX - (int64_t)HX;
    const int64_t y0 = (int64_t)ty * a.TY - (int64_t)H;
    const int64_t z0 = (int64_t)tz * a.TZ - (int64_t)Hz;
    for (uint32_t u = tid; u < g.BX; u += nthr) gxs[u] = wrap_coord(x0 + u, a.Lx);
    for (uint32_t v = tid; v < g.BY; v += nthr) gys[v] = wrap_coord(y0 + v, a.Ly);
    for (uint32_t w = tid; w < g.BZ; w += nthr) gzs[w] = (D == 3) ? wrap_coord(z0 + w, a.Lz) : 0u;
    for (uint32_t r = tid; r < 2u * (uint32_t)a.nbound; r += nthr) tbound[r] = a.Tb[r];
    if (kGrainsInLds)
        for (uint32_t q = tid; q < (uint32_t)a.Q; q += nthr) sB[q] = a.B[q];
    if (tid < 2) qcount[tid] = 0;
    __syncthreads();
    const uint32_t box_n = g.BX * g.BY * g.BZ;
    bool staged = false;
    if constexpr (sizeof(Spin) == 2) {
        if (g.vec) {
            // four spins per 8-byte load: box rows start at a global x that is a
            // multiple of 4 and Lx is a multiple of 4, so a group never wraps
            const uint32_t bx4 = g.BX >> 2, groups = box_n >> 2;
            for (uint32_t e0 = tid; e0 < groups; e0 += kUnroll * nthr) {
                uint64_t v[kUnroll];
#pragma unroll
                for (int j = 0; j < kUnroll; ++j) {
                    const uint32_t e = e0 + j * nthr;
                    const uint32_t ec = e < groups ? e : 0u;
                    const uint32_t r = fdiv(ec, g.m_bx4);
                    const uint32_t u4 = ec - __umul24(r, bx4);
                    const uint32_t w = (D == 3) ? fdiv(r, g.m_by) : 0u;
                    const uint32_t vv = r - __umul24(w, g.BY);
                    v[j] = *reinterpret_cast<const uint64_t*>(src + gxs[4 * u4] + a.Lx * (gys[vv] + a.Ly * gzs[w]));
                }
#pragma unroll
                for (int j = 0; j < kUnroll; ++j) {
                    const uint32_t e = e0 + j * nthr;
                    if (e < groups) *reinterpret_cast<uint64_t*>(box + 4 * e) = v[j];
                }
            }
            staged = true;
        }
    }
    for (uint32_t e0 = tid; !staged && e0 < box_n; e0 += kUnroll * nthr) {
        int32_t v[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const uint32_t e = e0 + j * nthr;
            const uint32_t ec = e < box_n ? e : 0u;
            const uint32_t r = fdiv(ec, g.m_bx);
            const uint32_t u = ec - __umul24(r, g.BX);
            const uint32_t w = (D == 3) ? fdiv(r, g.m_by) : 0u;
            const uint32_t vv = r - __umul24(w, g.BY);
            v[j] = (int32_t)src[gxs[u] + a.Lx * (gys[vv] + a.Ly * gzs[w])];
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const uint32_t e = e0 + j * nthr;
            if (e < box_n) box[e] = (Spin)v[j];
        }
    }
    if constexpr (kField) {
        for (uint32_t e = tid; e < box_n; e += nthr) {
            const uint32_t r = fdiv(e, g.m_bx);
            const uint32_t u = e - __umul24(r, g.BX);
            const uint32_t w = (D == 3) ? fdiv(r, g.m_by) : 0u;
            const uint32_t vv = r - __umul24(w, g.BY);
            fbox[e] = a.fsrc[gxs[u] + a.Lx * (gys[vv] + a.Ly * gzs[w])];
        }
    }
    __syncthreads();

    int off[M];
#pragma unroll
    for (int k = 0; k < M; ++k)
        off[k] = nbr_dx(NBR, k) + nbr_dy(NBR, k) * (int)g.BX + nbr_dz(NBR, k) * (int)(g.BX * g.BY);

    // parities of box coordinate 0 along each axis (global coordinate parity)
    const uint32_t px = (uint32_t)(x0 & 1), py = (uint32_t)(y0 & 1), pz = (uint32_t)(z0 & 1);
    const uint64_t lanes_below = (1ull << lane) - 1ull;

    unsigned long long drawn = 0;   // queued trials of this tile (thread 0; profiling only)
    for (uint32_t pass = 0; pass < g.P; ++pass) {
        const uint32_t gp = a.c0 + pass;   // pass counted from colour 0 of MC step t0
        const uint32_t c = gp % C;
        const uint32_t t = a.t0 + gp / C;
        const uint32_t lo = pass + 1;
        const uint32_t lox = lo + (HX - H);   // the same ring counted from the padded x edge
        const uint32_t loz = (D == 3) ? lo : 0;
        const uint32_t Wx = g.BX - 2 * lox;
        const uint32_t Wy = g.BY - 2 * lo;
        const uint32_t Wz = (D == 3) ? g.BZ - 2 * lo : 1;
        // colour-class enumeration: sites per row, rows per plane, planes
        const uint32_t per_row = Wx / 2;
        const uint32_t rows = kCheckerboard ? Wy : Wy / 2;
        const uint32_t planes = (kCheckerboard || D == 2) ? Wz : Wz / 2;
        const uint32_t total = per_row * rows * planes;
        const uint32_t m_row = g.m_pass[pass][0], m_rows = g.m_pass[pass][1];
        const uint32_t cx = c & 1u, cy = (c >> 1) & 1u, cz = (c >> 2) & 1u;

        // Metropolis trial of one queued site (packed box coordinates).  All
        // reads that do not depend on the random numbers (own spin and grain
        // energy, every neighbour, the site index) are issued before Philox
        // so that their latency overlaps it.
        auto trial = [&](uint32_t packed) __attribute__((always_inline)) {
            const uint32_t u = packed & 1023u, v = (packed >> 10) & 1023u, w = packed >> 20;
            const int idx = (int)(u + __umul24(g.BX, v + __umul24(g.BY, w)));
            const int32_t q = (int32_t)box[idx];
            int32_t nb[M];
#pragma unroll
            for (int k = 0; k < M; ++k) nb[k] = (int32_t)box[idx + off[k]];
            const uint32_t site = gxs[u] + a.Lx * (gys[v] + a.Ly * gzs[w]);
            // A spin outside [0, Q) never moves; it is tested with the
            // proposal below rather than by returning here, which would make
            // the neighbour and coordinate reads wait for q.
            const bool q_ok = (uint32_t)q < (uint32_t)a.Q;
            const int32_t bq = Bq[q_ok ? q : 0];
            const Philox2 r = philox_r01(site, t, c, 0u, a.k0, a.k1);
            int32_t qn;
            int32_t e_new = 0;   // field mode: the swept site's new field
            if (!a.uniform) {
                const uint32_t k = __umulhi(r.r0, (uint32_t)M);
                qn = nb[0];
#pragma unroll
                for (int kk = 1; kk < M; ++kk) qn = (k == (uint32_t)kk) ? nb[kk] : qn;
                if constexpr (kField)
                    e_new = a.frule ? 0 : fbox[idx + nbr_offset<NBR>(k, (int)g.BX, (int)(g.BX * g.BY))];
            } else {
                qn = q + 1 + (int32_t)__umulhi(r.r0, (uint32_t)(a.Q - 1));
                if (qn >= a.Q) qn -= a.Q;
            }
            if (!q_ok || qn == q || (uint32_t)qn >= (uint32_t)a.Q) return;
            if constexpr (kPair) {
                // dE = sum_k (Jp[q'][s_k] - Jp[q][s_k]) + B[q'] - B[q]; a
                // neighbour value outside [0, Q) bonds with nothing
                // (every load at an index valid for any neighbour and masked
                // after, so the 2M loads issue together instead of each pair
                // waiting in a branch of its own)
                const int32_t* Jq = a.Jp + (size_t)q * (uint32_t)a.Q;
                const int32_t* Jn = a.Jp + (size_t)qn * (uint32_t)a.Q;
                int32_t d = Bq[qn] - bq;
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    const int32_t in = -(int32_t)((uint32_t)nb[k] < (uint32_t)a.Q);
                    const int32_t sk = nb[k] & in;
                    d += (Jn[sk] - Jq[sk]) & in;
                }
                if (d <= 0 || r.r1 < a.Tg[min(d, a.Dmax)]) box[idx] = (Spin)qn;
                return;
            }
            int32_t dn;
            if constexpr (sizeof(Spin) == 2 && M % 2 == 0) {
                dn = like_difference16<M>(nb, q, qn);
            } else {
                int cq = 0, cn = 0;
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    cq += (nb[k] == q);
                    cn += (nb[k] == qn);
                }
                dn = cq - cn;
            }
            const int32_t dB = Bq[qn] - bq;
            if constexpr (kField) {
                // per-site field: dE gains e_new - e_i; threshold per d
                const int32_t d = a.J_fx * dn + dB + (e_new - fbox[idx]);
                if (d <= 0 || r.r1 < a.Tg[min(d, a.Dmax)]) {
                    box[idx] = (Spin)qn;
                    fbox[idx] = e_new;
                }
                return;
            }
            const int32_t d = a.J_fx * dn + dB;
            bool accept = d <= 0;
            if (!accept) {
                // T is non-increasing in d: the bucket's bounds decide almost every trial
                const int row = dn - a.dn_lo;
                const uint32_t col = (uint32_t)(dB + a.R);
                const uint32_t bucket = a.m_bw ? __umulhi(col, a.m_bw) : col / a.bw;
                const uint32_t bk = (uint32_t)row * (uint32_t)a.nb + bucket;
                if (r.r1 < tbound[2 * bk]) accept = true;
                else if (r.r1 < tbound[2 * bk + 1]) accept = r.r1 < a.T[row * a.TW + (int)col];
            }
            if (accept) box[idx] = (Spin)qn;
        };

        // Phase 1: enumerate colour c (every lane busy) and queue, through
        // one LDS atomic per wave, the sites that have a neighbour of another
        // spin.  Phase 2: full-width trials over the queue.
        uint32_t* qc = &qcount[pass & 1];
        if constexpr (kSwar) {
            // Checkerboard, 16-bit spins: a lane takes 4 consecutive sites of a
            // row as one 64-bit word, XORs it with its four (six) neighbour
            // words and tests the two colour-c fields.
            // Moore8 and Moore26: a pass takes the rows of one y (and z)
            // parity only, and in them the sites of one x parity
            constexpr bool kRowParity = NBR == HMC_MOORE8 || NBR == HMC_MOORE26;
            const uint32_t s_lo = lox >> 2, s_hi = (g.BX - lox - 1) >> 2;
            const uint32_t nseg = s_hi - s_lo + 1;
            const uint32_t rows_pl = kRowParity ? Wy / 2 : Wy;   // enumerated rows per plane
            const uint32_t totalS = nseg * rows_pl * (kRowParity && D == 3 ? Wz / 2 : Wz);
            const uint32_t plane = g.BX * g.BY;
            const uint32_t pbase = (px + py + pz) & 1u;
            // two words per lane and round: half the rounds, one LDS atomic
            // per wave for all four candidate fields
            for (uint32_t f0 = wave * kWave; f0 < totalS; f0 += 2 * nthr) {
                bool pa[2] = {false, false}, pb[2] = {false, false};
                uint32_t qa[2] = {0u, 0u}, qb[2] = {0u, 0u};
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                const uint32_t f = f0 + j * nthr + lane;
                if (f < totalS) {
                    const uint32_t rr = fdiv(f, m_row);
                    const uint32_t sg = s_lo + (f - __umul24(rr, nseg));
                    const uint32_t pl = (D == 3) ? fdiv(rr, m_rows) : 0u;
                    const uint32_t ri = rr - __umul24(pl, rows_pl);
                    const uint32_t v = kRowParity ? lo + 2 * ri + ((cy ^ (lo + py)) & 1u) : lo + ri;
                    const uint32_t w = (kRowParity && D == 3) ? loz + 2 * pl + ((cz ^ (loz + pz)) & 1u) : loz + pl;
                    const uint32_t row = __umul24(g.BX, v + __umul24(g.BY, w));
                    const uint32_t u0 = 4 * sg;
                    // first colour-c field of the word
                    const uint32_t k = kRowParity ? ((cx ^ px) & 1u) : ((c ^ (v + w + pbase)) & 1u);
                    const uint64_t S = *reinterpret_cast<const uint64_t*>(box + row + u0);
                    uint64_t x;   // per 16-bit field: nonzero where a neighbour differs
                    if (a.uniform) {
                        x = ~0ull;
                    } else if constexpr (kRowParity) {
                        // the word's neighbour sites: the words of the rows
                        // around it (3 in 2D, 9 in 3D), and all of those rows
                        // shifted one site each way.  A colour-c field has one
                        // x neighbour outside the word, before it (k = 0) or
                        // after it (k = 1): one load per row.
                        const uint32_t ue = k ? (u0 + 4 < g.BX ? u0 + 4 : g.BX - 1) : (u0 > 0 ? u0 - 1 : 0);
                        uint32_t fl = 0, fh = 0;
                        const uint32_t sl = (uint32_t)S, sh = (uint32_t)(S >> 32);
                        constexpr int kDz = D == 3 ? 1 : 0;
#pragma unroll
                        for (int dz = -kDz; dz <= kDz; ++dz) {
#pragma unroll
                            for (int dy = -1; dy <= 1; ++dy) {
                                const uint32_t rw = row + (uint32_t)(dy * (int)g.BX + dz * (int)plane);
                                const bool centre = dy == 0 && dz == 0;
                                const uint64_t W = centre ? S : *reinterpret_cast<const uint64_t*>(box + rw + u0);
                                const uint32_t e = (uint16_t)box[rw + ue];
                                const uint32_t wl = (uint32_t)W, wh = (uint32_t)(W >> 32);
                                const uint32_t mid = __builtin_amdgcn_alignbit(wh, wl, 16);   // sites 1, 2
                                fl |= (sl ^ ((wl << 16) | e)) | (sl ^ mid);
                                fh |= (sh ^ mid) | (sh ^ __builtin_amdgcn_alignbit(e, wh, 16));
                                if (!centre) {
                                    fl |= sl ^ wl;
                                    fh |= sh ^ wh;
                                }
                            }
                        }
                        x = ((uint64_t)fh << 32) | fl;
                    } else {
                        const uint64_t Up = *reinterpret_cast<const uint64_t*>(box + row - g.BX + u0);
                        const uint64_t Dn = *reinterpret_cast<const uint64_t*>(box + row + g.BX + u0);
                        const uint32_t sL = (uint16_t)box[row + (u0 > 0 ? u0 - 1 : 0)];
                        const uint32_t sR = (uint16_t)box[row + (u0 + 4 < g.BX ? u0 + 4 : g.BX - 1)];
                        // the word shifted one site each way, as 32-bit halves
                        // (funnel shifts instead of 64-bit shifts)
                        const uint32_t lo = (uint32_t)S, hi = (uint32_t)(S >> 32);
                        const uint32_t mid = __builtin_amdgcn_alignbit(hi, lo, 16);   // sites 1, 2
                        const uint32_t xl = (lo ^ ((lo << 16) | sL)) | (lo ^ mid);
                        const uint32_t xh = (hi ^ mid) | (hi ^ __builtin_amdgcn_alignbit(sR, hi, 16));
                        x = (((uint64_t)xh << 32) | xl) | (S ^ Up) | (S ^ Dn);
                        if (D == 3) {
                            const uint64_t Fr = *reinterpret_cast<const uint64_t*>(box + row - plane + u0);
                            const uint64_t Bk = *reinterpret_cast<const uint64_t*>(box + row + plane + u0);
                            x |= (S ^ Fr) | (S ^ Bk);
                        }
                    }
                    const uint32_t ua = u0 + k, ub = u0 + k + 2;
                    pa[j] = ua >= lox && ua < g.BX - lox && __builtin_amdgcn_ubfe((uint32_t)x, 16 * k, 16) != 0;
                    pb[j] = ub >= lox && ub < g.BX - lox && __builtin_amdgcn_ubfe((uint32_t)(x >> 32), 16 * k, 16) != 0;
                    qa[j] = ua | (v << 10) | (w << 20);
                    qb[j] = ub | (v << 10) | (w << 20);
                }
                }
                const uint64_t ma0 = __ballot(pa[0]), mb0 = __ballot(pb[0]);
                const uint64_t ma1 = __ballot(pa[1]), mb1 = __ballot(pb[1]);
                const uint32_t o1 = (uint32_t)__popcll(ma0);
                const uint32_t o2 = o1 + (uint32_t)__popcll(mb0);
                const uint32_t o3 = o2 + (uint32_t)__popcll(ma1);
                const uint32_t n = o3 + (uint32_t)__popcll(mb1);
                if (n) {
                    uint32_t base = 0;
                    if (lane == 0) base = atomicAdd(qc, n);
                    base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
                    if (pa[0]) queue[base + (uint32_t)__popcll(ma0 & lanes_below)] = qa[0];
                    if (pb[0]) queue[base + o1 + (uint32_t)__popcll(mb0 & lanes_below)] = qb[0];
                    if (pa[1]) queue[base + o2 + (uint32_t)__popcll(ma1 & lanes_below)] = qa[1];
                    if (pb[1]) queue[base + o3 + (uint32_t)__popcll(mb1 & lanes_below)] = qb[1];
                }
            }
        } else {
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
                            const uint32_t par = (lox + v + w + px + py + pz) & 1u;
                            u = lox + 2 * jj + ((c ^ par) & 1u);
                        } else {
                            u = lox + 2 * jj + ((cx ^ (lox + px)) & 1u);
                            v = lo + 2 * ri + ((cy ^ (lo + py)) & 1u);
                            w = (D == 3) ? lo + 2 * pl + ((cz ^ (lo + pz)) & 1u) : 0u;
                        }
                        const uint32_t idx = u + __umul24(g.BX, v + __umul24(g.BY, w));
                        const Spin s = box[idx];
                        bool diff = a.uniform != 0;
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
                        base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
                        if (push[j]) queue[base + (uint32_t)__popcll(mask & lanes_below)] = packed[j];
                    }
                }
            }
        }
        __syncthreads();
        const uint32_t count = *qc;
        if (tid == 0) {
            qcount[(pass + 1) & 1] = 0;
            drawn += count;
        }
        for (uint32_t e0 = tid; e0 < count; e0 += 2 * nthr) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const uint32_t e = e0 + j * nthr;
                if (e < count) trial(queue[e]);
            }
        }
        __syncthreads();
    }

    // one counter update per tile, spread over kTrialSlots addresses
    if (a.trials && tid == 0) atomicAdd(&a.trials[blockIdx.x & (kTrialSlots - 1)], drawn);

    // Interior back to global memory: flat over the tile, coalesced rows.
    const uint32_t tile_n = a.TX * a.TY * a.TZ;
    const uint32_t gx0 = gxs[HX];
    if constexpr (kField) {
        for (uint32_t e = tid; e < tile_n; e += nthr) {
            const uint32_t r = fdiv(e, g.m_tx);
            const uint32_t u = e - __umul24(r, a.TX);
            const uint32_t w = (D == 3) ? fdiv(r, g.m_ty) : 0u;
            const uint32_t vv = r - __umul24(w, a.TY);
            a.fdst[gx0 + u + a.Lx * (gys[H + vv] + a.Ly * gzs[Hz + w])] =
                fbox[(HX + u) + __umul24(g.BX, (H + vv) + __umul24(g.BY, Hz + w))];
        }
    }
    if constexpr (sizeof(Spin) == 2) {
        if (g.vec) {
            const uint32_t tx4 = a.TX >> 2, groups = tile_n >> 2;
            for (uint32_t e = tid; e < groups; e += nthr) {
                const uint32_t r = fdiv(e, g.m_tx4);
                const uint32_t u4 = e - __umul24(r, tx4);
                const uint32_t w = (D == 3) ? fdiv(r, g.m_ty) : 0u;
                const uint32_t vv = r - __umul24(w, a.TY);
                const uint64_t val =
                    *reinterpret_cast<const uint64_t*>(box + (HX + 4 * u4) + __umul24(g.BX, (H + vv) + __umul24(g.BY, Hz + w)));
                *reinterpret_cast<uint64_t*>(dst + gx0 + 4 * u4 + a.Lx * (gys[H + vv] + a.Ly * gzs[Hz + w])) = val;
            }
            return;
        }
    }
    for (uint32_t e = tid; e < tile_n; e += nthr) {
        const uint32_t r = fdiv(e, g.m_tx);
        const uint32_t u = e - __umul24(r, a.TX);
        const uint32_t w = (D == 3) ? fdiv(r, g.m_ty) : 0u;
        const uint32_t vv = r - __umul24(w, a.TY);
        const Spin val = box[(HX + u) + __umul24(g.BX, (H + vv) + __umul24(g.BY, Hz + w))];
        dst[gx0 + u + a.Lx * (gys[H + vv] + a.Ly * gzs[Hz + w])] = val;
    }
}

// One lattice: one workgroup per tile.
template <int NBR, typename Spin, bool kGrainsInLds, bool kSwar, bool kPair, bool kField = false>
__global__ void __launch_bounds__(kThreads) sweep_tile_kernel(LatArgs a, RunArgs g, uint32_t xcd_group) {
    extern __shared__ __align__(16) unsigned char smem[];
    // Consecutive workgroups are spread over the 8 XCDs round-robin; regroup
    // so that each XCD gets a contiguous run of tiles and the halos it reads
    // stay in its own L2.
    uint32_t b = blockIdx.x;
    if (xcd_group) b = (b & 7u) * xcd_group + (b >> 3);
    const uint32_t tx = b % a.ntx;
    const uint32_t ty = (b / a.ntx) % a.nty;
    const uint32_t tz = b / (a.ntx * a.nty);
    process_tile<NBR, Spin, kGrainsInLds, kSwar, kPair, kField>(a, g, tx, ty, tz, smem);
}

// Ensemble: persistent workgroups walk the ragged tile table of all lattices.
// tiles[i] = (lattice, tile index inside that lattice).  Launch j of a call
// advances every lattice from MC step t_base + j*k.
template <int NBR, typename Spin, bool kGrainsInLds, bool kSwar>
__global__ void __launch_bounds__(kThreads)
ensemble_kernel(RunArgs g, const EnsLat* __restrict__ lats, const uint2* __restrict__ tiles, uint32_t ntiles,
                uint32_t j, uint32_t k) {
    extern __shared__ __align__(16) unsigned char smem[];
    for (uint32_t i = blockIdx.x; i < ntiles; i += gridDim.x) {
        const uint2 tl = tiles[i];
        const EnsLat& e = lats[tl.x];
        LatArgs a = e.a;
        const uint32_t sel = (e.cur ^ j) & 1u;
        a.src = e.buf[sel];
        a.dst = e.buf[sel ^ 1u];
        a.t0 = e.t_base + j * k;
        const uint32_t tx = tl.y % a.ntx;
        const uint32_t ty = (tl.y / a.ntx) % a.nty;
        const uint32_t tz = tl.y / (a.ntx * a.nty);
        process_tile<NBR, Spin, kGrainsInLds, kSwar>(a, g, tx, ty, tz, smem);
        __syncthreads();
    }
}

// ----------------------------------------------------------------------
// 16-bit VN4 and Moore8 lattices in TX x TY tiles, K MC steps (K*C colour
// passes) per launch, neighbour trials: the method, random numbers and
// integer acceptance of process_tile with the box geometry fixed at compile
// time, so every index computation is a constant or a shift.  Per pass,
// phase 1 walks the rows of the pass region (Moore8: only those of the
// pass's y parity) in 4-site words from a fixed word column per thread,
// phase 2 runs the trials of the queued sites.  One routine per tile, run by
// a single-lattice kernel (one tile per workgroup) and by a persistent
// ensemble kernel over the tile table of all members.

constexpr size_t align16(size_t b) { return (b + 15) / 16 * 16; }

template <int NBR, int TX, int TY, int K>
struct Geom2D {
    static constexpr int M = Traits<NBR>::M, C = Traits<NBR>::C;
    static constexpr int P = K * C, H = P, HX = (P + 3) & ~3;
    static constexpr int BX = TX + 2 * HX, BY = TY + 2 * H, NBOX = BX * BY, NW = BX / 4;
    static constexpr int NWORDS = NBOX / 4, PRE = (NWORDS + kThreads - 1) / kThreads;
    // the colour class of the first (largest) pass region
    static constexpr int QCAP = (BX - 2 * (1 + HX - H)) * (BY - 2) / C + 1;
    static constexpr size_t kBoundOff = 0;                                  // uint32[2 * kBoundPairs]
    static constexpr size_t kCountOff = 8 * (size_t)kBoundPairs;            // uint32[2]
    static constexpr size_t kOffsetOff = kCountOff + 16;                    // int32[8]: neighbour offsets
    static constexpr size_t kGxOff = kOffsetOff + 32;                       // uint32[BX]
    static constexpr size_t kRowOff = kGxOff + align16(4 * (size_t)BX);     // uint32[BY]
    static constexpr size_t kBoxOff = kRowOff + align16(4 * (size_t)BY);    // int16[NBOX]
    static constexpr size_t kQueueOff = kBoxOff + align16(2 * (size_t)NBOX);
    static constexpr size_t kGrainOff = kQueueOff + align16(4 * (size_t)QCAP);   // int32[Q] (grains in LDS)
    static_assert(NBR == HMC_VN4 || NBR == HMC_MOORE8, "2D neighbourhoods");
    static_assert(TX % 4 == 0 && HX >= H, "tile and halo");
    static_assert(NBOX < 65536 && BY < 65536, "queue entries pack the box index and row in 16 bits each");
};

// Box offsets of the neighbours in LDS, written once per workgroup before
// its first tile (read by the trials after the tile's first barrier).
template <int NBR, int TX, int TY, int K>
__device__ __forceinline__ void init_offsets2d(unsigned char* smem) {
    using G = Geom2D<NBR, TX, TY, K>;
    constexpr int BX = G::BX;
    int32_t* noff = reinterpret_cast<int32_t*>(smem + G::kOffsetOff);
    const uint32_t tid = threadIdx.x;
    if (tid < (uint32_t)G::M) {   // neighbour k: +x -x +y -y (+1,+1) (-1,-1) (+1,-1) (-1,+1)
        const int sgn = (tid & 1u) ? -1 : 1;
        noff[tid] = tid < 2 ? sgn : (tid < 4 ? sgn * BX : (tid < 6 ? sgn * (1 + BX) : sgn * (1 - BX)));
    }
}

// One tile of lattice a (MC step t0 at its first pass, colour 0), box from
// src, interior to dst.  Ends past its last LDS access of the tile.
template <int NBR, int TX, int TY, int K, bool kGrainsInLds>
__device__ __forceinline__ void tile2d(const LatArgs& a, const int16_t* __restrict__ src, int16_t* __restrict__ dst,
                                       uint32_t t0, uint32_t tx, uint32_t ty, unsigned char* smem) {
    using G = Geom2D<NBR, TX, TY, K>;
    constexpr int BX = G::BX, BY = G::BY, NW = G::NW, H = G::H, HX = G::HX, P = G::P, M = G::M, C = G::C;
    constexpr bool kMoore = NBR == HMC_MOORE8;
    constexpr int kTrialUnroll = 2;   // trials in flight per thread
    uint32_t* tbound = reinterpret_cast<uint32_t*>(smem + G::kBoundOff);
    uint32_t* qcount = reinterpret_cast<uint32_t*>(smem + G::kCountOff);
    int32_t* noff = reinterpret_cast<int32_t*>(smem + G::kOffsetOff);
    uint32_t* gx = reinterpret_cast<uint32_t*>(smem + G::kGxOff);
    uint32_t* rowL = reinterpret_cast<uint32_t*>(smem + G::kRowOff);
    int16_t* box = reinterpret_cast<int16_t*>(smem + G::kBoxOff);
    uint64_t* boxw = reinterpret_cast<uint64_t*>(smem + G::kBoxOff);
    uint32_t* queue = reinterpret_cast<uint32_t*>(smem + G::kQueueOff);
    int32_t* sB = reinterpret_cast<int32_t*>(smem + G::kGrainOff);

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint64_t lanes_below = (1ull << lane) - 1ull;
    const uint32_t Lx = a.Lx, Ly = a.Ly;
    const int32_t x0 = (int32_t)(tx * TX) - HX, y0 = (int32_t)(ty * TY) - H;
    const int32_t* __restrict__ Bq = kGrainsInLds ? sB : a.B;
    for (uint32_t u = tid; u < (uint32_t)BX; u += kThreads) gx[u] = wrap_coord(x0 + (int32_t)u, Lx);
    for (uint32_t v = tid; v < (uint32_t)BY; v += kThreads) rowL[v] = Lx * wrap_coord(y0 + (int32_t)v, Ly);
    for (uint32_t r = tid; r < 2u * (uint32_t)a.nbound; r += kThreads) tbound[r] = a.Tb[r];
    if constexpr (kGrainsInLds)
        for (uint32_t q = tid; q < (uint32_t)a.Q; q += kThreads) sB[q] = a.B[q];
    if (tid < 2) qcount[tid] = 0;
    __syncthreads();
    {   // the box, four spins per 8-byte access (rows start at a multiple of 4)
        uint64_t w[G::PRE];
#pragma unroll
        for (int q = 0; q < G::PRE; ++q) {
            const uint32_t e2 = tid + (uint32_t)q * kThreads;
            const uint32_t ec = e2 < (uint32_t)G::NWORDS ? e2 : 0u;
            const uint32_t r = ec / NW, u4 = ec - r * NW;
            w[q] = *reinterpret_cast<const uint64_t*>(src + gx[4 * u4] + rowL[r]);
        }
#pragma unroll
        for (int q = 0; q < G::PRE; ++q) {
            const uint32_t e2 = tid + (uint32_t)q * kThreads;
            if (e2 < (uint32_t)G::NWORDS) boxw[e2] = w[q];
        }
    }
    __syncthreads();

    const uint32_t px = (uint32_t)x0 & 1u, py = (uint32_t)y0 & 1u;   // colour parity of box column/row 0
    unsigned long long drawn = 0;
    for (int p = 0; p < P; ++p) {
        const uint32_t c = (uint32_t)p % C, t = t0 + (uint32_t)p / C;
        const uint32_t R = (uint32_t)p + 1u;           // ring: the pass region is R sites inside the box
        const uint32_t lox = R + (uint32_t)(HX - H);
        const uint32_t s_lo = lox >> 2, s_hi = ((uint32_t)BX - lox - 1u) >> 2, nseg = s_hi - s_lo + 1u;
        // rows of the pass region (Moore8: of the pass's y parity only)
        const uint32_t nrows = kMoore ? ((uint32_t)BY - 2u * R) / 2u : (uint32_t)BY - 2u * R;
        const uint32_t vpar = kMoore ? ((c >> 1) ^ (R + py)) & 1u : 0u;
        const uint32_t rpi = kThreads / nseg;
        const uint32_t sg = s_lo + tid % nseg, i0 = tid / nseg;
        const bool tact = tid < rpi * nseg;
        const uint32_t u0 = 4 * sg;
        // first colour-c field of a word: Moore8 x & 1 = c & 1 (the same in
        // every row of the pass), VN4 (x + y) & 1 = c (alternating by row)
        const uint32_t kf0 = kMoore ? ((c ^ px) & 1u) : ((c ^ (R + px + py)) & 1u);
        // a colour-c field has one x neighbour outside the word: before it
        // (first field 0) or after it (first field 1)
        const uint32_t ue0 = kf0 ? (u0 + 4 < (uint32_t)BX ? u0 + 4 : (uint32_t)BX - 1) : (sg > 0 ? u0 - 1 : 0u);
        const uint32_t ue1 = kf0 ? (sg > 0 ? u0 - 1 : 0u) : (u0 + 4 < (uint32_t)BX ? u0 + 4 : (uint32_t)BX - 1);
        const uint32_t ua0 = u0 + kf0, ua1 = u0 + (kf0 ^ 1u);
        const bool oka0 = ua0 >= lox && ua0 < (uint32_t)BX - lox, okb0 = ua0 + 2 >= lox && ua0 + 2 < (uint32_t)BX - lox;
        const bool oka1 = ua1 >= lox && ua1 < (uint32_t)BX - lox, okb1 = ua1 + 2 >= lox && ua1 + 2 < (uint32_t)BX - lox;
        uint32_t* qc = &qcount[p & 1];
        const uint32_t iters = (nrows + rpi - 1) / rpi;
        for (uint32_t it = 0; it < iters; ++it) {
            const uint32_t ir = i0 + it * rpi;
            bool pa = false, pb = false;
            uint32_t ea = 0, eb = 0;
            if (tact && ir < nrows) {
                const uint32_t v = kMoore ? R + 2 * ir + vpar : R + ir;
                const bool odd = !kMoore && (ir & 1u);   // VN4: every other row has the other first field
                const uint32_t kf = odd ? kf0 ^ 1u : kf0;
                const uint32_t ue = odd ? ue1 : ue0;
                const uint32_t ua = odd ? ua1 : ua0;
                const bool oka = odd ? oka1 : oka0, okb = odd ? okb1 : okb0;
                const uint32_t wi = v * NW + sg;
                const uint64_t S = boxw[wi];
                const uint32_t sl = (uint32_t)S, sh = (uint32_t)(S >> 32);
                uint32_t fl = 0, fh = 0;
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy) {
                    const uint64_t W = dy == 0 ? S : boxw[wi + dy * NW];
                    const uint32_t wl = (uint32_t)W, wh = (uint32_t)(W >> 32);
                    if (dy == 0 || kMoore) {   // the row shifted one site each way
                        const uint32_t ev = (uint16_t)box[(v + dy) * BX + ue];
                        const uint32_t mid = __builtin_amdgcn_alignbit(wh, wl, 16);   // sites 1, 2
                        fl |= (sl ^ ((wl << 16) | ev)) | (sl ^ mid);
                        fh |= (sh ^ mid) | (sh ^ __builtin_amdgcn_alignbit(ev, wh, 16));
                    }
                    if (dy != 0) {
                        fl |= sl ^ wl;
                        fh |= sh ^ wh;
                    }
                }
                pa = oka && __builtin_amdgcn_ubfe(fl, 16 * kf, 16) != 0;
                pb = okb && __builtin_amdgcn_ubfe(fh, 16 * kf, 16) != 0;
                ea = (v * BX + ua) | (v << 16);
                eb = ea + 2;
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
        }
        __syncthreads();
        const uint32_t count = *qc;
        if (tid == 0) {
            qcount[(p + 1) & 1] = 0;
            drawn += count;
        }
        auto trial = [&](uint32_t en) __attribute__((always_inline)) {
            const uint32_t idx = en & 0xFFFFu, row = en >> 16;
            const uint32_t u = idx - row * BX;
            const int32_t q = box[idx];
            int32_t nb[M];
            nb[0] = box[idx + 1];
            nb[1] = box[idx - 1];
            nb[2] = box[idx + BX];
            nb[3] = box[idx - BX];
            if constexpr (M == 8) {
                nb[4] = box[idx + 1 + BX];
                nb[5] = box[idx - 1 - BX];
                nb[6] = box[idx + 1 - BX];
                nb[7] = box[idx - 1 + BX];
            }
            const uint32_t site = gx[u] + rowL[row];
            const bool q_ok = (uint32_t)q < (uint32_t)a.Q;   // a value outside [0, Q) never moves
            const int32_t bq = Bq[q_ok ? q : 0];
            const Philox2 r = philox_r01(site, t, c, 0u, a.k0, a.k1);
            const uint32_t kk = __umulhi(r.r0, (uint32_t)M);
            const int32_t qn = box[(int32_t)idx + noff[kk]];
            if (!q_ok || qn == q || (uint32_t)qn >= (uint32_t)a.Q) return;
            const int32_t dn = like_difference16<M>(nb, q, qn);
            const int32_t dB = Bq[qn] - bq;
            const int32_t d = a.J_fx * dn + dB;
            bool accept = d <= 0;
            if (!accept) {
                // T is non-increasing in d: the bucket's bounds decide almost every trial
                const int rowT = dn - a.dn_lo;
                const uint32_t col = (uint32_t)(dB + a.R);
                const uint32_t bucket = a.m_bw ? __umulhi(col, a.m_bw) : col / a.bw;
                const uint32_t bk = (uint32_t)rowT * (uint32_t)a.nb + bucket;
                if (r.r1 < tbound[2 * bk]) accept = true;
                else if (r.r1 < tbound[2 * bk + 1]) accept = r.r1 < a.T[rowT * a.TW + (int)col];
            }
            if (accept) box[idx] = (int16_t)qn;
        };
        for (uint32_t e0 = tid; e0 < count; e0 += kTrialUnroll * kThreads) {
#pragma unroll
            for (int q2 = 0; q2 < kTrialUnroll; ++q2) {
                const uint32_t en = e0 + q2 * kThreads;
                if (en < count) trial(queue[en]);
            }
        }
        __syncthreads();
    }
    if (a.trials && tid == 0) atomicAdd(&a.trials[blockIdx.x & (kTrialSlots - 1)], drawn);
    // the tile back to global memory, 8-byte words
    constexpr int TW4 = TX / 4;
    const uint32_t gx0 = gx[HX];
    for (uint32_t e2 = tid; e2 < (uint32_t)(TW4 * TY); e2 += kThreads) {
        const uint32_t vv = e2 / TW4, u4 = e2 - vv * TW4;
        const uint64_t val = boxw[(H + vv) * NW + HX / 4 + u4];
        *reinterpret_cast<uint64_t*>(dst + gx0 + 4 * u4 + rowL[H + vv]) = val;
    }
}

// One lattice, one tile per workgroup (XCD-grouped like sweep_tile_kernel).
template <int NBR, int TX, int TY, int K, bool kGrainsInLds>
__global__ void __launch_bounds__(kThreads) lat2d_kernel(LatArgs a, uint32_t xcd_group) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t b = blockIdx.x;
    if (xcd_group) b = (b & 7u) * xcd_group + (b >> 3);
    init_offsets2d<NBR, TX, TY, K>(smem);
    tile2d<NBR, TX, TY, K, kGrainsInLds>(a, static_cast<const int16_t*>(a.src), static_cast<int16_t*>(a.dst), a.t0,
                                    b % a.ntx, b / a.ntx, smem);
}

// Ensembles: persistent workgroups walk the tile table of all members.  Built
// for eight waves per SIMD (scalar registers held under 100, a few of them
// kept in vector lanes) so that two workgroups share a CU whenever their LDS
// fits: one issues while the other waits at a barrier or on LDS.
template <int NBR, int TX, int TY, int K, bool kGrainsInLds>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8)))
ens2d_kernel(const EnsLat* __restrict__ lats, const uint2* __restrict__ tiles, uint32_t ntiles, uint32_t j,
             uint32_t k) {
    extern __shared__ __align__(16) unsigned char smem[];
    init_offsets2d<NBR, TX, TY, K>(smem);
    for (uint32_t i = blockIdx.x; i < ntiles; i += gridDim.x) {
        const uint2 tl = tiles[i];
        const EnsLat& e = lats[tl.x];
        const uint32_t sel = (e.cur ^ j) & 1u;
        tile2d<NBR, TX, TY, K, kGrainsInLds>(e.a, static_cast<const int16_t*>(e.buf[sel]),
                                        static_cast<int16_t*>(e.buf[sel ^ 1u]), e.t_base + j * k,
                                        tl.y % e.a.ntx, tl.y / e.a.ntx, smem);
        __syncthreads();
    }
}

// ----------------------------------------------------------------------
// 16-bit Moore26 lattices (eight colours) in TX x TY x TZ tiles, P colour
// passes per launch starting at any colour, neighbour trials: the method,
// random numbers and integer acceptance of process_tile with the box
// geometry and the 26 neighbour offsets fixed at compile time.  A pass walks
// the box rows of its (y, z) parity in 4-site words from a fixed word column
// per thread; a word is compared with the nine rows around it, each also
// shifted one site each way, and its two fields of the pass's x parity are
// queued when a neighbour differs.  One tile per workgroup.

template <int TX, int TY, int TZ, int P>
struct Geom26 {
    static constexpr int M = 26, C = 8, H = P, HX = (P + 3) & ~3;
    static constexpr int BX = TX + 2 * HX, BY = TY + 2 * H, BZ = TZ + 2 * H, BXY = BX * BY, NBOX = BXY * BZ;
    static constexpr int NW = BX / 4, NROWS = BY * BZ, NWORDS = NW * NROWS;
    static constexpr int PRE = (NWORDS + kThreads - 1) / kThreads;
    // the colour class of the first (largest) pass region: an eighth of it
    static constexpr int QCAP = (BX - 2 * (1 + HX - H)) * (BY - 2) * (BZ - 2) / C + 1;
    static constexpr size_t kBoundOff = 0;                                  // uint32[2 * kBoundPairs]
    static constexpr size_t kCountOff = 8 * (size_t)kBoundPairs;            // uint32[2]
    static constexpr size_t kOffsetOff = kCountOff + 16;                    // int32[26]: neighbour offsets
    static constexpr size_t kGxOff = kOffsetOff + 128;                      // uint32[BX]
    static constexpr size_t kRowOff = kGxOff + align16(4 * (size_t)BX);     // uint32[NROWS]
    static constexpr size_t kBoxOff = kRowOff + align16(4 * (size_t)NROWS); // int16[NBOX]
    static constexpr size_t kQueueOff = kBoxOff + align16(2 * (size_t)NBOX);
    static constexpr size_t kGrainOff = kQueueOff + align16(4 * (size_t)QCAP);   // int32[Q] (grains in LDS)
    static_assert(TX % 4 == 0 && HX >= H && P <= 8, "tile and halo");
    static_assert(NBOX < 65536 && NROWS < 65536, "queue entries pack the box index and row in 16 bits each");
};

template <int TX, int TY, int TZ, int P, bool kGrainsInLds>
__global__ void __launch_bounds__(kThreads) lat26_kernel(LatArgs a, uint32_t xcd_group) {
    using G = Geom26<TX, TY, TZ, P>;
    constexpr int BX = G::BX, BY = G::BY, BXY = G::BXY, NW = G::NW, H = G::H, HX = G::HX;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* tbound = reinterpret_cast<uint32_t*>(smem + G::kBoundOff);
    uint32_t* qcount = reinterpret_cast<uint32_t*>(smem + G::kCountOff);
    int32_t* noff = reinterpret_cast<int32_t*>(smem + G::kOffsetOff);
    uint32_t* gx = reinterpret_cast<uint32_t*>(smem + G::kGxOff);
    uint32_t* rowL = reinterpret_cast<uint32_t*>(smem + G::kRowOff);
    int16_t* box = reinterpret_cast<int16_t*>(smem + G::kBoxOff);
    uint64_t* boxw = reinterpret_cast<uint64_t*>(smem + G::kBoxOff);
    uint32_t* queue = reinterpret_cast<uint32_t*>(smem + G::kQueueOff);
    int32_t* sB = reinterpret_cast<int32_t*>(smem + G::kGrainOff);
    const int16_t* __restrict__ src = static_cast<const int16_t*>(a.src);
    int16_t* __restrict__ dst = static_cast<int16_t*>(a.dst);
    const int32_t* __restrict__ Bq = kGrainsInLds ? sB : a.B;

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint64_t lanes_below = (1ull << lane) - 1ull;
    uint32_t b = blockIdx.x;
    if (xcd_group) b = (b & 7u) * xcd_group + (b >> 3);
    const uint32_t tx = b % a.ntx, ty = (b / a.ntx) % a.nty, tz = b / (a.ntx * a.nty);
    const int32_t x0 = (int32_t)(tx * TX) - HX, y0 = (int32_t)(ty * TY) - H, z0 = (int32_t)(tz * TZ) - H;

    if (tid < 26u) {   // box offset of neighbour k in the trial order
        const int k = (int)tid;
        noff[tid] = nbr_dx(HMC_MOORE26, k) + nbr_dy(HMC_MOORE26, k) * BX + nbr_dz(HMC_MOORE26, k) * BXY;
    }
    for (uint32_t u = tid; u < (uint32_t)BX; u += kThreads) gx[u] = wrap_coord(x0 + (int32_t)u, a.Lx);
    for (uint32_t r = tid; r < (uint32_t)G::NROWS; r += kThreads) {
        const uint32_t v = r % BY, w = r / BY;
        rowL[r] = a.Lx * (wrap_coord(y0 + (int32_t)v, a.Ly) + a.Ly * wrap_coord(z0 + (int32_t)w, a.Lz));
    }
    for (uint32_t r = tid; r < 2u * (uint32_t)a.nbound; r += kThreads) tbound[r] = a.Tb[r];
    if constexpr (kGrainsInLds)
        for (uint32_t q = tid; q < (uint32_t)a.Q; q += kThreads) sB[q] = a.B[q];
    if (tid < 2) qcount[tid] = 0;
    __syncthreads();
    {   // the box, four spins per 8-byte access (rows start at a multiple of 4)
        uint64_t wv[G::PRE];
#pragma unroll
        for (int q = 0; q < G::PRE; ++q) {
            const uint32_t e2 = tid + (uint32_t)q * kThreads;
            const uint32_t ec = e2 < (uint32_t)G::NWORDS ? e2 : 0u;
            const uint32_t r = ec / NW, u4 = ec - r * NW;
            wv[q] = *reinterpret_cast<const uint64_t*>(src + gx[4 * u4] + rowL[r]);
        }
#pragma unroll
        for (int q = 0; q < G::PRE; ++q) {
            const uint32_t e2 = tid + (uint32_t)q * kThreads;
            if (e2 < (uint32_t)G::NWORDS) boxw[e2] = wv[q];
        }
    }
    __syncthreads();

    // colour parity of box column, row and plane 0
    const uint32_t px = (uint32_t)x0 & 1u, py = (uint32_t)y0 & 1u, pz = (uint32_t)z0 & 1u;
    unsigned long long drawn = 0;
    for (int p = 0; p < P; ++p) {
        const uint32_t gp = a.c0 + (uint32_t)p;   // pass counted from colour 0 of MC step t0
        const uint32_t c = gp & 7u, t = a.t0 + (gp >> 3);
        const uint32_t cx = c & 1u, cy = (c >> 1) & 1u, cz = c >> 2;
        const uint32_t R = (uint32_t)p + 1u;           // ring: the pass region is R sites inside the box
        const uint32_t lox = R + (uint32_t)(HX - H);
        const uint32_t s_lo = lox >> 2, s_hi = ((uint32_t)BX - lox - 1u) >> 2, nseg = s_hi - s_lo + 1u;
        // rows of the pass's y and z parity
        const uint32_t ny = ((uint32_t)BY - 2u * R) / 2u, nz = ((uint32_t)G::BZ - 2u * R) / 2u, nrows = ny * nz;
        const uint32_t m_ny = magic(ny);
        const uint32_t vpar = (cy ^ (R + py)) & 1u, wpar = (cz ^ (R + pz)) & 1u;
        const uint32_t rpi = kThreads / nseg;
        const uint32_t sg = s_lo + tid % nseg, i0 = tid / nseg;
        const bool tact = tid < rpi * nseg;
        const uint32_t u0 = 4 * sg;
        const uint32_t kf = (cx ^ px) & 1u;   // first field of the pass's x parity in a word
        // a field of that parity has one x neighbour outside the word: before
        // it (first field 0) or after it (first field 1)
        const uint32_t ue = kf ? (u0 + 4 < (uint32_t)BX ? u0 + 4 : (uint32_t)BX - 1) : (sg > 0 ? u0 - 1 : 0u);
        const uint32_t ua = u0 + kf;
        const bool oka = ua >= lox && ua < (uint32_t)BX - lox, okb = ua + 2 >= lox && ua + 2 < (uint32_t)BX - lox;
        uint32_t* qc = &qcount[p & 1];
        const uint32_t iters = (nrows + rpi - 1) / rpi;
        for (uint32_t it = 0; it < iters; ++it) {
            const uint32_t ir = i0 + it * rpi;
            bool pa = false, pb = false;
            uint32_t ea = 0;
            if (tact && ir < nrows) {
                const uint32_t iz = fdiv(ir, m_ny), iy = ir - iz * ny;
                const uint32_t row = (R + 2 * iy + vpar) + (uint32_t)BY * (R + 2 * iz + wpar);
                const uint32_t wi = row * NW + sg;
                const uint64_t S = boxw[wi];
                const uint32_t sl = (uint32_t)S, sh = (uint32_t)(S >> 32);
                uint32_t fl = 0, fh = 0;
#pragma unroll
                for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
                    for (int dy = -1; dy <= 1; ++dy) {
                        const bool centre = dy == 0 && dz == 0;
                        const int dr = dy + dz * BY;
                        const uint64_t W = centre ? S : boxw[(int)wi + dr * NW];
                        const uint32_t ev = (uint16_t)box[((int)row + dr) * BX + (int)ue];
                        const uint32_t wl = (uint32_t)W, wh = (uint32_t)(W >> 32);
                        const uint32_t mid = __builtin_amdgcn_alignbit(wh, wl, 16);   // sites 1, 2
                        fl |= (sl ^ ((wl << 16) | ev)) | (sl ^ mid);
                        fh |= (sh ^ mid) | (sh ^ __builtin_amdgcn_alignbit(ev, wh, 16));
                        if (!centre) {
                            fl |= sl ^ wl;
                            fh |= sh ^ wh;
                        }
                    }
                }
                pa = oka && __builtin_amdgcn_ubfe(fl, 16 * kf, 16) != 0;
                pb = okb && __builtin_amdgcn_ubfe(fh, 16 * kf, 16) != 0;
                ea = (row * BX + ua) | (row << 16);
            }
            const uint64_t ma = __ballot(pa), mb = __ballot(pb);
            const uint32_t na = (uint32_t)__popcll(ma);
            const uint32_t n = na + (uint32_t)__popcll(mb);
            if (n) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(qc, n);
                base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
                if (pa) queue[base + (uint32_t)__popcll(ma & lanes_below)] = ea;
                if (pb) queue[base + na + (uint32_t)__popcll(mb & lanes_below)] = ea + 2;
            }
        }
        __syncthreads();
        const uint32_t count = *qc;
        if (tid == 0) {
            qcount[(p + 1) & 1] = 0;
            drawn += count;
        }
        auto trial = [&](uint32_t en) __attribute__((always_inline)) {
            const uint32_t idx = en & 0xFFFFu, row = en >> 16;
            const uint32_t u = idx - row * BX;
            const int32_t q = box[idx];
            int32_t nb[26];
#pragma unroll
            for (int k = 0; k < 26; ++k)
                nb[k] = box[(int)idx + nbr_dx(HMC_MOORE26, k) + nbr_dy(HMC_MOORE26, k) * BX +
                            nbr_dz(HMC_MOORE26, k) * BXY];
            const uint32_t site = gx[u] + rowL[row];
            const bool q_ok = (uint32_t)q < (uint32_t)a.Q;   // a value outside [0, Q) never moves
            const int32_t bq = Bq[q_ok ? q : 0];
            const Philox2 r = philox_r01(site, t, c, 0u, a.k0, a.k1);
            const uint32_t kk = __umulhi(r.r0, 26u);
            const int32_t qn = box[(int32_t)idx + noff[kk]];
            if (!q_ok || qn == q || (uint32_t)qn >= (uint32_t)a.Q) return;
            const int32_t dn = like_difference16<26>(nb, q, qn);
            const int32_t dB = Bq[qn] - bq;
            const int32_t d = a.J_fx * dn + dB;
            bool accept = d <= 0;
            if (!accept) {
                // T is non-increasing in d: the bucket's bounds decide almost every trial
                const int rowT = dn - a.dn_lo;
                const uint32_t col = (uint32_t)(dB + a.R);
                const uint32_t bucket = a.m_bw ? __umulhi(col, a.m_bw) : col / a.bw;
                const uint32_t bk = (uint32_t)rowT * (uint32_t)a.nb + bucket;
                if (r.r1 < tbound[2 * bk]) accept = true;
                else if (r.r1 < tbound[2 * bk + 1]) accept = r.r1 < a.T[rowT * a.TW + (int)col];
            }
            if (accept) box[idx] = (int16_t)qn;
        };
        for (uint32_t e0 = tid; e0 < count; e0 += 2 * kThreads) {
#pragma unroll
            for (int q2 = 0; q2 < 2; ++q2) {
                const uint32_t en = e0 + q2 * kThreads;
                if (en < count) trial(queue[en]);
            }
        }
        __syncthreads();
    }
    if (a.trials && tid == 0) atomicAdd(&a.trials[blockIdx.x & (kTrialSlots - 1)], drawn);
    // the tile back to global memory, 8-byte words
    constexpr int TW4 = TX / 4;
    const uint32_t gx0 = gx[HX];
    for (uint32_t e2 = tid; e2 < (uint32_t)(TW4 * TY * TZ); e2 += kThreads) {
        const uint32_t u4 = e2 % TW4, rr = e2 / TW4;
        const uint32_t vv = rr % TY, ww = rr / TY;
        const uint32_t brow = (H + vv) + BY * (H + ww);
        const uint64_t val = boxw[brow * NW + HX / 4 + u4];
        *reinterpret_cast<uint64_t*>(dst + gx0 + 4 * u4 + rowL[brow]) = val;
    }
}

template <int TX, int TY, int TZ, int P>
const void* pick26(int32_t maxQ, size_t* bytes) {
    using G = Geom26<TX, TY, TZ, P>;
    const int64_t limit = lds_limit_bytes();
    const bool lds = maxQ <= kLdsGrainLimit && (int64_t)(G::kGrainOff + 4 * (size_t)maxQ) <= limit;
    if (!lds && (int64_t)G::kGrainOff > limit) return nullptr;
    *bytes = G::kGrainOff + (lds ? 4 * (size_t)maxQ : 0);
    return lds ? reinterpret_cast<const void*>(&lat26_kernel<TX, TY, TZ, P, true>)
               : reinterpret_cast<const void*>(&lat26_kernel<TX, TY, TZ, P, false>);
}

// The compiled 2D kernel (single lattice or ensemble) for neighbourhood nbr
// and tiling t, and its LDS bytes, or null when there is none for t: Moore8
// 128x128 tiles with 3 MC steps per launch, and single VN4 lattices in
// 128x128 tiles with 6.  Against the general kernel on the same tiles (site
// updates/s): Moore8 2048^2 2.68 -> 3.08e11, 8192^2 3.00 -> 3.35e11, the
// 64-member ensemble of 29 M sites 2.94e11 either way; VN4 2048^2 4.23 ->
// 4.36e11.  VN4 64x64 tiles (1024^2: 2.17 -> 2.07e11) and VN4 ensembles
// (3.76 -> 3.71e11) stay with the general kernel.
template <int NBR, int TX, int TY, int K, bool kEnsemble>
const void* pick2d(int32_t maxQ, size_t* bytes) {
    using G = Geom2D<NBR, TX, TY, K>;
    const int64_t limit = lds_limit_bytes();
    // ensembles keep the grain energies in LDS only while two workgroups
    // still fit a CU (64 Moore8 members up to 2000 grains: 2.94 -> 3.82e11
    // site updates/s with them read through the caches instead)
    const int64_t fit = kEnsemble && 2 * (int64_t)G::kGrainOff <= limit ? limit / 2 : limit;
    const bool lds = maxQ <= kLdsGrainLimit && (int64_t)(G::kGrainOff + 4 * (size_t)maxQ) <= fit;
    if (!lds && (int64_t)G::kGrainOff > limit) return nullptr;
    *bytes = G::kGrainOff + (lds ? 4 * (size_t)maxQ : 0);
    if constexpr (kEnsemble)
        return lds ? reinterpret_cast<const void*>(&ens2d_kernel<NBR, TX, TY, K, true>)
                   : reinterpret_cast<const void*>(&ens2d_kernel<NBR, TX, TY, K, false>);
    return lds ? reinterpret_cast<const void*>(&lat2d_kernel<NBR, TX, TY, K, true>)
               : reinterpret_cast<const void*>(&lat2d_kernel<NBR, TX, TY, K, false>);
}

const void* compiled2d_for(int nbr, const Tiling& t, bool ensemble, int32_t maxQ, size_t* bytes) {
    if (nbr == HMC_MOORE26) {   // single lattices, 32x16x16 tiles, two or four colour passes
        if (ensemble || t.tx != 32 || t.ty != 16 || t.tz != 16) return nullptr;
        if (t.k == -2) return pick26<32, 16, 16, 2>(maxQ, bytes);
        if (t.k == -4) return pick26<32, 16, 16, 4>(maxQ, bytes);
        return nullptr;
    }
    if (t.tz != 1 && t.tz != 0) return nullptr;
    const bool t128 = t.tx == 128 && t.ty == 128, t256 = t.tx == 256 && t.ty == 128;
    if (nbr == HMC_MOORE8 && t.k == 3 && t128)
        return ensemble ? pick2d<HMC_MOORE8, 128, 128, 3, true>(maxQ, bytes)
                        : pick2d<HMC_MOORE8, 128, 128, 3, false>(maxQ, bytes);
    if (nbr == HMC_MOORE8 && t.k == 3 && t256)
        return ensemble ? pick2d<HMC_MOORE8, 256, 128, 3, true>(maxQ, bytes)
                        : pick2d<HMC_MOORE8, 256, 128, 3, false>(maxQ, bytes);
    if (nbr == HMC_VN4 && t.k == 6 && t128 && !ensemble) return pick2d<HMC_VN4, 128, 128, 6, false>(maxQ, bytes);
    if (nbr == HMC_VN4 && t.k == 4 && t256 && !ensemble) return pick2d<HMC_VN4, 256, 128, 4, false>(maxQ, bytes);
    return nullptr;
}

template <int NBR, bool kSwar>
const void* kernel_for(int spin, bool grains_in_lds, bool ensemble, bool pair, bool field) {
    if (ensemble) {
        if (pair || field) return nullptr;
        if (spin == HMC_I16)
            return grains_in_lds ? reinterpret_cast<const void*>(&ensemble_kernel<NBR, int16_t, true, kSwar>)
                                 : reinterpret_cast<const void*>(&ensemble_kernel<NBR, int16_t, false, kSwar>);
        return grains_in_lds ? reinterpret_cast<const void*>(&ensemble_kernel<NBR, int32_t, true, false>)
                             : reinterpret_cast<const void*>(&ensemble_kernel<NBR, int32_t, false, false>);
    }
    if (field) {   // per-site bulk field
        if (spin == HMC_I16)
            return grains_in_lds ? reinterpret_cast<const void*>(&sweep_tile_kernel<NBR, int16_t, true, kSwar, false, true>)
                                 : reinterpret_cast<const void*>(&sweep_tile_kernel<NBR, int16_t, false, kSwar, false, true>);
        return grains_in_lds ? reinterpret_cast<const void*>(&sweep_tile_kernel<NBR, int32_t, true, false, false, true>)
                             : reinterpret_cast<const void*>(&sweep_tile_kernel<NBR, int32_t, false, false, false, true>);
    }
    if (pair)   // bond energies from the pair table; grain energies read from global memory
        return spin == HMC_I16 ? reinterpret_cast<const void*>(&sweep_tile_kernel<NBR, int16_t, false, kSwar, true>)
                               : reinterpret_cast<const void*>(&sweep_tile_kernel<NBR, int32_t, false, false, true>);
    if (spin == HMC_I16)
        return grains_in_lds ? reinterpret_cast<const void*>(&sweep_tile_kernel<NBR, int16_t, true, kSwar, false>)
                             : reinterpret_cast<const void*>(&sweep_tile_kernel<NBR, int16_t, false, kSwar, false>);
    return grains_in_lds ? reinterpret_cast<const void*>(&sweep_tile_kernel<NBR, int32_t, true, false, false>)
                         : reinterpret_cast<const void*>(&sweep_tile_kernel<NBR, int32_t, false, false, false>);
}

// The 64-bit phase-1 path needs 16-bit spins and rows of a multiple of 4
// sites (8-byte aligned words).  Moore8 takes it from 128-site tiles on: the
// 64-member ensemble (128x128 tiles) gains 2.48 -> 2.57e11 site updates/s,
// while its members swept one by one with 64x64 tiles lose 1.10 -> 0.96e11.
bool use_swar(int nbr, int spin, uint32_t BX, int tx) {
    return spin == HMC_I16 && BX % 4 == 0 && (nbr != HMC_MOORE8 || tx >= 128);
}

const void* kernel_ptr(int nbr, int spin, bool grains_in_lds, bool ensemble, bool swar, bool pair = false,
                       bool field = false) {
    switch (nbr) {
    case HMC_VN4:
        return swar ? kernel_for<HMC_VN4, true>(spin, grains_in_lds, ensemble, pair, field)
                    : kernel_for<HMC_VN4, false>(spin, grains_in_lds, ensemble, pair, field);
    case HMC_MOORE8:
        return swar ? kernel_for<HMC_MOORE8, true>(spin, grains_in_lds, ensemble, pair, field)
                    : kernel_for<HMC_MOORE8, false>(spin, grains_in_lds, ensemble, pair, field);
    case HMC_VN6:
        return swar ? kernel_for<HMC_VN6, true>(spin, grains_in_lds, ensemble, pair, field)
                    : kernel_for<HMC_VN6, false>(spin, grains_in_lds, ensemble, pair, field);
    default:
        return swar ? kernel_for<HMC_MOORE26, true>(spin, grains_in_lds, ensemble, pair, field)
                    : kernel_for<HMC_MOORE26, false>(spin, grains_in_lds, ensemble, pair, field);
    }
}

struct Layout {
    uint32_t BX, BY, BZ, H;
    size_t box_off, queue_off, coord_off, grain_off, bytes;
    bool grains_in_lds;
    uint32_t HX;              // x halo (H, or H rounded up to 4 with vec)
    bool vec;                 // 8-byte staging and store of 16-bit spins
    size_t field_off;         // per-site field box (field mode)
};

// LDS layout of one tile: [bucket bounds, queue counters | box | queue | coords | grains].
Layout box_layout(int nbr, int ndim, size_t spin_bytes, int32_t maxQ, const Tiling& t, int passes, bool vec,
                  bool field = false) {
    Layout o{};
    o.H = (uint32_t)passes;
    o.HX = vec ? (uint32_t)((passes + 3) & ~3) : (uint32_t)passes;
    o.vec = vec;
    o.BX = (uint32_t)(t.tx + 2 * o.HX);
    o.BY = (uint32_t)(t.ty + 2 * passes);
    o.BZ = ndim == 3 ? (uint32_t)(t.tz + 2 * passes) : 1u;
    const size_t elems = (size_t)o.BX * o.BY * o.BZ;
    // The queue holds at most the colour class of the first (largest) pass
    // region, which is one ring inside the box (x from the padded edge):
    // every side of it is even, so the class is exactly 1/C of the region.
    const size_t W0x = o.BX - 2 * (1 + (o.HX - o.H)), W0y = o.BY - 2, W0z = ndim == 3 ? o.BZ - 2 : 1;
    const size_t qcap = W0x * W0y * W0z / (size_t)nbr_info(nbr).C + 1;
    o.box_off = kHeaderBytes;
    o.queue_off = o.box_off + (elems * spin_bytes + 15) / 16 * 16;
    o.coord_off = o.queue_off + (qcap * 4 + 15) / 16 * 16;
    o.grain_off = (o.coord_off + (size_t)(o.BX + o.BY + o.BZ) * 4 + 15) / 16 * 16;
    o.bytes = o.grain_off;
    o.grains_in_lds = false;
    const size_t with_grains = o.grain_off + (size_t)maxQ * 4;
    const size_t field_bytes = field ? 16 + elems * 4 : 0;   // the field box after the grains, aligned
    if (maxQ <= kLdsGrainLimit && (int64_t)(with_grains + field_bytes) <= lds_limit_bytes()) {
        o.grains_in_lds = true;
        o.bytes = with_grains;
    }
    o.field_off = (o.bytes + 15) / 16 * 16;
    if (field) o.bytes = o.field_off + elems * 4;   // per-site field box, int32
    return o;
}

// Four 16-bit spins per 8-byte access along x: needs int16 lattices whose
// tiles and x side are multiples of 4 and 8-byte aligned spin buffers (a
// borrowed buffer may be aligned to 2 bytes only).
bool vec_ok(const hmc_lattice* L, const Tiling& t) {
    return L->desc.spin == HMC_I16 && t.tx % 4 == 0 && L->desc.dims[0] % 4 == 0 &&
           reinterpret_cast<uintptr_t>(L->spins[0]) % 8 == 0 && reinterpret_cast<uintptr_t>(L->spins[1]) % 8 == 0;
}

Layout box_layout(const hmc_lattice* L, const Tiling& t, int passes) {
    if (vec_ok(L, t)) {
        const Layout v = box_layout(L->desc.nbr, L->ndim, L->spin_bytes, L->Q, t, passes, true, L->field);
        if ((int64_t)v.bytes <= lds_limit_bytes() && v.BX <= 1023) return v;
    }
    return box_layout(L->desc.nbr, L->ndim, L->spin_bytes, L->Q, t, passes, false, L->field);
}

RunArgs run_args(const Layout& lay, int nbr, const Tiling& t, int passes, bool swar) {
    RunArgs g{};
    g.BX = lay.BX; g.BY = lay.BY; g.BZ = lay.BZ;
    g.H = lay.H;
    g.HX = lay.HX;
    g.vec = lay.vec ? 1u : 0u;
    g.m_bx4 = magic(lay.BX / 4);
    g.m_tx4 = magic((uint32_t)t.tx / 4);
    g.P = (uint32_t)passes;
    g.box_off = (uint32_t)lay.box_off;
    g.queue_off = (uint32_t)lay.queue_off;
    g.coord_off = (uint32_t)lay.coord_off;
    g.grain_off = (uint32_t)lay.grain_off;
    g.field_off = (uint32_t)lay.field_off;
    g.m_bx = magic(lay.BX);
    g.m_by = magic(lay.BY);
    g.m_tx = magic((uint32_t)t.tx);
    g.m_ty = magic((uint32_t)t.ty);
    const bool cb = nbr == HMC_VN4 || nbr == HMC_VN6;
    for (int ps = 0; ps < passes; ++ps) {
        const uint32_t lo = (uint32_t)ps + 1;
        const uint32_t lox = lo + (lay.HX - lay.H);
        const uint32_t Wx = lay.BX - 2 * lox, Wy = lay.BY - 2 * lo;
        if (swar) {   // rows of 4-site segments
            const uint32_t nseg = ((lay.BX - lox - 1) >> 2) - (lox >> 2) + 1;
            g.m_pass[ps][0] = magic(nseg);
            g.m_pass[ps][1] = magic(nbr == HMC_MOORE8 || nbr == HMC_MOORE26 ? Wy / 2 : Wy);
        } else {
            g.m_pass[ps][0] = magic(Wx / 2);
            g.m_pass[ps][1] = magic(cb ? Wy : Wy / 2);
        }
    }
    return g;
}

LatArgs lat_args(const hmc_lattice* L, const Tiling& t, uint64_t seed) {
    const int* dims = L->desc.dims;
    LatArgs a{};
    a.B = L->dB;
    a.T = L->table.dev;
    a.Tb = L->table.bounds;
    a.rows = L->table.rows;
    a.Lx = (uint32_t)dims[0];
    a.Ly = (uint32_t)dims[1];
    a.Lz = L->ndim == 3 ? (uint32_t)dims[2] : 1u;
    a.TX = (uint32_t)t.tx;
    a.TY = (uint32_t)t.ty;
    a.TZ = L->ndim == 3 ? (uint32_t)t.tz : 1u;
    a.ntx = a.Lx / a.TX;
    a.nty = a.Ly / a.TY;
    a.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
    a.k1 = (uint32_t)(seed >> 32);
    a.J_fx = L->desc.J_fx;
    a.Q = L->Q;
    a.dn_lo = L->table.dn_lo;
    a.TW = L->table.TW;
    a.R = L->table.R;
    a.nb = L->table.nb;
    a.nbound = L->table.rows * L->table.nb;
    a.bw = (uint32_t)L->table.bw;
    // umulhi(col, m) = col / bw exactly while col * bw < 2^32 (bw >= 2); with a
    // single column (bw = 1, col = 0) any m gives 0; otherwise m = 0 selects
    // a plain division
    if (a.bw == 1) a.m_bw = 1u;
    else a.m_bw = (uint64_t)L->table.TW * (uint64_t)a.bw < (1ull << 32) ? magic(a.bw) : 0u;
    a.uniform = L->desc.proposal == HMC_PROP_UNIFORM ? 1u : 0u;
    a.trials = L->profiling ? L->d_trials : nullptr;
    return a;
}

int largest_even_divisor_at_most(int L, int target) {
    for (int d = std::min(L, target) & ~1; d >= 2; d -= 2)
        if (L % d == 0) return d;
    return 2;
}

hmc_status check_tiling(int nbr, int ndim, int C, size_t spin_bytes, int32_t maxQ, const int* dims, const Tiling& r,
                        bool field) {
    const int sides[3] = {r.tx, r.ty, r.tz};
    for (int ax = 0; ax < ndim; ++ax) {
        if (sides[ax] < 2 || sides[ax] % 2 != 0 || dims[ax] % sides[ax] != 0)
            return fail(HMC_E_INVAL, "tile side " + std::to_string(sides[ax]) +
                                         " must be an even divisor of the lattice side " + std::to_string(dims[ax]));
    }
    if (r.k == 0 || launch_passes(r, C) > kMaxPasses)
        return fail(HMC_E_INVAL, "colour passes per launch must be in [1, " + std::to_string(kMaxPasses) + "]");
    const Layout lay = box_layout(nbr, ndim, spin_bytes, maxQ, r, launch_passes(r, C), false, field);
    if (lay.BX > 1023 || lay.BY > 1023 || lay.BZ > 1023)
        return fail(HMC_E_INVAL, "tile + halo exceeds 1023 sites along an axis");
    if ((int64_t)lay.bytes > lds_limit_bytes())
        return fail(HMC_E_INVAL, "tile + halo needs " + std::to_string(lay.bytes) + " B of LDS, limit " +
                                     std::to_string(lds_limit_bytes()));
    return HMC_OK;
}

// Default tilings in order of preference (measured on the 1024^2 VN4 and
// 256^3 VN6 workloads); the first that fits the LDS after each side is cut to
// an even divisor of the lattice side is used.
std::vector<Tiling> default_tilings(int nbr) {
    auto T = [](int x, int y, int z, int k) {
        Tiling t;
        t.tx = x; t.ty = y; t.tz = z; t.k = k;
        return t;
    };
    switch (nbr) {
    case HMC_VN4: return {T(64, 64, 1, 6), T(64, 64, 1, 5), T(32, 32, 1, 4), T(16, 16, 1, 2)};
    case HMC_MOORE8: return {T(64, 64, 1, 2), T(32, 32, 1, 2), T(16, 16, 1, 1)};
    case HMC_VN6: return {T(64, 16, 16, 1), T(32, 32, 16, 1), T(32, 16, 16, 1), T(16, 16, 16, 1), T(8, 8, 8, 1)};
    // eight colours: four colour passes per launch keep the halo at four rings
    default: return {T(32, 16, 16, -4), T(16, 16, 16, -4), T(8, 8, 8, -2), T(4, 4, 4, -1)};
    }
}

}  // namespace

int lds_limit_bytes() {
    static int cached = -1;
    if (cached < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            cached = v;
        else
            cached = 65536;
    }
    return cached;
}

int device_cus() {
    static int cached = -1;
    if (cached < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cached = v;
        else
            cached = 256;
    }
    return cached;
}

// A 2D 16-bit VN4 or Moore8 problem with at least two 256x128 tiles per CU
// (n256: their number, -1 if a side does not divide) takes them, with 4
// (VN4) or 3 (Moore8) MC steps per launch; else one with at least one
// 128x128 tile per CU (n128) takes those, with 6 or 3 steps.  The halo of
// the fused passes is a smaller share of a big tile, and there are enough
// tiles to fill the chip.  VN4 site updates/s against 64x64 tiles: 2048^2
// 2.12 -> 3.40e11 (128x128); 4096^2 2.20 -> 4.25e11, 16384^2 2.41 ->
// 5.30e11 (256x128); Moore8 2048^2 1.16 -> 2.13e11, 8192^2 1.30 -> 3.09e11.
// 1024^2 (64 tiles of 128x128) keeps 64x64.
bool large_tiling(int nbr, int ndim, size_t spin_bytes, int64_t n128, int64_t n256, Tiling& out) {
    if (ndim != 2 || spin_bytes != 2 || (nbr != HMC_VN4 && nbr != HMC_MOORE8)) return false;
    out.tz = 1;
    if (n256 >= 2 * (int64_t)device_cus()) {
        out.tx = 256;
        out.ty = 128;
        out.k = nbr == HMC_VN4 ? 4 : 3;
        return true;
    }
    if (n128 >= device_cus()) {
        out.tx = 128;
        out.ty = 128;
        out.k = nbr == HMC_VN4 ? 6 : 3;
        return true;
    }
    return false;
}

hmc_status choose_tiling(const hmc_lattice* L, Tiling& t, bool explicit_request) {
    const int* dims = L->desc.dims;
    Tiling r = t;
    if (!explicit_request || r.tx == 0 || r.ty == 0 || (L->ndim == 3 && r.tz == 0) || r.k == 0) {
        const Tiling* tuned = tuned_tiling(L->desc, L->Q);
        if (tuned && r.tx == 0 && r.ty == 0 && r.tz == 0 && r.k == 0) {
            r = *tuned;
        } else {
            const Tiling req = r;
            std::vector<Tiling> cands;
            Tiling big;
            const int64_t n128 = (dims[0] % 128 == 0 && dims[1] % 128 == 0)
                                     ? (int64_t)(dims[0] / 128) * (dims[1] / 128) : -1;
            const int64_t n256 = (dims[0] % 256 == 0 && dims[1] % 128 == 0)
                                     ? (int64_t)(dims[0] / 256) * (dims[1] / 128) : -1;
            if (req.tx == 0 && req.ty == 0 && req.k == 0 &&
                large_tiling(L->desc.nbr, L->ndim, L->spin_bytes, n128, n256, big))
                cands.push_back(big);
            // the compiled six-neighbour kernel runs 32x16x16 tiles two
            // workgroups per CU (256^3: 2.63e11 site updates/s against 2.52e11
            // with 64x16x16 tiles one per CU)
            if (compiled_vn6_model(L)) {
                Tiling v;
                v.tx = 32; v.ty = 16; v.tz = 16; v.k = 1;
                cands.push_back(v);
            }
            // the compiled Moore26 kernel is fastest with two colour passes
            // per launch (128^3: 4.41e10 site updates/s; four passes 4.29e10,
            // the general kernel 3.93e10 with four and 3.60e10 with two)
            if (compiled_moore26_model(L) && dims[0] % 32 == 0 && dims[1] % 16 == 0 && dims[2] % 16 == 0) {
                Tiling v;
                v.tx = 32; v.ty = 16; v.tz = 16; v.k = -2;
                cands.push_back(v);
            }
            for (const Tiling& d : default_tilings(L->desc.nbr)) cands.push_back(d);
            for (const Tiling& d : cands) {
                r = req;
                if (r.tx == 0) r.tx = largest_even_divisor_at_most(dims[0], d.tx);
                if (r.ty == 0) r.ty = largest_even_divisor_at_most(dims[1], d.ty);
                if (L->ndim == 3 && r.tz == 0) r.tz = largest_even_divisor_at_most(dims[2], d.tz);
                if (L->ndim == 2) r.tz = 1;
                if (r.k == 0) r.k = d.k;
                const Layout lay = box_layout(L->desc.nbr, L->ndim, L->spin_bytes, L->Q, r, launch_passes(r, L->C),
                                              false, L->field);
                if ((int64_t)lay.bytes <= lds_limit_bytes()) break;
            }
        }
    }
    if (L->ndim == 2) r.tz = 1;
    HMC_TRY(check_tiling(L->desc.nbr, L->ndim, L->C, L->spin_bytes, L->Q, dims, r, L->field));
    t = r;
    return HMC_OK;
}

// A lattice over a caller's buffer keeps its state there between calls.
hmc_status settle_borrowed(hmc_lattice* L) {
    if (!L->borrowed || L->cur == 0) return HMC_OK;
    HMC_HIP(hipMemcpyAsync(L->spins[0], L->spins[1], (size_t)L->N * L->spin_bytes, hipMemcpyDeviceToDevice,
                           L->stream));
    if (L->field)
        HMC_HIP(hipMemcpyAsync(L->d_field[0], L->d_field[1], (size_t)L->N * 4, hipMemcpyDeviceToDevice, L->stream));
    L->cur = 0;
    return HMC_OK;
}

// The six-neighbour 16-bit model with neighbour trials, one bond energy and
// grain energies has a kernel of its own for its common tiles (one or two
// colour passes per launch).
bool compiled_vn6_model(const hmc_lattice* L) {
    return L->sweep_kernel == HMC_KERNEL_AUTO && L->desc.nbr == HMC_VN6 && L->desc.spin == HMC_I16 &&
           L->desc.proposal == HMC_PROP_NEIGHBOUR && !L->pair && !L->field && L->desc.J_fx < (1 << 23);
}

bool compiled_vn6(const hmc_lattice* L, const Tiling& t, const void** fn, size_t* bytes, int* per_cu) {
    return compiled_vn6_model(L) && launch_passes(t, L->C) <= 2 && vec_ok(L, t) &&
           vn6_kernel_for(t, L->Q, fn, bytes, per_cu);
}

bool compiled_moore26_model(const hmc_lattice* L) {
    return L->sweep_kernel == HMC_KERNEL_AUTO && L->desc.nbr == HMC_MOORE26 && L->desc.spin == HMC_I16 &&
           L->desc.proposal == HMC_PROP_NEIGHBOUR && !L->pair && !L->field && L->desc.dims[0] % 4 == 0;
}

// 16-bit VN4, Moore8 and Moore26 lattices with neighbour trials, one bond
// energy and grain energies take the compiled kernel for their tile (full
// launches).
bool compiled2d(const hmc_lattice* L, const Tiling& t, const void** fn, size_t* bytes) {
    if (L->sweep_kernel != HMC_KERNEL_AUTO || (L->ndim != 2 && L->desc.nbr != HMC_MOORE26) || L->desc.spin != HMC_I16 ||
        L->desc.proposal != HMC_PROP_NEIGHBOUR || L->pair || L->field || !vec_ok(L, t))
        return false;
    *fn = compiled2d_for(L->desc.nbr, t, false, L->Q, bytes);
    return *fn != nullptr;
}

hmc_status launch_sweep(hmc_lattice* L, float kT, int32_t n_mcs, uint64_t seed) {
    if (n_mcs == 0) return HMC_OK;
    if (L->pair || L->field) {
        HMC_TRY(build_direct_table(L, kT));
    } else {
        HMC_TRY(build_table(L->table, kT, L->M, L->desc.J_fx, L->Bmin, L->Bmax, L->stream));
        if (L->table.rows > kMaxRows) return fail(HMC_E_INTERNAL, "threshold table has too many rows");
    }
    Tiling t = L->tiling;
    HMC_TRY(choose_tiling(L, t, L->tiling_explicit));
    L->tiling = t;

    LatArgs a = lat_args(L, t, seed);
    if (L->pair || L->field) {   // threshold per energy change; the per-row bounds are not used
        a.Jp = L->d_Jp;
        a.Tg = L->d_Tg;
        a.Dmax = L->Tg_Dmax;
        a.nbound = 0;
        a.frule = L->frule;
    }
    const uint32_t ntiles = a.ntx * a.nty * (a.Lz / a.TZ);
    const uint32_t xcd_group = (ntiles % 8 == 0) ? ntiles / 8 : 0u;

    // Colour passes per launch.  A borrowed spin buffer must hold the result:
    // when the launch count would leave it in the second buffer, the last
    // launch is split in two (results do not depend on the split).
    const int P = launch_passes(t, L->C);
    std::vector<int> chunks;
    for (int64_t rem = (int64_t)n_mcs * L->C; rem > 0; rem -= std::min<int64_t>(P, rem))
        chunks.push_back((int)std::min<int64_t>(P, rem));
    if (L->borrowed && ((L->cur + (int)chunks.size()) & 1) && !chunks.empty() && chunks.back() >= 2) {
        const int pl = chunks.back();
        chunks.back() = pl / 2;
        chunks.push_back(pl - pl / 2);
    }
    const void* vfn = nullptr;
    size_t vbytes = 0;
    int per_cu = 1;
    const bool vn6 = compiled_vn6(L, t, &vfn, &vbytes, &per_cu);
    const void* cfn = nullptr;
    size_t cbytes = 0;
    const bool c2d = !vn6 && compiled2d(L, t, &cfn, &cbytes);
    Vn6Args va{};
    if (vn6) {
        va.B = a.B; va.T = a.T; va.Tb = a.Tb;
        va.Lx = a.Lx; va.Ly = a.Ly; va.Lz = a.Lz; va.ntx = a.ntx; va.nty = a.nty;
        va.k0 = a.k0; va.k1 = a.k1;
        va.J_fx = a.J_fx; va.Q = a.Q; va.dn_lo = a.dn_lo; va.TW = a.TW; va.R = a.R; va.nb = a.nb;
        va.nbound = a.nbound; va.bw = a.bw; va.m_bw = a.m_bw;
        va.ntiles = ntiles;
        va.trials = a.trials;
    }
    int64_t gp0 = 0;   // passes done in this call
    for (const int passes : chunks) {
        const Layout lay = box_layout(L, t, passes);
        const bool swar = use_swar(L->desc.nbr, L->desc.spin, lay.BX, t.tx);
        RunArgs g = run_args(lay, L->desc.nbr, t, passes, swar);
        // the compiled tile kernel runs every launch of all P passes (the 2D
        // ones start at colour 0; the Moore26 one takes the launch's colour)
        const bool full2d = c2d && passes == P && (L->desc.nbr == HMC_MOORE26 || gp0 % L->C == 0);
        const void* kfn = vn6 ? vfn : (full2d ? cfn : kernel_ptr(L->desc.nbr, L->desc.spin, lay.grains_in_lds, false,
                                                                 swar, L->pair, L->field));
        const size_t lds = vn6 ? vbytes : (full2d ? cbytes : lay.bytes);
        a.src = L->spins[L->cur];
        a.dst = L->spins[L->cur ^ 1];
        a.fsrc = L->d_field[L->cur];
        a.fdst = L->d_field[L->cur ^ 1];
        a.t0 = (uint32_t)(L->mcs + (uint64_t)(gp0 / L->C));
        a.c0 = (uint32_t)(gp0 % L->C);
        va.src = static_cast<const int16_t*>(a.src);
        va.dst = static_cast<int16_t*>(a.dst);
        va.t0 = a.t0;
        va.c0 = a.c0;
        va.npass = (uint32_t)passes;
        uint32_t xg = xcd_group;
        void* gargs[] = {&a, &g, &xg};
        void* vargs[] = {&va};
        void* cargs[] = {&a, &xg};
        void** args = vn6 ? vargs : (full2d ? cargs : gargs);
        // the compiled-tile kernel is persistent: one or two workgroups per
        // CU walk their share of the tiles
        const uint32_t grid = vn6 ? std::min<uint32_t>(ntiles, (uint32_t)(per_cu * device_cus())) : ntiles;
        va.xcd_blocks = (vn6 && grid % 8 == 0) ? 1u : 0u;
        if (L->profiling) {
            // Events bound to the dispatch itself: they time the kernel, not
            // the queue around it.
            if (L->events_used == L->events.size()) {
                hipEvent_t e0, e1;
                HMC_HIP(hipEventCreate(&e0));
                HMC_HIP(hipEventCreate(&e1));
                L->events.emplace_back(e0, e1);
            }
            const auto& ev = L->events[L->events_used++];
            HMC_HIP(hipExtLaunchKernel(kfn, dim3(grid), dim3(kThreads), args, lds, L->stream, ev.first,
                                       ev.second, 0));
            L->prof_launches += 1;
            L->prof_su += (int64_t)passes * L->N / L->C;
        } else {
            HMC_HIP(hipLaunchKernel(kfn, dim3(grid), dim3(kThreads), args, lds, L->stream));
        }
        L->cur ^= 1;
        gp0 += passes;
    }
    L->mcs += (uint64_t)n_mcs;
    return settle_borrowed(L);
}

// ------------------------------------------------------------------ ensemble

hmc_status ensemble_prepare(hmc_ensemble* E) {
    hmc_lattice* L0 = E->lats[0];
    int32_t maxQ = 0;
    std::vector<int> g(3, 0);
    for (hmc_lattice* L : E->lats) {
        maxQ = std::max(maxQ, L->Q);
        for (int ax = 0; ax < L0->ndim; ++ax) g[ax] = std::gcd(g[ax], L->desc.dims[ax]);
    }
    E->maxQ = maxQ;
    const int cus = device_cus();
    if (E->tiling.tx == 0 || E->tiling.k == 0) {
        // the single-lattice rule on the whole ensemble's 128x128 tiles (64
        // Moore8 members, 29 M sites: 251 -> 130 ms per 1000 steps)
        std::vector<Tiling> cands;
        bool div128 = true, div256 = true;
        int64_t n128 = 0, n256 = 0;
        for (const hmc_lattice* L : E->lats) {
            div128 = div128 && L->desc.dims[0] % 128 == 0 && L->desc.dims[1] % 128 == 0;
            div256 = div256 && L->desc.dims[0] % 256 == 0 && L->desc.dims[1] % 128 == 0;
            n128 += (int64_t)(L->desc.dims[0] / 128) * (L->desc.dims[1] / 128);
            n256 += (int64_t)(L->desc.dims[0] / 256) * (L->desc.dims[1] / 128);
        }
        Tiling big;
        if (large_tiling(L0->desc.nbr, L0->ndim, L0->spin_bytes, div128 ? n128 : -1, div256 ? n256 : -1, big))
            cands.push_back(big);
        for (const Tiling& d : default_tilings(L0->desc.nbr)) cands.push_back(d);
        Tiling t;
        for (const Tiling& d : cands) {
            t.tx = largest_even_divisor_at_most(g[0], d.tx);
            t.ty = largest_even_divisor_at_most(g[1], d.ty);
            t.tz = L0->ndim == 3 ? largest_even_divisor_at_most(g[2], d.tz) : 1;
            t.k = d.k > 0 ? d.k : 1;   // ensemble launches cover whole MC steps
            const Layout lay = box_layout(L0->desc.nbr, L0->ndim, L0->spin_bytes, maxQ, t, t.k * L0->C, false);
            if ((int64_t)lay.bytes <= lds_limit_bytes()) break;
        }
        E->tiling = t;
    }
    for (hmc_lattice* L : E->lats)
        HMC_TRY(check_tiling(L->desc.nbr, L->ndim, L->C, L->spin_bytes, maxQ, L->desc.dims, E->tiling, false));
    // ragged tile table: every tile of every lattice
    std::vector<uint2> tiles;
    for (size_t i = 0; i < E->lats.size(); ++i) {
        const hmc_lattice* L = E->lats[i];
        const uint32_t n = (uint32_t)(L->desc.dims[0] / E->tiling.tx) * (uint32_t)(L->desc.dims[1] / E->tiling.ty) *
                           (uint32_t)(L->ndim == 3 ? L->desc.dims[2] / E->tiling.tz : 1);
        for (uint32_t tIdx = 0; tIdx < n; ++tIdx) tiles.push_back(make_uint2((uint32_t)i, tIdx));
    }
    E->ntiles = (uint32_t)tiles.size();
    dev_free(E->d_tiles, E->tiles_bytes);
    E->d_tiles = nullptr;
    E->tiles_bytes = tiles.size() * sizeof(uint2);
    HMC_TRY(dev_alloc(&E->d_tiles, E->tiles_bytes, "ensemble tile table"));
    HMC_HIP(hipMemcpy(E->d_tiles, tiles.data(), E->tiles_bytes, hipMemcpyHostToDevice));
    if (!E->d_lats) {
        E->lats_bytes = E->lats.size() * sizeof(EnsLat);
        HMC_TRY(dev_alloc(&E->d_lats, E->lats_bytes, "ensemble descriptors"));
    }
    // four spins per 8-byte access when every member allows it and the
    // padded box still fits (the tile choice above did not pad)
    E->vec = true;
    for (const hmc_lattice* L : E->lats) E->vec = E->vec && vec_ok(L, E->tiling);
    if (E->vec) {
        for (int passes = 1; passes <= E->tiling.k * L0->C; ++passes) {
            const Layout v = box_layout(L0->desc.nbr, L0->ndim, L0->spin_bytes, maxQ, E->tiling, passes, true);
            E->vec = E->vec && (int64_t)v.bytes <= lds_limit_bytes() && v.BX <= 1023;
        }
    }
    const Layout lay = box_layout(L0->desc.nbr, L0->ndim, L0->spin_bytes, maxQ, E->tiling, E->tiling.k * L0->C,
                                  E->vec);
    // resident workgroups per CU: two 1024-thread groups fill the wave slots;
    // the LDS of a CU (equal to the per-group limit on gfx950) may allow fewer
    const int per_cu = std::max(1, std::min(2, (int)(lds_limit_bytes() / std::max<size_t>(lay.bytes, 1))));
    E->grid = std::max(1u, std::min(E->ntiles, (uint32_t)(cus * per_cu)));
    for (auto& kv : E->graphs) (void)hipGraphExecDestroy(kv.second);
    E->graphs.clear();
    E->prepared = true;
    return HMC_OK;
}

hmc_status launch_ensemble(hmc_ensemble* E, const float* kT, const uint64_t* seed, int32_t n_mcs) {
    if (n_mcs == 0) return HMC_OK;
    for (const hmc_lattice* L : E->lats)
        if (L->pair || L->field) return fail(HMC_E_STATE, "an ensemble member was given pair or per-site energies");
    if (!E->prepared) HMC_TRY(ensemble_prepare(E));
    hmc_lattice* L0 = E->lats[0];
    const int C = L0->C;
    std::vector<EnsLat> h(E->lats.size());
    for (size_t i = 0; i < E->lats.size(); ++i) {
        hmc_lattice* L = E->lats[i];
        HMC_TRY(build_table(L->table, kT[i], L->M, L->desc.J_fx, L->Bmin, L->Bmax, L->stream));
        if (L->table.rows > kMaxRows) return fail(HMC_E_INTERNAL, "threshold table has too many rows");
        h[i].a = lat_args(L, E->tiling, seed[i]);
        h[i].a.trials = nullptr;
        h[i].buf[0] = L->spins[0];
        h[i].buf[1] = L->spins[1];
        h[i].cur = (uint32_t)L->cur;
        h[i].t_base = (uint32_t)L->mcs;
    }
    // order after every member's pending work, its table and energy uploads included
    for (hmc_lattice* L : E->lats) {
        HMC_HIP(hipEventRecord(E->ev, L->stream));
        HMC_HIP(hipStreamWaitEvent(E->stream, E->ev, 0));
    }
    // Upload from pinned staging, two slots in turn: the host waits only for
    // the upload made two calls ago from the same slot (long finished in a
    // steady loop), never for the replay itself.
    const int slot = E->stage_slot;
    if (!E->h_stage[slot]) {
        HMC_HIP(hipHostMalloc(&E->h_stage[slot], E->lats_bytes, hipHostMallocDefault));
        HMC_HIP(hipEventCreateWithFlags(&E->stage_ev[slot], hipEventDisableTiming));
    }
    if (E->stage_used[slot]) HMC_HIP(hipEventSynchronize(E->stage_ev[slot]));
    std::memcpy(E->h_stage[slot], h.data(), E->lats_bytes);
    HMC_HIP(hipMemcpyAsync(E->d_lats, E->h_stage[slot], E->lats_bytes, hipMemcpyHostToDevice, E->stream));
    HMC_HIP(hipEventRecord(E->stage_ev[slot], E->stream));
    E->stage_used[slot] = true;
    E->stage_slot = slot ^ 1;

    auto it = E->graphs.find(n_mcs);
    if (it == E->graphs.end()) {
        hipGraph_t graph = nullptr;
        HMC_HIP(hipStreamBeginCapture(E->stream, hipStreamCaptureModeThreadLocal));
        hipError_t err = hipSuccess;
        int32_t remaining = n_mcs;
        uint32_t j = 0;
        const uint32_t kfull = (uint32_t)E->tiling.k;
        // 16-bit Moore8 members with neighbour trials in 128x128 tiles with 3
        // MC steps per launch: the compiled 2D kernel for every full launch
        bool c2 = L0->ndim == 2 && L0->desc.spin == HMC_I16 && E->vec;
        for (const hmc_lattice* L : E->lats) c2 = c2 && L->desc.proposal == HMC_PROP_NEIGHBOUR;
        size_t c2_bytes = 0;
        const void* c2_fn = c2 ? compiled2d_for(L0->desc.nbr, E->tiling, true, E->maxQ, &c2_bytes) : nullptr;
        const uint32_t c2_grid = std::max(1u, std::min(E->ntiles, (uint32_t)(device_cus() *
                                          std::max(1, std::min(2, (int)(lds_limit_bytes() / std::max<size_t>(c2_bytes, 1)))))));
        while (remaining > 0 && err == hipSuccess) {
            const int k = std::min<int32_t>(E->tiling.k, remaining);
            const EnsLat* dl = static_cast<const EnsLat*>(E->d_lats);
            const uint2* dt = static_cast<const uint2*>(E->d_tiles);
            uint32_t nt = E->ntiles, jj = j, kk = kfull;
            if (c2_fn && k == E->tiling.k) {
                void* args[] = {&dl, &dt, &nt, &jj, &kk};
                err = hipLaunchKernel(c2_fn, dim3(c2_grid), dim3(kThreads), args, c2_bytes, E->stream);
            } else {
                const int passes = k * C;
                const Layout lay = box_layout(L0->desc.nbr, L0->ndim, L0->spin_bytes, E->maxQ, E->tiling, passes,
                                              E->vec);
                const bool swar = use_swar(L0->desc.nbr, L0->desc.spin, lay.BX, E->tiling.tx);
                RunArgs g = run_args(lay, L0->desc.nbr, E->tiling, passes, swar);
                const void* kfn = kernel_ptr(L0->desc.nbr, L0->desc.spin, lay.grains_in_lds, true, swar);
                void* args[] = {&g, &dl, &dt, &nt, &jj, &kk};
                err = hipLaunchKernel(kfn, dim3(E->grid), dim3(kThreads), args, lay.bytes, E->stream);
            }
            remaining -= k;
            ++j;
        }
        const hipError_t e2 = hipStreamEndCapture(E->stream, &graph);
        if (err != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(err, "ensemble capture");
        }
        if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
        hipGraphExec_t exec = nullptr;
        const hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e3 != hipSuccess) return hip_fail(e3, "hipGraphInstantiate");
        it = E->graphs.emplace(n_mcs, exec).first;
        E->graph_launches = j;
    }
    const uint32_t launches = (uint32_t)((n_mcs + E->tiling.k - 1) / E->tiling.k);
    if (E->profiling) {   // events outside the graph, around its replay
        if (E->events_used == E->events.size()) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            HMC_HIP(hipEventCreate(&e0));
            HMC_HIP(hipEventCreate(&e1));
            E->events.emplace_back(e0, e1);
        }
        const auto& ev = E->events[E->events_used++];
        HMC_HIP(hipEventRecord(ev.first, E->stream));
        HMC_HIP(hipGraphLaunch(it->second, E->stream));
        HMC_HIP(hipEventRecord(ev.second, E->stream));
        E->prof_launches += launches;
        for (const hmc_lattice* L : E->lats) E->prof_su += (int64_t)L->N * n_mcs;
    } else {
        HMC_HIP(hipGraphLaunch(it->second, E->stream));
    }
    HMC_HIP(hipEventRecord(E->ev, E->stream));
    for (hmc_lattice* L : E->lats) {
        HMC_HIP(hipStreamWaitEvent(L->stream, E->ev, 0));
        L->cur ^= (int)(launches & 1u);
        L->mcs += (uint64_t)n_mcs;
        HMC_TRY(settle_borrowed(L));
    }
    return HMC_OK;
}

}  // namespace hmc
