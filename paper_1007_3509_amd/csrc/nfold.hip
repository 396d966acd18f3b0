// nfold.hip -- the n-fold way: rejection-free, continuous-time Metropolis
// dynamics of the Potts model, one lattice per wave.
//
// Zhang, Dingreville, Bartel, Lusk, arXiv:1007.3509, Sec. 1 and Sec. 4 name
// the n-fold way (Bortz, Kalos, Lebowitz 1975; Hassold and Holm 1993 for
// Potts grain growth) as the alternative to red/black updating.  It runs the
// single-site Metropolis process of Sec. 3 in continuous time without
// rejected trials: every site attempts at rate one per MC step, an attempt
// proposes one of S slots (the M neighbour spins, or the Q-1 other values in
// the symmetric trial mode) and succeeds with min(1, exp(-dE/kT)).  Slot k of
// site i therefore fires at rate w_ik / (S 2^32) with the integer weight
// w_ik = 2^32 (d <= 0) or T(d) (the sweep's threshold), and the next event
// comes after an Exp(W / (S 2^32)) waiting time and is (i, k) with
// probability w_ik / W, W the sum of every weight.
//
// Definitions fixed by the library (include/hmc.h): Philox4x32-10 with
// counter (lo32(n), hi32(n), 0x4E464F57, block) for event n; words 0 and 1
// give the rank r = floor(u W / 2^64) of the event among the cumulative
// weights in site order, then slot order; the following words give an Exp(1)
// variate by von Neumann's comparison method (1951) in 32.32 fixed point;
// dt = (E S) / W in double, t = t_last + dt; an event landing beyond t_end
// is left for the next call.
//
// MI355X layout.  One workgroup of one wave per lattice.  The lattice's
// spins and a 64-ary tree of weight sums sit in LDS (level 1 holds the sum
// of each run of 64 sites, every level above the sum of 64 entries of the
// one below, the root the total), so an event is a descent of at most three
// levels, each a 64-lane load and a wave-wide 64-bit prefix scan, followed by
// the weights of the site and its M neighbours recomputed before and after
// the flip and their differences added up the tree with LDS atomics.  Site
// weights are not stored: each lane recomputes the weight of its site from
// the spins in LDS when a descent reaches its run of 64.  Each event is a
// dependent chain in one wave, so the code avoids anything that lengthens
// it: the 64 random words are generated side by side, a site's table loads
// are issued together (no branch per slot), and an event's tree updates
// overlap the next event instead of ending in a barrier.  Batches put many
// lattices in one launch, one wave each, which is what fills the chip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace hmc {
namespace {

constexpr int kNfThreads = 64;                 // one wave per lattice
constexpr uint32_t kNfTag = 0x4E464F57u;
constexpr int kNfMaxLevels = 3;                // 64^3 sites: beyond any LDS-resident lattice
constexpr int64_t kNfEventsPerLaunch = 1 << 15;

enum : int32_t { kNfRunning = 0, kNfReached = 1, kNfNoEvent = 2, kNfBroken = 3 };

struct NfClock {
    double t_last;
    unsigned long long n_events;
    int32_t state;
    int32_t pad;
};

struct NfLat {
    void* spins;
    const int32_t* B;
    const uint32_t* Tg;          // T(d), d = 0..Dmax
    const int32_t* Jp;           // Q x Q, pair mode only
    NfClock* clock;
    double t_end;
    uint32_t Lx, Ly, Lz, N;
    uint32_t mx, my;             // ceil(2^32 / Lx), ceil(2^32 / Ly): division by multiply-high
    int32_t Q, J_fx, Dmax, S;
    uint32_t k0, k1;
};

struct NfLevels {
    int T;                       // stored levels 1..T; level T has <= 64 entries
    uint32_t n[kNfMaxLevels + 1];
    uint32_t off[kNfMaxLevels + 1];   // uint64 offsets of each level in the tree array
    uint32_t total;              // uint64 entries of every level
};

__host__ __device__ inline NfLevels nf_levels(uint32_t N) {
    NfLevels v{};
    v.n[0] = N;
    v.T = 0;
    uint32_t o = 0;
#pragma unroll
    for (int L = 1; L <= kNfMaxLevels; ++L) {   // unrolled: constant indices keep the table in registers
        const bool used = v.T == 0;              // still below the top level
        v.n[L] = used ? (v.n[L - 1] + 63u) / 64u : 0u;
        v.off[L] = o;
        o += v.n[L];
        if (used && (v.n[L] <= 64u || L == kNfMaxLevels)) v.T = L;
    }
    v.total = o;
    return v;
}

// LDS of one lattice: spins (16-byte aligned), the tree levels and root
// (uint64), the grain energies (int32).
__host__ __device__ inline size_t nf_spin_bytes_lds(uint32_t N, size_t spin_bytes) {
    return ((size_t)N * spin_bytes + 15) & ~(size_t)15;
}

inline size_t nf_lds_bytes(uint32_t N, size_t spin_bytes, int32_t Q) {
    const NfLevels lv = nf_levels(N);
    return nf_spin_bytes_lds(N, spin_bytes) + 8 * ((size_t)lv.total + 1) + 4 * (size_t)Q;
}

// ------------------------------------------------------------------ device

// A 64-bit value moved across lanes by one DPP pattern; lanes without a
// source (or outside row_mask) read 0.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, kCtrl, kRowMask, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), kCtrl, kRowMask, 0xF, true);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Inclusive prefix sum over the 64 lanes with DPP (no LDS round trips):
// shifts by 1, 2, 4, 8 inside each row of 16, then the last lane of row 0
// and 2 added to rows 1 and 3, then the last lane of row 1 to rows 2 and 3.
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) {
    v += dpp64<0x111, 0xF>(v);    // row_shr:1
    v += dpp64<0x112, 0xF>(v);    // row_shr:2
    v += dpp64<0x114, 0xF>(v);    // row_shr:4
    v += dpp64<0x118, 0xF>(v);    // row_shr:8
    v += dpp64<0x142, 0xA>(v);    // row_bcast:15 into rows 1 and 3
    v += dpp64<0x143, 0xC>(v);    // row_bcast:31 into rows 2 and 3
    return v;
}

__device__ __forceinline__ uint32_t lane_value(uint32_t v, int src) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, src);
}

__device__ __forceinline__ uint64_t lane_value64(uint64_t v, int src) {
    return ((uint64_t)lane_value((uint32_t)(v >> 32), src) << 32) | lane_value((uint32_t)v, src);
}

// Sum over the wave, in every lane.
__device__ __forceinline__ uint64_t wave_sum(uint64_t v) { return lane_value64(wave_incl_scan(v), 63); }

// First lane whose inclusive sum exceeds r (-1 if none), and r reduced by
// the sum of the lanes before it.
__device__ __forceinline__ int wave_pick(uint64_t v, uint64_t& r) {
    const uint64_t incl = wave_incl_scan(v);
    const unsigned long long m = __ballot(incl > r);
    if (m == 0ull) return -1;
    const int c = __ffsll((long long)m) - 1;
    r -= lane_value64(incl - v, c);
    return c;
}

// The words of one event's Philox stream.  Lane l computes block l / 4 and
// keeps its word l % 4, so the wave holds words 0..63 at once; words beyond
// them come from one further block at a time.  `desc` has bit k set when
// word k+1 < word k (k < 63), which lets a whole decreasing run be measured
// with one bit scan.
struct NfWords {
    uint32_t n_lo, n_hi, k0, k1;
    uint32_t wl;                 // lane l: word l
    uint64_t desc;
    uint32_t e0, e1, e2, e3;     // the current block beyond the first sixteen
    int w;                       // next word (uniform)
    __device__ void start(uint64_t n, uint32_t key0, uint32_t key1, int lane) {
        n_lo = (uint32_t)n;
        n_hi = (uint32_t)(n >> 32);
        k0 = key0;
        k1 = key1;
        uint32_t o[4];
        philox4x32_10(n_lo, n_hi, kNfTag, (uint32_t)(lane >> 2), k0, k1, o);
        const int c = lane & 3;
        wl = c == 0 ? o[0] : c == 1 ? o[1] : c == 2 ? o[2] : o[3];
        const uint32_t up = (uint32_t)__shfl_down((int)wl, 1, 64);   // word l+1
        desc = (uint64_t)__ballot(lane < 63 && up < wl);
        e0 = e1 = e2 = e3 = 0u;
        w = 0;
    }
    __device__ uint32_t word(int idx) const { return lane_value(wl, idx); }   // idx < 64, uniform
    __device__ uint32_t next() {
        const int idx = w++;
        if (idx < 64) return word(idx);
        const int c = idx & 3;
        if (c == 0) {
            uint32_t o[4];
            philox4x32_10(n_lo, n_hi, kNfTag, (uint32_t)(idx >> 2), k0, k1, o);
            e0 = o[0]; e1 = o[1]; e2 = o[2]; e3 = o[3];
        }
        return c == 0 ? e0 : c == 1 ? e1 : c == 2 ? e2 : e3;
    }
};

// von Neumann (1951): a trial takes u0 and the length n of the strictly
// decreasing run it starts (the word that ends the run is used up); odd n
// accepts E = K + u0 / 2^32, even n adds one to K.  Runs are cut at 64 words
// and K at 64.  A run that ends inside the first kWin words is measured from
// `desc` (c further words continue it, the next one breaks it); any other
// run is walked word by word.  kWin is 64 in the event loop; the self-test
// entry point also builds smaller windows so that both paths are exercised.
template <int kWin = 64>
__device__ __forceinline__ uint64_t nf_exponential(NfWords& w) {
    static_assert(kWin >= 2 && kWin <= 64, "the window lies in the wave's 64 words");
    const uint64_t desc = kWin == 64 ? w.desc : w.desc & ((1ull << (kWin - 1)) - 1);   // bits < kWin - 1
    uint64_t K = 0;
    // The first four trials as selects, without branches; an event needs
    // more, or meets a run that leaves the window, about once in fifty, and
    // the loop below then resumes where they stopped.
    {
        int p = w.w, pa = 0, ka = 0;
        bool done = false, stop = false;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int c = p <= kWin - 2 ? (int)__builtin_ctzll(~(desc >> p)) : 64;
            const bool go = !done && !stop;
            const bool inw = p + c <= kWin - 2;
            const bool acc = go && inw && !(c & 1);
            const bool rej = go && inw && (c & 1);
            stop = stop || (go && !inw);
            pa = acc ? p : pa;
            ka = acc ? (int)K : ka;
            done = done || acc;
            K += rej ? 1u : 0u;
            p = (acc || rej) ? p + c + 2 : p;
        }
        w.w = p;
        if (done) return ((uint64_t)ka << 32) | (uint64_t)w.word(pa);
    }
    for (;;) {
        uint32_t u0;
        int n;
        const int p = w.w;
        const int c = p <= kWin - 2 ? (int)__builtin_ctzll(~(desc >> p)) : 64;   // bit kWin-1 of desc is 0
        if (p + c <= kWin - 2) {
            u0 = w.word(p);
            n = c + 1;            // <= 61: p >= 2
            w.w = p + c + 2;
        } else {
            u0 = w.next();
            uint32_t prev = u0;
            n = 1;
            while (n < 64) {
                const uint32_t v = w.next();
                if (v < prev) {
                    prev = v;
                    ++n;
                } else {
                    break;
                }
            }
        }
        if (n & 1) return (K << 32) | (uint64_t)u0;
        if (++K == 64) return K << 32;
    }
}

template <int NBR>
__device__ __forceinline__ uint32_t nf_neighbour(const NfLat& a, uint32_t x, uint32_t y, uint32_t z, int k) {
    const int dx = nbr_dx(NBR, k), dy = nbr_dy(NBR, k), dz = nbr_dz(NBR, k);
    uint32_t xn = x, yn = y, zn = z;
    if (dx > 0) xn = x + 1 == a.Lx ? 0 : x + 1;
    if (dx < 0) xn = x == 0 ? a.Lx - 1 : x - 1;
    if (dy > 0) yn = y + 1 == a.Ly ? 0 : y + 1;
    if (dy < 0) yn = y == 0 ? a.Ly - 1 : y - 1;
    if (dz > 0) zn = z + 1 == a.Lz ? 0 : z + 1;
    if (dz < 0) zn = z == 0 ? a.Lz - 1 : z - 1;
    return xn + a.Lx * (yn + a.Ly * zn);
}

// Coordinates of site j: floor(j / L) = mulhi(j, ceil(2^32 / L)), exact
// while j * L < 2^32 (the host checks N * Lx and N * Ly).
__device__ __forceinline__ void nf_coords(const NfLat& a, uint32_t j, uint32_t& x, uint32_t& y, uint32_t& z) {
    const uint32_t yz = __umulhi(j, a.mx);
    x = j - yz * a.Lx;
    z = __umulhi(yz, a.my);
    y = yz - z * a.Ly;
}

template <int NBR>
constexpr int nf_M() {
    return NBR == HMC_VN4 ? 4 : NBR == HMC_MOORE8 ? 8 : NBR == HMC_VN6 ? 6 : 26;
}

template <int NBR>
__device__ __forceinline__ uint32_t nf_neighbour_of(const NfLat& a, uint32_t j, int k) {
    uint32_t x, y, z;
    nf_coords(a, j, x, y, z);
    uint32_t out = j;
#pragma unroll
    for (int m = 0; m < nf_M<NBR>(); ++m)
        if (m == k) out = nf_neighbour<NBR>(a, x, y, z, m);
    return out;
}

// Spin of the site and of its M neighbours.
template <int NBR, typename Spin>
__device__ __forceinline__ int32_t nf_gather(const Spin* s, const NfLat& a, uint32_t j, int32_t* nb) {
    uint32_t x, y, z;
    nf_coords(a, j, x, y, z);
#pragma unroll
    for (int k = 0; k < nf_M<NBR>(); ++k) nb[k] = (int32_t)s[nf_neighbour<NBR>(a, x, y, z, k)];
    return (int32_t)s[j];
}

// The lattice descriptors are read from device memory, so the compiler cannot
// tell that their pointers are global and would emit flat loads, which also
// hold up every later LDS wait; this cast makes them global loads.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* nf_global(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}

// Weight of moving a site with spin q and neighbour spins nb to spin c != q;
// B is the LDS copy of the grain energies.
template <int NBR, bool kPair>
__device__ __forceinline__ uint64_t nf_slot_weight(const NfLat& a, const int32_t* B, int32_t q, int32_t c,
                                                   const int32_t* nb) {
    constexpr int M = nf_M<NBR>();
    int64_t d;
    if constexpr (kPair) {
        const auto* rq = nf_global(a.Jp) + (int64_t)q * a.Q;
        const auto* rc = nf_global(a.Jp) + (int64_t)c * a.Q;
        int64_t acc = 0;
#pragma unroll
        for (int m = 0; m < M; ++m)   // a value outside [0, Q) bonds with nothing
            if ((uint32_t)nb[m] < (uint32_t)a.Q) acc += (int64_t)rc[nb[m]] - (int64_t)rq[nb[m]];
        d = acc;
    } else {
        int cq = 0, cc = 0;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            cq += nb[m] == q;
            cc += nb[m] == c;
        }
        d = (int64_t)a.J_fx * (cq - cc);   // unlike bonds after minus before
    }
    d += (int64_t)B[c] - (int64_t)B[q];
    if (d <= 0) return 1ull << 32;
    return (uint64_t)nf_global(a.Tg)[d < a.Dmax ? d : a.Dmax];
}

// Weights of the neighbour-mode slots of one site (spin q, in range; neighbour
// spins nb), summed over the slots with use[k] set.  Every slot's d and
// table index are formed without branches (a slot that is not used gets
// d = 0) and the M table loads are issued together: in a branch per slot
// each load waited for the one before it.
template <int NBR, bool kPair>
__device__ __forceinline__ uint64_t nf_slots_weight(const NfLat& a, const int32_t* B, int32_t q, const int32_t* nb,
                                                    const bool* use) {
    constexpr int M = nf_M<NBR>();
    if constexpr (kPair && M > 8) {   // 26 slots of 26 pair-table loads: one slot at a time
        uint64_t w = 0;
        for (int k = 0; k < M; ++k)
            if (use[k]) w += nf_slot_weight<NBR, kPair>(a, B, q, nb[k], nb);
        return w;
    }
    // d fits in 32 bits: setting energies keeps (largest bond) M + 2 max|B|
    // below 2^31.  Selections are masks, so that no slot becomes a branch.
    int32_t d[M];
    const int32_t bq = B[q];
    if constexpr (kPair) {
        const auto* rq = nf_global(a.Jp) + (int64_t)q * a.Q;
        int32_t nbs[M], in[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {   // a value outside [0, Q) bonds with nothing
            in[m] = -(int32_t)((uint32_t)nb[m] < (uint32_t)a.Q);
            nbs[m] = nb[m] & in[m];
        }
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int32_t c = use[k] ? nb[k] : q;
            const auto* rc = nf_global(a.Jp) + (int64_t)c * a.Q;
            int32_t acc = 0;
#pragma unroll
            for (int m = 0; m < M; ++m) acc += (rc[nbs[m]] - rq[nbs[m]]) & in[m];
            d[k] = (acc + B[c] - bq) & -(int32_t)use[k];
        }
    } else {
        // every grain energy read at an index valid for any slot (an unused
        // slot's value is masked off), so that no read waits for a branch
        int32_t bn[M];
#pragma unroll
        for (int m = 0; m < M; ++m) bn[m] = B[(uint32_t)nb[m] < (uint32_t)a.Q ? nb[m] : q];
        int cq = 0;
#pragma unroll
        for (int m = 0; m < M; ++m) cq += nb[m] == q;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            int cc = 0;
#pragma unroll
            for (int m = 0; m < M; ++m) cc += nb[m] == nb[k];
            // unlike bonds after minus before; an unused slot gets d = 0
            d[k] = (a.J_fx * (cq - cc) + bn[k] - bq) & -(int32_t)use[k];
        }
    }
    uint32_t t[M];
#pragma unroll
    for (int k = 0; k < M; ++k) t[k] = nf_global(a.Tg)[min(max(d[k], 0), a.Dmax)];   // d <= 0 reads T[0], unused
    uint64_t w = 0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const uint64_t wk = d[k] <= 0 ? (1ull << 32) : (uint64_t)t[k];
        w += wk & (0ull - (uint64_t)use[k]);
    }
    return w;
}

// Candidate spin of slot k in the symmetric trial mode.
__device__ __forceinline__ int32_t nf_uniform_candidate(const NfLat& a, int32_t q, int k) {
    const int32_t c = q + 1 + k;
    return c >= a.Q ? c - a.Q : c;
}

// Weight of site j; in the neighbour mode `only` < 0 counts every slot,
// otherwise slot `only` alone (its candidate returned in cand, -1 if empty).
// Values outside [0, Q) (a wrapped buffer may hold them) are inert, as in
// the sweep: such a site never moves and such a neighbour is never proposed.
template <int NBR, typename Spin, bool kUniform, bool kPair>
__device__ uint64_t nf_site_weight(const Spin* s, const NfLat& a, const int32_t* B, uint32_t j, int only,
                                   int32_t& cand) {
    int32_t nb[nf_M<NBR>()];
    const int32_t q = nf_gather<NBR>(s, a, j, nb);
    uint64_t w = 0;
    cand = -1;
    const bool q_ok = (uint32_t)q < (uint32_t)a.Q;
    if constexpr (kUniform) {
        if (!q_ok) return 0;
        for (int k = 0; k < a.S; ++k) w += nf_slot_weight<NBR, kPair>(a, B, q, nf_uniform_candidate(a, q, k), nb);
    } else {
        // no early exit for a site outside [0, Q): its slots are simply unused,
        // so the spin reads never wait for a branch on q
        bool use[nf_M<NBR>()];
#pragma unroll
        for (int k = 0; k < nf_M<NBR>(); ++k) {
            const bool valid = q_ok && nb[k] != q && (uint32_t)nb[k] < (uint32_t)a.Q;
            if (k == only) cand = valid ? nb[k] : -1;
            use[k] = (only < 0 || k == only) && valid;
        }
        w = nf_slots_weight<NBR, kPair>(a, B, q_ok ? q : 0, nb, use);
    }
    return w;
}

// Weight of site j in the neighbour mode as if site `at` held spin `val`
// (at = ~0: as it is); `only` < 0 counts every slot, otherwise slot `only`
// alone (its candidate returned in cand).  One code path for every lane of
// a pass, whatever it weighs.
template <int NBR, typename Spin, bool kPair>
__device__ uint64_t nf_site_weight_if(const Spin* s, const NfLat& a, const int32_t* B, uint32_t j, uint32_t at,
                                      int32_t val, int only, int32_t& cand) {
    constexpr int M = nf_M<NBR>();
    uint32_t x, y, z;
    nf_coords(a, j, x, y, z);
    int32_t nb[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const uint32_t n = nf_neighbour<NBR>(a, x, y, z, k);
        const int32_t v = (int32_t)s[n];
        nb[k] = n == at ? val : v;
    }
    const int32_t sj = (int32_t)s[j];
    const int32_t q = j == at ? val : sj;
    cand = -1;
    const bool q_ok = (uint32_t)q < (uint32_t)a.Q;
    bool use[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const bool valid = q_ok && nb[k] != q && (uint32_t)nb[k] < (uint32_t)a.Q;
        if (k == only) cand = valid ? nb[k] : -1;
        use[k] = (only < 0 || k == only) && valid;
    }
    return nf_slots_weight<NBR, kPair>(a, B, q_ok ? q : 0, nb, use);
}

template <int NBR, typename Spin, bool kUniform, bool kPair>
__device__ __forceinline__ uint64_t nf_site_weight(const Spin* s, const NfLat& a, const int32_t* B, uint32_t j) {
    int32_t unused;
    return nf_site_weight<NBR, Spin, kUniform, kPair>(s, a, B, j, -1, unused);
}

template <int NBR, typename Spin, bool kUniform, bool kPair>
__global__ __launch_bounds__(kNfThreads) void nfold_kernel(const NfLat* __restrict__ lats, int64_t max_events) {
    extern __shared__ __align__(16) unsigned char nf_lds[];
    const NfLat a = lats[blockIdx.x];
    const int lane = (int)threadIdx.x;
    NfClock* clk = a.clock;
    if (clk->state != kNfRunning) return;

    constexpr int M = nf_M<NBR>();
    static_assert(M < 32, "slot lanes and site lanes share the wave");
    const NfLevels lv = nf_levels(a.N);
    Spin* s = reinterpret_cast<Spin*>(nf_lds);
    uint64_t* tree = reinterpret_cast<uint64_t*>(nf_lds + nf_spin_bytes_lds(a.N, sizeof(Spin)));
    uint64_t* root = tree + lv.total;
    int32_t* B = reinterpret_cast<int32_t*>(root + 1);

    const auto* gs = nf_global(static_cast<const Spin*>(a.spins));
    for (uint32_t i = (uint32_t)lane; i < a.N; i += kNfThreads) s[i] = gs[i];
    for (int32_t q = lane; q < a.Q; q += kNfThreads) B[q] = nf_global(a.B)[q];
    __syncthreads();
    // level 1: the weight of every run of 64 sites
    for (uint32_t b = 0; b < lv.n[1]; ++b) {
        const uint32_t j = b * 64u + (uint32_t)lane;
        const uint64_t w = j < a.N ? nf_site_weight<NBR, Spin, kUniform, kPair>(s, a, B, j) : 0ull;
        const uint64_t tot = wave_sum(w);
        if (lane == 0) tree[lv.off[1] + b] = tot;
    }
    __syncthreads();
#pragma unroll
    for (int L = 2; L <= kNfMaxLevels; ++L) {   // unrolled: the level tables stay in registers
        if (L > lv.T) break;
        for (uint32_t b = 0; b < lv.n[L]; ++b) {
            const uint32_t c = b * 64u + (uint32_t)lane;
            const uint64_t v = c < lv.n[L - 1] ? tree[lv.off[L - 1] + c] : 0ull;
            const uint64_t tot = wave_sum(v);
            if (lane == 0) tree[lv.off[L] + b] = tot;
        }
        __syncthreads();
    }
    {
        uint32_t nT = lv.n[1], oT = lv.off[1];
#pragma unroll
        for (int L = 2; L <= kNfMaxLevels; ++L)
            if (L == lv.T) {
                nT = lv.n[L];
                oT = lv.off[L];
            }
        const uint64_t v = (uint32_t)lane < nT ? tree[oT + lane] : 0ull;
        const uint64_t tot = wave_sum(v);
        if (lane == 0) *root = tot;
    }
    __syncthreads();

    // Neighbourhoods of at most six take the speculative path below, which
    // keeps W in a register (the root in LDS is then only the initial sum).
    constexpr bool kSpec = !kUniform && M <= 6;
    uint64_t W_reg = *root;
    double t_last = clk->t_last;
    uint64_t n = clk->n_events;
    int32_t state = kNfRunning;
    for (int64_t done = 0; done < max_events; ++done) {
        const uint64_t W = kSpec ? W_reg : *root;
        if (W == 0ull) {
            state = kNfNoEvent;
            break;
        }
        NfWords wd;
        wd.start(n, a.k0, a.k1, lane);
        uint64_t u = wd.next();
        u |= (uint64_t)wd.next() << 32;
        const uint64_t E = nf_exponential<>(wd);
        const double t_next = t_last + (double)(E * (uint64_t)a.S) / (double)W;
        if (!(t_next <= a.t_end)) {
            state = kNfReached;
            break;
        }
        uint64_t r = __umul64hi(u, W);
        // descent: top level, ..., level 1, then the sites of one run
        uint32_t p = 0;
        bool ok = true;
#pragma unroll
        for (int L = kNfMaxLevels; L >= 1; --L) {
            if (L > lv.T || !ok) continue;
            const uint32_t c = p * 64u + (uint32_t)lane;
            const uint64_t v = c < lv.n[L] ? tree[lv.off[L] + c] : 0ull;
            const int pick = wave_pick(v, r);
            ok = pick >= 0 && p * 64u + (uint32_t)pick < lv.n[L];
            p = ok ? p * 64u + (uint32_t)pick : 0u;
        }
        uint32_t site = 0;
        if (ok) {
            const uint32_t j = p * 64u + (uint32_t)lane;
            const uint64_t w = j < a.N ? nf_site_weight<NBR, Spin, kUniform, kPair>(s, a, B, j) : 0ull;
            const int pick = wave_pick(w, r);
            ok = pick >= 0 && p * 64u + (uint32_t)pick < a.N;
            site = ok ? p * 64u + (uint32_t)pick : 0u;
        }
        // Neighbourhoods of at most six: one pass weighs the chosen site's
        // slots (lanes 0..M-1), the site and its neighbours before the flip
        // (lanes M..2M) and, for every slot it might take, after it (lanes
        // 2M+1 + s(M+1) + a), so no pass has to wait for the flip.
        if constexpr (kSpec) {
            if (!ok) {
                state = kNfBroken;
                break;
            }
            constexpr int kB = M, kA = 2 * M + 1;
            int role_a = -1, role_s = -1;
            if (lane >= kB && lane < kA) role_a = lane - kB;
            if (lane >= kA && lane < kA + M * (M + 1)) {
                role_s = (lane - kA) / (M + 1);
                role_a = lane - kA - role_s * (M + 1);
            }
            const uint32_t jr = role_a >= 1 ? nf_neighbour_of<NBR>(a, site, role_a - 1) : site;
            const int32_t val = (int32_t)s[nf_neighbour_of<NBR>(a, site, role_s >= 0 ? role_s : 0)];
            int32_t cand = -1;
            const uint64_t w = nf_site_weight_if<NBR, Spin, kPair>(s, a, B, jr, role_s >= 0 ? site : ~0u, val,
                                                                    role_a >= 0 ? -1 : lane, cand);
            const int pick = wave_pick(lane < M ? w : 0ull, r);
            const int32_t cnew = (int32_t)lane_value((uint32_t)cand, pick < 0 ? 0 : pick);
            if (pick < 0 || cnew < 0 || cnew >= a.Q) {   // the tree disagrees with the spins
                state = kNfBroken;
                break;
            }
            // lanes M..2M take the weight after the chosen flip from its lane
            const int src = kA + pick * (M + 1) + (role_a >= 0 && role_s < 0 ? role_a : 0);
            const uint64_t after = __shfl(w, src, 64);
            const bool upd = role_a >= 0 && role_s < 0;
            const uint64_t delta = upd ? after - w : 0ull;
            if (upd && delta != 0ull) {
                uint32_t idx = jr;
#pragma unroll
                for (int L = 1; L <= kNfMaxLevels; ++L) {
                    if (L > lv.T) break;
                    idx >>= 6;
                    atomicAdd(reinterpret_cast<unsigned long long*>(&tree[lv.off[L] + idx]), (unsigned long long)delta);
                }
            }
            // the new total from the M+1 site lanes
#pragma unroll
            for (int i = 0; i <= M; ++i) W_reg += lane_value64(delta, kB + i);
            if (lane == 0) s[site] = (Spin)cnew;
            // One wave per workgroup executes its LDS operations in order, so
            // the next event's reads see these writes without waiting for them
            // here; the fence keeps the compiler from moving accesses across.
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            t_last = t_next;
            ++n;
            continue;
        }
        // lanes 32..32+M: the site and its M neighbours, whose weights change
        const int aff = lane - 32;
        const bool act = aff >= 0 && aff <= M;
        const uint32_t ja = aff >= 1 && aff <= M ? nf_neighbour_of<NBR>(a, site, aff - 1) : site;
        int32_t cnew = -1;
        uint64_t before = 0;
        if constexpr (kUniform) {
            if (ok) {   // lane k takes slot k of the chosen site
                int32_t nb[M];
                const int32_t q = nf_gather<NBR>(s, a, site, nb);
                const int32_t cand = lane < a.S ? nf_uniform_candidate(a, q, lane) : -1;
                const uint64_t w = cand >= 0 ? nf_slot_weight<NBR, kPair>(a, B, q, cand, nb) : 0ull;
                const int pick = wave_pick(w, r);
                ok = pick >= 0;
                cnew = (int32_t)lane_value((uint32_t)cand, pick < 0 ? 0 : pick);
            }
            before = act ? nf_site_weight<NBR, Spin, kUniform, kPair>(s, a, B, ja) : 0ull;
        } else if (ok) {
            // one pass: lanes k < M weigh slot k of the chosen site, the site
            // lanes weigh every slot of their site (before the flip)
            int32_t cand = -1;
            const uint64_t w = nf_site_weight<NBR, Spin, kUniform, kPair>(s, a, B, act ? ja : site,
                                                                          act ? -1 : lane, cand);
            before = act ? w : 0ull;
            const int pick = wave_pick(lane < M ? w : 0ull, r);
            ok = pick >= 0;
            cnew = (int32_t)lane_value((uint32_t)cand, pick < 0 ? 0 : pick);
        }
        ok = ok && cnew >= 0 && cnew < a.Q;
        if (!ok) {   // the tree disagrees with the spins: stop and report
            state = kNfBroken;
            break;
        }
        __syncthreads();
        if (lane == 0) s[site] = (Spin)cnew;
        __syncthreads();
        const uint64_t after = act ? nf_site_weight<NBR, Spin, kUniform, kPair>(s, a, B, ja) : 0ull;
        if (act && after != before) {
            const unsigned long long delta = (unsigned long long)(after - before);
            uint32_t idx = ja;
#pragma unroll
            for (int L = 1; L <= kNfMaxLevels; ++L) {
                if (L > lv.T) break;
                idx >>= 6;
                atomicAdd(reinterpret_cast<unsigned long long*>(&tree[lv.off[L] + idx]), delta);
            }
            atomicAdd(reinterpret_cast<unsigned long long*>(root), delta);
        }
        __syncthreads();
        t_last = t_next;
        ++n;
    }
    Spin* out = static_cast<Spin*>(a.spins);
    for (uint32_t i = (uint32_t)lane; i < a.N; i += kNfThreads) out[i] = s[i];
    if (lane == 0) {
        clk->t_last = t_last;
        clk->n_events = n;
        clk->state = state;
    }
}

template <int NBR, typename Spin>
const void* nf_kernel_for(bool uniform, bool pair) {
    if (uniform) return reinterpret_cast<const void*>(&nfold_kernel<NBR, Spin, true, false>);
    if (pair) return reinterpret_cast<const void*>(&nfold_kernel<NBR, Spin, false, true>);
    return reinterpret_cast<const void*>(&nfold_kernel<NBR, Spin, false, false>);
}

template <int NBR>
const void* nf_kernel_spin(int spin, bool uniform, bool pair) {
    return spin == HMC_I16 ? nf_kernel_for<NBR, int16_t>(uniform, pair) : nf_kernel_for<NBR, int32_t>(uniform, pair);
}

const void* nf_kernel_ptr(int nbr, int spin, bool uniform, bool pair) {
    switch (nbr) {
    case HMC_VN4: return nf_kernel_spin<HMC_VN4>(spin, uniform, pair);
    case HMC_MOORE8: return nf_kernel_spin<HMC_MOORE8>(spin, uniform, pair);
    case HMC_VN6: return nf_kernel_spin<HMC_VN6>(spin, uniform, pair);
    default: return nf_kernel_spin<HMC_MOORE26>(spin, uniform, pair);
    }
}

// Launch arguments and clocks of a batch, kept per device between calls.
// T(d) for d = 0..Dmax at one kT.  Lattices of a batch that share kT share
// one table sized for the largest Dmax among them: the values depend on d
// and kT only, and one table stays in L2 where a table per lattice would not.
struct NfTable {
    uint32_t kT_bits = 0;
    int64_t Dmax = -1;
    uint32_t* dev = nullptr;
    size_t bytes = 0;
    uint64_t used = 0;
};
constexpr size_t kNfTablesKept = 4;                // tables kept per device between calls
constexpr size_t kNfTableCapBytes = 64ull << 20;

struct NfBuffers {
    void* d_lats = nullptr;
    size_t lats_bytes = 0;
    NfClock* d_clocks = nullptr;
    size_t clocks_bytes = 0;
    std::vector<NfTable> tables;
    uint64_t tick = 0;
};

// A table covering d = 0..Dmax at kT (a cached one with a larger Dmax
// serves as well); returns its device pointer and its Dmax.  A table used
// since call_tick (by an earlier lattice of the same call) is never evicted.
hmc_status nf_table(NfBuffers& b, float kT, int64_t Dmax, hipStream_t st, uint64_t call_tick, const uint32_t*& out,
                    int32_t& out_Dmax) {
    uint32_t bits;
    std::memcpy(&bits, &kT, sizeof bits);
    for (NfTable& t : b.tables)
        if (t.dev && t.kT_bits == bits && t.Dmax >= Dmax) {
            t.used = ++b.tick;
            out = t.dev;
            out_Dmax = (int32_t)t.Dmax;
            return HMC_OK;
        }
    const size_t bytes = (size_t)(Dmax + 1) * sizeof(uint32_t);
    if (Dmax > INT32_MAX || bytes > kNfTableCapBytes)
        return fail(HMC_E_RANGE, "n-fold way: threshold table would need " + std::to_string(bytes) + " bytes");
    NfTable* slot = nullptr;
    if (b.tables.size() >= kNfTablesKept)
        for (NfTable& t : b.tables)
            if (t.used < call_tick && (!slot || t.used < slot->used)) slot = &t;
    if (!slot) {
        b.tables.emplace_back();
        slot = &b.tables.back();
    }
    dev_free(slot->dev, slot->bytes);
    *slot = NfTable{};
    std::vector<uint32_t> host((size_t)Dmax + 1);
    host[0] = 0xFFFFFFFFu;   // d <= 0 never reads the table
    for (int64_t d = 1; d <= Dmax; ++d) host[(size_t)d] = threshold_value(d, kT);
    HMC_TRY(dev_alloc(reinterpret_cast<void**>(&slot->dev), bytes, "n-fold threshold table"));
    slot->bytes = bytes;
    HMC_HIP(hipMemcpyAsync(slot->dev, host.data(), bytes, hipMemcpyHostToDevice, st));
    HMC_HIP(hipStreamSynchronize(st));
    slot->kT_bits = bits;
    slot->Dmax = Dmax;
    slot->used = ++b.tick;
    out = slot->dev;
    out_Dmax = (int32_t)Dmax;
    return HMC_OK;
}
std::mutex g_nf_mutex;
std::vector<NfBuffers> g_nf_buffers;

hmc_status nf_buffers(int device, size_t n, NfBuffers*& out) {
    if ((size_t)device >= g_nf_buffers.size()) g_nf_buffers.resize((size_t)device + 1);
    NfBuffers& b = g_nf_buffers[(size_t)device];
    if (b.lats_bytes < n * sizeof(NfLat)) {
        dev_free(b.d_lats, b.lats_bytes);
        b.d_lats = nullptr;
        b.lats_bytes = 0;
        HMC_TRY(dev_alloc(&b.d_lats, n * sizeof(NfLat), "n-fold arguments"));
        b.lats_bytes = n * sizeof(NfLat);
    }
    if (b.clocks_bytes < n * sizeof(NfClock)) {
        dev_free(b.d_clocks, b.clocks_bytes);
        b.d_clocks = nullptr;
        b.clocks_bytes = 0;
        HMC_TRY(dev_alloc(reinterpret_cast<void**>(&b.d_clocks), n * sizeof(NfClock), "n-fold clocks"));
        b.clocks_bytes = n * sizeof(NfClock);
    }
    out = &b;
    return HMC_OK;
}

// One wave per event stream: the waiting-time variate of events n0, n0+1, ...
// drawn after the two selection words, with the event loop's own code.
template <int kWin>
__global__ __launch_bounds__(kNfThreads) void nfold_exponential_kernel(uint64_t n0, int64_t count, uint32_t k0,
                                                                       uint32_t k1, uint64_t* __restrict__ out) {
    const int lane = (int)threadIdx.x;
    for (int64_t e = blockIdx.x; e < count; e += gridDim.x) {
        NfWords wd;
        wd.start(n0 + (uint64_t)e, k0, k1, lane);
        (void)wd.next();
        (void)wd.next();
        const uint64_t E = nf_exponential<kWin>(wd);
        if (lane == 0) out[e] = E;
    }
}

}  // namespace

hmc_status nfold_exponentials(uint64_t seed, uint64_t n0, int64_t count, int32_t window, uint64_t* out) {
    const void* kfn = window == 64   ? reinterpret_cast<const void*>(&nfold_exponential_kernel<64>)
                      : window == 16 ? reinterpret_cast<const void*>(&nfold_exponential_kernel<16>)
                      : window == 7  ? reinterpret_cast<const void*>(&nfold_exponential_kernel<7>)
                      : window == 4  ? reinterpret_cast<const void*>(&nfold_exponential_kernel<4>)
                                     : nullptr;
    if (!kfn) return fail(HMC_E_INVAL, "window must be 4, 7, 16 or 64");
    if (count < 0 || (count > 0 && !out)) return fail(HMC_E_INVAL, "NULL output or count < 0");
    if (count > (1ll << 26)) return fail(HMC_E_RANGE, "count must be at most 2^26");
    if (count == 0) return HMC_OK;
    void* d = nullptr;
    const size_t bytes = (size_t)count * sizeof(uint64_t);
    HMC_TRY(dev_alloc(&d, bytes, "n-fold exponentials"));
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    uint64_t* dout = static_cast<uint64_t*>(d);
    void* kargs[] = {&n0, &count, &k0, &k1, &dout};
    const unsigned grid = (unsigned)std::min<int64_t>(count, 4096);
    hipError_t e = hipLaunchKernel(kfn, dim3(grid), dim3(kNfThreads), kargs, 0, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out, d, bytes, hipMemcpyDeviceToHost);
    dev_free(d, bytes);
    if (e != hipSuccess) return hip_fail(e, "n-fold exponentials");
    return HMC_OK;
}

size_t nfold_lds_bytes(int64_t N, size_t spin_bytes, int32_t Q) { return nf_lds_bytes((uint32_t)N, spin_bytes, Q); }

hmc_status launch_nfold(hmc_lattice* const* lats, int32_t count, const float* kT, double mcs, const uint64_t* seed) {
    for (int32_t b = 0; b < count; ++b)   // the weight tree has at most kNfMaxLevels levels of 64-way sums
        if (lats[b]->N > (1ll << (6 * kNfMaxLevels)))
            return fail(HMC_E_RANGE, "n-fold way: at most 64^3 sites per lattice");
    hmc_lattice* L0 = lats[0];
    const bool uniform = L0->desc.proposal == HMC_PROP_UNIFORM;
    size_t lds = 0;
    std::vector<NfLat> args((size_t)count);
    std::vector<NfClock> clocks((size_t)count);
    // the largest energy change of each lattice, and of each temperature
    std::vector<int64_t> Dmax((size_t)count);
    std::vector<std::pair<uint32_t, int64_t>> groups;   // (kT bits, largest Dmax)
    for (int32_t b = 0; b < count; ++b) {
        const hmc_lattice* L = lats[b];
        const int64_t bond = L->pair ? L->Jp_max : L->desc.J_fx;
        Dmax[(size_t)b] = (int64_t)L->M * bond + ((int64_t)L->Bmax - L->Bmin);
        uint32_t bits;
        std::memcpy(&bits, &kT[b], sizeof bits);
        bool found = false;
        for (auto& g : groups)
            if (g.first == bits) {
                g.second = std::max(g.second, Dmax[(size_t)b]);
                found = true;
            }
        if (!found) groups.emplace_back(bits, Dmax[(size_t)b]);
    }
    std::lock_guard<std::mutex> lock(g_nf_mutex);
    NfBuffers* buf = nullptr;
    HMC_TRY(nf_buffers(L0->device, (size_t)count, buf));
    const uint64_t call_tick = buf->tick + 1;
    for (int32_t b = 0; b < count; ++b) {
        hmc_lattice* L = lats[b];
        // the batch runs on the first lattice's stream: wait for work still
        // queued on another lattice's stream (an idle stream costs a query)
        if (L->stream != L0->stream) {
            const hipError_t q = hipStreamQuery(L->stream);
            if (q == hipErrorNotReady) HMC_HIP(hipStreamSynchronize(L->stream));
            else if (q != hipSuccess) return hip_fail(q, "hipStreamQuery");
        }
        NfLat& a = args[(size_t)b];
        uint32_t bits;
        std::memcpy(&bits, &kT[b], sizeof bits);
        int64_t gmax = Dmax[(size_t)b];
        for (const auto& g : groups)
            if (g.first == bits) gmax = g.second;
        HMC_TRY(nf_table(*buf, kT[b], gmax, L0->stream, call_tick, a.Tg, a.Dmax));
        a.spins = L->spins[L->cur];
        a.B = L->dB;
        a.Jp = L->pair ? L->d_Jp : nullptr;
        a.t_end = L->nf_t_now + mcs;
        a.Lx = (uint32_t)L->desc.dims[0];
        a.Ly = (uint32_t)L->desc.dims[1];
        a.Lz = (uint32_t)(L->ndim == 3 ? L->desc.dims[2] : 1);
        a.N = (uint32_t)L->N;
        a.mx = (uint32_t)(((1ull << 32) + a.Lx - 1) / a.Lx);
        a.my = (uint32_t)(((1ull << 32) + a.Ly - 1) / a.Ly);
        a.Q = L->Q;
        a.J_fx = L->desc.J_fx;
        a.S = uniform ? L->Q - 1 : L->M;
        a.k0 = (uint32_t)(seed[b] & 0xFFFFFFFFu);
        a.k1 = (uint32_t)(seed[b] >> 32);
        clocks[(size_t)b] = NfClock{L->nf_t_last, (unsigned long long)L->nf_events, kNfRunning, 0};
        lds = std::max(lds, nf_lds_bytes(a.N, L->spin_bytes, L->Q));
    }
    for (int32_t b = 0; b < count; ++b) args[(size_t)b].clock = buf->d_clocks + b;
    hipStream_t st = L0->stream;
    HMC_HIP(hipMemcpyAsync(buf->d_lats, args.data(), args.size() * sizeof(NfLat), hipMemcpyHostToDevice, st));
    HMC_HIP(hipMemcpyAsync(buf->d_clocks, clocks.data(), clocks.size() * sizeof(NfClock), hipMemcpyHostToDevice,
                           st));
    const void* kfn = nf_kernel_ptr(L0->desc.nbr, L0->desc.spin, uniform, L0->pair);
    const NfLat* d_lats = static_cast<const NfLat*>(buf->d_lats);
    int64_t cap = kNfEventsPerLaunch;
    void* kargs[] = {&d_lats, &cap};
    for (;;) {
        if (L0->profiling) {
            if (L0->events_used == L0->events.size()) {
                hipEvent_t e0, e1;
                HMC_HIP(hipEventCreate(&e0));
                HMC_HIP(hipEventCreate(&e1));
                L0->events.emplace_back(e0, e1);
            }
            const auto& ev = L0->events[L0->events_used++];
            HMC_HIP(hipExtLaunchKernel(kfn, dim3((unsigned)count), dim3(kNfThreads), kargs, lds, st, ev.first,
                                       ev.second, 0));
            L0->prof_launches += 1;
        } else {
            HMC_HIP(hipLaunchKernel(kfn, dim3((unsigned)count), dim3(kNfThreads), kargs, lds, st));
        }
        HMC_HIP(hipMemcpyAsync(clocks.data(), buf->d_clocks, clocks.size() * sizeof(NfClock), hipMemcpyDeviceToHost,
                               st));
        HMC_HIP(hipStreamSynchronize(st));
        bool running = false;
        for (const NfClock& c : clocks) {
            if (c.state == kNfBroken) return fail(HMC_E_INTERNAL, "n-fold way: weight tree out of step with the spins");
            running = running || c.state == kNfRunning;
        }
        if (!running) break;
    }
    for (int32_t b = 0; b < count; ++b) {
        hmc_lattice* L = lats[b];
        L->nf_t_last = clocks[(size_t)b].t_last;
        L->nf_events = clocks[(size_t)b].n_events;
        L->nf_t_now = args[(size_t)b].t_end;
    }
    return HMC_OK;
}

}  // namespace hmc
