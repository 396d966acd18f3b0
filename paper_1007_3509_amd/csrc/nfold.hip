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
// one below, the root the total), so an event is a descent of at most four
// levels, each a 64-lane load and a wave-wide 64-bit prefix scan, followed by
// the weights of the site and its M neighbours recomputed before and after
// the flip and their differences added up the tree with LDS atomics.  Site
// weights are not stored: each lane recomputes the weight of its site from
// the spins in LDS when a descent reaches its run of 64.  Batches put many
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
constexpr int kNfMaxLevels = 4;                // 64^4 sites: beyond any LDS-resident lattice
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

__host__ __device__ inline size_t nf_spin_bytes_lds(uint32_t N, size_t spin_bytes) {
    return ((size_t)N * spin_bytes + 15) & ~(size_t)15;
}

inline size_t nf_lds_bytes(uint32_t N, size_t spin_bytes) {
    const NfLevels lv = nf_levels(N);
    return nf_spin_bytes_lds(N, spin_bytes) + 8 * ((size_t)lv.total + 1);
}

// ------------------------------------------------------------------ device

__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t u = __shfl_up(v, (unsigned)o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// First lane whose inclusive sum exceeds r (-1 if none), and r reduced by
// the sum of the lanes before it.
__device__ __forceinline__ int wave_pick(uint64_t v, int lane, uint64_t& r) {
    const uint64_t incl = wave_incl_scan(v, lane);
    const unsigned long long m = __ballot(incl > r);
    if (m == 0ull) return -1;
    const int c = __ffsll((long long)m) - 1;
    r -= __shfl(incl - v, c, 64);
    return c;
}

struct NfWords {               // the words of one event's Philox stream
    uint32_t n_lo, n_hi, k0, k1, j;
    uint32_t b0, b1, b2, b3;
    int used;
    __device__ uint32_t next() {
        if (used == 4) {
            uint32_t o[4];
            philox4x32_10(n_lo, n_hi, kNfTag, j++, k0, k1, o);
            b0 = o[0]; b1 = o[1]; b2 = o[2]; b3 = o[3];
            used = 0;
        }
        const uint32_t w = used == 0 ? b0 : used == 1 ? b1 : used == 2 ? b2 : b3;
        ++used;
        return w;
    }
};

// von Neumann (1951): a trial takes u0 and the length n of the strictly
// decreasing run it starts; odd n accepts E = K + u0 / 2^32, even n adds one
// to K.  Runs are cut at 64 words and K at 64.
__device__ __forceinline__ uint64_t nf_exponential(NfWords& w) {
    uint64_t K = 0;
    for (;;) {
        const uint32_t u0 = w.next();
        uint32_t prev = u0;
        int n = 1;
        while (n < 64) {
            const uint32_t v = w.next();
            if (v < prev) {
                prev = v;
                ++n;
            } else {
                break;
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

template <int NBR>
constexpr int nf_M() {
    return NBR == HMC_VN4 ? 4 : NBR == HMC_MOORE8 ? 8 : NBR == HMC_VN6 ? 6 : 26;
}

// Spin of the site and of its M neighbours.
template <int NBR, typename Spin>
__device__ __forceinline__ int32_t nf_gather(const Spin* s, const NfLat& a, uint32_t j, int32_t* nb) {
    const uint32_t x = j % a.Lx;
    const uint32_t yz = j / a.Lx;
    const uint32_t y = yz % a.Ly;
    const uint32_t z = yz / a.Ly;
#pragma unroll
    for (int k = 0; k < nf_M<NBR>(); ++k) nb[k] = (int32_t)s[nf_neighbour<NBR>(a, x, y, z, k)];
    return (int32_t)s[j];
}

// Weight of moving a site with spin q and neighbour spins nb to spin c != q.
template <int NBR, bool kPair>
__device__ __forceinline__ uint64_t nf_slot_weight(const NfLat& a, int32_t q, int32_t c, const int32_t* nb) {
    constexpr int M = nf_M<NBR>();
    int64_t d;
    if constexpr (kPair) {
        const int32_t* rq = a.Jp + (int64_t)q * a.Q;
        const int32_t* rc = a.Jp + (int64_t)c * a.Q;
        int64_t acc = 0;
#pragma unroll
        for (int m = 0; m < M; ++m) acc += (int64_t)rc[nb[m]] - (int64_t)rq[nb[m]];
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
    d += (int64_t)a.B[c] - (int64_t)a.B[q];
    if (d <= 0) return 1ull << 32;
    return (uint64_t)a.Tg[d < a.Dmax ? d : a.Dmax];
}

// Candidate spin of slot k (-1 if the slot is empty).
template <bool kUniform>
__device__ __forceinline__ int32_t nf_candidate(const NfLat& a, int32_t q, const int32_t* nb, int k) {
    if constexpr (kUniform) {
        int32_t c = q + 1 + k;
        return c >= a.Q ? c - a.Q : c;
    } else {
        return nb[k] == q ? -1 : nb[k];
    }
}

template <int NBR, typename Spin, bool kUniform, bool kPair>
__device__ uint64_t nf_site_weight(const Spin* s, const NfLat& a, uint32_t j) {
    int32_t nb[nf_M<NBR>()];
    const int32_t q = nf_gather<NBR>(s, a, j, nb);
    uint64_t w = 0;
    if constexpr (kUniform) {
        for (int k = 0; k < a.S; ++k) w += nf_slot_weight<NBR, kPair>(a, q, nf_candidate<true>(a, q, nb, k), nb);
    } else {
#pragma unroll
        for (int k = 0; k < nf_M<NBR>(); ++k)
            if (nb[k] != q) w += nf_slot_weight<NBR, kPair>(a, q, nb[k], nb);
    }
    return w;
}

template <int NBR, typename Spin, bool kUniform, bool kPair>
__global__ __launch_bounds__(kNfThreads) void nfold_kernel(const NfLat* __restrict__ lats, int64_t max_events) {
    extern __shared__ __align__(16) unsigned char nf_lds[];
    const NfLat a = lats[blockIdx.x];
    const int lane = (int)threadIdx.x;
    NfClock* clk = a.clock;
    if (clk->state != kNfRunning) return;

    const NfLevels lv = nf_levels(a.N);
    Spin* s = reinterpret_cast<Spin*>(nf_lds);
    uint64_t* tree = reinterpret_cast<uint64_t*>(nf_lds + nf_spin_bytes_lds(a.N, sizeof(Spin)));
    uint64_t* root = tree + lv.total;

    const Spin* gs = static_cast<const Spin*>(a.spins);
    for (uint32_t i = (uint32_t)lane; i < a.N; i += kNfThreads) s[i] = gs[i];
    __syncthreads();
    // level 1: the weight of every run of 64 sites
    for (uint32_t b = 0; b < lv.n[1]; ++b) {
        const uint32_t j = b * 64u + (uint32_t)lane;
        const uint64_t w = j < a.N ? nf_site_weight<NBR, Spin, kUniform, kPair>(s, a, j) : 0ull;
        const uint64_t tot = __shfl(wave_incl_scan(w, lane), 63, 64);
        if (lane == 0) tree[lv.off[1] + b] = tot;
    }
    __syncthreads();
#pragma unroll
    for (int L = 2; L <= kNfMaxLevels; ++L) {   // unrolled: the level tables stay in registers
        if (L > lv.T) break;
        for (uint32_t b = 0; b < lv.n[L]; ++b) {
            const uint32_t c = b * 64u + (uint32_t)lane;
            const uint64_t v = c < lv.n[L - 1] ? tree[lv.off[L - 1] + c] : 0ull;
            const uint64_t tot = __shfl(wave_incl_scan(v, lane), 63, 64);
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
        const uint64_t tot = __shfl(wave_incl_scan(v, lane), 63, 64);
        if (lane == 0) *root = tot;
    }
    __syncthreads();

    double t_last = clk->t_last;
    uint64_t n = clk->n_events;
    int32_t state = kNfRunning;
    constexpr int M = nf_M<NBR>();
    for (int64_t done = 0; done < max_events; ++done) {
        const uint64_t W = *root;
        if (W == 0ull) {
            state = kNfNoEvent;
            break;
        }
        NfWords wd{(uint32_t)n, (uint32_t)(n >> 32), a.k0, a.k1, 0u, 0u, 0u, 0u, 0u, 4};
        uint64_t u = wd.next();
        u |= (uint64_t)wd.next() << 32;
        const uint64_t E = nf_exponential(wd);
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
            const int pick = wave_pick(v, lane, r);
            ok = pick >= 0;
            p = p * 64u + (uint32_t)(ok ? pick : 0);
        }
        int32_t q = 0, nb[M];
        int32_t cnew = -1;
        uint32_t site = 0;
        if (ok) {
            const uint32_t j = p * 64u + (uint32_t)lane;
            const uint64_t w = j < a.N ? nf_site_weight<NBR, Spin, kUniform, kPair>(s, a, j) : 0ull;
            const int pick = wave_pick(w, lane, r);
            ok = pick >= 0;
            site = p * 64u + (uint32_t)(pick < 0 ? 0 : pick);
        }
        if (ok) {
            // the slot: lane k takes slot k of the chosen site
            q = nf_gather<NBR>(s, a, site, nb);
            uint64_t w = 0;
            int32_t cand = -1;
            if (lane < a.S) {
                if constexpr (kUniform) {
                    cand = nf_candidate<true>(a, q, nb, lane);
                } else {
#pragma unroll
                    for (int k = 0; k < M; ++k)
                        if (k == lane) cand = nf_candidate<false>(a, q, nb, k);
                }
                if (cand >= 0) w = nf_slot_weight<NBR, kPair>(a, q, cand, nb);
            }
            const int pick = wave_pick(w, lane, r);
            ok = pick >= 0;
            cnew = __shfl(cand, pick < 0 ? 0 : pick, 64);
            ok = ok && cnew >= 0;
        }
        if (!ok) {   // the tree disagrees with the spins: stop and report
            state = kNfBroken;
            break;
        }
        // the site and its M neighbours change weight
        uint32_t ja = site;
        const bool act = lane <= M;
        if (lane >= 1 && lane <= M) {
            const uint32_t x = site % a.Lx, yz = site / a.Lx;
#pragma unroll
            for (int k = 0; k < M; ++k)
                if (k == lane - 1) ja = nf_neighbour<NBR>(a, x, yz % a.Ly, yz / a.Ly, k);
        }
        const uint64_t before = act ? nf_site_weight<NBR, Spin, kUniform, kPair>(s, a, ja) : 0ull;
        __syncthreads();
        if (lane == 0) s[site] = (Spin)cnew;
        __syncthreads();
        const uint64_t after = act ? nf_site_weight<NBR, Spin, kUniform, kPair>(s, a, ja) : 0ull;
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
struct NfBuffers {
    void* d_lats = nullptr;
    size_t lats_bytes = 0;
    NfClock* d_clocks = nullptr;
    size_t clocks_bytes = 0;
};
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

}  // namespace

size_t nfold_lds_bytes(int64_t N, size_t spin_bytes) { return nf_lds_bytes((uint32_t)N, spin_bytes); }

hmc_status launch_nfold(hmc_lattice* const* lats, int32_t count, const float* kT, double mcs, const uint64_t* seed) {
    hmc_lattice* L0 = lats[0];
    const bool uniform = L0->desc.proposal == HMC_PROP_UNIFORM;
    size_t lds = 0;
    std::vector<NfLat> args((size_t)count);
    std::vector<NfClock> clocks((size_t)count);
    for (int32_t b = 0; b < count; ++b) {
        hmc_lattice* L = lats[b];
        HMC_HIP(hipStreamSynchronize(L->stream));
        HMC_TRY(build_direct_table(L, kT[b]));
        NfLat& a = args[(size_t)b];
        a.spins = L->spins[L->cur];
        a.B = L->dB;
        a.Tg = L->d_Tg;
        a.Jp = L->pair ? L->d_Jp : nullptr;
        a.t_end = L->nf_t_now + mcs;
        a.Lx = (uint32_t)L->desc.dims[0];
        a.Ly = (uint32_t)L->desc.dims[1];
        a.Lz = (uint32_t)(L->ndim == 3 ? L->desc.dims[2] : 1);
        a.N = (uint32_t)L->N;
        a.Q = L->Q;
        a.J_fx = L->desc.J_fx;
        a.Dmax = L->Tg_Dmax;
        a.S = uniform ? L->Q - 1 : L->M;
        a.k0 = (uint32_t)(seed[b] & 0xFFFFFFFFu);
        a.k1 = (uint32_t)(seed[b] >> 32);
        clocks[(size_t)b] = NfClock{L->nf_t_last, (unsigned long long)L->nf_events, kNfRunning, 0};
        lds = std::max(lds, nf_lds_bytes(a.N, L->spin_bytes));
    }
    std::lock_guard<std::mutex> lock(g_nf_mutex);
    NfBuffers* buf = nullptr;
    HMC_TRY(nf_buffers(L0->device, (size_t)count, buf));
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
        HMC_TRY(settle_borrowed(L));
        if (L != L0) HMC_HIP(hipStreamSynchronize(L->stream));
    }
    return HMC_OK;
}

}  // namespace hmc
