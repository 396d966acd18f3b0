// common.hpp -- internal declarations shared by the libhmc translation units.
//
// Nothing here is part of the ABI (include/hmc.h is).  The lattice object,
// error plumbing, device-memory accounting and the Philox4x32-10 generator
// (Salmon, Moraes, Dror, Shaw, SC'11) used by both the host (Voronoi seed
// points) and the kernels (Metropolis trials).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "hmc.h"

namespace hmc {

// ------------------------------------------------------------------ errors

void set_error(const std::string& msg);
hmc_status fail(hmc_status code, const std::string& msg);
hmc_status hip_fail(hipError_t e, const char* what);

#define HMC_HIP(call)                                             \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return ::hmc::hip_fail(e_, #call);  \
    } while (0)

#define HMC_TRY(call)                         \
    do {                                      \
        hmc_status s_ = (call);               \
        if (s_ != HMC_OK) return s_;          \
    } while (0)

// Device allocation with the optional HMC_MAX_BYTES cap.
hmc_status dev_alloc(void** p, size_t bytes, const char* what);
void dev_free(void* p, size_t bytes);

// ------------------------------------------------------------------ Philox

struct Philox2 {   // the two words the sweep consumes
    uint32_t r0, r1;
};

// a ^ b ^ c; on the device one three-input logic instruction (truth table
// 0x96) in place of two exclusive ors
__host__ __device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
    return a ^ b ^ c;
#endif
}

// Philox4x32-10: ten rounds of two 32x32->64 products on counter words 0 and
// 2 with the round key mixed into the high halves; Weyl key schedule.
__host__ __device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                       uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)0xD2511F53u * c0;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(pb >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(pa >> 32), c3, k1);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

__device__ __forceinline__ Philox2 philox_r01(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1) {
    uint32_t o[4];
    philox4x32_10(c0, c1, c2, c3, k0, k1, o);
    return Philox2{o[0], o[1]};
}

// ------------------------------------------------------- like neighbours

// (neighbours equal to q) - (neighbours equal to qn) over M 16-bit spin
// values (M even).  The values go two to a register as 16-bit halves; per
// half, min(x ^ y, 1) is 1 where two spins differ, so one packed minimum
// tests two neighbours, and the difference of the likes is the difference of
// the unlikes taken the other way round.
template <int M>
__device__ __forceinline__ int32_t like_difference16(const int32_t* nb, int32_t q, int32_t qn) {
    static_assert(M % 2 == 0 && M <= 64, "pairs of neighbours, per-half counts below 2^15");
    auto pack = [](int32_t hi, int32_t lo) __attribute__((always_inline)) {
        return __builtin_amdgcn_perm((uint32_t)hi, (uint32_t)lo, 0x05040100u);
    };
    auto ne = [](uint32_t x) __attribute__((always_inline)) -> uint32_t {
        uint32_t r;
        asm("v_pk_min_u16 %0, %1, %2" : "=v"(r) : "v"(x), "s"(0x00010001u));
        return r;
    };
    const uint32_t qq = pack(q, q), nn = pack(qn, qn);
    uint32_t uq = 0, un = 0;
#pragma unroll
    for (int k = 0; k < M; k += 2) {
        const uint32_t p = pack(nb[k + 1], nb[k]);
        uq += ne(p ^ qq);
        un += ne(p ^ nn);
    }
    const uint32_t D = un + (uint32_t)(M / 2) * 0x00010001u - uq;   // per half in [0, M]
    return (int32_t)((D & 0xFFFFu) + (D >> 16)) - M;
}

// --------------------------------------------------------------- geometry

struct NbrInfo {
    int M;      // neighbours
    int C;      // colours
    int ndim;
};
NbrInfo nbr_info(int nbr);

// Offsets (dx, dy, dz) of neighbour k in the fixed trial order:
// VN4 +x,-x,+y,-y; VN6 adds +z,-z; Moore8 adds (+1,+1),(-1,-1),(+1,-1),(-1,+1);
// Moore26 runs over {-1,0,1}^3 without the centre, lexicographic in (dz,dy,dx).
__host__ __device__ constexpr int nbr_dx(int nbr, int k) {
    if (nbr == HMC_MOORE26) return ((k < 13 ? k : k + 1) % 3) - 1;
    if (k == 0) return 1;
    if (k == 1) return -1;
    if (nbr == HMC_MOORE8 && (k == 4 || k == 6)) return 1;
    if (nbr == HMC_MOORE8 && (k == 5 || k == 7)) return -1;
    return 0;
}
__host__ __device__ constexpr int nbr_dy(int nbr, int k) {
    if (nbr == HMC_MOORE26) return (((k < 13 ? k : k + 1) / 3) % 3) - 1;
    if (k == 2) return 1;
    if (k == 3) return -1;
    if (nbr == HMC_MOORE8 && (k == 4 || k == 7)) return 1;
    if (nbr == HMC_MOORE8 && (k == 5 || k == 6)) return -1;
    return 0;
}
__host__ __device__ constexpr int nbr_dz(int nbr, int k) {
    if (nbr == HMC_MOORE26) return ((k < 13 ? k : k + 1) / 9) - 1;
    if (nbr == HMC_VN6 && k == 4) return 1;
    if (nbr == HMC_VN6 && k == 5) return -1;
    return 0;
}

// ----------------------------------------------------- threshold table

// T(d) for every d > 0 the lattice can produce, laid out as
// T[(dn - dn_lo) * TW + (dB + R)] with dn = c(q) - c(q'), dB = B[q'] - B[q],
// R = max B - min B, TW = 2R + 1.
// Each row is split into nb buckets of bw consecutive columns; bounds[2*k]
// is T at the largest d of bucket k (a lower bound of T over the bucket),
// bounds[2*k+1] T at its smallest positive d (an upper bound).  T is
// non-increasing in d, so a trial whose r1 falls outside [lower, upper) is
// decided by the bucket's two numbers alone; kBoundPairs bounds the count.
constexpr int kBoundPairs = 512;
struct Table {
    uint32_t* dev = nullptr;      // rows * TW entries (the current slot)
    uint32_t* bounds = nullptr;   // 2 * rows * nb entries
    size_t bytes = 0;             // allocation behind dev (bounds included)
    // two device slots, each filled from its own pinned staging buffer: a
    // new table goes to the slot the queued sweeps do not read, in stream
    // order, without the host waiting for them
    uint32_t* slot_dev[2] = {nullptr, nullptr};
    size_t slot_bytes[2] = {0, 0};
    uint32_t* pin[2] = {nullptr, nullptr};
    size_t pin_bytes[2] = {0, 0};
    hipEvent_t uploaded[2] = {nullptr, nullptr};
    int slot = 0;
    int32_t dn_lo = 0, rows = 0, R = 0, TW = 1;
    int32_t nb = 1, bw = 1;       // buckets per row, columns per bucket
    uint32_t kT_bits = 0;
    int32_t Bmin = 0, Bmax = 0;
    bool valid = false;
};
uint32_t threshold_value(int64_t d, float kT);
struct TableLayout {
    int32_t dn_lo = 0, rows = 0, R = 0, TW = 1, nb = 1, bw = 1;
};
// The table and its bucket bounds on the host: rows * TW entries followed by
// 2 * rows * nb bounds (entries whose d <= 0 hold 2^32 - 1, never read).
hmc_status table_host(float kT, int M, int32_t J_fx, int32_t Bmin, int32_t Bmax, TableLayout& lay,
                      std::vector<uint32_t>& host);
hmc_status build_table(Table& tab, float kT, int M, int32_t J_fx, int32_t Bmin, int32_t Bmax,
                       hipStream_t stream);
// Threshold table T(d) for every d in [0, Dmax] (pair bond energies,
// per-site field).
hmc_status build_direct_table(hmc_lattice* L, float kT);
void free_table(Table& tab);

// ---------------------------------------------------------------- tiling

struct Tiling {
    // interior tile; k > 0: MC steps per launch, k < 0: -k colour passes per
    // launch (part of an MC step), 0: automatic
    int32_t tx = 0, ty = 0, tz = 0, k = 0;
};
inline int launch_passes(const Tiling& t, int C) { return t.k > 0 ? t.k * C : -t.k; }

// Arguments of the six-neighbour 16-bit sweep kernel with compile-time tile
// geometry (sweep_vn6.hip); one or two colour passes per launch.
struct Vn6Args {
    const int16_t* src;
    int16_t* dst;
    const int32_t* B;
    const uint32_t* T;            // threshold table (rows x TW)
    const uint32_t* Tb;           // per-bucket (lower, upper) bounds of T
    uint32_t Lx, Ly, Lz, ntx, nty;
    uint32_t t0, c0, npass;       // MC step and colour of the first pass; passes (1 or 2)
    uint32_t k0, k1;              // Philox key
    int32_t J_fx, Q, dn_lo, TW, R, nb, nbound;
    uint32_t bw, m_bw;
    uint32_t ntiles;              // tiles of the lattice; workgroups walk them in turn
    uint32_t xcd_blocks;          // 1: each XCD's workgroups take one contiguous block of tiles
    unsigned long long* trials;   // profiling: Philox draws, or null
};
// The specialised kernel for tile t (its dynamic LDS size and the
// workgroups per CU it is built for: two when its LDS fits twice) given Q
// grains, or false when t is not one of its compiled tiles or does not fit
// the LDS.
bool vn6_kernel_for(const Tiling& t, int32_t Q, const void** fn, size_t* lds_bytes, int* per_cu);

// --------------------------------------------------------------- lattice

}  // namespace hmc

constexpr int kTrialSlots = 1024;   // spread of the profiling trial counters (power of two)

struct hmc_lattice_s {
    hmc_lattice_desc desc{};
    int32_t Q = 0;
    int64_t N = 0;
    int M = 0, C = 0, ndim = 0;
    size_t spin_bytes = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;

    void* spins[2] = {nullptr, nullptr};
    int cur = 0;
    bool borrowed = false;                  // spins[0] belongs to the caller
    void* snap = nullptr;
    uint64_t snap_mcs = 0;
    bool has_snap = false;
    uint64_t mcs = 0;

    int32_t* dB = nullptr;
    std::vector<int32_t> hB;
    // pinned staging of grain-energy uploads (stream-ordered, no host wait)
    int32_t* hB_pinned = nullptr;
    hipEvent_t hB_uploaded = nullptr;
    int32_t Bmin = 0, Bmax = 0;
    hmc::Table table;

    uint32_t* d_areas = nullptr;            // Q counts
    unsigned long long* d_stats = nullptr;  // 1 + max bins
    int32_t* d_gbin = nullptr;
    int32_t stats_bins_cap = 0;

    hmc::Tiling tiling;
    bool tiling_explicit = false;
    int32_t sweep_kernel = 0;               // HMC_KERNEL_AUTO or HMC_KERNEL_GENERIC

    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    size_t events_used = 0;
    int64_t prof_launches = 0, prof_su = 0;
    unsigned long long* d_trials = nullptr;   // kTrialSlots counters of Philox draws while profiling
    unsigned long long* d_count = nullptr;    // boundary-site count

    // bond energy per pair of spins (Eq. (7)'s J_{q_i,q_n}); off: uniform J_fx
    bool pair = false;
    int32_t* d_Jp = nullptr;                  // int32[Q*Q]
    int32_t Jp_max = 0;
    uint32_t* d_Tg = nullptr;                 // T(d), d = 0..Tg_Dmax
    size_t Tg_bytes = 0;
    uint32_t Tg_kT_bits = 0;
    int32_t Tg_Dmax = -1;

    // per-site bulk field (Eq. (7)'s b_i inside grains), ping-pong with the spins
    bool field = false;
    int32_t* d_field[2] = {nullptr, nullptr};
    int32_t* field_snap = nullptr;
    int32_t Fmin = 0, Fmax = 0;               // bounds of every value the field can hold
    uint32_t frule = 0;                       // 0 carry, 1 recrystallise

    // clock of the n-fold way (continuous time in MC steps, separate from mcs)
    double nf_t_now = 0.0;                    // time the lattice has been advanced to
    double nf_t_last = 0.0;                   // time of the last executed event
    uint64_t nf_events = 0;                   // events executed (the event counter of the RNG)
    double snap_nf_t_now = 0.0, snap_nf_t_last = 0.0;
    uint64_t snap_nf_events = 0;
};

namespace hmc {

}  // namespace hmc

struct hmc_ensemble_s {
    std::vector<hmc_lattice*> lats;     // borrowed
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    hmc::Tiling tiling;                 // shared by all members
    bool tiling_explicit = false;
    bool prepared = false;
    int32_t maxQ = 0;
    bool vec = false;                   // members staged four 16-bit spins per 8-byte access
    void* d_tiles = nullptr;            // uint2 (lattice, tile) per tile
    size_t tiles_bytes = 0;
    uint32_t ntiles = 0;
    void* d_lats = nullptr;             // one descriptor per member
    size_t lats_bytes = 0;
    // pinned host staging of the descriptors, two slots used in turn; the
    // event after each upload says when its slot may be rewritten
    void* h_stage[2] = {nullptr, nullptr};
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    bool stage_used[2] = {false, false};
    int stage_slot = 0;
    uint32_t grid = 0;
    std::map<int32_t, hipGraphExec_t> graphs;   // captured launch sequences by n_mcs
    uint32_t graph_launches = 0;
    // event pairs around each graph replay while profiling
    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    size_t events_used = 0;
    int64_t prof_launches = 0, prof_su = 0;
};

namespace hmc {

// Kernels (defined in their .hip files).
hmc_status launch_sweep(hmc_lattice* L, float kT, int32_t n_mcs, uint64_t seed);
hmc_status ensemble_prepare(hmc_ensemble* E);
hmc_status launch_ensemble(hmc_ensemble* E, const float* kT, const uint64_t* seed, int32_t n_mcs);
// Autotuned tiling for this lattice shape, or nullptr (tune.hip).
const Tiling* tuned_tiling(const hmc_lattice_desc& d, int32_t Q);
void record_tuning(const hmc_lattice_desc& d, const Tiling& t, double us_per_mcs);
hmc_status choose_tiling(const hmc_lattice* L, Tiling& t, bool explicit_request);
// True when sweeps of L with tiling t run the compiled-tile kernel.
bool compiled_vn6(const hmc_lattice* L, const Tiling& t, const void** fn, size_t* bytes, int* per_cu);
bool compiled_vn6_model(const hmc_lattice* L);
bool compiled2d(const hmc_lattice* L, const Tiling& t, const void** fn, size_t* bytes);
bool compiled_moore26_model(const hmc_lattice* L);
hmc_status launch_voronoi(hmc_lattice* L, uint64_t vseed);
hmc_status launch_boundary_count(hmc_lattice* L);
hmc_status launch_histogram(hmc_lattice* L);   // fills L->d_areas
hmc_status launch_bin_stats(hmc_lattice* L, const int32_t* d_gbin, int32_t n_bins);
// The same two steps on raw device buffers: per-spin areas of N spins
// (values outside [0, Q) not counted) into d_areas[Q], then the
// present-grain count and per-bin areas into d_stats[1 + n_bins] (d_gbin may
// be null when n_bins is 0).  Both clear their outputs with a kernel first.
hmc_status launch_areas(const void* spins, bool i16, uint64_t N, uint32_t Q, uint32_t* d_areas, hipStream_t stream);
hmc_status launch_bins(const uint32_t* d_areas, int32_t Q, const int32_t* d_gbin, int32_t n_bins,
                       unsigned long long* d_stats, hipStream_t stream);
int lds_limit_bytes();
hmc_status settle_borrowed(hmc_lattice* L);

// n-fold way (nfold.hip): LDS a lattice needs, and a batch run of lattices
// that share neighbourhood, spin type, trial mode and bond model.
size_t nfold_lds_bytes(int64_t N, size_t spin_bytes, int32_t Q);
hmc_status nfold_exponentials(uint64_t seed, uint64_t n0, int64_t count, int32_t window, uint64_t* out);
hmc_status launch_nfold(hmc_lattice* const* lats, int32_t count, const float* kT, double mcs, const uint64_t* seed);

}  // namespace hmc
