// mcp.hip -- Monte Carlo crystal plasticity (MCP) on the GPU, FP64.
//
// Sec. 2 of the paper: rate-independent small-deformation crystal
// plasticity in which one slip system is activated per step.  Candidates are
// the systems whose resolved shear stress exceeds the slip resistance; the
// elastic energy E_a of the crystal after activating candidate a alone sets
// p_a = exp(-beta E_a) / Z (Eq. (1)); system i is taken when
// S_{i-1} <= R < S_i over the cumulative probabilities (Eq. (2)).  Table 1
// gives the nickel constants.  The stored dislocation energy follows Eq. (4):
// E_rho = 2 sigma_f^2 / G.
//
// Readings (the paper does not fix them): "C22" of Table 1 is C12; MPa
// units with beta = 1000 / MPa; FCC {111}<110> systems in a fixed order;
// Voce hardening tau_c(G) = tau_s - (tau_s - tau_0) exp(-h0 G / (tau_s -
// tau_0)); linearised single-slip return dgamma = (|tau| - tau_c) /
// (P:C:P + h); the input strain is the total strain from the virgin crystal
// applied in K = ceil(max|eps_ij| / 1e-5) <= 200 equal sub-steps; sigma_f is
// the slip resistance; G = (C11 - C12 + 3 C44) / 5; R is the 53-bit fraction
// of Philox(key = seed, counter = (sample, step, 0, 0x4D435053)).
//
// Sixteen lanes per crystal (one per slip system).  Symmetric tensors are
// 6-vectors (xx, yy, zz, yz, xz, xy) with tensor shear components; the
// slip-system projections P_a, C:P_a and P_a:C:P_a are built on the host and
// sit in constant memory.
// Products and sums are not contracted into FMAs, so the arithmetic follows
// the written expressions.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "common.hpp"

namespace hmc {

namespace {

constexpr double kC11 = 250800.0, kC12 = 150000.0, kC44 = 123500.0;   // MPa (Table 1)
constexpr double kTau0 = 8.0, kTauS = 122.0, kH0 = 440.0, kBeta = 1000.0;
constexpr int kMcpThreads = 128;
constexpr int64_t kGroupBatchMax = 4096;   // up to this many crystals: sixteen lanes per crystal

struct SlipTable {
    double P[12][6];
    double CP[12][6];
    double PCP[12];
};
__constant__ SlipTable c_slip;

struct Sym {
    double xx, yy, zz, yz, xz, xy;
};

__device__ __forceinline__ Sym stiffness(const Sym& e) {
#pragma clang fp contract(off)
    const double tr = e.xx + e.yy + e.zz;
    Sym s;
    s.xx = kC12 * tr + (kC11 - kC12) * e.xx;
    s.yy = kC12 * tr + (kC11 - kC12) * e.yy;
    s.zz = kC12 * tr + (kC11 - kC12) * e.zz;
    s.yz = 2.0 * kC44 * e.yz;
    s.xz = 2.0 * kC44 * e.xz;
    s.xy = 2.0 * kC44 * e.xy;
    return s;
}

// 1/2 sigma : S : sigma for the cubic compliance S
__device__ __forceinline__ double elastic_energy(const Sym& s) {
#pragma clang fp contract(off)
    const double den = (kC11 - kC12) * (kC11 + 2.0 * kC12);
    const double S11 = (kC11 + kC12) / den, S12 = -kC12 / den;
    const double tr = s.xx + s.yy + s.zz;
    const double exx = S12 * tr + (S11 - S12) * s.xx;
    const double eyy = S12 * tr + (S11 - S12) * s.yy;
    const double ezz = S12 * tr + (S11 - S12) * s.zz;
    const double g = 1.0 / (2.0 * kC44);
    const double diag = s.xx * exx + s.yy * eyy + s.zz * ezz;
    const double off = s.yz * (s.yz * g) + s.xz * (s.xz * g) + s.xy * (s.xy * g);
    return 0.5 * (diag + 2.0 * off);
}

__device__ __forceinline__ double resolved(const Sym& s, int a) {
#pragma clang fp contract(off)
    const double* P = c_slip.P[a];
    return s.xx * P[0] + s.yy * P[1] + s.zz * P[2] + 2.0 * (s.yz * P[3] + s.xz * P[4] + s.xy * P[5]);
}

__device__ __forceinline__ Sym slipped(const Sym& s, int a, double sgn_dg) {
#pragma clang fp contract(off)
    const double* CP = c_slip.CP[a];
    Sym r;
    r.xx = s.xx - sgn_dg * CP[0];
    r.yy = s.yy - sgn_dg * CP[1];
    r.zz = s.zz - sgn_dg * CP[2];
    r.yz = s.yz - sgn_dg * CP[3];
    r.xz = s.xz - sgn_dg * CP[4];
    r.xy = s.xy - sgn_dg * CP[5];
    return r;
}

__device__ __forceinline__ double voce(double gamma) {
#pragma clang fp contract(off)
    return kTauS - (kTauS - kTau0) * exp(-kH0 * gamma / (kTauS - kTau0));
}

// Crystal set-up shared by both kernels: the strain rotated into the crystal
// frame, the number of sub-steps K and the stress increment per sub-step.
__device__ __forceinline__ void crystal_setup(const double* eu, const double* e6, int& K, Sym& dsig) {
#pragma clang fp contract(off)
    // passive rotation sample -> crystal (Bunge ZXZ)
    const double c1 = cos(eu[0]), s1 = sin(eu[0]), c = cos(eu[1]), sn = sin(eu[1]), c2 = cos(eu[2]), s2 = sin(eu[2]);
    double g[3][3];
    g[0][0] = c1 * c2 - s1 * s2 * c; g[0][1] = s1 * c2 + c1 * s2 * c; g[0][2] = s2 * sn;
    g[1][0] = -c1 * s2 - s1 * c2 * c; g[1][1] = -s1 * s2 + c1 * c2 * c; g[1][2] = c2 * sn;
    g[2][0] = s1 * sn; g[2][1] = -c1 * sn; g[2][2] = c;
    const double es[3][3] = {{e6[0], e6[5], e6[4]}, {e6[5], e6[1], e6[3]}, {e6[4], e6[3], e6[2]}};
    double maxabs = 0.0;
    for (int i = 0; i < 6; ++i) maxabs = fmax(maxabs, fabs(e6[i]));
    double ec[3][3];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) {
            double acc = 0.0;
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) acc += g[i][p] * es[p][q] * g[k][q];
            ec[i][k] = acc;
        }
    K = (int)ceil(maxabs / 1e-5);
    K = K < 1 ? 1 : (K > 200 ? 200 : K);
    Sym de;
    de.xx = ec[0][0] / K; de.yy = ec[1][1] / K; de.zz = ec[2][2] / K;
    de.yz = ec[1][2] / K; de.xz = ec[0][2] / K; de.xy = ec[0][1] / K;
    dsig = stiffness(de);
}

__device__ __forceinline__ double mcp_uniform(uint64_t sample, int step, uint32_t k0, uint32_t k1) {
    uint32_t o[4];
    philox4x32_10((uint32_t)sample, (uint32_t)step, 0u, 0x4D435053u, k0, k1, o);
    return (double)((((uint64_t)o[0] << 32) | o[1]) >> 11) * (1.0 / 9007199254740992.0);
}

// One thread per crystal (large batches: every lane does useful work).
__global__ void __launch_bounds__(kMcpThreads)
mcp_thread_kernel(const double* __restrict__ euler, const double* __restrict__ eps, int eps_stride, int64_t n,
                  uint32_t k0, uint32_t k1, uint64_t sample0, const int32_t* __restrict__ sample_ids,
                  double* __restrict__ E_out, double* __restrict__ tauc_out) {
#pragma clang fp contract(off)
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    // the sample index keys the crystal's random stream
    const uint64_t sample = sample_ids ? (uint64_t)sample_ids[s] : sample0 + (uint64_t)s;
    int K;
    Sym dsig;
    crystal_setup(euler + 3 * s, eps + (int64_t)eps_stride * s, K, dsig);
    Sym sig{0, 0, 0, 0, 0, 0};
    double gamma = 0.0, tc = kTau0;
    for (int step = 1; step <= K; ++step) {
        Sym str;
        str.xx = sig.xx + dsig.xx; str.yy = sig.yy + dsig.yy; str.zz = sig.zz + dsig.zz;
        str.yz = sig.yz + dsig.yz; str.xz = sig.xz + dsig.xz; str.xy = sig.xy + dsig.xy;
        uint32_t cand = 0;   // bit a set: system a is a candidate
        double tau[12];
#pragma unroll
        for (int a = 0; a < 12; ++a) {
            tau[a] = resolved(str, a);
            if (fabs(tau[a]) > tc) cand |= 1u << a;
        }
        if (!cand) {
            sig = str;
            continue;
        }
        const double h = kH0 * exp(-kH0 * gamma / (kTauS - kTau0));
        // energies of the candidates, then Eq. (1) and Eq. (2) in system order
        double E[12], dg[12];
        double Emin = INFINITY;
#pragma unroll
        for (int a = 0; a < 12; ++a) {
            if (!(cand & (1u << a))) continue;
            dg[a] = (fabs(tau[a]) - tc) / (c_slip.PCP[a] + h);
            const double sgn = tau[a] > 0.0 ? 1.0 : -1.0;
            E[a] = elastic_energy(slipped(str, a, sgn * dg[a]));
            Emin = fmin(Emin, E[a]);
        }
        double w[12], Z = 0.0;
#pragma unroll
        for (int a = 0; a < 12; ++a) {
            w[a] = (cand & (1u << a)) ? exp(-kBeta * (E[a] - Emin)) : 0.0;
            if (cand & (1u << a)) Z += w[a];
        }
        const double R = mcp_uniform(sample, step, k0, k1);
        int pick = -1, last = -1;
        double S = 0.0;
#pragma unroll
        for (int a = 0; a < 12; ++a) {
            if (!(cand & (1u << a))) continue;
            const double p = w[a] / Z;
            S += p;
            if (pick < 0 && S - p <= R && R < S) pick = a;
            last = a;
        }
        if (pick < 0) pick = last;
        double dgp = 0.0, taup = 0.0;
#pragma unroll
        for (int a = 0; a < 12; ++a)
            if (a == pick) { dgp = dg[a]; taup = tau[a]; }
        sig = slipped(str, pick, (taup > 0.0 ? 1.0 : -1.0) * dgp);
        gamma += dgp;
        tc = voce(gamma);
    }
    const double G = (kC11 - kC12 + 3.0 * kC44) / 5.0;
    E_out[s] = 2.0 * tc * tc / G;
    if (tauc_out) tauc_out[s] = tc;
}

// Sixteen lanes per crystal, lane j owning slip system j (j < 12), for small
// batches where one thread per crystal would leave the chip idle and the
// serial sub-steps set the time: the resolved shears, candidate returns,
// energies and Eq. (1) weights of a step are computed side by side; Z and the
// cumulative intervals of Eq. (2) are then summed in system order by every
// lane of the group from the gathered weights, so the arithmetic and its
// order are those of the one-thread kernel and the results are identical.
constexpr int kGroup = 16;

__global__ void __launch_bounds__(kMcpThreads)
mcp_group_kernel(const double* __restrict__ euler, const double* __restrict__ eps, int eps_stride, int64_t n,
                 uint32_t k0, uint32_t k1, uint64_t sample0, const int32_t* __restrict__ sample_ids,
                 double* __restrict__ E_out, double* __restrict__ tauc_out) {
#pragma clang fp contract(off)
    const int64_t s = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kGroup;
    const int j = (int)(threadIdx.x % kGroup);
    if (s >= n) return;   // whole groups leave together
    const int a = j < 12 ? j : 11;   // lanes 12..15 mirror system 11 and never become candidates
    const uint32_t gbase = (threadIdx.x & 63u) & ~(uint32_t)(kGroup - 1);
    const uint64_t sample = sample_ids ? (uint64_t)sample_ids[s] : sample0 + (uint64_t)s;
    int K;
    Sym dsig;
    crystal_setup(euler + 3 * s, eps + (int64_t)eps_stride * s, K, dsig);
    Sym sig{0, 0, 0, 0, 0, 0};
    double gamma = 0.0, tc = kTau0;
    for (int step = 1; step <= K; ++step) {
        Sym str;
        str.xx = sig.xx + dsig.xx; str.yy = sig.yy + dsig.yy; str.zz = sig.zz + dsig.zz;
        str.yz = sig.yz + dsig.yz; str.xz = sig.xz + dsig.xz; str.xy = sig.xy + dsig.xy;
        const double tau = resolved(str, a);
        const bool is_cand = j < 12 && fabs(tau) > tc;
        const uint32_t cand = (uint32_t)(__ballot(is_cand) >> gbase) & 0xFFFu;   // bit b: system b
        if (!cand) {
            sig = str;
            continue;
        }
        const double h = kH0 * exp(-kH0 * gamma / (kTauS - kTau0));
        double dg = 0.0, E = INFINITY;
        if (is_cand) {
            dg = (fabs(tau) - tc) / (c_slip.PCP[a] + h);
            const double sgn = tau > 0.0 ? 1.0 : -1.0;
            E = elastic_energy(slipped(str, a, sgn * dg));
        }
        double Emin = E;   // the minimum does not depend on the order
        for (int off = kGroup / 2; off >= 1; off >>= 1) Emin = fmin(Emin, __shfl_xor(Emin, off, kGroup));
        const double w = is_cand ? exp(-kBeta * (E - Emin)) : 0.0;
        double wall[12];
#pragma unroll
        for (int b = 0; b < 12; ++b) wall[b] = __shfl(w, b, kGroup);
        double Z = 0.0;
#pragma unroll
        for (int b = 0; b < 12; ++b)
            if (cand & (1u << b)) Z += wall[b];
        const double R = mcp_uniform(sample, step, k0, k1);
        int pick = -1, last = -1;
        double S = 0.0;
#pragma unroll
        for (int b = 0; b < 12; ++b) {
            if (!(cand & (1u << b))) continue;
            const double p = wall[b] / Z;
            S += p;
            if (pick < 0 && S - p <= R && R < S) pick = b;
            last = b;
        }
        if (pick < 0) pick = last;
        const double dgp = __shfl(dg, pick, kGroup), taup = __shfl(tau, pick, kGroup);
        sig = slipped(str, pick, (taup > 0.0 ? 1.0 : -1.0) * dgp);
        gamma += dgp;
        tc = voce(gamma);
    }
    if (j == 0) {
        const double G = (kC11 - kC12 + 3.0 * kC44) / 5.0;
        E_out[s] = 2.0 * tc * tc / G;
        if (tauc_out) tauc_out[s] = tc;
    }
}

SlipTable build_slip_table() {
    static const double normals[4][3] = {{1, 1, 1}, {-1, 1, 1}, {1, -1, 1}, {1, 1, -1}};
    static const double dirs[6][3] = {{1, -1, 0}, {1, 0, -1}, {0, 1, -1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
    SlipTable t{};
    int a = 0;
    for (int ni = 0; ni < 4; ++ni)
        for (int di = 0; di < 6; ++di) {
            const double* nn = normals[ni];
            const double* dd = dirs[di];
            if (nn[0] * dd[0] + nn[1] * dd[1] + nn[2] * dd[2] != 0.0) continue;
            double n[3], d[3];
            for (int k = 0; k < 3; ++k) {
                n[k] = nn[k] / std::sqrt(3.0);
                d[k] = dd[k] / std::sqrt(2.0);
            }
            // P = sym(d (x) n) as (xx, yy, zz, yz, xz, xy)
            const double P[6] = {d[0] * n[0], d[1] * n[1], d[2] * n[2], 0.5 * (d[1] * n[2] + d[2] * n[1]),
                                 0.5 * (d[0] * n[2] + d[2] * n[0]), 0.5 * (d[0] * n[1] + d[1] * n[0])};
            const double tr = P[0] + P[1] + P[2];
            double CP[6];
            for (int k = 0; k < 3; ++k) CP[k] = kC12 * tr + (kC11 - kC12) * P[k];
            for (int k = 3; k < 6; ++k) CP[k] = 2.0 * kC44 * P[k];
            double pcp = 0.0;
            for (int k = 0; k < 3; ++k) pcp += P[k] * CP[k];
            for (int k = 3; k < 6; ++k) pcp += 2.0 * P[k] * CP[k];
            for (int k = 0; k < 6; ++k) {
                t.P[a][k] = P[k];
                t.CP[a][k] = CP[k];
            }
            t.PCP[a] = pcp;
            ++a;
        }
    return t;
}

}  // namespace

hmc_status mcp_solve_device(const double* d_euler, const double* d_eps, int64_t n, uint64_t seed, uint64_t sample0,
                            double* d_E, double* d_tauc, hipStream_t stream, int eps_stride,
                            const int32_t* d_sample_ids) {
    static bool uploaded = false;
    if (!uploaded) {
        const SlipTable t = build_slip_table();
        HMC_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_slip), &t, sizeof t, 0, hipMemcpyHostToDevice));
        uploaded = true;
    }
    if (n == 0) return HMC_OK;
    const uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFu), k1 = (uint32_t)(seed >> 32);
    if (n <= kGroupBatchMax) {
        const uint64_t blocks = ((uint64_t)n * kGroup + kMcpThreads - 1) / kMcpThreads;
        mcp_group_kernel<<<dim3((unsigned)blocks), kMcpThreads, 0, stream>>>(d_euler, d_eps, eps_stride, n, k0, k1,
                                                                             sample0, d_sample_ids, d_E, d_tauc);
    } else {
        const uint64_t blocks = ((uint64_t)n + kMcpThreads - 1) / kMcpThreads;
        mcp_thread_kernel<<<dim3((unsigned)blocks), kMcpThreads, 0, stream>>>(d_euler, d_eps, eps_stride, n, k0, k1,
                                                                              sample0, d_sample_ids, d_E, d_tauc);
    }
    HMC_HIP(hipGetLastError());
    return HMC_OK;
}

}  // namespace hmc

using namespace hmc;

extern "C" hmc_status hmc_mcp_solve(const double* euler, const double* eps, int64_t n, uint64_t seed,
                                    uint64_t sample0, int32_t on_device, double* E_out, double* tauc_out) {
    set_error("");
    if (n < 0 || (n > 0 && (!euler || !eps || !E_out))) return fail(HMC_E_INVAL, "NULL argument or n < 0");
    if (n >= (1ll << 31)) return fail(HMC_E_INVAL, "n must be below 2^31");
    if (n == 0) return HMC_OK;
    if (on_device) {
        HMC_TRY(mcp_solve_device(euler, eps, n, seed, sample0, E_out, tauc_out, nullptr, 6, nullptr));
        HMC_HIP(hipStreamSynchronize(nullptr));
        return HMC_OK;
    }
    for (int64_t i = 0; i < 6 * n; ++i)
        if (!std::isfinite(eps[i])) return fail(HMC_E_INVAL, "non-finite strain");
    void *de = nullptr, *dp = nullptr, *dE = nullptr, *dT = nullptr;
    const size_t be = (size_t)n * 3 * 8, bp = (size_t)n * 6 * 8, bE = (size_t)n * 8;
    hmc_status st = dev_alloc(&de, be, "mcp euler");
    if (st == HMC_OK) st = dev_alloc(&dp, bp, "mcp strain");
    if (st == HMC_OK) st = dev_alloc(&dE, bE, "mcp energy");
    if (st == HMC_OK && tauc_out) st = dev_alloc(&dT, bE, "mcp tau_c");
    hipError_t e = hipSuccess;
    if (st == HMC_OK) e = hipMemcpy(de, euler, be, hipMemcpyHostToDevice);
    if (st == HMC_OK && e == hipSuccess) e = hipMemcpy(dp, eps, bp, hipMemcpyHostToDevice);
    if (st == HMC_OK && e == hipSuccess)
        st = mcp_solve_device((const double*)de, (const double*)dp, n, seed, sample0, (double*)dE, (double*)dT, nullptr,
                              6, nullptr);
    if (st == HMC_OK && e == hipSuccess) e = hipMemcpy(E_out, dE, bE, hipMemcpyDeviceToHost);
    if (st == HMC_OK && e == hipSuccess && tauc_out) e = hipMemcpy(tauc_out, dT, bE, hipMemcpyDeviceToHost);
    dev_free(de, be);
    dev_free(dp, bp);
    dev_free(dE, bE);
    dev_free(dT, bE);
    if (st != HMC_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "mcp solve");
    return HMC_OK;
}
