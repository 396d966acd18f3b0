// pair.hip -- bond energies per pair of grains on the GPU.
//
// Eq. (7) of Zhang, Dingreville, Bartel, Lusk (arXiv:1007.3509) writes the
// bond energy J for each pair of spins (q_i, q_n); the closing section names
// misorientation-dependent boundary energy as the use of that freedom.  The
// paper gives no law; the Read-Shockley low-angle form (Read and Shockley,
// Phys. Rev. 78 (1950) 275) is used:
//   J(theta) = J_max (theta/theta_m) (1 - ln(theta/theta_m))  (theta < theta_m),
//   J(theta) = J_max                                          (theta >= theta_m),
// theta the misorientation angle of the two grains: the smallest rotation
// angle of g_b g_a^T over the 24 proper rotations of the cube (g Bunge ZXZ,
// passive sample -> crystal).  Fixed point: round-half-even(J * 65536).
//
// One thread per pair (a < b) writes both entries, so the table is exactly
// symmetric; the diagonal is zero.  Products and sums are not contracted into
// FMAs, so the arithmetic follows the written expressions.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "common.hpp"

namespace hmc {
namespace {

constexpr int kPairThreads = 256;

struct CubeRotations {
    int8_t perm[24][3];
    int8_t sign[24][3];
};
__constant__ CubeRotations c_cube;

CubeRotations cube_rotations() {
    // signed permutation matrices of determinant +1: row r has sign[r] in column perm[r]
    static const int P[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    static const int parity[6] = {1, -1, -1, 1, 1, -1};
    CubeRotations t{};
    int n = 0;
    for (int p = 0; p < 6; ++p)
        for (int m = 0; m < 8; ++m) {
            const int s[3] = {(m & 1) ? -1 : 1, (m & 2) ? -1 : 1, (m & 4) ? -1 : 1};
            if (parity[p] * s[0] * s[1] * s[2] != 1) continue;
            for (int r = 0; r < 3; ++r) {
                t.perm[n][r] = (int8_t)P[p][r];
                t.sign[n][r] = (int8_t)s[r];
            }
            ++n;
        }
    return t;
}

__global__ void __launch_bounds__(kPairThreads)
orientation_kernel(const double* __restrict__ euler, int32_t Q, double* __restrict__ G) {
#pragma clang fp contract(off)
    const int32_t q = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= Q) return;
    const double* e = euler + 3 * (size_t)q;
    const double c1 = cos(e[0]), s1 = sin(e[0]), c = cos(e[1]), s = sin(e[1]), c2 = cos(e[2]), s2 = sin(e[2]);
    double* g = G + 9 * (size_t)q;
    g[0] = c1 * c2 - s1 * s2 * c;  g[1] = s1 * c2 + c1 * s2 * c;  g[2] = s2 * s;
    g[3] = -c1 * s2 - s1 * c2 * c; g[4] = -s1 * s2 + c1 * c2 * c; g[5] = c2 * s;
    g[6] = s1 * s;                 g[7] = -c1 * s;                g[8] = c;
}

__global__ void __launch_bounds__(kPairThreads)
pair_energy_kernel(const double* __restrict__ G, int32_t Q, double J_max, double theta_m, int32_t* __restrict__ Jp) {
#pragma clang fp contract(off)
    const int32_t b = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    const int32_t a = (int32_t)blockIdx.y;
    if (b >= Q || b < a) return;
    if (a == b) {
        Jp[(size_t)a * Q + a] = 0;
        return;
    }
    const double* ga = G + 9 * (size_t)a;
    const double* gb = G + 9 * (size_t)b;
    double dg[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += gb[3 * i + k] * ga[3 * j + k];
            dg[i][j] = acc;
        }
    double best = -2.0;
    for (int m = 0; m < 24; ++m) {
        double tr = 0.0;   // trace of R dg, R[i][perm[i]] = sign[i]
        for (int i = 0; i < 3; ++i) tr += (double)c_cube.sign[m][i] * dg[c_cube.perm[m][i]][i];
        best = tr > best ? tr : best;
    }
    double cth = (best - 1.0) / 2.0;
    cth = cth > 1.0 ? 1.0 : (cth < -1.0 ? -1.0 : cth);
    const double theta = acos(cth) * (180.0 / 3.14159265358979323846);
    double J;
    if (theta <= 0.0) J = 0.0;
    else if (theta >= theta_m) J = J_max;
    else {
        const double x = theta / theta_m;
        J = J_max * x * (1.0 - log(x));
    }
    const int32_t v = (int32_t)rint(J * 65536.0);
    Jp[(size_t)a * Q + b] = v;
    Jp[(size_t)b * Q + a] = v;
}

}  // namespace
}  // namespace hmc

using namespace hmc;

extern "C" hmc_status hmc_misorientation_energy(const double* euler, int32_t Q, double J_max, double theta_m_deg,
                                                int32_t on_device, int32_t* Jp_out) {
    set_error("");
    if (!euler || !Jp_out) return fail(HMC_E_INVAL, "NULL argument");
    if (Q < 1 || Q > 46340) return fail(HMC_E_INVAL, "Q must be in [1, 46340]");
    if (!(J_max >= 0.0) || !std::isfinite(J_max) || J_max * 65536.0 > (double)(1 << 24))
        return fail(HMC_E_INVAL, "J_max must be in [0, 256]");
    if (!(theta_m_deg > 0.0) || !std::isfinite(theta_m_deg)) return fail(HMC_E_INVAL, "theta_m must be positive");
    static bool uploaded = false;
    if (!uploaded) {
        const CubeRotations t = cube_rotations();
        HMC_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_cube), &t, sizeof t, 0, hipMemcpyHostToDevice));
        uploaded = true;
    }
    const size_t be = (size_t)Q * 24, bg = (size_t)Q * 72, bj = (size_t)Q * (size_t)Q * 4;
    void *de = nullptr, *dG = nullptr, *dJ = nullptr;
    hmc_status st = HMC_OK;
    if (!on_device) st = dev_alloc(&de, be, "orientations");
    if (st == HMC_OK) st = dev_alloc(&dG, bg, "rotation matrices");
    if (st == HMC_OK && !on_device) st = dev_alloc(&dJ, bj, "pair energies");
    hipError_t e = hipSuccess;
    const double* d_euler = on_device ? euler : static_cast<const double*>(de);
    int32_t* d_J = on_device ? Jp_out : static_cast<int32_t*>(dJ);
    if (st == HMC_OK && !on_device) e = hipMemcpy(de, euler, be, hipMemcpyHostToDevice);
    if (st == HMC_OK && e == hipSuccess) {
        orientation_kernel<<<(unsigned)((Q + kPairThreads - 1) / kPairThreads), kPairThreads>>>(
            d_euler, Q, static_cast<double*>(dG));
        pair_energy_kernel<<<dim3((unsigned)((Q + kPairThreads - 1) / kPairThreads), (unsigned)Q), kPairThreads>>>(
            static_cast<const double*>(dG), Q, J_max, theta_m_deg, d_J);
        e = hipGetLastError();
    }
    if (st == HMC_OK && e == hipSuccess) e = hipDeviceSynchronize();
    if (st == HMC_OK && e == hipSuccess && !on_device) e = hipMemcpy(Jp_out, dJ, bj, hipMemcpyDeviceToHost);
    dev_free(de, be);
    dev_free(dG, bg);
    dev_free(dJ, bj);
    if (st != HMC_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "misorientation energy");
    return HMC_OK;
}
