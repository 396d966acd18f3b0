// mlp.hip -- learned stored-energy surrogate: a 9-64-64-1 tanh MLP trained
// and evaluated by the library's own kernels (FP32), and the driver that
// turns its predictions into per-grain bulk energies for the sweep.
//
// The network stands in for the per-grain crystal-plasticity update of
// Sec. 2 (mcp.hip) that produces the stored dislocation energy of Eq. (4),
// which enters Eq. (7) as the grain's bulk energy (Sec. 3, Sec. 6).
//
// Inputs: Bunge angles (phi1, Phi, phi2) and the six strain components
// (e11, e22, e33, e23, e13, e12); features: the Rodrigues vector of the
// orientation's cubic-symmetry equivalent in the fundamental zone, over
// sqrt 2 - 1, and e_ij / 2e-3, so every orientation and the strain box
// [-2e-3, 2e-3]^6 map into [-1,1]^9.  Target: E_rho standardised by the
// training mean and standard deviation.  Loss: mean squared error.  Adam
// (Kingma & Ba, 2015), beta1 0.9, beta2 0.999, eps 1e-8; Xavier-uniform
// initial weights from Philox; learning rate decays on a cosine to 1/10.
//
// Parameter vector (4865 floats): W1[64][9], b1[64], W2[64][64], b2[64],
// w3[64], b3.
//
// Training step on a batch of B samples: one workgroup per tile of 32
// samples computes the forward pass, the back-propagated deltas and the
// tile's gradient (the weights and the tile's activations sit in LDS) and
// writes it to its own slot; a second kernel sums the slots in a fixed order
// (reproducible) and applies Adam.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace hmc {
hmc_status mcp_solve_device(const double* d_euler, const double* d_eps, int64_t n, uint64_t seed, uint64_t sample0,
                            double* d_E, double* d_tauc, hipStream_t stream, int eps_stride,
                            const int32_t* d_sample_ids);
}

namespace {

using namespace hmc;

constexpr int kIn = 9, kHid = 64;
constexpr int kNP = kHid * kIn + kHid + kHid * kHid + kHid + kHid + 1;   // 4865
constexpr int oW1 = 0, ob1 = kHid * kIn, oW2 = ob1 + kHid, ob2 = oW2 + kHid * kHid, ow3 = ob2 + kHid,
              ob3 = ow3 + kHid;
constexpr int kTile = 32;          // samples per workgroup in training
constexpr int kTileThreads = 256;
constexpr double kStrainBox = 2e-3;
constexpr double kPi = 3.14159265358979323846;

// ------------------------------------------------------------------ kernels

// The orientation's three inputs: the Rodrigues vector of its cubic
// symmetry-equivalent with the smallest rotation angle (the cubic
// fundamental zone), scaled by 1/(sqrt 2 - 1) into [-1, 1].  The stored
// energy depends on the orientation only up to the 24 rotations of the cubic
// crystal (they permute the slip systems and leave the stiffness alone), so
// the network learns it on one zone, where it has no copies and no wrap.
__device__ __forceinline__ void orientation_features(const double* e, float* x) {
    const double c1 = cos(e[0]), s1 = sin(e[0]), c = cos(e[1]), sn = sin(e[1]), c2 = cos(e[2]), s2 = sin(e[2]);
    // Bunge passive matrix (crystal <- sample)
    const double g[3][3] = {{c1 * c2 - s1 * s2 * c, s1 * c2 + c1 * s2 * c, s2 * sn},
                            {-c1 * s2 - s1 * c2 * c, -s1 * s2 + c1 * c2 * c, c2 * sn},
                            {s1 * sn, -c1 * sn, c}};
    // the cubic rotation S (a signed permutation, det +1) with the largest
    // trace of S g: rows of S g are sign[i] * row perm[i] of g
    const int perms[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {0, 2, 1}, {2, 1, 0}, {1, 0, 2}};
    double best = -4.0;
    int bp = 0, bs = 0;
    for (int p = 0; p < 6; ++p) {
        const int parity = p < 3 ? 1 : -1;
        for (int sg = 0; sg < 8; ++sg) {
            const int a = (sg & 1) ? -1 : 1, b = (sg & 2) ? -1 : 1, d = (sg & 4) ? -1 : 1;
            if (a * b * d * parity != 1) continue;
            const double tr = a * g[perms[p][0]][0] + b * g[perms[p][1]][1] + d * g[perms[p][2]][2];
            if (tr > best) {
                best = tr;
                bp = p;
                bs = sg;
            }
        }
    }
    const double sgn[3] = {(bs & 1) ? -1.0 : 1.0, (bs & 2) ? -1.0 : 1.0, (bs & 4) ? -1.0 : 1.0};
    double h[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) h[i][j] = sgn[i] * g[perms[bp][i]][j];
    // Rodrigues vector n tan(theta/2) = (antisymmetric part) / (1 + trace)
    const double den = 1.0 + best;
    const double k = 1.0 / (0.41421356237309503 * den);
    x[0] = (float)((h[2][1] - h[1][2]) * k);
    x[1] = (float)((h[0][2] - h[2][0]) * k);
    x[2] = (float)((h[1][0] - h[0][1]) * k);
}

__global__ void features_kernel(const double* __restrict__ euler, const double* __restrict__ eps, int eps_stride,
                                int64_t n, float* __restrict__ X) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float* x = X + kIn * s;
    orientation_features(euler + 3 * s, x);
    for (int k = 0; k < 6; ++k) x[3 + k] = (float)(eps[(int64_t)eps_stride * s + k] / kStrainBox);
}

__global__ void targets_kernel(const double* __restrict__ E, int64_t n, double mean, double inv_std,
                               float* __restrict__ t) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) t[s] = (float)((E[s] - mean) * inv_std);
}

// One tile of kTile samples: forward, deltas and the tile's gradient.
// sel: sample indices of the batch (nullptr: consecutive from b0).
__global__ void __launch_bounds__(kTileThreads)
train_tile_kernel(const float* __restrict__ theta, const float* __restrict__ X, const float* __restrict__ t,
                  const uint32_t* __restrict__ sel, int64_t b0, int32_t B, float* __restrict__ partial) {
    __shared__ float W[kNP];
    __shared__ float xs[kTile][kIn];
    __shared__ float H1[kTile][kHid];
    __shared__ float H2[kTile][kHid + 1];   // becomes D2
    __shared__ float D1[kTile][kHid + 1];
    __shared__ float dy[kTile];
    const int tid = threadIdx.x;
    const int tile = blockIdx.x;
    for (int p = tid; p < kNP; p += blockDim.x) W[p] = theta[p];
    for (int e = tid; e < kTile * kIn; e += blockDim.x) {
        const int s = e / kIn, j = e % kIn;
        const int64_t gi = (int64_t)tile * kTile + s;
        const int64_t idx = sel ? (int64_t)sel[b0 + gi] : b0 + gi;
        xs[s][j] = X[idx * kIn + j];
    }
    __syncthreads();
    // H1 = tanh(W1 x + b1)
    for (int e = tid; e < kTile * kHid; e += blockDim.x) {
        const int s = e / kHid, i = e % kHid;
        float a = W[ob1 + i];
        for (int j = 0; j < kIn; ++j) a += W[oW1 + i * kIn + j] * xs[s][j];
        H1[s][i] = tanhf(a);
    }
    __syncthreads();
    // H2 = tanh(W2 h1 + b2)
    for (int e = tid; e < kTile * kHid; e += blockDim.x) {
        const int s = e / kHid, i = e % kHid;
        float a = W[ob2 + i];
        for (int j = 0; j < kHid; ++j) a += W[oW2 + i * kHid + j] * H1[s][j];
        H2[s][i] = tanhf(a);
    }
    __syncthreads();
    float* g = partial + (size_t)tile * (kNP + 1);
    // y, dL/dy = 2 (y - t) / B, tile loss
    if (tid < kTile) {
        const int64_t gi = (int64_t)tile * kTile + tid;
        const int64_t idx = sel ? (int64_t)sel[b0 + gi] : b0 + gi;
        float y = W[ob3];
        for (int i = 0; i < kHid; ++i) y += W[ow3 + i] * H2[tid][i];
        const float r = y - t[idx];
        dy[tid] = 2.0f * r / (float)B;
        D1[tid][kHid] = r * r;   // scratch column for the loss
    }
    __syncthreads();
    if (tid == 0) {
        float L = 0.0f, db3 = 0.0f;
        for (int s = 0; s < kTile; ++s) {
            L += D1[s][kHid];
            db3 += dy[s];
        }
        g[ob3] = db3;
        g[kNP] = L;
    }
    // dw3 = sum_s dy h2
    for (int i = tid; i < kHid; i += blockDim.x) {
        float a = 0.0f;
        for (int s = 0; s < kTile; ++s) a += dy[s] * H2[s][i];
        g[ow3 + i] = a;
    }
    __syncthreads();
    // D2 = dy w3 (1 - h2^2), in place
    for (int e = tid; e < kTile * kHid; e += blockDim.x) {
        const int s = e / kHid, i = e % kHid;
        const float h = H2[s][i];
        H2[s][i] = dy[s] * W[ow3 + i] * (1.0f - h * h);
    }
    __syncthreads();
    // dW2 = sum_s D2 h1^T, db2 = sum_s D2
    for (int e = tid; e < kHid * kHid; e += blockDim.x) {
        const int i = e / kHid, j = e % kHid;
        float a = 0.0f;
        for (int s = 0; s < kTile; ++s) a += H2[s][i] * H1[s][j];
        g[oW2 + e] = a;
    }
    for (int i = tid; i < kHid; i += blockDim.x) {
        float a = 0.0f;
        for (int s = 0; s < kTile; ++s) a += H2[s][i];
        g[ob2 + i] = a;
    }
    // D1 = (W2^T D2) (1 - h1^2)
    for (int e = tid; e < kTile * kHid; e += blockDim.x) {
        const int s = e / kHid, j = e % kHid;
        float a = 0.0f;
        for (int i = 0; i < kHid; ++i) a += W[oW2 + i * kHid + j] * H2[s][i];
        const float h = H1[s][j];
        D1[s][j] = a * (1.0f - h * h);
    }
    __syncthreads();
    // dW1 = sum_s D1 x^T, db1 = sum_s D1
    for (int e = tid; e < kHid * kIn; e += blockDim.x) {
        const int i = e / kIn, j = e % kIn;
        float a = 0.0f;
        for (int s = 0; s < kTile; ++s) a += D1[s][i] * xs[s][j];
        g[oW1 + e] = a;
    }
    for (int i = tid; i < kHid; i += blockDim.x) {
        float a = 0.0f;
        for (int s = 0; s < kTile; ++s) a += D1[s][i];
        g[ob1 + i] = a;
    }
}

// Sum the tiles' gradients in tile order; optionally apply one Adam step.
__global__ void reduce_adam_kernel(const float* __restrict__ partial, int ntiles, float* __restrict__ theta,
                                   float* __restrict__ m, float* __restrict__ v, float lr, float c1, float c2,
                                   int apply, float* __restrict__ grad_out, float* __restrict__ loss_out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kNP) return;
    float gsum = 0.0f;
    for (int k = 0; k < ntiles; ++k) gsum += partial[(size_t)k * (kNP + 1) + p];
    if (p == kNP) {
        if (loss_out) *loss_out = gsum;
        return;
    }
    if (grad_out) grad_out[p] = gsum;
    if (apply) {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float mm = b1 * m[p] + (1.0f - b1) * gsum;
        const float vv = b2 * v[p] + (1.0f - b2) * gsum * gsum;
        m[p] = mm;
        v[p] = vv;
        theta[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    }
}

// Adam with a gradient given from outside (one step).
__global__ void adam_kernel(const float* __restrict__ g, float* __restrict__ theta, float* __restrict__ m,
                            float* __restrict__ v, float lr, float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNP) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mm = b1 * m[p] + (1.0f - b1) * g[p];
    const float vv = b2 * v[p] + (1.0f - b2) * g[p] * g[p];
    m[p] = mm;
    v[p] = vv;
    theta[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

constexpr int kPredThreads = 256;
constexpr int kPredLanes = 4;                             // lanes per sample
constexpr int kPredSamples = kPredThreads / kPredLanes;   // samples per workgroup
constexpr int kPredUnits = kHid / kPredLanes;             // hidden units per lane

// Workgroups of kPredThreads lanes for n samples.
inline unsigned predict_blocks(int64_t n) { return (unsigned)((n + kPredSamples - 1) / kPredSamples); }

// A surrogate query's inputs and outputs: features formed from the grains'
// orientations and one strain (read with stride 0) as features_kernel forms
// them, and the energies quantised as quantise_kernel does.
struct QueryIO {
    const double* euler;   // n x 3
    const double* eps;     // 6
    double qscale;         // E_scale * 65536
    int32_t* B;            // n
};

// Inference, four lanes per sample: each lane forms a quarter of the hidden
// units of both layers (every unit's sum in the same order as one lane
// alone would), the first layer is shared through LDS, and the four partial
// output sums are added in a fixed order.  kQuery: the features and the
// quantised energies of a surrogate query in the same launch (q).
template <bool kQuery>
__global__ void __launch_bounds__(kPredThreads)
predict_kernel(const float* __restrict__ theta, const float* __restrict__ X, int64_t n, double mean, double sdev,
               double* __restrict__ E_out, float* __restrict__ y_std_out, QueryIO q) {
    __shared__ float W[kNP];
    __shared__ float H1[kPredSamples][kHid];
    for (int p = threadIdx.x; p < kNP; p += blockDim.x) W[p] = theta[p];
    __syncthreads();
    const int ls = threadIdx.x / kPredLanes, part = threadIdx.x % kPredLanes;
    const int64_t s = (int64_t)blockIdx.x * kPredSamples + ls;
    const bool live = s < n;
    float x[kIn];
    if constexpr (kQuery) {
        const double* e = q.euler + 3 * (live ? s : 0);
        orientation_features(e, x);
        for (int k = 0; k < 6; ++k) x[3 + k] = (float)(q.eps[k] / kStrainBox);
    } else {
        for (int j = 0; j < kIn; ++j) x[j] = live ? X[s * kIn + j] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < kPredUnits; ++q) {
        const int i = part * kPredUnits + q;
        float a = W[ob1 + i];
#pragma unroll
        for (int j = 0; j < kIn; ++j) a += W[oW1 + i * kIn + j] * x[j];
        H1[ls][i] = tanhf(a);
    }
    // the four lanes of a sample sit in one wave, whose LDS operations run in order
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float h1[kHid];
#pragma unroll
    for (int j = 0; j < kHid; ++j) h1[j] = H1[ls][j];
    float y = 0.0f;
    for (int q = 0; q < kPredUnits; ++q) {
        const int i = part * kPredUnits + q;
        float a = W[ob2 + i];
#pragma unroll
        for (int j = 0; j < kHid; ++j) a += W[oW2 + i * kHid + j] * h1[j];
        y += W[ow3 + i] * tanhf(a);
    }
    // partial sums of lanes 1..3 of the sample to lane 0, added in lane order
    const float y1 = __shfl_down(y, 1, kPredLanes), y2 = __shfl_down(y, 2, kPredLanes),
                y3 = __shfl_down(y, 3, kPredLanes);
    if (!live || part != 0) return;
    const float out = ((W[ob3] + y) + y1) + (y2 + y3);
    if (y_std_out) y_std_out[s] = out;
    const double E = (double)out * sdev + mean;
    if (E_out) E_out[s] = E;
    if constexpr (kQuery) q.B[s] = (int32_t)rint(E * q.qscale);   // round half to even
}

__global__ void quantise_kernel(const double* __restrict__ E, int32_t n, double scale, int32_t* __restrict__ B) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) B[i] = (int32_t)rint(E[i] * scale);   // round half to even
}

// --------------------------------------------------------------- host side

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hmc_status ensure(size_t b, const char* what) {
        if (b <= bytes) return HMC_OK;
        dev_free(p, bytes);
        p = nullptr;
        bytes = 0;
        HMC_TRY(dev_alloc(&p, b, what));
        bytes = b;
        return HMC_OK;
    }
    void release() {
        dev_free(p, bytes);
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

// Pinned host memory: the destination of a query's read-backs, which from
// pageable memory go through a staged copy.
struct HostBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hmc_status ensure(size_t b, const char* what) {
        if (b <= bytes) return HMC_OK;
        release();
        hipError_t e = hipHostMalloc(&p, b, hipHostMallocDefault);
        if (e != hipSuccess) {
            p = nullptr;
            return hip_fail(e, what);
        }
        bytes = b;
        return HMC_OK;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

uint32_t philox_u32(uint64_t seed, uint32_t a, uint32_t b, uint32_t tag) {
    uint32_t o[4];
    philox4x32_10(a, b, 0u, tag, (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), o);
    return o[0];
}

}  // namespace

struct hmc_mlp_s {
    hipStream_t stream = nullptr;
    hipEvent_t ready = nullptr;     // orders work on other streams after the handle's own
    DevBuf theta, m, v;
    int64_t step = 0;
    double mean = 0.0, sdev = 1.0;
    DevBuf X, t, partial, sel, loss, grad, euler, eps, E, Eaudit, Bq, audit_idx;
    HostBuf readback;   // a query's predictions, audit energies and quantised energies
};

namespace {

hmc_status upload_or_alias(const double* src, size_t bytes, int32_t on_device, DevBuf& buf, const double** out,
                           hipStream_t s, const char* what) {
    if (on_device) {
        *out = src;
        return HMC_OK;
    }
    HMC_TRY(buf.ensure(bytes, what));
    HMC_HIP(hipMemcpyAsync(buf.p, src, bytes, hipMemcpyHostToDevice, s));
    *out = buf.as<double>();
    return HMC_OK;
}

hmc_status make_features(hmc_mlp* M, const double* euler, const double* eps, int64_t n, int32_t on_device) {
    const double *de = nullptr, *dp = nullptr;
    HMC_TRY(upload_or_alias(euler, (size_t)n * 3 * 8, on_device, M->euler, &de, M->stream, "mlp euler"));
    HMC_TRY(upload_or_alias(eps, (size_t)n * 6 * 8, on_device, M->eps, &dp, M->stream, "mlp strain"));
    HMC_TRY(M->X.ensure((size_t)n * kIn * 4, "mlp features"));
    const unsigned blocks = (unsigned)((n + 255) / 256);
    features_kernel<<<blocks, 256, 0, M->stream>>>(de, dp, 6, n, M->X.as<float>());
    HMC_HIP(hipGetLastError());
    return HMC_OK;
}

}  // namespace

using namespace hmc;

extern "C" {

hmc_status hmc_mlp_create(uint64_t seed, hmc_mlp** out) {
    set_error("");
    if (!out) return fail(HMC_E_INVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(HMC_E_DEVICE, "no HIP device available");
    hmc_mlp* M = new hmc_mlp();
    hmc_status st = HMC_OK;
    hipError_t e = hipStreamCreateWithFlags(&M->stream, hipStreamNonBlocking);
    if (e != hipSuccess) st = hip_fail(e, "mlp stream");
    if (st == HMC_OK) st = M->theta.ensure(kNP * 4, "mlp parameters");
    if (st == HMC_OK) st = M->m.ensure(kNP * 4, "adam m");
    if (st == HMC_OK) st = M->v.ensure(kNP * 4, "adam v");
    if (st == HMC_OK) {
        // Xavier-uniform weights, zero biases
        std::vector<float> th(kNP, 0.0f);
        auto fill = [&](int off, int rows, int cols) {
            const double a = std::sqrt(6.0 / (rows + cols));
            for (int k = 0; k < rows * cols; ++k) {
                const double u = (double)(philox_u32(seed, (uint32_t)(off + k), 0u, 0x4D4C5049u) >> 8) *
                                 (1.0 / 16777216.0);
                th[off + k] = (float)((2.0 * u - 1.0) * a);
            }
        };
        fill(oW1, kHid, kIn);
        fill(oW2, kHid, kHid);
        fill(ow3, 1, kHid);
        e = hipMemcpy(M->theta.p, th.data(), kNP * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(M->m.p, 0, kNP * 4);
        if (e == hipSuccess) e = hipMemset(M->v.p, 0, kNP * 4);
        if (e != hipSuccess) st = hip_fail(e, "mlp init");
    }
    if (st != HMC_OK) {
        M->theta.release();
        M->m.release();
        M->v.release();
        if (M->stream) (void)hipStreamDestroy(M->stream);
        delete M;
        return st;
    }
    *out = M;
    return HMC_OK;
}

hmc_status hmc_mlp_free(hmc_mlp* M) {
    set_error("");
    if (!M) return HMC_OK;
    (void)hipStreamSynchronize(M->stream);
    for (DevBuf* b : {&M->theta, &M->m, &M->v, &M->X, &M->t, &M->partial, &M->sel, &M->loss, &M->grad, &M->euler,
                      &M->eps, &M->E, &M->Eaudit, &M->Bq, &M->audit_idx})
        b->release();
    M->readback.release();
    if (M->ready) (void)hipEventDestroy(M->ready);
    (void)hipStreamDestroy(M->stream);
    delete M;
    return HMC_OK;
}

hmc_status hmc_mlp_get_params(hmc_mlp* M, float* host_dst, double* norm_out) {
    set_error("");
    if (!M || !host_dst) return fail(HMC_E_INVAL, "NULL argument");
    HMC_HIP(hipStreamSynchronize(M->stream));
    HMC_HIP(hipMemcpy(host_dst, M->theta.p, kNP * 4, hipMemcpyDeviceToHost));
    if (norm_out) {
        norm_out[0] = M->mean;
        norm_out[1] = M->sdev;
    }
    return HMC_OK;
}

hmc_status hmc_mlp_set_params(hmc_mlp* M, const float* host_src, const double* norm) {
    set_error("");
    if (!M || !host_src) return fail(HMC_E_INVAL, "NULL argument");
    for (int p = 0; p < kNP; ++p)
        if (!std::isfinite(host_src[p])) return fail(HMC_E_INVAL, "non-finite parameter");
    HMC_HIP(hipStreamSynchronize(M->stream));
    HMC_HIP(hipMemcpy(M->theta.p, host_src, kNP * 4, hipMemcpyHostToDevice));
    HMC_HIP(hipMemset(M->m.p, 0, kNP * 4));
    HMC_HIP(hipMemset(M->v.p, 0, kNP * 4));
    M->step = 0;
    if (norm) {
        if (!(norm[1] > 0.0) || !std::isfinite(norm[0])) return fail(HMC_E_INVAL, "bad normalisation");
        M->mean = norm[0];
        M->sdev = norm[1];
    }
    return HMC_OK;
}

// Gradient of the mean squared error over n samples given as scaled
// features X (n x 9) and standardised targets t (host float arrays).
hmc_status hmc_mlp_loss_grad(hmc_mlp* M, const float* X, const float* t, int32_t n, float* loss_out,
                             float* grad_out) {
    set_error("");
    if (!M || !X || !t || !loss_out || !grad_out) return fail(HMC_E_INVAL, "NULL argument");
    if (n < kTile || n % kTile != 0 || n > (1 << 24))
        return fail(HMC_E_INVAL, "n must be a positive multiple of 32");
    HMC_TRY(M->X.ensure((size_t)n * kIn * 4, "mlp features"));
    HMC_TRY(M->t.ensure((size_t)n * 4, "mlp targets"));
    const int ntiles = n / kTile;
    HMC_TRY(M->partial.ensure((size_t)ntiles * (kNP + 1) * 4, "mlp partial gradients"));
    HMC_TRY(M->grad.ensure(kNP * 4, "mlp gradient"));
    HMC_TRY(M->loss.ensure(4, "mlp loss"));
    HMC_HIP(hipMemcpyAsync(M->X.p, X, (size_t)n * kIn * 4, hipMemcpyHostToDevice, M->stream));
    HMC_HIP(hipMemcpyAsync(M->t.p, t, (size_t)n * 4, hipMemcpyHostToDevice, M->stream));
    train_tile_kernel<<<ntiles, kTileThreads, 0, M->stream>>>(M->theta.as<float>(), M->X.as<float>(),
                                                              M->t.as<float>(), nullptr, 0, n,
                                                              M->partial.as<float>());
    HMC_HIP(hipGetLastError());
    reduce_adam_kernel<<<(kNP + 1 + 255) / 256, 256, 0, M->stream>>>(M->partial.as<float>(), ntiles,
                                                                     M->theta.as<float>(), M->m.as<float>(),
                                                                     M->v.as<float>(), 0.0f, 1.0f, 1.0f, 0,
                                                                     M->grad.as<float>(), M->loss.as<float>());
    HMC_HIP(hipGetLastError());
    float lsum = 0.0f;
    HMC_HIP(hipMemcpyAsync(grad_out, M->grad.p, kNP * 4, hipMemcpyDeviceToHost, M->stream));
    HMC_HIP(hipMemcpyAsync(&lsum, M->loss.p, 4, hipMemcpyDeviceToHost, M->stream));
    HMC_HIP(hipStreamSynchronize(M->stream));
    *loss_out = lsum / (float)n;
    return HMC_OK;
}

// One Adam step with a host-supplied gradient (step counter advances).
hmc_status hmc_mlp_adam_step(hmc_mlp* M, const float* grad, float lr) {
    set_error("");
    if (!M || !grad) return fail(HMC_E_INVAL, "NULL argument");
    HMC_TRY(M->grad.ensure(kNP * 4, "mlp gradient"));
    HMC_HIP(hipMemcpyAsync(M->grad.p, grad, kNP * 4, hipMemcpyHostToDevice, M->stream));
    M->step += 1;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)M->step));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)M->step));
    adam_kernel<<<(kNP + 255) / 256, 256, 0, M->stream>>>(M->grad.as<float>(), M->theta.as<float>(),
                                                          M->m.as<float>(), M->v.as<float>(), lr, c1, c2);
    HMC_HIP(hipGetLastError());
    HMC_HIP(hipStreamSynchronize(M->stream));
    return HMC_OK;
}

hmc_status hmc_mlp_train(hmc_mlp* M, const double* euler, const double* eps, const double* E, int64_t n,
                         int32_t on_device, int32_t epochs, int32_t batch, float lr, uint64_t seed,
                         float* final_loss) {
    set_error("");
    if (!M || !euler || !eps || !E) return fail(HMC_E_INVAL, "NULL argument");
    if (n < kTile || n >= (1ll << 31)) return fail(HMC_E_INVAL, "n must be in [32, 2^31)");
    if (epochs < 1 || batch < kTile || batch % kTile != 0) return fail(HMC_E_INVAL, "bad epochs or batch");
    if (!(lr > 0.0f)) return fail(HMC_E_INVAL, "lr must be positive");
    batch = (int32_t)std::min<int64_t>(batch, n / kTile * kTile);
    // targets: mean and standard deviation in double on the host
    std::vector<double> hE((size_t)n);
    if (on_device) HMC_HIP(hipMemcpy(hE.data(), E, (size_t)n * 8, hipMemcpyDeviceToHost));
    else std::memcpy(hE.data(), E, (size_t)n * 8);
    double mean = 0.0;
    for (double x : hE) {
        if (!std::isfinite(x)) return fail(HMC_E_INVAL, "non-finite training target");
        mean += x;
    }
    mean /= (double)n;
    double var = 0.0;
    for (double x : hE) var += (x - mean) * (x - mean);
    const double sdev = std::sqrt(var / (double)n);
    if (!(sdev > 0.0)) return fail(HMC_E_INVAL, "training targets have zero spread");
    M->mean = mean;
    M->sdev = sdev;
    HMC_TRY(make_features(M, euler, eps, n, on_device));
    const double* dE = nullptr;
    HMC_TRY(upload_or_alias(E, (size_t)n * 8, on_device, M->E, &dE, M->stream, "mlp energies"));
    HMC_TRY(M->t.ensure((size_t)n * 4, "mlp targets"));
    targets_kernel<<<(unsigned)((n + 255) / 256), 256, 0, M->stream>>>(dE, n, mean, 1.0 / sdev, M->t.as<float>());
    HMC_HIP(hipGetLastError());
    const int ntiles = batch / kTile;
    const int64_t nbatches = n / batch;
    HMC_TRY(M->partial.ensure((size_t)ntiles * (kNP + 1) * 4, "mlp partial gradients"));
    HMC_TRY(M->sel.ensure((size_t)n * 4, "mlp permutation"));
    HMC_TRY(M->loss.ensure((size_t)nbatches * 4, "mlp losses"));
    std::vector<uint32_t> perm((size_t)n);
    const int64_t total_steps = (int64_t)epochs * nbatches;
    int64_t k = 0;
    for (int32_t ep = 0; ep < epochs; ++ep) {
        // Fisher-Yates with Philox draws (epoch, position)
        for (int64_t i = 0; i < n; ++i) perm[(size_t)i] = (uint32_t)i;
        for (int64_t i = n - 1; i > 0; --i) {
            const uint64_t r = philox_u32(seed, (uint32_t)ep, (uint32_t)i, 0x53485546u);
            const int64_t j = (int64_t)((r * (uint64_t)(i + 1)) >> 32);
            std::swap(perm[(size_t)i], perm[(size_t)j]);
        }
        HMC_HIP(hipMemcpyAsync(M->sel.p, perm.data(), (size_t)n * 4, hipMemcpyHostToDevice, M->stream));
        for (int64_t b = 0; b < nbatches; ++b, ++k) {
            const double frac = (double)k / (double)std::max<int64_t>(1, total_steps - 1);
            const float lr_k = (float)(lr * (0.1 + 0.9 * 0.5 * (1.0 + std::cos(kPi * frac))));
            M->step += 1;
            const float c1 = (float)(1.0 - std::pow(0.9, (double)M->step));
            const float c2 = (float)(1.0 - std::pow(0.999, (double)M->step));
            train_tile_kernel<<<ntiles, kTileThreads, 0, M->stream>>>(M->theta.as<float>(), M->X.as<float>(),
                                                                      M->t.as<float>(), M->sel.as<uint32_t>(),
                                                                      b * batch, batch, M->partial.as<float>());
            reduce_adam_kernel<<<(kNP + 1 + 255) / 256, 256, 0, M->stream>>>(
                M->partial.as<float>(), ntiles, M->theta.as<float>(), M->m.as<float>(), M->v.as<float>(), lr_k, c1,
                c2, 1, nullptr, M->loss.as<float>() + b);
        }
        HMC_HIP(hipGetLastError());
        // the host permutation buffer is reused next epoch: wait for the upload
        HMC_HIP(hipStreamSynchronize(M->stream));
    }
    if (final_loss) {
        std::vector<float> l((size_t)nbatches);
        HMC_HIP(hipMemcpy(l.data(), M->loss.p, (size_t)nbatches * 4, hipMemcpyDeviceToHost));
        double s = 0.0;
        for (float x : l) s += x;
        *final_loss = (float)(s / ((double)nbatches * batch));
    }
    return HMC_OK;
}

// E_rho (MPa) predicted for n crystals (double in/out, host or device).
hmc_status hmc_mlp_predict(hmc_mlp* M, const double* euler, const double* eps, int64_t n, int32_t on_device,
                           double* E_out) {
    set_error("");
    if (!M || (n > 0 && (!euler || !eps || !E_out))) return fail(HMC_E_INVAL, "NULL argument");
    if (n < 0 || n >= (1ll << 31)) return fail(HMC_E_INVAL, "n out of range");
    if (n == 0) return HMC_OK;
    HMC_TRY(make_features(M, euler, eps, n, on_device));
    double* dout = E_out;
    if (!on_device) {
        HMC_TRY(M->E.ensure((size_t)n * 8, "mlp predictions"));
        dout = M->E.as<double>();
    }
    predict_kernel<false><<<predict_blocks(n), kPredThreads, 0, M->stream>>>(
        M->theta.as<float>(), M->X.as<float>(), n, M->mean, M->sdev, dout, nullptr, QueryIO{});
    HMC_HIP(hipGetLastError());
    if (!on_device) HMC_HIP(hipMemcpyAsync(E_out, dout, (size_t)n * 8, hipMemcpyDeviceToHost, M->stream));
    HMC_HIP(hipStreamSynchronize(M->stream));
    return HMC_OK;
}

// Standardised network outputs for scaled features (host float arrays).
hmc_status hmc_mlp_forward(hmc_mlp* M, const float* X, int32_t n, float* y_out) {
    set_error("");
    if (!M || !X || !y_out || n < 1) return fail(HMC_E_INVAL, "NULL argument or n < 1");
    HMC_TRY(M->X.ensure((size_t)n * kIn * 4, "mlp features"));
    HMC_TRY(M->t.ensure((size_t)n * 4, "mlp outputs"));
    HMC_HIP(hipMemcpyAsync(M->X.p, X, (size_t)n * kIn * 4, hipMemcpyHostToDevice, M->stream));
    predict_kernel<false><<<predict_blocks(n), kPredThreads, 0, M->stream>>>(
        M->theta.as<float>(), M->X.as<float>(), n, 0.0, 1.0, nullptr, M->t.as<float>(), QueryIO{});
    HMC_HIP(hipGetLastError());
    HMC_HIP(hipMemcpyAsync(y_out, M->t.p, (size_t)n * 4, hipMemcpyDeviceToHost, M->stream));
    HMC_HIP(hipStreamSynchronize(M->stream));
    return HMC_OK;
}

hmc_status hmc_mlp_infer(hmc_mlp* M, const float* X_dev, float* y_dev, int64_t n, void* stream) {
    set_error("");
    if (!M || !X_dev || !y_dev || n < 0) return fail(HMC_E_INVAL, "NULL argument or n < 0");
    if (n >= (int64_t)1 << 40) return fail(HMC_E_INVAL, "n too large");
    if (n == 0) return HMC_OK;
    hipStream_t s = stream ? static_cast<hipStream_t>(stream) : M->stream;
    if (s != M->stream) {
        // the parameters may still be in flight on the handle's stream
        if (!M->ready) HMC_HIP(hipEventCreateWithFlags(&M->ready, hipEventDisableTiming));
        HMC_HIP(hipEventRecord(M->ready, M->stream));
        HMC_HIP(hipStreamWaitEvent(s, M->ready, 0));
    }
    predict_kernel<false><<<predict_blocks(n), kPredThreads, 0, s>>>(
        M->theta.as<float>(), X_dev, n, 0.0, 1.0, nullptr, y_dev, QueryIO{});
    HMC_HIP(hipGetLastError());
    return HMC_OK;
}

// Per-grain bulk energies for the sweep from the stored dislocation energy
// of every grain under one macroscopic strain: B[q] = round-half-even(
// E_rho[q] * E_scale * 65536).  mode 0: network with audit and fallback;
// mode 1: the crystal-plasticity solver for every grain (the method without
// the network).
hmc_status hmc_surrogate_update(hmc_lattice* L, hmc_mlp* M, const double* euler, const double* eps6, double E_scale,
                                int32_t mode, int32_t n_audit, double audit_tol, uint64_t seed,
                                int32_t* used_solver, double* audit_err, int32_t* B_out) {
    set_error("");
    if (!L || !euler || !eps6 || !used_solver || !audit_err) return fail(HMC_E_INVAL, "NULL argument");
    if (mode == 0 && !M) return fail(HMC_E_INVAL, "mode 0 needs a network");
    if (mode != 0 && mode != 1) return fail(HMC_E_INVAL, "mode must be 0 or 1");
    if (!(E_scale > 0.0) || !std::isfinite(E_scale)) return fail(HMC_E_INVAL, "E_scale must be positive");
    const int32_t Q = L->Q;
    hmc_mlp* W = M;
    hmc_mlp scratch_holder;   // buffers when no network is given
    if (!W) W = &scratch_holder;
    struct ReleaseAtExit {    // the holder's read-back memory, once the energies are set
        HostBuf* b;
        ~ReleaseAtExit() {
            if (b) b->release();
        }
    } release_readback{W == &scratch_holder ? &W->readback : nullptr};
    if (!W->stream) W->stream = L->stream;
    // every grain under the same strain: one 6-vector read with stride 0
    bool in_box = true;
    for (int k = 0; k < 6; ++k) {
        if (!std::isfinite(eps6[k])) return fail(HMC_E_INVAL, "non-finite strain");
        if (std::fabs(eps6[k]) > kStrainBox * (1.0 + 1e-12)) in_box = false;
    }
    const int32_t na = std::max(0, std::min(n_audit, Q));
    hmc_status st = W->euler.ensure((size_t)Q * 24, "grain orientations");
    if (st == HMC_OK) st = W->eps.ensure(48, "grain strain");
    if (st == HMC_OK) st = W->E.ensure((size_t)Q * 8, "grain energies");
    if (st == HMC_OK) st = W->Bq.ensure((size_t)Q * 4, "quantised energies");
    if (st == HMC_OK && na > 0) st = W->audit_idx.ensure((size_t)na * 4, "audit grains");
    if (st == HMC_OK && na > 0) st = W->Eaudit.ensure((size_t)na * 32, "audit orientations and energies");
    hipError_t e = hipSuccess;
    if (st == HMC_OK) e = hipMemcpyAsync(W->euler.p, euler, (size_t)Q * 24, hipMemcpyHostToDevice, W->stream);
    if (st == HMC_OK && e == hipSuccess) e = hipMemcpyAsync(W->eps.p, eps6, 48, hipMemcpyHostToDevice, W->stream);
    if (st == HMC_OK) st = W->readback.ensure((size_t)Q * 12 + (size_t)na * 8, "query read-back");
    double* predicted = st == HMC_OK ? W->readback.as<double>() : nullptr;
    double* Es = predicted ? predicted + Q : nullptr;
    int32_t* B = Es ? reinterpret_cast<int32_t*>(Es + na) : nullptr;
    bool solver = mode == 1 || !in_box;
    double err = 0.0;
    if (st == HMC_OK && e == hipSuccess && !solver) {
        // features, inference and the energies quantised in one launch, ahead
        // of the audit's decision: an accepted query needs no second round trip
        {
            const QueryIO q{W->euler.as<double>(), W->eps.as<double>(), E_scale * 65536.0, W->Bq.as<int32_t>()};
            predict_kernel<true><<<predict_blocks(Q), kPredThreads, 0, W->stream>>>(
                W->theta.as<float>(), nullptr, Q, W->mean, W->sdev, W->E.as<double>(), nullptr, q);
            e = hipGetLastError();
        }
        // audit: n_audit grains drawn with Philox, solved exactly with their
        // own random streams, i.e. the values the fallback would give them
        std::vector<int32_t> ids((size_t)na);
        if (st == HMC_OK && e == hipSuccess && na > 0) {
            std::vector<double> ae((size_t)na * 3);
            for (int32_t a = 0; a < na; ++a) {
                ids[a] = (int32_t)(((uint64_t)philox_u32(seed, (uint32_t)a, 1u, 0x41554449u) * (uint64_t)Q) >> 32);
                std::memcpy(&ae[(size_t)a * 3], euler + (size_t)ids[a] * 3, 24);
            }
            double* d_ae = W->Eaudit.as<double>();
            e = hipMemcpyAsync(W->audit_idx.p, ids.data(), (size_t)na * 4, hipMemcpyHostToDevice, W->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(d_ae, ae.data(), (size_t)na * 24, hipMemcpyHostToDevice, W->stream);
            if (e == hipSuccess)
                st = mcp_solve_device(d_ae, W->eps.as<double>(), na, seed, 0, d_ae + (size_t)na * 3, nullptr,
                                      W->stream, 0, W->audit_idx.as<int32_t>());
            if (st == HMC_OK && e == hipSuccess)
                e = hipMemcpyAsync(Es, d_ae + (size_t)na * 3, (size_t)na * 8, hipMemcpyDeviceToHost, W->stream);
        }
        if (st == HMC_OK && e == hipSuccess)
            e = hipMemcpyAsync(predicted, W->E.p, (size_t)Q * 8, hipMemcpyDeviceToHost, W->stream);
        if (st == HMC_OK && e == hipSuccess)
            e = hipMemcpyAsync(B, W->Bq.p, (size_t)Q * 4, hipMemcpyDeviceToHost, W->stream);
        if (st == HMC_OK && e == hipSuccess) e = hipStreamSynchronize(W->stream);
        if (st == HMC_OK && e == hipSuccess) {
            for (int32_t q = 0; q < Q; ++q)
                if (!std::isfinite(predicted[(size_t)q])) err = INFINITY;
            for (int32_t a = 0; a < na && std::isfinite(err); ++a)
                err = std::max(err, std::fabs(predicted[(size_t)ids[a]] - Es[(size_t)a]) / std::fabs(Es[(size_t)a]));
            if (!(err <= audit_tol)) solver = true;
        }
    }
    if (st == HMC_OK && e == hipSuccess && solver) {
        st = mcp_solve_device(W->euler.as<double>(), W->eps.as<double>(), Q, seed, 0, W->E.as<double>(), nullptr,
                              W->stream, 0, nullptr);
        if (st == HMC_OK) {
            quantise_kernel<<<(Q + 255) / 256, 256, 0, W->stream>>>(W->E.as<double>(), Q, E_scale * 65536.0,
                                                                     W->Bq.as<int32_t>());
            e = hipGetLastError();
        }
        if (st == HMC_OK && e == hipSuccess)
            e = hipMemcpyAsync(B, W->Bq.p, (size_t)Q * 4, hipMemcpyDeviceToHost, W->stream);
        if (st == HMC_OK && e == hipSuccess) e = hipStreamSynchronize(W->stream);
    }
    if (W == &scratch_holder) {
        (void)hipStreamSynchronize(W->stream);   // no copy may still target the read-back memory
        for (DevBuf* b : {&W->X, &W->euler, &W->eps, &W->E, &W->Bq, &W->audit_idx, &W->Eaudit}) b->release();
    }
    if (st != HMC_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "surrogate update");
    HMC_TRY(hmc_set_grain_energy(L, B, Q, 0));
    if (B_out) std::memcpy(B_out, B, (size_t)Q * 4);
    *used_solver = solver ? 1 : 0;
    *audit_err = err;
    return HMC_OK;
}

}  // extern "C"
