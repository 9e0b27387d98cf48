// Learned two-sided diagonal preconditioner for the LSQR solves.
//
// Per index i of z = (x, y, tau), a feature vector (QCPD_NFEAT floats) is read off the
// operator F: its Jacobi column and row norms, the kind of row (x, zero, nonneg, SOC, PSD,
// exp, tau), the diagonal of DPi at the solution, |P_ii| and the stored entries in the row.
// A 3-layer FP32 MLP (QCPD_NFEAT -> 64 -> 64 -> 2, tanh) maps it to log corrections of the
// Jacobi column and row scales. The models are trained on the two-sided equilibration scales
// the library computes for training problems, so one inference pass replaces the
// equilibration sweeps at setup.
//
// FP32 parameter blob (QCPD_MLP_PARAMS floats):
//   mu[F] sd[F]        feature standardisation (set from data, not trained)
//   W1[64][F] b1[64]   W2[64][64] b2[64]   W3[2][64] b3[2]     (W[out][in], row-major)
//
// All reductions run in a fixed order; no floating-point atomics.
#include <math.h>

#include <algorithm>
#include <mutex>

#include "qcpd_internal.h"

namespace qcpd {

constexpr int kF = QCPD_NFEAT;
constexpr int kH = QCPD_MLP_HIDDEN;
constexpr int kOut = 2;
constexpr int oMU = 0, oSD = kF, oW1 = 2 * kF, oB1 = oW1 + kH * kF, oW2 = oB1 + kH,
              oB2 = oW2 + kH * kH, oW3 = oB2 + kH, oB3 = oW3 + kOut * kH, kNParam = oB3 + kOut;
static_assert(kNParam == QCPD_MLP_PARAMS, "parameter blob layout");
static_assert(kH == 64, "one hidden unit per lane");
constexpr int kTrain0 = 2 * kF;  // first trained parameter

// ---------------------------------------------------------------------------------------
// features and targets
// ---------------------------------------------------------------------------------------

__global__ void k_features(Problem p, FeatMeta fm, const double *jcol, const double *jrow,
                           float *feat) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.N) return;
    float f[kF];
#pragma unroll
    for (int k = 0; k < kF; ++k) f[k] = 0.f;
    f[0] = (float)(-log(jcol[i]));
    f[1] = (float)(-log(jrow[i]));
    const int n = p.n;
    if (i < n) {
        f[2] = 1.f;
        f[9] = 1.f;
        double pii = 0.0;
        for (int k = p.Prp[i]; k < p.Prp[i + 1]; ++k)
            if (p.Pci[k] == i) pii = p.Pv[k];
        f[10] = (float)log1p(fabs(pii));
        f[11] = (float)log1p((double)(p.Prp[i + 1] - p.Prp[i] + p.Trp[i + 1] - p.Trp[i]));
    } else if (i < p.N - 1) {
        const int r = i - n;
        const int kind = r < fm.n_zero ? 3 : r < fm.n_diag ? 4 : r < fm.soc_end ? 5
                         : r < fm.psd_end ? 6 : 7;
        f[kind] = 1.f;
        f[9] = (float)p.jdiag[r];
        f[11] = (float)log1p((double)(p.Arp[r + 1] - p.Arp[r]));
    } else {
        f[8] = 1.f;
        f[9] = 1.f;
        f[11] = (float)log1p((double)(p.n + p.m));
    }
#pragma unroll
    for (int k = 0; k < kF; ++k) feat[(size_t)i * kF + k] = f[k];
}

__global__ void k_targets(int N, const double *jcol, const double *jrow, const double *ecol,
                          const double *erow, float *target) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    target[2 * (size_t)i] = (float)log(ecol[i] / jcol[i]);
    target[2 * (size_t)i + 1] = (float)log(erow[i] / jrow[i]);
}

// ---------------------------------------------------------------------------------------
// initialisation: standardisation from data, Glorot-uniform weights from a counter hash
// ---------------------------------------------------------------------------------------

// SplitMix64 finaliser (Steele, Lea, Flood 2014).
__device__ inline uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_feat_stats(const float *feat, int nrows, float *w) {
    __shared__ double s1[256], s2[256];
    const int tid = threadIdx.x;
    for (int k = 0; k < kF; ++k) {
        double a = 0.0, b = 0.0;
        for (int r = tid; r < nrows; r += 256) {
            const double v = feat[(size_t)r * kF + k];
            a += v;
            b += v * v;
        }
        s1[tid] = a;
        s2[tid] = b;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (tid < h) {
                s1[tid] += s1[tid + h];
                s2[tid] += s2[tid + h];
            }
            __syncthreads();
        }
        if (tid == 0) {
            const double mu = s1[0] / nrows;
            const double var = fmax(0.0, s2[0] / nrows - mu * mu);
            const double sd = sqrt(var);
            w[oMU + k] = (float)mu;
            w[oSD + k] = sd > 1e-3 ? (float)sd : 1.f;
        }
        __syncthreads();
    }
}

__global__ void k_init_weights(float *w, uint64_t seed) {
    const int pi = kTrain0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (pi >= kNParam) return;
    int fan_in = 0, fan_out = 0;
    if (pi < oB1) { fan_in = kF; fan_out = kH; }
    else if (pi >= oW2 && pi < oB2) { fan_in = kH; fan_out = kH; }
    else if (pi >= oW3 && pi < oB3) { fan_in = kH; fan_out = kOut; }
    if (fan_in == 0) {  // biases
        w[pi] = 0.f;
        return;
    }
    const uint64_t z = splitmix64(seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(pi + 1)));
    const double u = (double)(z >> 11) * 0x1.0p-53;  // [0, 1)
    const double a = sqrt(6.0 / (fan_in + fan_out));
    w[pi] = (float)((2.0 * u - 1.0) * a);
}

// ---------------------------------------------------------------------------------------
// inference: one thread per index, the weights broadcast from LDS
// ---------------------------------------------------------------------------------------

__device__ inline void mlp_forward(const float *w, const float *x, float *o) {
    float xn[kF], h1[kH], h2[kH];
#pragma unroll
    for (int k = 0; k < kF; ++k) xn[k] = (x[k] - w[oMU + k]) / w[oSD + k];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float a = w[oB1 + j];
#pragma unroll
        for (int k = 0; k < kF; ++k) a = fmaf(w[oW1 + j * kF + k], xn[k], a);
        h1[j] = tanhf(a);
    }
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float a = w[oB2 + j];
#pragma unroll
        for (int k = 0; k < kH; ++k) a = fmaf(w[oW2 + j * kH + k], h1[k], a);
        h2[j] = tanhf(a);
    }
#pragma unroll
    for (int j = 0; j < kOut; ++j) {
        float a = w[oB3 + j];
#pragma unroll
        for (int k = 0; k < kH; ++k) a = fmaf(w[oW3 + j * kH + k], h2[k], a);
        o[j] = a;
    }
}

__global__ __launch_bounds__(256) void k_mlp_predict(const float *feat, int nrows, const float *w,
                                                     float *out) {
    __shared__ float ws[kNParam];
    for (int k = threadIdx.x; k < kNParam; k += blockDim.x) ws[k] = w[k];
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    float x[kF], o[kOut];
#pragma unroll
    for (int k = 0; k < kF; ++k) x[k] = feat[(size_t)i * kF + k];
    mlp_forward(ws, x, o);
    out[2 * (size_t)i] = o[0];
    out[2 * (size_t)i + 1] = o[1];
}

// scales = Jacobi scales times exp(MLP corrections), the corrections clamped to [-30, 30]
__global__ __launch_bounds__(256) void k_mlp_scales(const float *feat, int N, const float *w,
                                                    const double *jcol, const double *jrow,
                                                    double *col, double *row) {
    __shared__ float ws[kNParam];
    for (int k = threadIdx.x; k < kNParam; k += blockDim.x) ws[k] = w[k];
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    float x[kF], o[kOut];
#pragma unroll
    for (int k = 0; k < kF; ++k) x[k] = feat[(size_t)i * kF + k];
    mlp_forward(ws, x, o);
    const double c0 = isfinite(o[0]) ? fmin(fmax((double)o[0], -30.0), 30.0) : 0.0;
    const double c1 = isfinite(o[1]) ? fmin(fmax((double)o[1], -30.0), 30.0) : 0.0;
    col[i] = jcol[i] * exp(c0);
    row[i] = jrow[i] * exp(c1);
}

// ---------------------------------------------------------------------------------------
// training: gradient of the mean squared error, then Adam
// ---------------------------------------------------------------------------------------

// Each workgroup takes a contiguous range of rows in passes of kR rows. A pass keeps its
// activations and back-propagated errors in LDS; lane j of a wavefront owns hidden unit j
// in the forward and backward sweeps (weights read transposed for the forward sweep so that
// the lanes' LDS reads are consecutive). Thread t accumulates the gradient of parameters
// kTrain0 + t + 256 s in registers; the per-block partials go to the workspace and are
// summed in block order by k_grad_reduce.
constexpr int kR = 16;
constexpr int kOwn = (kNParam - kTrain0 + 255) / 256;

constexpr int kMaxGradBlocks = 256;
int grad_blocks(int nrows) { return std::max(1, std::min(kMaxGradBlocks, div_up(nrows, 4 * kR))); }

__global__ __launch_bounds__(256) void k_mlp_grad(const float *feat, const float *target, int nrows,
                                                  const float *w, float *part) {
    __shared__ float ws[kNParam];
    __shared__ float w1t[kF * kH], w2t[kH * kH];
    __shared__ float X[kR][kF], H1[kR][kH], H2[kR][kH], D1[kR][kH], D2[kR][kH], D3[kR][kOut];
    const int tid = threadIdx.x;
    for (int k = tid; k < kNParam; k += 256) ws[k] = w[k];
    for (int e = tid; e < kF * kH; e += 256) {
        const int j = e / kF, k = e % kF;
        w1t[k * kH + j] = w[oW1 + e];
    }
    for (int e = tid; e < kH * kH; e += 256) {
        const int j = e / kH, k = e % kH;
        w2t[k * kH + j] = w[oW2 + e];
    }
    float g[kOwn];
#pragma unroll
    for (int s = 0; s < kOwn; ++s) g[s] = 0.f;
    float loss = 0.f;
    const int per_block = (nrows + (int)gridDim.x - 1) / (int)gridDim.x;
    const int r_begin = blockIdx.x * per_block, r_end = min(nrows, r_begin + per_block);
    const float inv_rows = 1.f / nrows;
    __syncthreads();
    for (int r0 = r_begin; r0 < r_end; r0 += kR) {
        const int nr = min(kR, r_end - r0);
        for (int e = tid; e < kR * kF; e += 256) {
            const int r = e / kF, k = e % kF;
            X[r][k] = r < nr ? (feat[(size_t)(r0 + r) * kF + k] - ws[oMU + k]) / ws[oSD + k] : 0.f;
        }
        __syncthreads();
        for (int e = tid; e < kR * kH; e += 256) {
            const int r = e / kH, j = e % kH;
            float a = ws[oB1 + j];
#pragma unroll
            for (int k = 0; k < kF; ++k) a = fmaf(w1t[k * kH + j], X[r][k], a);
            H1[r][j] = tanhf(a);
        }
        __syncthreads();
        for (int e = tid; e < kR * kH; e += 256) {
            const int r = e / kH, j = e % kH;
            float a = ws[oB2 + j];
#pragma unroll 16
            for (int k = 0; k < kH; ++k) a = fmaf(w2t[k * kH + j], H1[r][k], a);
            H2[r][j] = tanhf(a);
        }
        __syncthreads();
        if (tid < kR * kOut) {
            const int r = tid / kOut, j = tid % kOut;
            float a = ws[oB3 + j];
            for (int k = 0; k < kH; ++k) a = fmaf(ws[oW3 + j * kH + k], H2[r][k], a);
            const float diff = r < nr ? a - target[(size_t)(r0 + r) * kOut + j] : 0.f;
            loss = fmaf(diff, diff, loss);
            D3[r][j] = 2.f * diff * inv_rows;
        }
        __syncthreads();
        for (int e = tid; e < kR * kH; e += 256) {
            const int r = e / kH, j = e % kH;
            float a = 0.f;
#pragma unroll
            for (int k = 0; k < kOut; ++k) a = fmaf(ws[oW3 + k * kH + j], D3[r][k], a);
            D2[r][j] = a * (1.f - H2[r][j] * H2[r][j]);
        }
        __syncthreads();
        for (int e = tid; e < kR * kH; e += 256) {
            const int r = e / kH, j = e % kH;
            float a = 0.f;
#pragma unroll 16
            for (int k = 0; k < kH; ++k) a = fmaf(ws[oW2 + k * kH + j], D2[r][k], a);
            D1[r][j] = a * (1.f - H1[r][j] * H1[r][j]);
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kOwn; ++s) {
            const int pi = kTrain0 + tid + 256 * s;
            if (pi >= kNParam) break;
            float a = 0.f;
            if (pi < oB1) {
                const int j = (pi - oW1) / kF, k = (pi - oW1) % kF;
                for (int r = 0; r < nr; ++r) a = fmaf(D1[r][j], X[r][k], a);
            } else if (pi < oW2) {
                const int j = pi - oB1;
                for (int r = 0; r < nr; ++r) a += D1[r][j];
            } else if (pi < oB2) {
                const int j = (pi - oW2) / kH, k = (pi - oW2) % kH;
                for (int r = 0; r < nr; ++r) a = fmaf(D2[r][j], H1[r][k], a);
            } else if (pi < oW3) {
                const int j = pi - oB2;
                for (int r = 0; r < nr; ++r) a += D2[r][j];
            } else if (pi < oB3) {
                const int j = (pi - oW3) / kH, k = (pi - oW3) % kH;
                for (int r = 0; r < nr; ++r) a = fmaf(D3[r][j], H2[r][k], a);
            } else {
                const int j = pi - oB3;
                for (int r = 0; r < nr; ++r) a += D3[r][j];
            }
            g[s] += a;
        }
        __syncthreads();
    }
    float *gp = part + (size_t)blockIdx.x * (kNParam + 1);
#pragma unroll
    for (int s = 0; s < kOwn; ++s) {
        const int pi = kTrain0 + tid + 256 * s;
        if (pi < kNParam) gp[pi] = g[s];
    }
    if (tid < kTrain0) gp[tid] = 0.f;
    // loss of the block, summed in thread order (H1 is free after the last pass)
    float *ls = &H1[0][0];
    ls[tid] = loss;
    __syncthreads();
    if (tid == 0) {
        float t = 0.f;
        for (int k = 0; k < 256; ++k) t += ls[k];
        gp[kNParam] = t;
    }
}

// grad[p] = sum over blocks in block order; grad[kNParam] = mean squared error per row
__global__ void k_grad_reduce(const float *part, int nblocks, int nrows, float *grad) {
    const int pi = blockIdx.x * blockDim.x + threadIdx.x;
    if (pi > kNParam) return;
    float t = 0.f;
    for (int b = 0; b < nblocks; ++b) t += part[(size_t)b * (kNParam + 1) + pi];
    grad[pi] = pi == kNParam ? t / nrows : t;
}

// Adam (Kingma and Ba 2015) on the trained parameters
__global__ void k_adam(const float *grad, float *w, float *m, float *v, int step, float lr,
                       float b1, float b2, float eps) {
    const int pi = kTrain0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (pi >= kNParam) return;
    const float g = grad[pi];
    const float mm = b1 * m[pi] + (1.f - b1) * g;
    const float vv = b2 * v[pi] + (1.f - b2) * g * g;
    m[pi] = mm;
    v[pi] = vv;
    const float mh = mm / (1.f - powf(b1, (float)step));
    const float vh = vv / (1.f - powf(b2, (float)step));
    w[pi] -= lr * mh / (sqrtf(vh) + eps);
}

// ---------------------------------------------------------------------------------------
// fixed scratch of qcpd_mlp_grad_noalloc: the per-workgroup partial gradients of the largest
// k_mlp_grad launch (kMaxGradBlocks workgroups), 5.27 MB, one copy per GPU for the life of
// the process. In host code `scratch` names a host-side stand-in; kernels are given the
// device address that hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------------------
constexpr size_t kScratchFloats = (size_t)kMaxGradBlocks * (kNParam + 1);
static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, resolved once per device.
hipError_t scratch_address(float **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = static_cast<float *>(ptr);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

// ---------------------------------------------------------------------------------------
// launchers used by the handle API
// ---------------------------------------------------------------------------------------

hipError_t launch_features(const Problem &p, const FeatMeta &fm, const double *jcol,
                           const double *jrow, float *feat, hipStream_t s) {
    hipLaunchKernelGGL(k_features, dim3(div_up(p.N, 256)), dim3(256), 0, s, p, fm, jcol, jrow, feat);
    return hipGetLastError();
}

hipError_t launch_targets(int N, const double *jcol, const double *jrow, const double *ecol,
                          const double *erow, float *target, hipStream_t s) {
    hipLaunchKernelGGL(k_targets, dim3(div_up(N, 256)), dim3(256), 0, s, N, jcol, jrow, ecol, erow,
                       target);
    return hipGetLastError();
}

hipError_t launch_mlp_scales(const float *feat, int N, const float *w, const double *jcol,
                             const double *jrow, double *col, double *row, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_scales, dim3(div_up(N, 256)), dim3(256), 0, s, feat, N, w, jcol, jrow,
                       col, row);
    return hipGetLastError();
}

}  // namespace qcpd

using namespace qcpd;

extern "C" {

qcpd_status qcpd_mlp_init(const float *feat, int32_t nrows, uint64_t seed, float *weights,
                          void *stream) {
    if (!feat || nrows < 1 || !weights) return QCPD_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_feat_stats, dim3(1), dim3(256), 0, s, feat, nrows, weights);
    hipLaunchKernelGGL(k_init_weights, dim3(div_up(kNParam - kTrain0, 256)), dim3(256), 0, s, weights,
                       seed);
    if (hipGetLastError() != hipSuccess) return QCPD_ERR_HIP;
    return hipStreamSynchronize(s) == hipSuccess ? QCPD_OK : QCPD_ERR_HIP;
}

qcpd_status qcpd_mlp_predict(const float *feat, int32_t nrows, const float *weights, float *out,
                             void *stream) {
    if (!feat || nrows < 0 || !weights || !out) return QCPD_ERR_INVALID_ARG;
    if (nrows == 0) return QCPD_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_mlp_predict, dim3(div_up(nrows, 256)), dim3(256), 0, s, feat, nrows, weights,
                       out);
    return hipGetLastError() == hipSuccess ? QCPD_OK : QCPD_ERR_HIP;
}

int64_t qcpd_mlp_workspace_floats(int32_t nrows) {
    if (nrows < 1) return 0;
    return (int64_t)grad_blocks(nrows) * (kNParam + 1);
}

qcpd_status qcpd_mlp_grad(const float *feat, const float *target, int32_t nrows,
                          const float *weights, float *workspace, float *grad, void *stream) {
    if (!feat || !target || nrows < 1 || !weights || !workspace || !grad) return QCPD_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nb = grad_blocks(nrows);
    hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(256), 0, s, feat, target, nrows, weights, workspace);
    hipLaunchKernelGGL(k_grad_reduce, dim3(div_up(kNParam + 1, 256)), dim3(256), 0, s, workspace, nb,
                       nrows, grad);
    return hipGetLastError() == hipSuccess ? QCPD_OK : QCPD_ERR_HIP;
}

qcpd_status qcpd_mlp_grad_noalloc(const float *feat, const float *target, int32_t nrows,
                                  const float *weights, float *grad, void *stream) {
    if (!feat || !target || nrows < 1 || !weights || !grad) return QCPD_ERR_INVALID_ARG;
    const int nb = grad_blocks(nrows);
    if ((size_t)nb * (kNParam + 1) > kScratchFloats) return QCPD_ERR_INVALID_ARG;
    float *part = nullptr;
    if (scratch_address(&part) != hipSuccess) return QCPD_ERR_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // k_mlp_grad writes every slot of its nb partial rows, so nothing needs clearing
    hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(256), 0, s, feat, target, nrows, weights, part);
    hipLaunchKernelGGL(k_grad_reduce, dim3(div_up(kNParam + 1, 256)), dim3(256), 0, s, part, nb,
                       nrows, grad);
    return hipGetLastError() == hipSuccess ? QCPD_OK : QCPD_ERR_HIP;
}

qcpd_status qcpd_mlp_adam(const float *grad, float *weights, float *adam_m, float *adam_v,
                          int32_t step, float lr, void *stream) {
    if (!grad || !weights || !adam_m || !adam_v || step < 1 || !(lr > 0.f)) return QCPD_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_adam, dim3(div_up(kNParam - kTrain0, 256)), dim3(256), 0, s, grad, weights,
                       adam_m, adam_v, step, lr, 0.9f, 0.999f, 1e-8f);
    return hipGetLastError() == hipSuccess ? QCPD_OK : QCPD_ERR_HIP;
}

}  // extern "C"
