// Kernels of the per-tile cost model (an 8 -> 64 -> 64 -> V multilayer
// perceptron with ReLU): inference with argmin, the masked-MSE gradient and
// the Adam update.  The model is tiny (about 5K parameters), so the design
// aims at determinism rather than speed: one thread evaluates one feature
// row with the parameters staged in LDS (every thread reads the same weight
// at the same time, an LDS broadcast); weight gradients are sums over the
// batch taken by one thread per parameter in row order, in FP64.
#include <hip/hip_runtime.h>

#include "spmm_internal.h"

namespace spmm {
namespace {

constexpr int kIn = SPMM_NUM_FEATURES;
constexpr int kH = SPMM_MLP_HIDDEN;
constexpr int kV = SPMM_NUM_VARIANTS;
constexpr int kP = SPMM_MLP_PARAMS;
constexpr int kRowsPerBlock = 64;

__device__ __forceinline__ void stage_params(const float* __restrict__ params, float* w) {
    for (int i = threadIdx.x; i < kP; i += blockDim.x) w[i] = params[i];
    __syncthreads();
}

// Forward pass of one feature row; a1 and a2 are the hidden activations.
__device__ __forceinline__ void forward(const float* w, const float* x, float* a1, float* a2, float* out) {
    const float* W1 = w + SPMM_MLP_OFF_W1;
    const float* B1 = w + SPMM_MLP_OFF_B1;
    const float* W2 = w + SPMM_MLP_OFF_W2;
    const float* B2 = w + SPMM_MLP_OFF_B2;
    const float* W3 = w + SPMM_MLP_OFF_W3;
    const float* B3 = w + SPMM_MLP_OFF_B3;
#pragma unroll
    for (int j = 0; j < kH; ++j) a1[j] = B1[j];
#pragma unroll
    for (int i = 0; i < kIn; ++i)
#pragma unroll
        for (int j = 0; j < kH; ++j) a1[j] = fmaf(x[i], W1[i * kH + j], a1[j]);
#pragma unroll
    for (int j = 0; j < kH; ++j) a1[j] = fmaxf(a1[j], 0.0f);
#pragma unroll
    for (int j = 0; j < kH; ++j) a2[j] = B2[j];
    for (int i = 0; i < kH; ++i) {
        const float ai = a1[i];
#pragma unroll
        for (int j = 0; j < kH; ++j) a2[j] = fmaf(ai, W2[i * kH + j], a2[j]);
    }
#pragma unroll
    for (int j = 0; j < kH; ++j) a2[j] = fmaxf(a2[j], 0.0f);
#pragma unroll
    for (int v = 0; v < kV; ++v) out[v] = B3[v];
#pragma unroll
    for (int j = 0; j < kH; ++j)
#pragma unroll
        for (int v = 0; v < kV; ++v) out[v] = fmaf(a2[j], W3[j * kV + v], out[v]);
}

__global__ __launch_bounds__(kRowsPerBlock) void mlp_predict_kernel(const float* __restrict__ params,
                                                                    const float* __restrict__ feat, int64_t n,
                                                                    float* __restrict__ out,
                                                                    uint8_t* __restrict__ choice) {
    __shared__ float w[kP];
    stage_params(params, w);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[kIn], a1[kH], a2[kH], o[kV];
#pragma unroll
    for (int q = 0; q < kIn; ++q) x[q] = feat[i * kIn + q];
    forward(w, x, a1, a2, o);
    int best = 0;
#pragma unroll
    for (int v = 1; v < kV; ++v)
        if (o[v] < o[best]) best = v;
    if (out)
#pragma unroll
        for (int v = 0; v < kV; ++v) out[i * kV + v] = o[v];
    if (choice) choice[i] = (uint8_t)best;
}

// Number of measured targets (exact integer count, one block).
__global__ __launch_bounds__(256) void mask_count_kernel(const uint8_t* __restrict__ mask, const int32_t* idx,
                                                         int64_t n, uint32_t* __restrict__ count) {
    __shared__ uint32_t red[256];
    uint32_t c = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int64_t r = idx ? idx[i] : i;
#pragma unroll
        for (int v = 0; v < kV; ++v) c += mask ? (mask[r * kV + v] != 0) : 1u;
    }
    red[threadIdx.x] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) count[0] = red[0];
}

// Per row b of the batch (row idx[b] of the data, or b): forward pass, the
// loss term sum_v m (out - y)^2, and the backward deltas
//   d3 = 2 m (out - y) / M, d2 = (d3 W3^T) o [z2 > 0], d1 = (d2 W2^T) o [z1 > 0]
// stored with the inputs and activations for the weight-gradient sums.
__global__ __launch_bounds__(kRowsPerBlock) void mlp_backprop_kernel(
    const float* __restrict__ params, const float* __restrict__ feat, const float* __restrict__ target,
    const uint8_t* __restrict__ mask, const int32_t* __restrict__ idx, int64_t n,
    const uint32_t* __restrict__ count, float* __restrict__ sx, float* __restrict__ sa1,
    float* __restrict__ sa2, float* __restrict__ sd1, float* __restrict__ sd2, float* __restrict__ sd3,
    double* __restrict__ sloss) {
    __shared__ float w[kP];
    stage_params(params, w);
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const int64_t r = idx ? idx[b] : b;
    const float inv_m = 1.0f / (float)(count[0] > 0 ? count[0] : 1u);
    float x[kIn], a1[kH], a2[kH], o[kV];
#pragma unroll
    for (int q = 0; q < kIn; ++q) x[q] = feat[r * kIn + q];
    forward(w, x, a1, a2, o);
    float d3[kV];
    double l = 0.0;
#pragma unroll
    for (int v = 0; v < kV; ++v) {
        const bool m = mask ? mask[r * kV + v] != 0 : true;
        const float e = o[v] - target[r * kV + v];
        d3[v] = m ? 2.0f * e * inv_m : 0.0f;
        if (m) l += (double)e * (double)e;
    }
    sloss[b] = l;
    const float* W2 = w + SPMM_MLP_OFF_W2;
    const float* W3 = w + SPMM_MLP_OFF_W3;
#pragma unroll
    for (int q = 0; q < kIn; ++q) sx[b * kIn + q] = x[q];
#pragma unroll
    for (int v = 0; v < kV; ++v) sd3[b * kV + v] = d3[v];
    float d2[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float s = 0.0f;
#pragma unroll
        for (int v = 0; v < kV; ++v) s = fmaf(d3[v], W3[j * kV + v], s);
        d2[j] = a2[j] > 0.0f ? s : 0.0f;
        sa1[b * kH + j] = a1[j];
        sa2[b * kH + j] = a2[j];
        sd2[b * kH + j] = d2[j];
    }
    for (int i = 0; i < kH; ++i) {
        float s = 0.0f;
#pragma unroll
        for (int j = 0; j < kH; ++j) s = fmaf(d2[j], W2[i * kH + j], s);
        sd1[b * kH + i] = a1[i] > 0.0f ? s : 0.0f;
    }
}

// grad[p] for every parameter p: a sum over the batch rows in order, FP64.
//   W1[i][j] = sum_b x[b][i] d1[b][j]     b1[j] = sum_b d1[b][j]
//   W2[i][j] = sum_b a1[b][i] d2[b][j]    b2[j] = sum_b d2[b][j]
//   W3[j][v] = sum_b a2[b][j] d3[b][v]    b3[v] = sum_b d3[b][v]
__global__ __launch_bounds__(256) void mlp_wgrad_kernel(const float* __restrict__ sx, const float* __restrict__ sa1,
                                                        const float* __restrict__ sa2, const float* __restrict__ sd1,
                                                        const float* __restrict__ sd2, const float* __restrict__ sd3,
                                                        int64_t n, float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kP) return;
    const float* a = nullptr;  // left factor, a[b * lda + ia] (NULL for a bias)
    const float* d = nullptr;  // right factor, d[b * ldd + jd]
    int lda = 0, ia = 0, ldd = 0, jd = 0;
    if (p < SPMM_MLP_OFF_B1) {
        a = sx, lda = kIn, ia = p / kH, d = sd1, ldd = kH, jd = p % kH;
    } else if (p < SPMM_MLP_OFF_W2) {
        d = sd1, ldd = kH, jd = p - SPMM_MLP_OFF_B1;
    } else if (p < SPMM_MLP_OFF_B2) {
        const int q = p - SPMM_MLP_OFF_W2;
        a = sa1, lda = kH, ia = q / kH, d = sd2, ldd = kH, jd = q % kH;
    } else if (p < SPMM_MLP_OFF_W3) {
        d = sd2, ldd = kH, jd = p - SPMM_MLP_OFF_B2;
    } else if (p < SPMM_MLP_OFF_B3) {
        const int q = p - SPMM_MLP_OFF_W3;
        a = sa2, lda = kH, ia = q / kV, d = sd3, ldd = kV, jd = q % kV;
    } else {
        d = sd3, ldd = kV, jd = p - SPMM_MLP_OFF_B3;
    }
    double s = 0.0;
    if (a) {
        for (int64_t b = 0; b < n; ++b) s += (double)a[b * lda + ia] * (double)d[b * ldd + jd];
    } else {
        for (int64_t b = 0; b < n; ++b) s += (double)d[b * ldd + jd];
    }
    grad[p] = (float)s;
}

// loss = sum_b sloss[b] / max(1, M), one block, fixed tree.
__global__ __launch_bounds__(256) void loss_reduce_kernel(const double* __restrict__ sloss, int64_t n,
                                                          const uint32_t* __restrict__ count,
                                                          double* __restrict__ loss) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += sloss[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] / (double)(count[0] > 0 ? count[0] : 1u);
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, float* __restrict__ m,
                                                   float* __restrict__ v, const float* __restrict__ g, int np,
                                                   float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

}  // namespace

hipError_t launch_mlp_predict(const float* params, const float* feat, int64_t n, float* out, uint8_t* choice,
                              hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(mlp_predict_kernel, dim3((unsigned)((n + kRowsPerBlock - 1) / kRowsPerBlock)),
                           dim3(kRowsPerBlock), 0, s, params, feat, n, out, choice);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* params, const float* feat, const float* target, const uint8_t* mask,
                           const int32_t* idx, int64_t n, const MlpScratch& w, float* grad, double* loss,
                           hipStream_t s) {
    hipLaunchKernelGGL(mask_count_kernel, dim3(1), dim3(256), 0, s, mask, idx, n, w.count);
    if (n > 0)
        hipLaunchKernelGGL(mlp_backprop_kernel, dim3((unsigned)((n + kRowsPerBlock - 1) / kRowsPerBlock)),
                           dim3(kRowsPerBlock), 0, s, params, feat, target, mask, idx, n, w.count, w.x, w.a1,
                           w.a2, w.d1, w.d2, w.d3, w.loss_rows);
    hipLaunchKernelGGL(mlp_wgrad_kernel, dim3((kP + 255) / 256), dim3(256), 0, s, w.x, w.a1, w.a2, w.d1, w.d2,
                       w.d3, n, grad);
    if (loss) hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(256), 0, s, w.loss_rows, n, w.count, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, float* m, float* v, const float* g, int np, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3((np + 255) / 256), dim3(256), 0, s, p, m, v, g, np, lr, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

}  // namespace spmm
