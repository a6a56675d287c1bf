// X quantisation kernels: FP32 -> BF16, FP32 -> OCP FP8 E4M3 with a
// per-column scale s_j = 448 / max_i |X[i][j]|.
//
// Column absmax: |x| >= 0, so comparing FP32 bit patterns as unsigned
// integers orders the values; the reduction uses integer atomicMax, which is
// exact and order-independent (deterministic).  NaN inputs are not expected
// (X is finite); an infinity gives s_j = 0 and saturated codes.
#include <hip/hip_runtime.h>

#include "spmm_internal.h"

namespace spmm {
namespace {

__global__ void colmax_init(uint32_t* m, int k) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < k) m[j] = 0u;
}

// Every thread keeps the running max of one column (the grid stride is a
// multiple of k), then the block merges per column in LDS and issues one
// global atomicMax per column.
__global__ __launch_bounds__(256) void colmax_kernel(const float* __restrict__ X, int64_t n, int k,
                                                     int64_t ldx, uint32_t* __restrict__ m) {
    __shared__ uint32_t red[64];
    const int per_block = (256 / k) * k;
    if (threadIdx.x < 64) red[threadIdx.x] = 0u;
    __syncthreads();
    uint32_t best = 0u;
    if ((int)threadIdx.x < per_block) {
        const int j = threadIdx.x % k;
        const int64_t rows_per_step = (int64_t)gridDim.x * (per_block / k);
        for (int64_t i = (int64_t)blockIdx.x * (per_block / k) + threadIdx.x / k; i < n; i += rows_per_step) {
            const uint32_t b = __float_as_uint(X[i * ldx + j]) & 0x7FFFFFFFu;
            best = b > best ? b : best;
        }
        atomicMax(&red[j], best);
    }
    __syncthreads();
    if ((int)threadIdx.x < k) atomicMax(&m[threadIdx.x], red[threadIdx.x]);
}

// s_j = 448 / absmax_j (IEEE FP32 division), or 1 for an all-zero column.
__global__ void colscale_finalize(uint32_t* m, int k) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < k) {
        const float a = __uint_as_float(m[j]);
        reinterpret_cast<float*>(m)[j] = a > 0.0f ? __fdiv_rn(448.0f, a) : 1.0f;
    }
}

// Nearest BF16 (ties to even); NaN stays a quiet NaN with its sign.
__device__ __forceinline__ uint16_t to_bf16(float x) {
    const uint32_t b = __float_as_uint(x);
    if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu)) return (uint16_t)((b >> 16) | 0x0040u);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

// Nearest OCP E4M3 (ties to even), saturating to +-448; NaN -> S.1111.111.
__device__ __forceinline__ uint8_t to_e4m3(float x) {
    const uint32_t b = __float_as_uint(x);
    const uint32_t sign = (b >> 24) & 0x80u;
    const uint32_t mag = b & 0x7FFFFFFFu;
    if (mag > 0x7F800000u) return (uint8_t)(sign | 0x7Fu);          // NaN
    if (mag >= 0x43E00000u) return (uint8_t)(sign | 0x7Eu);         // >= 448 (incl. inf)
    if (mag < 0x3C800000u) {                                        // < 2^-6: step 2^-9
        const float q = __builtin_rintf(__uint_as_float(mag) * 512.0f);  // exact scale, RNE
        return (uint8_t)(sign | (uint32_t)q);                       // q = 8 is the min normal
    }
    // normal: keep 3 fraction bits, round to nearest even on the dropped 20
    const uint32_t r = (mag + 0x7FFFFu + ((mag >> 20) & 1u)) >> 20;
    return (uint8_t)(sign | (r - ((127u - 7u) << 3)));
}

__global__ __launch_bounds__(256) void quant_bf16_kernel(const float* __restrict__ X, int64_t n, int k,
                                                         int64_t ldx, uint16_t* __restrict__ Q,
                                                         int64_t ldq) {
    const int64_t total = n * k;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / k;
        const int j = (int)(t - i * k);
        Q[i * ldq + j] = to_bf16(X[i * ldx + j]);
    }
}

__global__ __launch_bounds__(256) void quant_fp8_kernel(const float* __restrict__ X, int64_t n, int k,
                                                        int64_t ldx, const float* __restrict__ s,
                                                        uint8_t* __restrict__ Q, int64_t ldq) {
    const int64_t total = n * k;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / k;
        const int j = (int)(t - i * k);
        const float prod = __fmul_rn(X[i * ldx + j], s[j]);
        Q[i * ldq + j] = to_e4m3(prod);
    }
}

}  // namespace

hipError_t launch_quantize(const float* X, int64_t n, int k, int64_t ldx, int dtype, void* Xq,
                           int64_t ldq, float* col_scale, bool scales_given, hipStream_t s) {
    const int64_t total = n * (int64_t)k;
    const int blocks = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (total + 255) / 256));
    if (dtype == SPMM_X_BF16) {
        if (total)
            hipLaunchKernelGGL(quant_bf16_kernel, dim3(blocks), dim3(256), 0, s, X, n, k, ldx,
                               static_cast<uint16_t*>(Xq), ldq);
        return hipGetLastError();
    }
    uint32_t* m = reinterpret_cast<uint32_t*>(col_scale);
    if (!scales_given) {
        hipLaunchKernelGGL(colmax_init, dim3(1), dim3(64), 0, s, m, k);
        if (n)
            hipLaunchKernelGGL(colmax_kernel, dim3(std::min<int64_t>(2048, (n + 3) / 4)), dim3(256), 0, s,
                               X, n, k, ldx, m);
        hipLaunchKernelGGL(colscale_finalize, dim3(1), dim3(64), 0, s, m, k);
    }
    if (total)
        hipLaunchKernelGGL(quant_fp8_kernel, dim3(blocks), dim3(256), 0, s, X, n, k, ldx, col_scale,
                           static_cast<uint8_t*>(Xq), ldq);
    return hipGetLastError();
}

}  // namespace spmm
