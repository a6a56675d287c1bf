// Kernels of the applications built on the SpMM (Section 4): PageRank
// (Section 4.1) and NMF by multiplicative updates (Section 4.3).
//
// Reductions (dangling mass, L1 residual, Gram matrices) are deterministic:
// a fixed grid, each thread summing its grid-stride elements in order, a
// fixed-shape tree inside the block, and one block adding the per-block
// partials in block order.  PageRank reductions are FP64; Gram matrices are
// accumulated in FP64 and rounded to FP32 once.
#include <hip/hip_runtime.h>

#include "spmm_internal.h"

namespace spmm {
namespace {

constexpr int kRedThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kRedThreads) void pr_init_kernel(float* pr, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        pr[i] = v;
}

// x'[i] = PR(v) / L(v) for v = old_of_new[i] (0 where L(v) = 0), written in
// the handle's column order; the block partials of the dangling mass
// sum_{L(v)=0} PR(v) go to dpart[blockIdx.x].
__global__ __launch_bounds__(kRedThreads) void pr_prepare_kernel(const float* __restrict__ pr,
                                                               const uint32_t* __restrict__ outdeg,
                                                               const int32_t* __restrict__ old_of_new,
                                                               int64_t n, float* __restrict__ xp,
                                                               double* __restrict__ dpart) {
    __shared__ double red[kRedThreads];
    double dang = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = old_of_new ? old_of_new[i] : i;
        const float p = pr[v];
        const uint32_t L = outdeg[v];
        xp[i] = L ? p / (float)L : 0.0f;
        if (!L) dang += (double)p;
    }
    const double s = block_sum(dang, red);
    if (threadIdx.x == 0) dpart[blockIdx.x] = s;
}

// out[0] = sum of part[0..np) in a fixed order (one block).
__global__ __launch_bounds__(1024) void reduce_partials_kernel(const double* __restrict__ part, int np,
                                                               double* __restrict__ out) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// PR'(u) = (1-d)/N + d (y(u) + D/N), evaluated in FP64 and stored as FP32;
// block partials of sum |PR'(u) - PR(u)| go to rpart.
__global__ __launch_bounds__(kRedThreads) void pr_update_kernel(float* __restrict__ pr,
                                                              const float* __restrict__ y, int64_t n,
                                                              double damping, const double* __restrict__ D,
                                                              int redistribute, double* __restrict__ rpart) {
    __shared__ double red[kRedThreads];
    const double invN = 1.0 / (double)n;
    const double base = (1.0 - damping) * invN + (redistribute ? damping * D[0] * invN : 0.0);
    double r = 0.0;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const double nv = base + damping * (double)y[u];
        const float nf = (float)nv;
        r += fabs((double)nf - (double)pr[u]);
        pr[u] = nf;
    }
    const double s = block_sum(r, red);
    if (threadIdx.x == 0) rpart[blockIdx.x] = s;
}

// Per-block partial Gram matrices part[b][a * r + c] = sum_i M[i][a] M[i][c]
// over the block's rows, in FP64.
__global__ __launch_bounds__(kRedThreads) void gram_partial_kernel(const float* __restrict__ M, int64_t n,
                                                                 int r, double* __restrict__ part) {
    extern __shared__ float rows[];  // 64 rows x r
    const int rr = r * r;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};  // pairs threadIdx.x + 256 q, r <= 32
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * per, i1 = i0 + per < n ? i0 + per : n;
    for (int64_t b = i0; b < i1; b += 64) {
        const int nb = (int)(i1 - b < 64 ? i1 - b : 64);
        for (int t = threadIdx.x; t < nb * r; t += blockDim.x) rows[t] = M[b * r + t];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int p = threadIdx.x + 256 * q;
            if (p < rr) {
                const int a = p / r, c = p % r;
                double s = acc[q];
                for (int i = 0; i < nb; ++i) s += (double)rows[i * r + a] * (double)rows[i * r + c];
                acc[q] = s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int p = threadIdx.x + 256 * q;
        if (p < rr) part[(size_t)blockIdx.x * rr + p] = acc[q];
    }
}

// G[p] = FP32(sum_b part[b][p]) in block order.
__global__ __launch_bounds__(1024) void gram_final_kernel(const double* __restrict__ part, int nb, int r,
                                                          float* __restrict__ G) {
    const int rr = r * r;
    for (int p = threadIdx.x; p < rr; p += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[(size_t)b * rr + p];
        G[p] = (float)s;
    }
}

// Multiplicative update of one factor, row by row:
//   M[i][j] <- M[i][j] * S[i][j] / (sum_l M[i][l] G[l][j] + eps)
// (S = A^T W with G = W^T W for H; S = A H with G = H^T H for W).
__global__ __launch_bounds__(kRedThreads) void mu_update_kernel(float* __restrict__ M, const float* __restrict__ S,
                                                              const float* __restrict__ G, int64_t n, int r,
                                                              float eps) {
    __shared__ float g[32 * 32];
    for (int t = threadIdx.x; t < r * r; t += blockDim.x) g[t] = G[t];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float m[32];
#pragma unroll
        for (int l = 0; l < 32; ++l) m[l] = l < r ? M[i * r + l] : 0.0f;
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            if (j < r) {
                float den = 0.0f;
#pragma unroll
                for (int l = 0; l < 32; ++l)
                    if (l < r) den = fmaf(m[l], g[l * r + j], den);
                M[i * r + j] = m[j] * S[i * r + j] / (den + eps);
            }
        }
    }
}

}  // namespace

constexpr int kRedBlocks = 1024;

hipError_t launch_pr_init(float* pr, int64_t n, float v, hipStream_t s) {
    hipLaunchKernelGGL(pr_init_kernel, dim3(1024), dim3(kRedThreads), 0, s, pr, n, v);
    return hipGetLastError();
}

hipError_t launch_pr_prepare(const float* pr, const uint32_t* outdeg, const int32_t* old_of_new, int64_t n,
                             float* xp, double* dpart, double* D, hipStream_t s) {
    hipLaunchKernelGGL(pr_prepare_kernel, dim3(kRedBlocks), dim3(kRedThreads), 0, s, pr, outdeg, old_of_new,
                       n, xp, dpart);
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(1024), 0, s, dpart, kRedBlocks, D);
    return hipGetLastError();
}

hipError_t launch_pr_update(float* pr, const float* y, int64_t n, double damping, const double* D,
                            int redistribute, double* rpart, double* resid_slot, hipStream_t s) {
    hipLaunchKernelGGL(pr_update_kernel, dim3(kRedBlocks), dim3(kRedThreads), 0, s, pr, y, n, damping, D,
                       redistribute, rpart);
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(1024), 0, s, rpart, kRedBlocks, resid_slot);
    return hipGetLastError();
}

int gram_blocks() { return kRedBlocks; }

hipError_t launch_gram(const float* M, int64_t n, int r, double* part, float* G, hipStream_t s) {
    hipLaunchKernelGGL(gram_partial_kernel, dim3(kRedBlocks), dim3(kRedThreads), 64 * r * sizeof(float), s, M, n,
                       r, part);
    hipLaunchKernelGGL(gram_final_kernel, dim3(1), dim3(1024), 0, s, part, kRedBlocks, r, G);
    return hipGetLastError();
}

hipError_t launch_mu_update(float* M, const float* S, const float* G, int64_t n, int r, float eps, hipStream_t s) {
    const unsigned blocks = (unsigned)std::min<int64_t>(8192, (n + kRedThreads - 1) / kRedThreads + 1);
    hipLaunchKernelGGL(mu_update_kernel, dim3(blocks), dim3(kRedThreads), 0, s, M, S, G, n, r, eps);
    return hipGetLastError();
}

}  // namespace spmm
