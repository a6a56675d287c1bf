// Dense kernels of the block Krylov-Schur eigensolver.  The basis V is a
// tall, narrow FP32 matrix (n rows, at most a few hundred columns, row-major):
//   ts_tn   C = A^T B            (A n x p, p <= 512, B n x q, q <= 16, p q <= 1024;
//                                 C p x q FP64, row-major)
//   ts_nn   W = alpha W + beta A C   (C p x q FP64; W must not alias A)
//   fill_uniform  X[i][c] uniform in [-1/2, 1/2) from a counter-based hash.
// Products are exact in FP64 (two FP32 factors) and sums are FP64 in a fixed
// order, so every result is deterministic for a given n.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "spmm_internal.h"

namespace spmm {
namespace {

constexpr int kTsThreads = 256;
constexpr int kTsMaxBlocks = 2048;  // row ranges of C = A^T B, one partial each
constexpr int kTsMaxOut = 1024;     // p * q
constexpr int kTsMaxP = 512;        // columns of A in C = A^T B
constexpr int kTsMaxQ = 16;         // columns of B in C = A^T B
constexpr int kNnCols = 32;         // columns of A staged in LDS per step of W += A C

// Row ranges for C = A^T B: a function of n only, so results are
// reproducible for a given n.
int tn_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(kTsMaxBlocks, (n + 63) / 64)); }

// part[(a * q + c) * nblk + blk] = sum over block blk's rows i of A[i][a] B[i][c],
// for the columns a in [256 y, 256 y + pc) of blockIdx.y = y.  The block's
// threads form G = 256 / pc groups of pc lanes; lane a of group g reads
// A[i][a] for the rows i = r0 + g, r0 + g + G, ... (a group reads a row's
// slice of A contiguously) and B[i][0..q) (one address per group), keeping q
// FP64 sums; the groups are then added in order through LDS.
template <int Q>
__global__ __launch_bounds__(kTsThreads) void ts_tn_partial_kernel(const float* __restrict__ A, int64_t lda, int p,
                                                                   const float* __restrict__ B, int64_t ldb, int q,
                                                                   int64_t n, double* __restrict__ part) {
    // rows per batch: all loads of a batch are issued before the first FMA;
    // sums for c >= q repeat column q - 1 (a valid address, no branch) and
    // are never written out
    constexpr int U = Q <= 4 ? 8 : (Q <= 8 ? 4 : 2);
    __shared__ double red[kTsThreads * Q];
    const int nblk = gridDim.x;
    const int a0 = blockIdx.y * kTsThreads;
    const int pc = min(kTsThreads, p - a0);
    const int G = kTsThreads / pc;
    const int g = threadIdx.x / pc, a = threadIdx.x - g * pc;
    const int64_t per = (n + nblk - 1) / nblk;
    const int64_t r0 = std::min<int64_t>(n, (int64_t)blockIdx.x * per);
    const int64_t r1 = std::min<int64_t>(n, r0 + per);
    double acc[Q];
#pragma unroll
    for (int c = 0; c < Q; ++c) acc[c] = 0.0;
    if (g < G) {
        const float* ac = A + a0 + a;
        int64_t i = r0 + g;
        for (; i + (int64_t)(U - 1) * G < r1; i += (int64_t)U * G) {
            float x[U], y[U][Q];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t r = i + (int64_t)u * G;
                x[u] = ac[r * lda];
#pragma unroll
                for (int c = 0; c < Q; ++c) y[u][c] = B[r * ldb + (c < q ? c : q - 1)];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int c = 0; c < Q; ++c) acc[c] += (double)x[u] * (double)y[u][c];
        }
        for (; i < r1; i += G) {
            const double xv = (double)ac[i * lda];
#pragma unroll
            for (int c = 0; c < Q; ++c) acc[c] += xv * (double)B[i * ldb + (c < q ? c : q - 1)];
        }
    }
#pragma unroll
    for (int c = 0; c < Q; ++c) red[threadIdx.x * Q + c] = acc[c];
    __syncthreads();
    for (int o = threadIdx.x; o < pc * q; o += kTsThreads) {
        const int aa = o / q, c = o - (o / q) * q;
        double s = 0.0;
        for (int gg = 0; gg < G; ++gg) s += red[(gg * pc + aa) * Q + c];
        part[((size_t)(a0 + aa) * q + c) * nblk + blockIdx.x] = s;
    }
}

// C[o] = sum over blk of part[o * nblk + blk]: one block per output, a
// strided sum per thread and a fixed-shape tree, so the order never varies.
__global__ __launch_bounds__(kTsThreads) void ts_tn_final_kernel(const double* __restrict__ part, int nblk,
                                                                 double* __restrict__ C) {
    __shared__ double red[kTsThreads];
    const int o = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kTsThreads) s += part[(size_t)o * nblk + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kTsThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) C[o] = red[0];
}

// W[i][c0 + c] = alpha W[i][c0 + c] + beta sum_a A[i][a] C[a][c0 + c] for the
// output columns [c0, c0 + QC) of blockIdx.y: one thread per row (256 rows
// per block).  A is staged through LDS 32 columns at a time with coalesced
// loads (row stride 33 floats: the per-thread row reads hit distinct banks),
// with the matching 32 rows of C (every thread reads the same entry: an LDS
// broadcast).
template <int QC>
__global__ __launch_bounds__(kTsThreads) void ts_nn_kernel(const float* __restrict__ A, int64_t lda, int p,
                                                           const double* __restrict__ C, int q, double alpha,
                                                           double beta, float* __restrict__ W, int64_t ldw,
                                                           int64_t n) {
    __shared__ float sa[kTsThreads * (kNnCols + 1)];
    __shared__ double sc[kNnCols * QC];
    const int64_t row0 = (int64_t)blockIdx.x * kTsThreads;
    const int c0 = blockIdx.y * QC;
    const int qc = min(QC, q - c0);
    double acc[QC];
#pragma unroll
    for (int c = 0; c < QC; ++c) acc[c] = 0.0;
    for (int a0 = 0; a0 < p; a0 += kNnCols) {
        const int pw = min(kNnCols, p - a0);
        // thread t loads column t % 32 of rows t / 32 + 8 j: all 32 loads in flight together
        constexpr int kRowsPerPass = kTsThreads / kNnCols;
        const int cc = threadIdx.x % kNnCols;
        float v[kNnCols];
#pragma unroll
        for (int j = 0; j < kNnCols; ++j) {
            const int64_t i = row0 + threadIdx.x / kNnCols + j * kRowsPerPass;
            v[j] = (cc < pw && i < n) ? A[i * lda + a0 + cc] : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < kNnCols; ++j) sa[(threadIdx.x / kNnCols + j * kRowsPerPass) * (kNnCols + 1) + cc] = v[j];
        // this slice of C (rows a0 .. a0 + pw), zero past q and past pw
        for (int e = threadIdx.x; e < kNnCols * QC; e += kTsThreads) {
            const int r = e / QC, c = e - (e / QC) * QC;
            sc[e] = (r < pw && c < qc) ? C[(size_t)(a0 + r) * q + c0 + c] : 0.0;
        }
        __syncthreads();
        for (int a = 0; a < pw; ++a) {
            const double x = (double)sa[threadIdx.x * (kNnCols + 1) + a];
#pragma unroll
            for (int c = 0; c < QC; ++c) acc[c] += x * sc[a * QC + c];
        }
        __syncthreads();
    }
    const int64_t i = row0 + threadIdx.x;
    if (i < n) {
        float* w = W + i * ldw + c0;
#pragma unroll
        for (int c = 0; c < QC; ++c)
            if (c < qc) w[c] = (float)((alpha != 0.0 ? alpha * (double)w[c] : 0.0) + beta * acc[c]);
    }
}

// SplitMix64 (Steele, Lea and Flood, 2014) of a counter: the value for
// element (i, c) depends only on seed, i and c.
__device__ inline uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(kTsThreads) void fill_uniform_kernel(float* __restrict__ X, int64_t ldx, int q,
                                                                  int64_t n, uint64_t seed) {
    const int64_t total = n * q;
    for (int64_t t = (int64_t)blockIdx.x * kTsThreads + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * kTsThreads) {
        const int64_t i = t / q;
        const int c = (int)(t - i * q);
        const uint64_t r = splitmix64(seed ^ splitmix64((uint64_t)i * 64u + (uint64_t)c));
        X[i * ldx + c] = (float)(r >> 40) * (1.0f / 16777216.0f) - 0.5f;
    }
}

unsigned grid_for(int64_t total) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(16384, (total + kTsThreads - 1) / kTsThreads));
}

}  // namespace

int ts_max_outputs() { return kTsMaxOut; }
int ts_max_width() { return kTsMaxP; }
size_t ts_partial_doubles() { return (size_t)kTsMaxBlocks * kTsMaxOut; }

hipError_t launch_ts_tn(const float* A, int64_t lda, int p, const float* B, int64_t ldb, int q, int64_t n,
                        double* part, double* C, hipStream_t s) {
    if (p < 1 || q < 1 || p > kTsMaxP || q > kTsMaxQ || p * q > kTsMaxOut || n < 0) return hipErrorInvalidValue;
    const int nblk = tn_blocks(n);
    const dim3 grid(nblk, (p + kTsThreads - 1) / kTsThreads);
    if (q == 1)
        hipLaunchKernelGGL(ts_tn_partial_kernel<1>, grid, dim3(kTsThreads), 0, s, A, lda, p, B, ldb, q, n, part);
    else if (q == 2)
        hipLaunchKernelGGL(ts_tn_partial_kernel<2>, grid, dim3(kTsThreads), 0, s, A, lda, p, B, ldb, q, n, part);
    else if (q <= 4)
        hipLaunchKernelGGL(ts_tn_partial_kernel<4>, grid, dim3(kTsThreads), 0, s, A, lda, p, B, ldb, q, n, part);
    else if (q <= 8)
        hipLaunchKernelGGL(ts_tn_partial_kernel<8>, grid, dim3(kTsThreads), 0, s, A, lda, p, B, ldb, q, n, part);
    else
        hipLaunchKernelGGL(ts_tn_partial_kernel<16>, grid, dim3(kTsThreads), 0, s, A, lda, p, B, ldb, q, n, part);
    hipLaunchKernelGGL(ts_tn_final_kernel, dim3(p * q), dim3(kTsThreads), 0, s, part, nblk, C);
    return hipGetLastError();
}

hipError_t launch_ts_nn(const float* A, int64_t lda, int p, const double* C, int q, double alpha, double beta,
                        float* W, int64_t ldw, int64_t n, hipStream_t s) {
    if (p < 1 || q < 1 || n < 0) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    const unsigned gx = (unsigned)((n + kTsThreads - 1) / kTsThreads);
    if (q == 1)
        hipLaunchKernelGGL(ts_nn_kernel<1>, dim3(gx, 1), dim3(kTsThreads), 0, s, A, lda, p, C, q, alpha, beta, W, ldw, n);
    else if (q == 2)
        hipLaunchKernelGGL(ts_nn_kernel<2>, dim3(gx, 1), dim3(kTsThreads), 0, s, A, lda, p, C, q, alpha, beta, W, ldw, n);
    else if (q <= 4)
        hipLaunchKernelGGL(ts_nn_kernel<4>, dim3(gx, 1), dim3(kTsThreads), 0, s, A, lda, p, C, q, alpha, beta, W, ldw, n);
    else if (q <= 8)
        hipLaunchKernelGGL(ts_nn_kernel<8>, dim3(gx, 1), dim3(kTsThreads), 0, s, A, lda, p, C, q, alpha, beta, W, ldw, n);
    else if (q <= 16)
        hipLaunchKernelGGL(ts_nn_kernel<16>, dim3(gx, 1), dim3(kTsThreads), 0, s, A, lda, p, C, q, alpha, beta, W, ldw, n);
    else
        hipLaunchKernelGGL(ts_nn_kernel<32>, dim3(gx, (q + 31) / 32), dim3(kTsThreads), 0, s, A, lda, p, C, q, alpha,
                           beta, W, ldw, n);
    return hipGetLastError();
}

hipError_t launch_fill_uniform(float* X, int64_t ldx, int q, int64_t n, uint64_t seed, hipStream_t s) {
    if (q < 1 || q > 64 || n < 0) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_uniform_kernel, dim3(grid_for(n * q)), dim3(kTsThreads), 0, s, X, ldx, q, n, seed);
    return hipGetLastError();
}

}  // namespace spmm
