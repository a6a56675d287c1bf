// Dense kernels of the block Krylov-Schur eigensolver.  The basis V is a
// tall, narrow FP32 matrix (n rows, at most a few hundred columns), row-major
// or stored as contiguous blocks of columns (a ColLayout gives the address
// of element (i, c)):
//   ts_tn   C = A^T B            (A n x p, p <= 512, B n x q row-major, q <= 16,
//                                 p q <= 2048; C p x q FP64, row-major)
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
constexpr int kTsWaves = kTsThreads / 64;
constexpr int kTsMaxBlocks = 2048;  // row ranges of C = A^T B, one partial each
constexpr int kTsMaxOut = 2048;     // p * q
constexpr int kTsMaxP = 512;        // columns of A in C = A^T B
constexpr int kTsMaxQ = 16;         // columns of B in C = A^T B
constexpr int kTnCols = 64;         // columns of A per blockIdx.y in C = A^T B
constexpr int kTnU = 8;             // rows per lane per batch in C = A^T B

// Row ranges for C = A^T B: a function of n only, so results are
// reproducible for a given n.
int tn_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(kTsMaxBlocks, (n + 63) / 64)); }

__device__ inline int pow2_at_least(int x) {
    int v = 1;
    while (v < x) v <<= 1;
    return v;
}

// part[(a * q + c) * nblk + blk] = sum over block blk's rows i of A[i][a] B[i][c]
// for the columns a in [64 y, 64 y + pc) of blockIdx.y = y.  Each wavefront
// owns batches of rows: its lanes form 64 / ncol row slots of ncol lanes
// (ncol = pc rounded up to a power of two), lane (slot, a) reads A[i][a] for
// U rows i of its slot, and the batch's rows of B are loaded once, coalesced,
// into the wavefront's own LDS region and read from there (one address per
// slot).  Loads use clamped, always-valid indices, so a batch's loads are all
// in flight before its first FMA; invalid rows and columns contribute 0.
// The lanes' FP64 sums are then added in a fixed order through LDS.
template <int Q>
__global__ __launch_bounds__(kTsThreads) void ts_tn_partial_kernel(const float* __restrict__ A, ColLayout LA, int p,
                                                                   const float* __restrict__ B, int64_t ldb, int q,
                                                                   int64_t n, double* __restrict__ part) {
    __shared__ double smem[kTsThreads * Q];   // B batches during the sweep, then the lanes' sums
    const int nblk = gridDim.x;
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
    float* sb = reinterpret_cast<float*>(smem) + wv * 64 * Q;   // this wavefront's B rows, 64 x Q floats
    const int a0 = blockIdx.y * kTnCols;
    const int pc = min(kTnCols, p - a0);
    const int ncol = pow2_at_least(pc);
    const int rs = 64 / ncol;                                     // row slots per wavefront
    const int U = min(kTnU, 64 / rs);                             // rows per slot per batch
    const int RB = rs * U;                                        // rows per batch (<= 64)
    const int slot = lane / ncol, col = lane - (lane / ncol) * ncol;
    const bool active = col < pc;
    const float* ac = A + col_off(LA, a0 + (active ? col : 0));
    const int64_t lda = LA.ld;
    const int64_t per = (n + nblk - 1) / nblk;
    const int64_t r0 = std::min<int64_t>(n, (int64_t)blockIdx.x * per);
    const int64_t r1 = std::min<int64_t>(n, r0 + per);
    double acc[Q];
#pragma unroll
    for (int c = 0; c < Q; ++c) acc[c] = 0.0;
    for (int64_t base = r0 + (int64_t)wv * RB; base < r1; base += (int64_t)kTsWaves * RB) {
        const int nr = (int)std::min<int64_t>(RB, r1 - base);
        float y[Q];   // B entries this lane stages: rows e / Q of the batch for e = lane + 64 j
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            const int e = lane + 64 * j;
            const int r = min(e / Q, nr - 1), c = min(e % Q, q - 1);
            y[j] = B[(base + r) * ldb + c];
        }
        float x[kTnU];
#pragma unroll
        for (int u = 0; u < kTnU; ++u) {
            const int r = min(slot + u * rs, nr - 1);
            x[u] = ac[(base + r) * lda];
        }
#pragma unroll
        for (int j = 0; j < Q; ++j) sb[lane + 64 * j] = y[j];
        // the wavefront's own LDS region: order its writes before its reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int u = 0; u < kTnU; ++u) {
            const int r = slot + u * rs;
            const double xv = (u < U && r < nr && active) ? (double)x[u] : 0.0;
            const float* br = sb + min(r, nr - 1) * Q;
#pragma unroll
            for (int c = 0; c < Q; ++c) acc[c] += xv * (double)br[c];
        }
        // all lanes have read this batch before the next one overwrites it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < Q; ++c) smem[threadIdx.x * Q + c] = acc[c];
    __syncthreads();
    for (int o = threadIdx.x; o < pc * q; o += kTsThreads) {
        const int aa = o / q, c = o - (o / q) * q;
        double s = 0.0;
        for (int w = 0; w < kTsWaves; ++w)
            for (int sl = 0; sl < rs; ++sl) s += smem[(w * 64 + sl * ncol + aa) * Q + c];
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

// W = alpha W + beta A C for q <= 16 output columns (QC >= q), W row-major
// with row stride ldw: one thread per row, 256 rows per block.  A is staged through LDS CW columns at a
// time with coalesced loads (row stride CW + 1 floats: the per-thread row
// reads hit distinct banks), with the matching CW rows of C (every thread
// reads the same entry: a broadcast).  The block's 256 x q results go back
// through LDS so that W is read and written with consecutive lanes on
// consecutive elements.
template <int QC, int CW>
__global__ __launch_bounds__(kTsThreads) void ts_nn_kernel(const float* __restrict__ A, ColLayout LA, int p,
                                                           const double* __restrict__ C, int q, double alpha,
                                                           double beta, float* __restrict__ W, int64_t ldw,
                                                           int64_t n) {
    constexpr int kA = (kTsThreads * (CW + 1) + 1) / 2;     // doubles holding the A tile (floats)
    constexpr int kOut = kTsThreads * QC;                    // doubles of the result tile
    __shared__ double sbuf[kA > kOut ? kA : kOut];
    __shared__ double sc[CW * QC];
    float* sa = reinterpret_cast<float*>(sbuf);
    const int64_t row0 = (int64_t)blockIdx.x * kTsThreads;
    const int rows = (int)std::min<int64_t>(kTsThreads, n - row0);
    double acc[QC];
#pragma unroll
    for (int c = 0; c < QC; ++c) acc[c] = 0.0;
    constexpr int kRowsPerPass = kTsThreads / CW;
    const int cc = threadIdx.x % CW;
    for (int a0 = 0; a0 < p; a0 += CW) {
        const int pw = min(CW, p - a0);
        // thread t loads column t % CW of rows t / CW + (256 / CW) j
        float v[CW];
        const float* ap = A + col_off(LA, a0 + min(cc, pw - 1));
#pragma unroll
        for (int j = 0; j < CW; ++j) {
            const int r = min(threadIdx.x / CW + j * kRowsPerPass, rows - 1);
            v[j] = ap[(row0 + r) * LA.ld];
        }
#pragma unroll
        for (int j = 0; j < CW; ++j) sa[(threadIdx.x / CW + j * kRowsPerPass) * (CW + 1) + cc] = cc < pw ? v[j] : 0.0f;
        for (int e = threadIdx.x; e < CW * QC; e += kTsThreads) {
            const int r = e / QC, c = e - (e / QC) * QC;
            sc[e] = (r < pw && c < q) ? C[(size_t)(a0 + r) * q + c] : 0.0;
        }
        __syncthreads();
        for (int a = 0; a < pw; ++a) {
            const double x = (double)sa[threadIdx.x * (CW + 1) + a];
#pragma unroll
            for (int c = 0; c < QC; ++c) acc[c] += x * sc[a * QC + c];
        }
        __syncthreads();
    }
    double* so = sbuf;
#pragma unroll
    for (int c = 0; c < QC; ++c) so[threadIdx.x * QC + c] = acc[c];
    __syncthreads();
    for (int e = threadIdx.x; e < rows * q; e += kTsThreads) {
        const int r = e / q, c = e - (e / q) * q;
        float* w = W + (row0 + r) * ldw + c;
        const double old = alpha != 0.0 ? alpha * (double)*w : 0.0;
        *w = (float)(old + beta * so[r * QC + c]);
    }
}

// W = alpha W + beta A C for wide C (the restart and the Ritz vectors): a
// 64-row x 64-column tile of W per block, 4 x 4 of it per thread, with
// 32-column slices of A and the matching 32 x 64 slice of C staged in LDS.
__global__ __launch_bounds__(kTsThreads) void ts_nn_wide_kernel(const float* __restrict__ A, ColLayout LA, int p,
                                                                const double* __restrict__ C, int q, double alpha,
                                                                double beta, float* __restrict__ W, ColLayout LW,
                                                                int64_t n) {
    constexpr int TR = 64, TC = 64, KA = 32;
    __shared__ float sa[TR * (KA + 1)];
    __shared__ double sc[KA * TC];
    const int64_t row0 = (int64_t)blockIdx.x * TR;
    const int c0 = blockIdx.y * TC;
    const int rows = (int)std::min<int64_t>(TR, n - row0);
    const int cols = min(TC, q - c0);
    const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;    // rows 4 ty .. +3, columns 4 tx .. +3
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int a0 = 0; a0 < p; a0 += KA) {
        const int pw = min(KA, p - a0);
        float v[TR * KA / kTsThreads];
#pragma unroll
        for (int j = 0; j < TR * KA / kTsThreads; ++j) {
            const int e = threadIdx.x + kTsThreads * j;
            const int r = min(e / KA, rows - 1), k = min(e % KA, pw - 1);
            v[j] = A[col_off(LA, a0 + k) + (row0 + r) * LA.ld];
        }
        double u[KA * TC / kTsThreads];
#pragma unroll
        for (int j = 0; j < KA * TC / kTsThreads; ++j) {
            const int e = threadIdx.x + kTsThreads * j;
            const int k = min(e / TC, pw - 1), c = min(e % TC, cols - 1);
            u[j] = C[(size_t)(a0 + k) * q + c0 + c];
        }
#pragma unroll
        for (int j = 0; j < TR * KA / kTsThreads; ++j) {
            const int e = threadIdx.x + kTsThreads * j;
            sa[(e / KA) * (KA + 1) + e % KA] = (e % KA) < pw ? v[j] : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < KA * TC / kTsThreads; ++j) sc[threadIdx.x + kTsThreads * j] = u[j];
        __syncthreads();
        for (int k = 0; k < pw; ++k) {
            double xa[4], cb[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) xa[i] = (double)sa[(4 * ty + i) * (KA + 1) + k];
#pragma unroll
            for (int j = 0; j < 4; ++j) cb[j] = sc[k * TC + 4 * tx + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += xa[i] * cb[j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = 4 * ty + i;
        if (r >= rows) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = 4 * tx + j;
            if (c >= cols) continue;
            float* w = W + col_off(LW, c0 + c) + (row0 + r) * LW.ld;
            const double old = alpha != 0.0 ? alpha * (double)*w : 0.0;
            *w = (float)(old + beta * acc[i][j]);
        }
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

hipError_t launch_ts_tn(const float* A, ColLayout LA, int p, const float* B, int64_t ldb, int q, int64_t n,
                        double* part, double* C, hipStream_t s) {
    if (p < 1 || q < 1 || p > kTsMaxP || q > kTsMaxQ || p * q > kTsMaxOut || n < 0 || LA.bw < 1)
        return hipErrorInvalidValue;
    const int nblk = tn_blocks(n);
    if (n == 0) {
        // no rows: C = 0 (one empty row range)
        hipLaunchKernelGGL(ts_tn_final_kernel, dim3(p * q), dim3(kTsThreads), 0, s, part, 0, C);
        return hipGetLastError();
    }
    const dim3 grid(nblk, (p + kTnCols - 1) / kTnCols);
    if (q == 1)
        hipLaunchKernelGGL(ts_tn_partial_kernel<1>, grid, dim3(kTsThreads), 0, s, A, LA, p, B, ldb, q, n, part);
    else if (q == 2)
        hipLaunchKernelGGL(ts_tn_partial_kernel<2>, grid, dim3(kTsThreads), 0, s, A, LA, p, B, ldb, q, n, part);
    else if (q <= 4)
        hipLaunchKernelGGL(ts_tn_partial_kernel<4>, grid, dim3(kTsThreads), 0, s, A, LA, p, B, ldb, q, n, part);
    else if (q <= 8)
        hipLaunchKernelGGL(ts_tn_partial_kernel<8>, grid, dim3(kTsThreads), 0, s, A, LA, p, B, ldb, q, n, part);
    else
        hipLaunchKernelGGL(ts_tn_partial_kernel<16>, grid, dim3(kTsThreads), 0, s, A, LA, p, B, ldb, q, n, part);
    hipLaunchKernelGGL(ts_tn_final_kernel, dim3(p * q), dim3(kTsThreads), 0, s, part, nblk, C);
    return hipGetLastError();
}

template <int QC>
static void launch_nn_q(const float* A, ColLayout LA, int p, const double* C, int q, double alpha, double beta,
                        float* W, int64_t ldw, int64_t n, hipStream_t s) {
    const dim3 grid((unsigned)((n + kTsThreads - 1) / kTsThreads));
    if (p <= 8)
        hipLaunchKernelGGL((ts_nn_kernel<QC, 8>), grid, dim3(kTsThreads), 0, s, A, LA, p, C, q, alpha, beta, W, ldw, n);
    else
        hipLaunchKernelGGL((ts_nn_kernel<QC, 32>), grid, dim3(kTsThreads), 0, s, A, LA, p, C, q, alpha, beta, W, ldw, n);
}

hipError_t launch_ts_nn(const float* A, ColLayout LA, int p, const double* C, int q, double alpha, double beta,
                        float* W, ColLayout LW, int64_t n, hipStream_t s) {
    if (p < 1 || q < 1 || n < 0 || LA.bw < 1 || LW.bw < 1) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    // the row-per-thread kernel writes W as one row-major block
    const bool one_block = q <= LW.bw;
    if (one_block && q == 1)
        launch_nn_q<1>(A, LA, p, C, q, alpha, beta, W, LW.ld, n, s);
    else if (one_block && q == 2)
        launch_nn_q<2>(A, LA, p, C, q, alpha, beta, W, LW.ld, n, s);
    else if (one_block && q <= 4)
        launch_nn_q<4>(A, LA, p, C, q, alpha, beta, W, LW.ld, n, s);
    else if (one_block && q <= 8)
        launch_nn_q<8>(A, LA, p, C, q, alpha, beta, W, LW.ld, n, s);
    else if (one_block && q <= 16)
        launch_nn_q<16>(A, LA, p, C, q, alpha, beta, W, LW.ld, n, s);
    else
        hipLaunchKernelGGL(ts_nn_wide_kernel, dim3((unsigned)((n + 63) / 64), (q + 63) / 64), dim3(kTsThreads), 0, s,
                           A, LA, p, C, q, alpha, beta, W, LW, n);
    return hipGetLastError();
}

hipError_t launch_fill_uniform(float* X, int64_t ldx, int q, int64_t n, uint64_t seed, hipStream_t s) {
    if (q < 1 || q > 64 || n < 0) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_uniform_kernel, dim3(grid_for(n * q)), dim3(kTsThreads), 0, s, X, ldx, q, n, seed);
    return hipGetLastError();
}

}  // namespace spmm
