// Untiled CSR SpMM kernels for gfx950 (the V-csr baseline of the format
// comparison): rows in order of descending degree, columns in the handle's
// column order, FP32 sums in registers.
//
// Three row classes, by length (rows are sorted, so each class is a
// contiguous range of the row order):
//   group rows  (length <= kCsrWaveMin): G = KC / VW lanes per row, each lane
//               sums VW columns of its row in order; P = 64 / G rows per
//               wavefront have similar lengths, so the lanes stay in step;
//   wave rows   (length <= kCsrPiece): one wavefront per row, P lane groups
//               stride over it, a shuffle butterfly sums the groups;
//   split rows  (longer): pieces of kCsrPiece entries, one wavefront each,
//               write partial sums; a combine kernel adds a row's pieces in
//               piece order.
// Every Y row is written once (rows without entries get zeros); the order
// of every sum is fixed, so results are deterministic.
#include <hip/hip_runtime.h>

#include "spmm_internal.h"

namespace spmm {
namespace {

template <int VW>
struct XV;
template <>
struct XV<1> {
    static __device__ __forceinline__ void ld(const float* p, float* v) { v[0] = *p; }
};
template <>
struct XV<2> {
    static __device__ __forceinline__ void ld(const float* p, float* v) {
        const float2 t = *reinterpret_cast<const float2*>(p);
        v[0] = t.x;
        v[1] = t.y;
    }
};
template <>
struct XV<4> {
    static __device__ __forceinline__ void ld(const float* p, float* v) {
        const float4 t = *reinterpret_cast<const float4*>(p);
        v[0] = t.x;
        v[1] = t.y;
        v[2] = t.z;
        v[3] = t.w;
    }
};

// Rows [r0, r1) of the row order, G lanes per row.
template <int KC, int VW, int U>
__global__ __launch_bounds__(256) void csr_group_rows(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                     const float* __restrict__ X, int64_t ldx, float* __restrict__ Y,
                                                     int64_t ldy, const int32_t* __restrict__ rmap, int64_t r0,
                                                     int64_t r1) {
    constexpr int G = KC / VW;
    const int64_t r = r0 + ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int g = threadIdx.x % G;
    if (r >= r1) return;
    const int64_t b = rp[r], e = rp[r + 1];
    float s[VW];
#pragma unroll
    for (int i = 0; i < VW; ++i) s[i] = 0.0f;
    for (int64_t p = b; p < e; p += U) {
        int32_t c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = ci[min(p + u, e - 1)];
        float x[U][VW];
#pragma unroll
        for (int u = 0; u < U; ++u) XV<VW>::ld(X + (int64_t)c[u] * ldx + g * VW, x[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (p + u < e) {
#pragma unroll
                for (int i = 0; i < VW; ++i) s[i] += x[u][i];
            }
        }
    }
    float* y = Y + (int64_t)rmap[r] * ldy + g * VW;
#pragma unroll
    for (int i = 0; i < VW; ++i) y[i] = s[i];
}

// One wavefront per segment {row, first entry, end entry, partial slot};
// slot < 0 writes the Y row, else the partial slot.
template <int KC, int VW, int U>
__global__ __launch_bounds__(256) void csr_wave_segs(const int64_t* __restrict__ seg, int64_t nseg,
                                                    const int32_t* __restrict__ ci, const float* __restrict__ X,
                                                    int64_t ldx, float* __restrict__ Y, int64_t ldy,
                                                    const int32_t* __restrict__ rmap, float* __restrict__ part) {
    constexpr int G = KC / VW, P = 64 / G;
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (w >= nseg) return;
    const int lane = threadIdx.x & 63, g = lane % G, slot = lane / G;
    const int64_t r = seg[4 * w], b = seg[4 * w + 1], e = seg[4 * w + 2], pt = seg[4 * w + 3];
    float s[VW];
#pragma unroll
    for (int i = 0; i < VW; ++i) s[i] = 0.0f;
    for (int64_t p = b + slot; p < e; p += (int64_t)P * U) {
        int32_t c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = ci[min(p + (int64_t)u * P, e - 1)];
        float x[U][VW];
#pragma unroll
        for (int u = 0; u < U; ++u) XV<VW>::ld(X + (int64_t)c[u] * ldx + g * VW, x[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (p + (int64_t)u * P < e) {
#pragma unroll
                for (int i = 0; i < VW; ++i) s[i] += x[u][i];
            }
        }
    }
#pragma unroll
    for (int m = G; m < 64; m <<= 1)
#pragma unroll
        for (int i = 0; i < VW; ++i) s[i] += __shfl_xor(s[i], m);
    if (slot == 0) {
        float* y = pt < 0 ? Y + (int64_t)rmap[r] * ldy + g * VW : part + pt * KC + g * VW;
#pragma unroll
        for (int i = 0; i < VW; ++i) y[i] = s[i];
    }
}

// Split row j (row srow[j]): the sum of its partial slots pb[j] .. pb[j+1]-1
// in slot order.  One block per split row, one thread per column.
__global__ void csr_combine(const int64_t* __restrict__ srow, const int64_t* __restrict__ pb, int64_t ns,
                            const float* __restrict__ part, int kc, float* __restrict__ Y, int64_t ldy,
                            const int32_t* __restrict__ rmap) {
    const int64_t j = blockIdx.x;
    const int c = threadIdx.x;
    if (j >= ns || c >= kc) return;
    float s = 0.0f;
    for (int64_t q = pb[j]; q < pb[j + 1]; ++q) s += part[q * kc + c];
    Y[(int64_t)rmap[srow[j]] * ldy + c] = s;
}

template <int KC, int VW>
hipError_t launch_chunk(const Handle& H, const float* X, int64_t ldx, float* Y, int64_t ldy, hipStream_t st) {
    constexpr int G = KC / VW;
    constexpr int U = KC <= 2 ? 8 : KC <= 8 ? 4 : 8;
    const CsrStore& C = H.csr;
    if (C.n_seg)
        hipLaunchKernelGGL((csr_wave_segs<KC, VW, U>), dim3((unsigned)((C.n_seg + 3) / 4)), dim3(256), 0, st, C.d_seg,
                           C.n_seg, C.d_col, X, ldx, Y, ldy, H.d_row_old, C.d_part);
    const int64_t rows = H.n_rows - C.n_wave_rows;
    if (rows > 0) {
        const int64_t threads = rows * G;
        hipLaunchKernelGGL((csr_group_rows<KC, VW, U>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st,
                           C.d_rp, C.d_col, X, ldx, Y, ldy, H.d_row_old, C.n_wave_rows, H.n_rows);
    }
    if (C.n_split)
        hipLaunchKernelGGL(csr_combine, dim3((unsigned)C.n_split), dim3(64), 0, st, C.d_srow, C.d_pb, C.n_split,
                           C.d_part, KC, Y, ldy, H.d_row_old);
    return hipGetLastError();
}

template <int KC>
hipError_t launch_vw(const Handle& H, const float* X, int64_t ldx, float* Y, int64_t ldy, hipStream_t st, int vw) {
    if constexpr (KC >= 4)
        if (vw == 4) return launch_chunk<KC, 4>(H, X, ldx, Y, ldy, st);
    if constexpr (KC >= 2)
        if (vw == 2) return launch_chunk<KC, 2>(H, X, ldx, Y, ldy, st);
    return launch_chunk<KC, 1>(H, X, ldx, Y, ldy, st);
}

}  // namespace

hipError_t launch_csr(const Handle& H, const float* X, int64_t ldx, int k, float* Y, int64_t ldy, hipStream_t st) {
    for (int c0 = 0; c0 < k;) {
        const int rem = k - c0;
        const int kc = rem >= 32 ? 32 : rem >= 16 ? 16 : rem >= 8 ? 8 : rem >= 4 ? 4 : rem >= 2 ? 2 : 1;
        int vw = kc >= 4 ? 4 : kc;
        while (vw > 1 && ((ldx % vw) != 0 || (c0 % vw) != 0 || (reinterpret_cast<uintptr_t>(X) % (vw * 4u)) != 0))
            vw >>= 1;
        const float* Xc = X + c0;
        float* Yc = Y + c0;
        hipError_t e;
        switch (kc) {
            case 32: e = launch_vw<32>(H, Xc, ldx, Yc, ldy, st, vw); break;
            case 16: e = launch_vw<16>(H, Xc, ldx, Yc, ldy, st, vw); break;
            case 8: e = launch_vw<8>(H, Xc, ldx, Yc, ldy, st, vw); break;
            case 4: e = launch_vw<4>(H, Xc, ldx, Yc, ldy, st, vw); break;
            case 2: e = launch_vw<2>(H, Xc, ldx, Yc, ldy, st, vw); break;
            default: e = launch_vw<1>(H, Xc, ldx, Yc, ldy, st, vw); break;
        }
        if (e != hipSuccess) return e;
        c0 += kc;
    }
    return hipSuccess;
}

}  // namespace spmm
