// SpMM kernels for gfx950 (CDNA4, wave64).
//
// Y = A X over the encoded tile store.  Each work item is processed by ONE
// wavefront that owns an LDS accumulator for the h rows of its tile row --
// the GPU counterpart of the per-thread output buffer of MulTRows in
// Algorithm 1, which merges every tile product of a tile row locally and
// writes each output row once.  A workgroup holds up to four independent
// wavefronts (four items); the wavefronts never synchronise with each
// other.
//
// Within an item the entries arrive in three streams, each with its own
// mapping onto the 64 lanes (G = KC / VW lanes cover the KC columns of one
// X row, VW columns per lane, so P = 64 / G entries are in flight per step):
//   COO  - one entry per lane group: gather X[col], add into acc[row].
//   LR   - one row segment per lane group: the lane walks its segment,
//          sums in registers, then adds once into acc[row].
//   WR   - one row segment per wavefront: the P lane groups stride over the
//          segment, then a butterfly of cross-lane shuffles sums them.
// Accumulator updates are LDS atomic adds (ds_add_f32): rows repeat across
// tiles and segments, and only one wavefront ever touches an accumulator.
//
// Tile rows with more non-zeros than one item holds are split; every piece
// writes its accumulator to a partial slot and the last piece to finish sums
// the slots of its tile row in slot order.  Y receives plain stores only.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "spmm_internal.h"

namespace spmm {
namespace {

// Wavefront-level barrier: LDS operations of one wavefront execute in
// order; the fences keep the compiler from moving them across this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- X loads
// Load VW consecutive X elements and widen them to FP32.
template <typename XT, int VW>
struct XLd;

template <int VW>
struct XLd<float, VW> {
    static __device__ __forceinline__ void load(const float* p, float* v) {
        if constexpr (VW == 4) {
            float4 t = *reinterpret_cast<const float4*>(p);
            v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
        } else if constexpr (VW == 2) {
            float2 t = *reinterpret_cast<const float2*>(p);
            v[0] = t.x; v[1] = t.y;
        } else {
            v[0] = *p;
        }
    }
};

// BF16: the upper 16 bits of an FP32 value.
template <int VW>
struct XLd<uint16_t, VW> {
    static __device__ __forceinline__ void load(const uint16_t* p, float* v) {
        if constexpr (VW == 4) {
            uint2 t = *reinterpret_cast<const uint2*>(p);
            v[0] = __uint_as_float(t.x << 16); v[1] = __uint_as_float(t.x & 0xFFFF0000u);
            v[2] = __uint_as_float(t.y << 16); v[3] = __uint_as_float(t.y & 0xFFFF0000u);
        } else if constexpr (VW == 2) {
            uint32_t t = *reinterpret_cast<const uint32_t*>(p);
            v[0] = __uint_as_float(t << 16); v[1] = __uint_as_float(t & 0xFFFF0000u);
        } else {
            v[0] = __uint_as_float((uint32_t)*p << 16);
        }
    }
};

// OCP FP8 E4M3.  Placing the code's sign, 4 exponent and 3 fraction bits in
// the matching fields of an FP16 value gives exactly value * 2^-8 (FP16 has
// exponent bias 15 = 7 + 8 and holds every E4M3 subnormal as a subnormal),
// so two codes decode with a few bit operations and FP16 -> FP32
// conversions.  The factor 2^8 is restored, exactly, at write-out.
__device__ __forceinline__ uint32_t e4m3_pair_to_f16x2(uint32_t w) {
    // bytes 0 and 2 of w -> FP16 halves 0 and 1
    return ((w & 0x00800080u) << 8) | ((w & 0x007F007Fu) << 7);
}
__device__ __forceinline__ float f16lo(uint32_t h) {
    return __half2float(__ushort_as_half((unsigned short)(h & 0xFFFFu)));
}
__device__ __forceinline__ float f16hi(uint32_t h) {
    return __half2float(__ushort_as_half((unsigned short)(h >> 16)));
}

template <int VW>
struct XLd<uint8_t, VW> {
    static __device__ __forceinline__ void load(const uint8_t* p, float* v) {
        if constexpr (VW == 4) {
            uint32_t w = *reinterpret_cast<const uint32_t*>(p);
            uint32_t a = e4m3_pair_to_f16x2(w), b = e4m3_pair_to_f16x2(w >> 8);
            v[0] = f16lo(a); v[1] = f16lo(b); v[2] = f16hi(a); v[3] = f16hi(b);
        } else if constexpr (VW == 2) {
            uint32_t w = *reinterpret_cast<const uint16_t*>(p);
            uint32_t a = e4m3_pair_to_f16x2(w), b = e4m3_pair_to_f16x2(w >> 8);
            v[0] = f16lo(a); v[1] = f16lo(b);
        } else {
            v[0] = f16lo(e4m3_pair_to_f16x2(*p));
        }
    }
};

template <typename XT>
struct OutScale {
    // FP8 accumulators hold (A X_q) * 2^-8; Y = that * 2^8 / s_j.
    static __device__ __forceinline__ float apply(float y, const float* s, uint32_t c) {
        if constexpr (sizeof(XT) == 1) return (y * 256.0f) / s[c];
        else return y;
    }
};

template <int KC, int VW, typename XT>
__global__ __launch_bounds__(256) void spmm_items(
    const ItemDesc* __restrict__ items, uint32_t n_items, const uint8_t* __restrict__ blob,
    uint64_t blob_bias, const XT* __restrict__ X, int64_t ldx, float* __restrict__ Y, int64_t ldy,
    float* __restrict__ part, const CombineDesc* __restrict__ combine,
    uint32_t* __restrict__ count, const float* __restrict__ yscale, uint32_t h, uint32_t wshift,
    int64_t n_rows, int has_val) {
    constexpr int G = KC / VW;
    constexpr int P = 64 / G;
    extern __shared__ float lds[];
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const uint32_t it = blockIdx.x * (blockDim.x >> 6) + wave;
    if (it >= n_items) return;
    float* acc = lds + (size_t)wave * h * KC;
    const ItemDesc d = items[it];
    const uint8_t* base = blob + (d.blob_off - blob_bias);

    for (uint32_t i = lane; i < h * KC; i += 64) acc[i] = 0.0f;
    wave_sync();

    const int g = lane % G;
    const uint32_t slot = lane / G;
    const int c0 = g * VW;

    // ---- COO stream: one entry per lane group
    {
        const uint32_t* ent = reinterpret_cast<const uint32_t*>(base);
        const float* cval = reinterpret_cast<const float*>(base + 4 * (size_t)d.n_coo);
        const uint2* ctile = reinterpret_cast<const uint2*>(base + d.o_coo_tile);
        uint32_t cur = 0;
        for (uint32_t pb = 0; pb < d.n_coo; pb += P) {
            const uint32_t e = pb + slot;
            const uint32_t pe = pb + P;
            uint32_t ord = cur;
            for (uint32_t t = cur + 1; t < d.n_coo_tiles; ++t) {
                const uint32_t st = ctile[t].y;
                if (st >= pe) break;
                if (e >= st) ord = t;
            }
            if (e < d.n_coo) {
                const uint32_t en = ent[e];
                const uint32_t J = ctile[ord].x;
                const XT* xp = X + (((int64_t)J << wshift) + (en & 0xFFFFu)) * ldx + c0;
                float x[VW];
                XLd<XT, VW>::load(xp, x);
                const float v = has_val ? cval[e] : 1.0f;
                float* a = acc + (en >> 16) * KC + c0;
#pragma unroll
                for (int i = 0; i < VW; ++i) atomicAdd(a + i, v * x[i]);
            }
            while (cur + 1 < d.n_coo_tiles && ctile[cur + 1].y <= pe) ++cur;
        }
    }

    const uint16_t* cols = reinterpret_cast<const uint16_t*>(base + d.o_cols);
    const float* colv = reinterpret_cast<const float*>(base + d.o_col_val);

    // ---- LR stream: one row segment per lane group
    {
        const uint32_t* ldesc = reinterpret_cast<const uint32_t*>(base + d.o_lr_desc);
        const uint32_t* lstart = reinterpret_cast<const uint32_t*>(base + d.o_lr_start);
        const uint32_t* lJ = reinterpret_cast<const uint32_t*>(base + d.o_lr_J);
        for (uint32_t pb = 0; pb < d.n_lr; pb += P) {
            const uint32_t si = pb + slot;
            if (si < d.n_lr) {
                const uint32_t ds = ldesc[si];
                const uint32_t J = lJ[ds >> 16];
                const uint32_t a = lstart[si], b = lstart[si + 1];
                const XT* xb = X + ((int64_t)J << wshift) * ldx + c0;
                float s[VW];
#pragma unroll
                for (int i = 0; i < VW; ++i) s[i] = 0.0f;
                for (uint32_t t = a; t < b; ++t) {
                    float x[VW];
                    XLd<XT, VW>::load(xb + (int64_t)cols[t] * ldx, x);
                    const float v = has_val ? colv[t] : 1.0f;
#pragma unroll
                    for (int i = 0; i < VW; ++i) s[i] += v * x[i];
                }
                float* ap = acc + (ds & 0xFFFFu) * KC + c0;
#pragma unroll
                for (int i = 0; i < VW; ++i) atomicAdd(ap + i, s[i]);
            }
        }
    }

    // ---- WR stream: one row segment per wavefront
    {
        const uint4* wr = reinterpret_cast<const uint4*>(base + d.o_wr);
        for (uint32_t q = 0; q < d.n_wr; ++q) {
            const uint4 sg = wr[q];  // {J, row, first col, length}
            const XT* xb = X + ((int64_t)sg.x << wshift) * ldx + c0;
            float s[VW];
#pragma unroll
            for (int i = 0; i < VW; ++i) s[i] = 0.0f;
            for (uint32_t t = slot; t < sg.w; t += P) {
                float x[VW];
                XLd<XT, VW>::load(xb + (int64_t)cols[sg.z + t] * ldx, x);
                const float v = has_val ? colv[sg.z + t] : 1.0f;
#pragma unroll
                for (int i = 0; i < VW; ++i) s[i] += v * x[i];
            }
#pragma unroll
            for (int m = G; m < 64; m <<= 1)
#pragma unroll
                for (int i = 0; i < VW; ++i) s[i] += __shfl_xor(s[i], m);
            if (slot == 0) {
                float* ap = acc + sg.y * KC + c0;
#pragma unroll
                for (int i = 0; i < VW; ++i) atomicAdd(ap + i, s[i]);
            }
        }
    }

    wave_sync();
    const int64_t row0 = (int64_t)d.slab * h;
    const int64_t left = n_rows - row0;
    const uint32_t rows = left < (int64_t)h ? (uint32_t)left : h;
    const uint32_t total = rows * KC;
    if (d.part < 0) {
        for (uint32_t i = lane; i < total; i += 64) {
            const uint32_t r = i / KC, c = i % KC;
            Y[(row0 + r) * ldy + c] = OutScale<XT>::apply(acc[i], yscale, c);
        }
        return;
    }
    // Split tile row: publish this item's partial sums; the last item of the
    // tile row to finish adds all partial slots in slot order (so the result
    // does not depend on which item finishes last), writes Y, and re-arms
    // the counter for the next launch.
    float* pp = part + (size_t)d.part * h * KC;
    for (uint32_t i = lane; i < total; i += 64) pp[i] = acc[i];
    __threadfence();
    uint32_t old = 0;
    if (lane == 0) old = atomicAdd(&count[d.cid], 1u);
    old = __shfl(old, 0);
    const CombineDesc cd = combine[d.cid];
    if (old != cd.part_end - cd.part_begin - 1) return;
    __threadfence();
    const float* p0 = part + (size_t)cd.part_begin * h * KC;
    const size_t stride = (size_t)h * KC;
    const uint32_t np = cd.part_end - cd.part_begin;
    for (uint32_t i = lane; i < total; i += 64) {
        float s = 0.0f;
        for (uint32_t q = 0; q < np; ++q) s += __builtin_nontemporal_load(p0 + q * stride + i);
        const uint32_t r = i / KC, c = i % KC;
        Y[(row0 + r) * ldy + c] = OutScale<XT>::apply(s, yscale, c);
    }
    if (lane == 0) atomicExch(&count[d.cid], 0u);
}

template <typename XT, int KC, int VW>
hipError_t launch_one(const Handle& H, const RunArgs& a, const XT* X, float* Y,
                      const float* yscale) {
    const uint32_t per_wave = H.h * KC * 4u;
    uint32_t wpb = 65536u / per_wave;
    wpb = wpb < 1 ? 1 : (wpb > 4 ? 4 : wpb);
    const uint32_t grid = (a.n_items + wpb - 1) / wpb;
    if (grid)
        hipLaunchKernelGGL((spmm_items<KC, VW, XT>), dim3(grid), dim3(64 * wpb),
                           (size_t)per_wave * wpb, a.stream, a.items, a.n_items, a.blob,
                           a.blob_bias, X, a.ldx, Y, a.ldy, H.d_part, a.combine, a.count, yscale,
                           H.h, H.wshift, (int64_t)H.n_rows, (int)H.has_val);
    return hipGetLastError();
}

template <typename XT, int KC>
hipError_t launch_vw(const Handle& H, const RunArgs& a, const XT* X, float* Y,
                     const float* yscale, int vw) {
    if constexpr (KC >= 4) {
        if (vw == 4) return launch_one<XT, KC, 4>(H, a, X, Y, yscale);
    }
    if constexpr (KC >= 2) {
        if (vw == 2) return launch_one<XT, KC, 2>(H, a, X, Y, yscale);
    }
    return launch_one<XT, KC, 1>(H, a, X, Y, yscale);
}

template <typename XT>
hipError_t launch_typed(const Handle& H, const RunArgs& a) {
    const XT* X = static_cast<const XT*>(a.X);
    const int cap = kc_cap(H);
    for (int c0 = 0; c0 < a.k;) {
        const int rem = a.k < c0 + cap ? a.k - c0 : cap;
        const int kc = rem >= 32 ? 32 : rem >= 16 ? 16 : rem >= 8 ? 8 : rem >= 4 ? 4 : rem >= 2 ? 2 : 1;
        int vw = kc >= 4 ? 4 : kc;
        while (vw > 1 && ((a.ldx % vw) != 0 || (c0 % vw) != 0 ||
                          (reinterpret_cast<uintptr_t>(X) % (vw * sizeof(XT))) != 0))
            vw >>= 1;
        const XT* Xc = X + c0;
        float* Yc = a.Y + c0;
        const float* sc = a.col_scale ? a.col_scale + c0 : nullptr;
        hipError_t e;
        switch (kc) {
            case 32: e = launch_vw<XT, 32>(H, a, Xc, Yc, sc, vw); break;
            case 16: e = launch_vw<XT, 16>(H, a, Xc, Yc, sc, vw); break;
            case 8: e = launch_vw<XT, 8>(H, a, Xc, Yc, sc, vw); break;
            case 4: e = launch_vw<XT, 4>(H, a, Xc, Yc, sc, vw); break;
            case 2: e = launch_vw<XT, 2>(H, a, Xc, Yc, sc, vw); break;
            default: e = launch_vw<XT, 1>(H, a, Xc, Yc, sc, vw); break;
        }
        if (e != hipSuccess) return e;
        c0 += kc;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_spmm(const Handle& H, const RunArgs& a) {
    switch (a.dtype) {
        case SPMM_X_BF16: return launch_typed<uint16_t>(H, a);
        case SPMM_X_FP8_E4M3: return launch_typed<uint8_t>(H, a);
        default: return launch_typed<float>(H, a);
    }
}

}  // namespace spmm
