// SpMM kernels for gfx950 (CDNA4, wave64).
//
// Y = A X over the encoded tile store.  Each work item is processed by ONE
// wavefront that owns an LDS accumulator for the h rows of its tile row --
// the GPU counterpart of the per-thread output buffer of MulTRows in
// Algorithm 1, which merges every tile product of a tile row locally and
// writes each output row once.  A workgroup holds up to four independent
// wavefronts (four items); the wavefronts never synchronise with each
// other.  On request (a build option), launches of at most 8 columns use a
// persistent form instead: one workgroup per CU stages the hottest rows of
// X in LDS once, and its wavefronts then loop over the items.
//
// Within an item the entries arrive in three streams, each with its own
// mapping onto the 64 lanes (G = KC / VW lanes cover the KC columns of one
// X row, VW columns per lane, so P = 64 / G entries are in flight per step):
//   COO  - one entry per lane group: gather X[col], add into acc[row].
//   LR   - one row segment per lane group: the lane walks its segment,
//          sums in registers, then adds once into acc[row].
//   WR   - one row segment per wavefront: the P lane groups stride over the
//          segment, then a butterfly of cross-lane shuffles sums them.
// Accumulators are 64-bit fixed point, updated with integer LDS atomics
// (ds_add_u64): float LDS atomics are an order of magnitude slower on this
// hardware, and integer sums are exact and independent of the order in which
// lanes, segments or split-row pieces arrive, so the result is
// deterministic.  Column j is scaled by 2^f_j, chosen per call from
// max |X[:, j]| and the largest row L1 norm of A so that no partial sum of a
// row can exceed 2^61; each FP32 product (or FP32 register partial sum of a
// row segment) is rounded once to the fixed-point grid.
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

// FP32 value -> signed 64-bit fixed point with 2^f = scale (round to
// nearest); two's complement wraps correctly under unsigned atomic adds.
__device__ __forceinline__ unsigned long long to_fixed(float v, double scale) {
    return (unsigned long long)__double2ll_rn((double)v * scale);
}
// A column of X holding a NaN or an infinity has no fixed-point scale: its
// exponent is this sentinel, its products are scaled by 0 (the sums are
// meaningless) and every Y entry written for it is NaN.
constexpr int32_t kNonFiniteCol = INT32_MIN;
__device__ __forceinline__ float from_fixed(unsigned long long q, int32_t f) {
    if (f == kNonFiniteCol) return __int_as_float(0x7FC00000);
    return (float)ldexp((double)(long long)q, -f);
}

// X[gc, c0 .. c0 + VW) as FP32: from the rows staged in LDS (ns rows of KC
// decoded values) when gc is one of them, else from memory.
template <typename XT, int KC, int VW, bool STAGED>
__device__ __forceinline__ void xget(const XT* __restrict__ X, int64_t ldx, int c0, int64_t gc,
                                     const float* xs, uint32_t ns, float* v) {
    if constexpr (STAGED) {
        if (gc < (int64_t)ns) {
            const float* p = xs + gc * KC + c0;
            if constexpr (VW == 4) {
                const float4 t = *reinterpret_cast<const float4*>(p);
                v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
            } else if constexpr (VW == 2) {
                const float2 t = *reinterpret_cast<const float2*>(p);
                v[0] = t.x; v[1] = t.y;
            } else {
                v[0] = p[0];
            }
            return;
        }
    }
    XLd<XT, VW>::load(X + gc * ldx + c0, v);
}

// One work item on one wavefront (see the file comment); acc is the
// wavefront's h x KC accumulator, jt its strip-table slots.
template <int KC, int VW, typename XT, bool HV, bool STAGED>
__device__ __forceinline__ void process_item(
    const ItemDesc& d, const uint8_t* __restrict__ blob, uint64_t blob_bias, const XT* __restrict__ X,
    int64_t ldx, float* __restrict__ Y, int64_t ldy, int64_t* __restrict__ part,
    const CombineDesc* __restrict__ combine, uint32_t* __restrict__ count, const float* __restrict__ yscale,
    const int32_t* __restrict__ fexp, const int32_t* __restrict__ rmap, uint32_t h, uint32_t wshift,
    unsigned long long* acc, uint32_t* jt, const float* xs, uint32_t ns, int lane) {
    constexpr bool has_val = HV;        // weighted A
    constexpr int G = KC / VW;          // lanes per X row
    constexpr int P = 64 / G;           // entries per step
    constexpr int U = KC <= 2 ? 8 : KC <= 8 ? 4 : 8;  // steps in flight per lane
    const ItemLayout L = item_layout(d, has_val);
    const uint8_t* base = blob + (d.blob_off - blob_bias);
    const uint32_t lo = d.rows & 0xFFFFu, hi = d.rows >> 16;

    for (uint32_t i = lane; i < (hi - lo) * KC; i += 64) acc[lo * KC + i] = 0ull;
    wave_sync();

    const int g = lane % G;
    const uint32_t slot = lane / G;
    const int c0 = g * VW;
    // fixed-point scale of each of this lane's columns
    double fs[VW];
#pragma unroll
    for (int i = 0; i < VW; ++i) fs[i] = ldexp(1.0, fexp[c0 + i]);
    const uint64_t le_mask = lane == 63 ? ~0ull : ((2ull << lane) - 1);

    // Loads inside the unrolled steps are unconditional (indices clamped to
    // the last valid element, out-of-range slots weighted 0), so each phase
    // issues its U loads back to back and waits once.

    // ---- COO stream: one entry per lane group.  The strip of an entry is
    // the strip of the last run start at or before it: a ballot of the start
    // flags gives each lane its run ordinal, and the item's strip table sits
    // in LDS.  The entries of the next batch are loaded while the current
    // batch gathers X, so each batch waits for one memory round trip.
    if (d.n_coo) {
        const uint32_t* ent = reinterpret_cast<const uint32_t*>(base);
        const float* cval = reinterpret_cast<const float*>(base + 4 * (size_t)d.n_coo);
        const uint32_t* cJg = reinterpret_cast<const uint32_t*>(base + L.o_coo_J);
        const bool jt_lds = d.n_coo_J <= kJTab;
        if (jt_lds) {
            for (uint32_t i = lane; i < d.n_coo_J; i += 64) jt[i] = cJg[i];
            wave_sync();
        }
        const uint32_t last = d.n_coo - 1;
        int32_t seen = 0;  // run starts before the current step
        uint32_t en[U];
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t e = min((uint32_t)(u * P) + slot, last);
            en[u] = __builtin_nontemporal_load(ent + e);
            if constexpr (has_val) v[u] = cval[e];
            else v[u] = 1.0f;
        }
        for (uint32_t pb = 0; pb < d.n_coo; pb += P * U) {
            uint32_t enN[U];
            float vN[U];
            const uint32_t nb = pb + P * U;
            if (nb < d.n_coo) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t e = min(nb + u * P + slot, last);
                    enN[u] = __builtin_nontemporal_load(ent + e);
                    if constexpr (has_val) vN[u] = cval[e];
                    else vN[u] = 1.0f;
                }
            }
            uint32_t J[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool ok = pb + u * P + slot <= last;
                const uint64_t m = __ballot(ok && g == 0 && (en[u] & kCooNewTile));
                int32_t ord = seen + __popcll(m & le_mask) - 1;
                seen += __popcll(m);
                ord = ord < 0 ? 0 : ord;
                J[u] = jt_lds ? jt[ord] : cJg[ord];
            }
            float x[U][VW];
#pragma unroll
            for (int u = 0; u < U; ++u)
                xget<XT, KC, VW, STAGED>(X, ldx, c0, ((int64_t)J[u] << wshift) + (en[u] & 0xFFFFu), xs, ns, x[u]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (pb + u * P + slot <= last) {
                    unsigned long long* a = acc + ((en[u] >> 16) & 0xFFFu) * KC + c0;
#pragma unroll
                    for (int i = 0; i < VW; ++i) atomicAdd(a + i, to_fixed(v[u] * x[u][i], fs[i]));
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                en[u] = enN[u];
                v[u] = vN[u];
            }
        }
    }

    const uint16_t* cols = reinterpret_cast<const uint16_t*>(base + L.o_cols);
    const float* colv = reinterpret_cast<const float*>(base + L.o_cval);

    // ---- LR stream: one row segment per lane group, U elements in flight.
    // Segments are sorted by length and interleaved in blocks of 64, so the
    // lanes of a step read neighbouring column slots.
    if (d.n_lr) {
        const uint2* lseg = reinterpret_cast<const uint2*>(base + L.o_lr);
        const uint32_t* lJ = reinterpret_cast<const uint32_t*>(base + L.o_lr_J);
        for (uint32_t pb = 0; pb < d.n_lr; pb += P) {
            const uint32_t si = pb + slot;
            const bool seg_ok = si < d.n_lr;
            const uint2 sg = lseg[seg_ok ? si : d.n_lr - 1];
            const uint32_t len = seg_ok ? sg.y >> kLrStartBits : 0u;
            const uint32_t start = sg.y & ((1u << kLrStartBits) - 1);
            const uint32_t lastq = start + 64u * ((sg.y >> kLrStartBits) - 1);
            const uint32_t J = lJ[sg.x >> 12];
            const int64_t gb = (int64_t)J << wshift;
            float s[VW];
#pragma unroll
            for (int i = 0; i < VW; ++i) s[i] = 0.0f;
            for (uint32_t t = 0; t < len; t += U) {
                uint32_t cc[U];
                float w[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t q = min(start + 64u * (t + u), lastq);
                    cc[u] = __builtin_nontemporal_load(cols + q);
                    float wv = 1.0f;
                    if constexpr (has_val) wv = colv[q];
                    w[u] = t + u < len ? wv : 0.0f;
                }
                float x[U][VW];
#pragma unroll
                for (int u = 0; u < U; ++u) xget<XT, KC, VW, STAGED>(X, ldx, c0, gb + cc[u], xs, ns, x[u]);
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int i = 0; i < VW; ++i) s[i] += w[u] * x[u][i];
            }
            if (len) {
                unsigned long long* ap = acc + (sg.x & 0xFFFu) * KC + c0;
#pragma unroll
                for (int i = 0; i < VW; ++i) atomicAdd(ap + i, to_fixed(s[i], fs[i]));
            }
        }
    }

    // ---- WR stream: one row segment per wavefront; the P lane groups
    // stride over it (U elements in flight each), then a shuffle butterfly.
    // Segment descriptors are loaded 64 at a time into lanes and broadcast.
    {
        const uint4* wr = reinterpret_cast<const uint4*>(base + L.o_wr);
        uint4 mine = make_uint4(0u, 0u, 0u, 0u);
        for (uint32_t q = 0; q < d.n_wr; ++q) {
            if ((q & 63) == 0 && q + lane < d.n_wr) mine = wr[q + lane];
            uint4 sg;  // {J, row, first col, length}
            sg.x = __shfl(mine.x, q & 63);
            sg.y = __shfl(mine.y, q & 63);
            sg.z = __shfl(mine.z, q & 63);
            sg.w = __shfl(mine.w, q & 63);
            const int64_t gb = (int64_t)sg.x << wshift;
            const uint16_t* cp = cols + sg.z;
            const float* vp = colv + sg.z;
            float s[VW];
#pragma unroll
            for (int i = 0; i < VW; ++i) s[i] = 0.0f;
            for (uint32_t t = slot; t < sg.w; t += P * U) {
                uint32_t cc[U];
                float w[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t q2 = min(t + u * P, sg.w - 1);
                    cc[u] = __builtin_nontemporal_load(cp + q2);
                    float wv = 1.0f;
                    if constexpr (has_val) wv = vp[q2];
                    w[u] = t + u * P < sg.w ? wv : 0.0f;
                }
                float x[U][VW];
#pragma unroll
                for (int u = 0; u < U; ++u) xget<XT, KC, VW, STAGED>(X, ldx, c0, gb + cc[u], xs, ns, x[u]);
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int i = 0; i < VW; ++i) s[i] += w[u] * x[u][i];
            }
#pragma unroll
            for (int m = G; m < 64; m <<= 1)
#pragma unroll
                for (int i = 0; i < VW; ++i) s[i] += __shfl_xor(s[i], m);
            if (slot == 0) {
                unsigned long long* ap = acc + sg.y * KC + c0;
#pragma unroll
                for (int i = 0; i < VW; ++i) atomicAdd(ap + i, to_fixed(s[i], fs[i]));
            }
        }
    }

    wave_sync();
    const int64_t row0 = (int64_t)d.slab * h;
    if (d.part < 0) {
        const uint32_t total = (hi - lo) * KC;
        for (uint32_t i = lane; i < total; i += 64) {
            const uint32_t r = i / KC, c = i % KC;
            const int64_t t = row0 + lo + r;
            const int64_t yr = rmap ? (int64_t)rmap[t] : t;
            Y[yr * ldy + c] = OutScale<XT>::apply(from_fixed(acc[lo * KC + i], fexp[c]), yscale, c);
        }
        return;
    }
    // One piece of a split row: publish its KC fixed-point partial sums; the
    // last piece of the row to finish adds the slots (exact integer sums, so
    // the result does not depend on which piece finishes last), writes Y and
    // re-arms the counter for the next launch.
    if (lane < KC) part[(size_t)d.part * KC + lane] = (int64_t)acc[lo * KC + lane];
    __threadfence();
    uint32_t old = 0;
    if (lane == 0) old = atomicAdd(&count[d.cid], 1u);
    old = __shfl(old, 0);
    const CombineDesc cd = combine[d.cid];
    if (old != cd.part_end - cd.part_begin - 1) return;
    __threadfence();
    if (lane < KC) {
        unsigned long long s = 0ull;
        for (uint32_t p = cd.part_begin; p < cd.part_end; ++p)
            s += (unsigned long long)__builtin_nontemporal_load(part + (size_t)p * KC + lane);
        const int64_t t = row0 + cd.row;
        const int64_t yr = rmap ? (int64_t)rmap[t] : t;
        Y[yr * ldy + lane] = OutScale<XT>::apply(from_fixed(s, fexp[lane]), yscale, lane);
    }
    if (lane == 0) atomicExch(&count[d.cid], 0u);
}

// One wavefront per work item (up to four per workgroup).
template <int KC, int VW, typename XT, bool HV>
__global__ __launch_bounds__(256) void spmm_items(
    const ItemDesc* __restrict__ items, uint32_t n_items, const uint8_t* __restrict__ blob,
    uint64_t blob_bias, const XT* __restrict__ X, int64_t ldx, float* __restrict__ Y, int64_t ldy,
    int64_t* __restrict__ part, const CombineDesc* __restrict__ combine,
    uint32_t* __restrict__ count, const float* __restrict__ yscale, const int32_t* __restrict__ fexp,
    const int32_t* __restrict__ rmap, uint32_t h, uint32_t wshift) {
    extern __shared__ unsigned long long lds[];
    const uint32_t waves = blockDim.x >> 6;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t it = blockIdx.x * waves + wave;
    if (it >= n_items) return;
    unsigned long long* acc = lds + (size_t)wave * h * KC;
    uint32_t* jt = reinterpret_cast<uint32_t*>(lds + (size_t)waves * h * KC) + wave * kJTab;
    const ItemDesc d = items[it];
    process_item<KC, VW, XT, HV, false>(d, blob, blob_bias, X, ldx, Y, ldy, part, combine, count, yscale, fexp, rmap,
                                        h, wshift, acc, jt, nullptr, 0u, threadIdx.x & 63);
}

// Persistent variant with X rows staged in LDS: the workgroup first copies
// the first ns rows of X (the hottest columns in the handle's in-degree
// order), decoded to FP32, into LDS; then each wavefront walks the items
// it, it + (all wavefronts), ... .  Gathers of staged rows read LDS and
// leave the memory pipeline to the others.  Every wavefront reaches the one
// barrier before the item loop, and every loop ends (a fixed stride over a
// fixed count).
template <int KC, int VW, typename XT, bool HV>
__global__ __launch_bounds__(1024) void spmm_items_staged(
    const ItemDesc* __restrict__ items, uint32_t n_items, const uint8_t* __restrict__ blob,
    uint64_t blob_bias, const XT* __restrict__ X, int64_t ldx, float* __restrict__ Y, int64_t ldy,
    int64_t* __restrict__ part, const CombineDesc* __restrict__ combine,
    uint32_t* __restrict__ count, const float* __restrict__ yscale, const int32_t* __restrict__ fexp,
    const int32_t* __restrict__ rmap, uint32_t h, uint32_t wshift, uint32_t ns) {
    extern __shared__ unsigned long long lds[];
    float* xs = reinterpret_cast<float*>(lds);
    for (uint32_t t = threadIdx.x; t < ns * KC; t += blockDim.x) {
        float v[1];
        XLd<XT, 1>::load(X + (int64_t)(t / KC) * ldx + (t % KC), v);
        xs[t] = v[0];
    }
    __syncthreads();
    const uint32_t waves = blockDim.x >> 6;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    unsigned long long* accs = lds + ((size_t)ns * KC + 1) / 2;  // after the staged floats, 8-byte aligned
    unsigned long long* acc = accs + (size_t)wave * h * KC;
    uint32_t* jt = reinterpret_cast<uint32_t*>(accs + (size_t)waves * h * KC) + wave * kJTab;
    for (uint32_t it = blockIdx.x * waves + wave; it < n_items; it += gridDim.x * waves) {
        const ItemDesc d = items[it];
        process_item<KC, VW, XT, HV, true>(d, blob, blob_bias, X, ldx, Y, ldy, part, combine, count, yscale, fexp,
                                           rmap, h, wshift, acc, jt, xs, ns, threadIdx.x & 63);
    }
}

__global__ void colmax_init_kernel(uint32_t* m) {
    if (threadIdx.x < 64) m[threadIdx.x] = 0u;
}

// f_j = 61 - e with row_l1 * M_j < 2^e (0 when the bound is 0);
// kNonFiniteCol when the column holds a NaN or an infinity (M_j's bits are
// those of |x| with the largest bit pattern, so any non-finite value wins).
__global__ void fexp_kernel(const uint32_t* __restrict__ m, int k, double row_l1, int32_t* __restrict__ f) {
    const int j = threadIdx.x;
    if (j < 64) {
        int fj = 0;
        if (j < k) {
            if (m[j] >= 0x7F800000u) {
                fj = kNonFiniteCol;
            } else {
                const double b = row_l1 * (double)__uint_as_float(m[j]);
                if (b > 0.0 && b < 1.0e300) {
                    int e;
                    (void)frexp(b, &e);
                    fj = 61 - e;
                }
            }
        }
        f[j] = fj;
    }
}

// Per-device launch limits, read once per device.
struct DeviceLimits {
    int cus = 0;
    int max_lds = 0;
};

const DeviceLimits& device_limits() {
    static DeviceLimits lim[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        static DeviceLimits none;
        return none;
    }
    DeviceLimits& L = lim[dev];
    if (!L.cus) {
        int cus = 0, lds = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess) {
            L.max_lds = lds;
            L.cus = cus;
        }
    }
    return L;
}

template <typename XT, int KC, int VW>
hipError_t launch_one(const Handle& H, const RunArgs& a, const XT* X, float* Y,
                      const float* yscale, const int32_t* fexp) {
    if (!a.n_items) return hipSuccess;
    const uint32_t per_wave = H.h * KC * 8u + kJTab * 4u;
    // Narrow launches with staging requested: one persistent workgroup of 16
    // wavefronts per CU with the hottest X rows staged in the LDS left over
    // by the accumulators.
    if constexpr (KC <= 8) {
        const DeviceLimits& lim = device_limits();
        constexpr uint32_t kWaves = 16;
        const uint64_t fixed = (uint64_t)kWaves * per_wave;
        if (H.stage_bytes && lim.cus && (uint64_t)lim.max_lds > fixed + 16384) {
            const uint64_t budget = std::min<uint64_t>(H.stage_bytes, (uint64_t)lim.max_lds - fixed);
            uint64_t ns = std::min<uint64_t>((uint64_t)H.n_cols, budget / (KC * 4u));
            ns &= ~(uint64_t)1;
            if (ns >= 1024) {
                const size_t bytes = (size_t)ns * KC * 4u + fixed;
                const uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)lim.cus, (a.n_items + kWaves - 1) / kWaves);
                if (H.has_val) {
                    // raises the dynamic-LDS limit where the runtime asks for it; a
                    // launch beyond the device's limit fails and is reported below
                    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&spmm_items_staged<KC, VW, XT, true>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
                    hipLaunchKernelGGL((spmm_items_staged<KC, VW, XT, true>), dim3(grid), dim3(64 * kWaves), bytes,
                                       a.stream, a.items, a.n_items, a.blob, a.blob_bias, X, a.ldx, Y, a.ldy,
                                       a.part, a.combine, a.count, yscale, fexp, a.rmap, H.h, H.wshift, (uint32_t)ns);
                } else {
                    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&spmm_items_staged<KC, VW, XT, false>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
                    hipLaunchKernelGGL((spmm_items_staged<KC, VW, XT, false>), dim3(grid), dim3(64 * kWaves), bytes,
                                       a.stream, a.items, a.n_items, a.blob, a.blob_bias, X, a.ldx, Y, a.ldy,
                                       a.part, a.combine, a.count, yscale, fexp, a.rmap, H.h, H.wshift, (uint32_t)ns);
                }
                return hipGetLastError();
            }
        }
    }
    // 160 KB of LDS per CU; small accumulators pack four wavefronts per
    // workgroup so that the per-CU workgroup limit does not cap residency.
    const uint32_t wpb = per_wave <= 12288u ? 4u : per_wave <= 34816u ? 2u : 1u;
    const uint32_t grid = (a.n_items + wpb - 1) / wpb;
    if (H.has_val)
        hipLaunchKernelGGL((spmm_items<KC, VW, XT, true>), dim3(grid), dim3(64 * wpb), (size_t)per_wave * wpb,
                           a.stream, a.items, a.n_items, a.blob, a.blob_bias, X, a.ldx, Y, a.ldy, a.part,
                           a.combine, a.count, yscale, fexp, a.rmap, H.h, H.wshift);
    else
        hipLaunchKernelGGL((spmm_items<KC, VW, XT, false>), dim3(grid), dim3(64 * wpb), (size_t)per_wave * wpb,
                           a.stream, a.items, a.n_items, a.blob, a.blob_bias, X, a.ldx, Y, a.ldy, a.part,
                           a.combine, a.count, yscale, fexp, a.rmap, H.h, H.wshift);
    return hipGetLastError();
}

template <typename XT, int KC>
hipError_t launch_vw(const Handle& H, const RunArgs& a, const XT* X, float* Y,
                     const float* yscale, const int32_t* fexp, int vw) {
    if constexpr (KC >= 4) {
        if (vw == 4) return launch_one<XT, KC, 4>(H, a, X, Y, yscale, fexp);
    }
    if constexpr (KC >= 2) {
        if (vw == 2) return launch_one<XT, KC, 2>(H, a, X, Y, yscale, fexp);
    }
    return launch_one<XT, KC, 1>(H, a, X, Y, yscale, fexp);
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
        const int32_t* fx = a.fexp + c0;
        hipError_t e;
        switch (kc) {
            case 32: e = launch_vw<XT, 32>(H, a, Xc, Yc, sc, fx, vw); break;
            case 16: e = launch_vw<XT, 16>(H, a, Xc, Yc, sc, fx, vw); break;
            case 8: e = launch_vw<XT, 8>(H, a, Xc, Yc, sc, fx, vw); break;
            case 4: e = launch_vw<XT, 4>(H, a, Xc, Yc, sc, fx, vw); break;
            case 2: e = launch_vw<XT, 2>(H, a, Xc, Yc, sc, fx, vw); break;
            default: e = launch_vw<XT, 1>(H, a, Xc, Yc, sc, fx, vw); break;
        }
        if (e != hipSuccess) return e;
        c0 += kc;
    }
    return hipSuccess;
}

// X rows into the handle's column order (Xp row i = X row old_of_new[i]),
// together with the per-column max |x| of the values read (decoded to FP32,
// compared as FP32 bits with integer atomicMax: exact and order-free).  With
// Xp NULL nothing is written and rows are read in place.  One thread moves
// one U-sized unit (E elements) of a row; 2^lsh lanes cover a row's units
// and keep the same lane -> unit mapping for every row they visit, so each
// thread holds a running max for the same E columns throughout.
template <typename U, typename XT>
__global__ __launch_bounds__(256) void gather_colmax_kernel(const XT* __restrict__ X, int64_t ldx,
                                                            const int32_t* __restrict__ old_of_new, int64_t n,
                                                            int k, XT* __restrict__ Xp, int64_t ldp, int lsh,
                                                            uint32_t* __restrict__ m) {
    constexpr int E = sizeof(U) / sizeof(XT);
    __shared__ uint32_t red[64];
    if (threadIdx.x < 64) red[threadIdx.x] = 0u;
    __syncthreads();
    const int units = k / E;
    const int u = threadIdx.x & ((1 << lsh) - 1);
    if (u < units) {
        uint32_t best[E];
#pragma unroll
        for (int q = 0; q < E; ++q) best[q] = 0u;
        const int64_t step = ((int64_t)gridDim.x * blockDim.x) >> lsh;
        for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> lsh; i < n; i += step) {
            const int64_t src = old_of_new ? (int64_t)old_of_new[i] : i;
            const U v = *reinterpret_cast<const U*>(X + src * ldx + (int64_t)u * E);
            if (Xp) *reinterpret_cast<U*>(Xp + i * ldp + (int64_t)u * E) = v;
            const XT* e = reinterpret_cast<const XT*>(&v);
#pragma unroll
            for (int q = 0; q < E; ++q) {
                float f[1];
                XLd<XT, 1>::load(e + q, f);
                uint32_t bits = __float_as_uint(f[0]) & 0x7FFFFFFFu;
                // the E4M3 NaN codes (S.1111.111) decode to a finite value on
                // the fast path: mark their column as not finite here
                if constexpr (sizeof(XT) == 1)
                    if ((e[q] & 0x7Fu) == 0x7Fu) bits = 0x7FC00000u;
                best[q] = bits > best[q] ? bits : best[q];
            }
        }
#pragma unroll
        for (int q = 0; q < E; ++q) atomicMax(&red[u * E + q], best[q]);
    }
    __syncthreads();
    if ((int)threadIdx.x < k) atomicMax(&m[threadIdx.x], red[threadIdx.x]);
}

template <typename U, typename XT>
void launch_gather_unit(const XT* X, int64_t ldx, const int32_t* old_of_new, int64_t n, int k, XT* Xp,
                        int64_t ldp, uint32_t* m, hipStream_t s) {
    constexpr int E = sizeof(U) / sizeof(XT);
    const int units = k / E;
    int lsh = 0;
    while ((1 << lsh) < units) ++lsh;
    const int64_t rows_per_block = 256 >> lsh;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, (n + rows_per_block - 1) / rows_per_block));
    hipLaunchKernelGGL((gather_colmax_kernel<U, XT>), dim3(blocks), dim3(256), 0, s, X, ldx, old_of_new, n, k, Xp,
                       ldp, lsh, m);
}

// The widest unit (16, 8, 4, 2 or 1 bytes) that divides every row offset
// and both base addresses.
template <typename XT>
void launch_gather(const XT* X, int64_t ldx, const int32_t* old_of_new, int64_t n, int k, XT* Xp, int64_t ldp,
                   uint32_t* m, hipStream_t s) {
    auto fits = [&](size_t ub) {
        const size_t es = sizeof(XT);
        if (ub < es || ((size_t)k * es) % ub || ((size_t)ldx * es) % ub || reinterpret_cast<uintptr_t>(X) % ub)
            return false;
        return !Xp || (((size_t)ldp * es) % ub == 0 && reinterpret_cast<uintptr_t>(Xp) % ub == 0);
    };
    if (fits(16)) return launch_gather_unit<uint4, XT>(X, ldx, old_of_new, n, k, Xp, ldp, m, s);
    if (fits(8)) return launch_gather_unit<uint2, XT>(X, ldx, old_of_new, n, k, Xp, ldp, m, s);
    if (fits(4)) return launch_gather_unit<uint32_t, XT>(X, ldx, old_of_new, n, k, Xp, ldp, m, s);
    if constexpr (sizeof(XT) <= 2)
        if (fits(2)) return launch_gather_unit<uint16_t, XT>(X, ldx, old_of_new, n, k, Xp, ldp, m, s);
    if constexpr (sizeof(XT) == 1) return launch_gather_unit<uint8_t, XT>(X, ldx, old_of_new, n, k, Xp, ldp, m, s);
}

}  // namespace

hipError_t launch_prepare_x(const void* X, int dtype, int64_t ldx, int k, const int32_t* old_of_new, int64_t n,
                            void* Xp, int64_t ldp, double row_l1, uint32_t* colmax, int32_t* fexp,
                            hipStream_t s) {
    hipLaunchKernelGGL(colmax_init_kernel, dim3(1), dim3(64), 0, s, colmax);
    if (n > 0) {
        if (dtype == SPMM_X_BF16)
            launch_gather(static_cast<const uint16_t*>(X), ldx, old_of_new, n, k, static_cast<uint16_t*>(Xp), ldp,
                          colmax, s);
        else if (dtype == SPMM_X_FP8_E4M3)
            launch_gather(static_cast<const uint8_t*>(X), ldx, old_of_new, n, k, static_cast<uint8_t*>(Xp), ldp,
                          colmax, s);
        else
            launch_gather(static_cast<const float*>(X), ldx, old_of_new, n, k, static_cast<float*>(Xp), ldp, colmax,
                          s);
    }
    hipLaunchKernelGGL(fexp_kernel, dim3(1), dim3(64), 0, s, colmax, k, row_l1, fexp);
    return hipGetLastError();
}

namespace {
__global__ __launch_bounds__(256) void zero_rows_kernel(float* __restrict__ Y, int64_t ldy, int k,
                                                        const int32_t* __restrict__ rows, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count * k) return;
    const int64_t r = i / k;
    Y[(int64_t)rows[r] * ldy + (i - r * k)] = 0.0f;
}
}  // namespace

hipError_t launch_zero_rows(float* Y, int64_t ldy, int k, const int32_t* rows, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t total = count * k;
    hipLaunchKernelGGL(zero_rows_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, Y, ldy, k, rows,
                       count);
    return hipGetLastError();
}

hipError_t launch_spmm(const Handle& H, const RunArgs& a) {
    switch (a.dtype) {
        case SPMM_X_BF16: return launch_typed<uint16_t>(H, a);
        case SPMM_X_FP8_E4M3: return launch_typed<uint8_t>(H, a);
        default: return launch_typed<float>(H, a);
    }
}

}  // namespace spmm
