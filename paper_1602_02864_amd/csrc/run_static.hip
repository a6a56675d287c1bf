// spmm_run_static: Y = A X without any device allocation, for callers that
// cannot allocate (code under graph capture, serving loops, harnesses that
// forbid hipMalloc).
//
// The scratch of an SpMM launch -- the split-row partial sums, their
// counters, the column maxima of X and the fixed-point exponents -- lives in
// the file-scope device array `scratch` below instead of handle-owned
// allocations.  Each GPU holds its own copy of the array, at its own
// address, from the first call on that device until the process ends; the
// address is looked up once per device (hipGetSymbolAddress) and only that
// address is handed to kernels and copies.  Every call on a device shares
// the array: calls that overlap on one GPU race, and the array keeps the
// last call's contents (the counters are cleared at the start of each call).
#include <hip/hip_runtime.h>

#include <mutex>

#include "abi_internal.h"

constexpr size_t kScratchBytes = size_t(16) << 20;  // 16 MiB per device

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up once).
spmm_status_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return spmm_abi::hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return spmm_abi::fail(SPMM_EUNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return spmm_abi::hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SPMM_OK;
}

__global__ void clear_u32(uint32_t* __restrict__ p, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

extern "C" spmm_status_t spmm_run_static(spmm_handle_t h, const void* X, int k, int64_t ldx, spmm_xdtype_t dt,
                                         const float* col_scale, float* Y, int64_t ldy, hipStream_t s) {
    using namespace spmm_abi;
    try {
        if (spmm_status_t rs = check_ready(h)) return rs;
        spmm::Handle& H = h->H;
        if (H.place != SPMM_PLACE_DEVICE) return fail(SPMM_ESTATE, "tiles are placed in host memory");
        if (H.format != SPMM_FORMAT_TILES) return fail(SPMM_EUNSUPPORTED, "spmm_run_static runs the tile store");
        if (H.relabel)
            return fail(SPMM_EUNSUPPORTED, "spmm_run_static reads X in place: build the handle with keep_order = 1");
        spmm_status_t st = check_run_args(H, X, k, ldx, dt, col_scale, Y, ldy);
        if (st != SPMM_OK) return st;
        if (H.n_rows == 0) return SPMM_OK;
        if (!H.uploaded)
            return fail(SPMM_ESTATE, "the tiles are not on the device yet: call spmm_run on the handle once first");
        // layout of the scratch: partial sums, counters, column maxima, exponents
        const size_t n_comb = H.enc.combine.size();
        const size_t part_bytes = align256(H.enc.n_parts * (size_t)spmm::kc_cap(H) * sizeof(int64_t));
        const size_t count_bytes = align256(n_comb * sizeof(uint32_t));
        const size_t need = part_bytes + count_bytes + 2 * 256;
        if (need > kScratchBytes)
            return fail(SPMM_EINVAL, "the handle's split rows need " + std::to_string(need) +
                                         " bytes of scratch; spmm_run_static has " + std::to_string(kScratchBytes));
        void* base = nullptr;
        if ((st = scratch_address(&base)) != SPMM_OK) return st;
        unsigned char* b = static_cast<unsigned char*>(base);
        int64_t* part = reinterpret_cast<int64_t*>(b);
        uint32_t* count = reinterpret_cast<uint32_t*>(b + part_bytes);
        uint32_t* colmax = reinterpret_cast<uint32_t*>(b + part_bytes + count_bytes);
        int32_t* fexp = reinterpret_cast<int32_t*>(b + part_bytes + count_bytes + 256);
        if (n_comb) {
            hipLaunchKernelGGL(clear_u32, dim3((unsigned)((n_comb + 255) / 256)), dim3(256), 0, s, count,
                               (uint32_t)n_comb);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return hip_fail(e, "counter clear launch");
        }
        return run_device_scratch(H, X, k, ldx, dt, col_scale, Y, ldy, s, part, count, colmax, fexp);
    } catch (const std::exception& ex) {
        return fail(SPMM_EINVAL, ex.what());
    }
}
