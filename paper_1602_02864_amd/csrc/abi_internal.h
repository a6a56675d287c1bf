// Helpers shared by the C ABI translation units (abi.cpp, selector.cpp):
// error reporting, device residency of a handle, and the SpMM dispatch.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "spmm_internal.h"

struct spmm_handle_s {
    spmm::Handle H;
};

namespace spmm_abi {

// Record msg as the thread's last error and return st.
spmm_status_t fail(spmm_status_t st, const std::string& msg);
spmm_status_t hip_fail(hipError_t e, const char* what);

// SPMM_EINVAL for a NULL handle, SPMM_ESTATE for one whose slab-wise build
// has not ended, else SPMM_OK.
spmm_status_t check_ready(spmm_handle_t h);

// Release every device and pinned buffer of H; H.uploaded becomes false.
void free_device(spmm::Handle& H);
// Upload the encoded work (once) and size the split-row partial slots.
spmm_status_t prepare_device(spmm::Handle& H);
// Y = A X on s: optional X gather into handle column order, fixed-point
// exponents, SpMM launches.
spmm_status_t run_device(spmm::Handle& H, const void* X, int k, int64_t ldx, int dt, const float* col_scale,
                         float* Y, int64_t ldy, hipStream_t s, bool x_in_handle_order);
// spmm_run's work with caller-given scratch (see abi.cpp); allocates nothing.
spmm_status_t run_device_scratch(spmm::Handle& H, const void* X, int k, int64_t ldx, int dt,
                                 const float* col_scale, float* Y, int64_t ldy, hipStream_t s, int64_t* part,
                                 uint32_t* count, uint32_t* colmax, int32_t* fexp);
// Argument checks shared by the run entry points.
spmm_status_t check_run_args(const spmm::Handle& H, const void* X, int k, int64_t ldx, spmm_xdtype_t dt,
                             const float* col_scale, const float* Y, int64_t ldy);
// The SpMM launches alone, given fixed-point exponents and X in handle order.
spmm_status_t launch_items_only(spmm::Handle& H, const void* X, int k, int64_t ldx, int dt,
                                const float* col_scale, float* Y, int64_t ldy, hipStream_t s,
                                const int32_t* fexp);

// Scoped device buffers for the drivers that need a workspace.  With
// sync_on(s), the stream the buffers are used on is synchronised before they
// are freed, so an error return in the middle of queued work cannot free
// memory that kernels still use.
struct DevBufs {
    std::vector<void*> p;
    hipStream_t stream = nullptr;
    bool sync_first = false;
    void sync_on(hipStream_t s) {
        stream = s;
        sync_first = true;
    }
    ~DevBufs() {
        if (sync_first && !p.empty()) (void)hipStreamSynchronize(stream);
        for (void* q : p) (void)hipFree(q);
    }
    template <typename T>
    T* get(size_t count) {
        void* q = nullptr;
        if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return nullptr;
        p.push_back(q);
        return static_cast<T*>(q);
    }
};

}  // namespace spmm_abi
