// A plain streaming read of device memory: the HBM rate a simple kernel
// attains, measured beside the SpMM so that the nominal peak is in context.
#include <hip/hip_runtime.h>

#include "spmm_internal.h"

namespace spmm {
namespace {

// Every 16-byte vector of p is read once (four loads in flight per thread);
// the sum is stored only when it equals a value no input of this use
// produces, which keeps the loads without writing anything in practice.
__global__ __launch_bounds__(256) void read_probe_kernel(const float4* __restrict__ p, uint64_t n4,
                                                         float* __restrict__ sink) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float acc = 0.0f;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        const float4 a = p[i], b = p[i + stride], c = p[i + 2 * stride], d = p[i + 3 * stride];
        acc += (a.x + b.y) + (c.z + d.w);
    }
    for (; i < n4; i += stride) acc += p[i].x;
    if (acc == -1.0f) sink[0] = acc;
}

}  // namespace

hipError_t launch_read_probe(const void* buf, uint64_t bytes, float* sink, hipStream_t s) {
    const uint64_t n4 = bytes / 16;
    if (n4) hipLaunchKernelGGL(read_probe_kernel, dim3(8192), dim3(256), 0, s, static_cast<const float4*>(buf), n4, sink);
    return hipGetLastError();
}

}  // namespace spmm
