// Measurement utility: streaming-read bandwidth of the device, the reference
// ceiling for the SpMM's matrix stream (not part of the method).
#include <hip/hip_runtime.h>

#include <string>

#include "common.hpp"

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace xct {

// Streaming read of a buffer (16-byte non-temporal loads, grid-stride), the
// reference ceiling for the SpMM's matrix stream.
__global__ void __launch_bounds__(256) k_read_probe(const u32x4 *p, int64_t n, uint32_t *sink) {
    uint32_t acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const u32x4 v = __builtin_nontemporal_load(p + i);
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;  // keeps the loads; practically never stores
}
}  // namespace xct

using namespace xct;

extern "C" int xct_read_bandwidth(const void *buf, int64_t bytes, int reps, double *gbps, void *stream) {
    if (!buf || !gbps || bytes < 16 || reps < 1) return fail(XCT_ERR_INVALID, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = bytes / 16;
    uint32_t *sink = nullptr;
    XCT_HIP_TRY(hipMalloc(&sink, sizeof(uint32_t)));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = XCT_OK;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    const int grid = 4096;
    if (he == hipSuccess) {
        hipLaunchKernelGGL(k_read_probe, dim3(grid), dim3(256), 0, st, (const u32x4 *)buf, n, sink);
        he = hipEventRecord(e0, st);
    }
    for (int r = 0; r < reps && he == hipSuccess; ++r) {
        hipLaunchKernelGGL(k_read_probe, dim3(grid), dim3(256), 0, st, (const u32x4 *)buf, n, sink);
        he = hipGetLastError();
    }
    if (he == hipSuccess) he = hipEventRecord(e1, st);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (he != hipSuccess) rc = fail(XCT_ERR_HIP, std::string("read probe: ") + hipGetErrorString(he));
    else *gbps = (double)n * 16.0 * reps / (ms * 1e-3) / 1e9;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    return rc;
}

