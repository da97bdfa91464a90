// Plain streaming kernels that measure the memory roofline the Yee kernels
// are compared with: a copy (one read and one write per element), a read
// only and a write only pass, 16 bytes per lane per access, with a
// grid-stride loop over four resident workgroups per CU.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/fdtd.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) probe_copy(const v4f* __restrict__ in, v4f* __restrict__ out,
                                                  size_t n) {
    for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        __builtin_nontemporal_store(in[i], &out[i]);
}

__global__ void __launch_bounds__(256) probe_read(const v4f* __restrict__ in, float* sink,
                                                  size_t n) {
    float s = 0.f;
    for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const v4f v = in[i];
        s += (v.x + v.y) + (v.z + v.w);
    }
    // the buffer holds zeros, so this store never happens; it keeps the loads
    if (s != 0.f) sink[threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) probe_write(v4f* __restrict__ out, size_t n) {
    const v4f v = {1.f, 2.f, 3.f, 4.f};
    for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        __builtin_nontemporal_store(v, &out[i]);
}

}  // namespace

extern "C" int fdtd_stream_probe(int32_t kind, int64_t bytes, int32_t reps, void* stream,
                                 double* ms_per_pass, double* gbs) {
    if (kind < FDTD_PROBE_COPY || kind > FDTD_PROBE_WRITE || bytes <= 0 || bytes % 16 != 0 ||
        reps < 1 || reps > 1000 || !ms_per_pass || !gbs)
        return FDTD_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return FDTD_EDEVICE;
    void *a = nullptr, *b = nullptr;
    float* sink = nullptr;
    if (hipMalloc(&a, (size_t)bytes) != hipSuccess) return FDTD_ENOMEM;
    if (hipMalloc(&b, (size_t)bytes) != hipSuccess || hipMalloc(&sink, 256 * sizeof(float)) != hipSuccess) {
        (void)hipFree(a);
        (void)hipFree(b);
        return FDTD_ENOMEM;
    }
    int rc = FDTD_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const size_t n = (size_t)bytes / 16;
    const dim3 grid((unsigned)(4 * (cus > 0 ? cus : 1))), block(256);
    auto pass = [&]() {
        if (kind == FDTD_PROBE_COPY)
            hipLaunchKernelGGL(probe_copy, grid, block, 0, s, (const v4f*)a, (v4f*)b, n);
        else if (kind == FDTD_PROBE_READ)
            hipLaunchKernelGGL(probe_read, grid, block, 0, s, (const v4f*)a, sink, n);
        else
            hipLaunchKernelGGL(probe_write, grid, block, 0, s, (v4f*)b, n);
    };
    do {
        if (hipMemsetAsync(a, 0, (size_t)bytes, s) != hipSuccess ||
            hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            rc = FDTD_EDEVICE;
            break;
        }
        pass();   // warm-up
        if (hipEventRecord(e0, s) != hipSuccess) { rc = FDTD_EDEVICE; break; }
        for (int r = 0; r < reps; ++r) pass();
        float ms = 0.f;
        if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = FDTD_EDEVICE;
            break;
        }
        const double moved = (kind == FDTD_PROBE_COPY ? 2.0 : 1.0) * (double)bytes;
        *ms_per_pass = (double)ms / reps;
        *gbs = moved / (*ms_per_pass * 1e-3) / 1e9;
    } while (false);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(a);
    (void)hipFree(b);
    (void)hipFree(sink);
    return rc;
}
