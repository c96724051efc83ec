// Diagnostic: the read bandwidth this device delivers to a plain streaming
// kernel, the practical ceiling against which the row-streaming solves are
// judged (the published HBM peak is not reachable by reads alone).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>

#include "sssp.h"

namespace sssp {
int set_error(int code, const char* msg);  // api.cpp
}

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

// Each thread reads 16-byte words i, i + stride, ... with 16 loads in flight and
// folds them into one value, stored only if it equals a fixed pattern (a store
// the compiler cannot rule out, so it keeps the loads); nontemporal, like the
// whole-GPU solve.
__global__ __launch_bounds__(1024) void k_stream_read(const v4i* __restrict__ p, size_t words,
                                                      int32_t* __restrict__ sink) {
    constexpr int U = 16;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    int acc = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride * U) {
        v4i r[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const size_t j = i + (size_t)q * stride;
            r[q] = j < words ? __builtin_nontemporal_load(p + j) : v4i{0, 0, 0, 0};
        }
#pragma unroll
        for (int q = 0; q < U; ++q) acc ^= r[q].x ^ r[q].y ^ r[q].z ^ r[q].w;
    }
    if (acc == 0x5eed5eed && sink) sink[0] = acc;
}

}  // namespace

extern "C" int sssp_stream_read(const void* buf, int64_t bytes, int32_t* sink, void* stream) {
    if (!buf || bytes < 16 || ((uintptr_t)buf & 15)) return sssp::set_error(SSSP_EINVAL, "bad buffer");
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return sssp::set_error(SSSP_EDEVICE, "device query failed");
    hipLaunchKernelGGL(k_stream_read, dim3(8 * cus), dim3(1024), 0, (hipStream_t)stream,
                       static_cast<const v4i*>(buf), (size_t)bytes / 16, sink);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        char msg[256];
        snprintf(msg, sizeof msg, "stream read launch: %s", hipGetErrorString(e));
        return sssp::set_error(SSSP_EDEVICE, msg);
    }
    return SSSP_OK;
}
