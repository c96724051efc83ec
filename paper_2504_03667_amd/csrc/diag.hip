// Diagnostic: the read bandwidth this device delivers to a plain streaming
// kernel, the practical ceiling against which the row-streaming solves are
// measured (the published HBM peak is not reachable by reads alone).
//
// Workgroups claim fixed-size chunks from a counter until none is left, so
// faster XCDs read more chunks than slower ones: a static split (every
// workgroup the same share) ends when the slowest XCD ends and measures less.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <mutex>
#include <vector>

#include "sssp.h"

namespace sssp {
int set_error(int code, const char* msg);  // api.cpp
}

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kThreads = 1024;
constexpr int kInFlight = 16;                  // 16-byte loads in flight per thread
constexpr int64_t kDefaultChunk = 256 << 10;   // bytes per claim

// claims: next chunk index; exits: workgroups done.  The last workgroup out
// zeroes both, so the next launch starts from zero without a host memset.
struct ReadCounters {
    unsigned long long claims;
    unsigned long long exits;
};

__global__ __launch_bounds__(kThreads) void k_stream_read(const v4i* __restrict__ p, uint64_t words,
                                                          uint32_t chunk_words, ReadCounters* __restrict__ rc,
                                                          uint32_t* __restrict__ fold) {
    __shared__ unsigned long long s_chunk;
    __shared__ uint32_t s_fold[kThreads / 64];
    const uint64_t nchunks = (words + chunk_words - 1) / chunk_words;
    uint32_t acc = 0;
    for (;;) {
        if (threadIdx.x == 0)
            s_chunk = __hip_atomic_fetch_add(&rc->claims, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint64_t c = s_chunk;
        __syncthreads();
        if (c >= nchunks) break;
        const uint64_t base = c * chunk_words;
        const uint32_t len = (uint32_t)min((uint64_t)chunk_words, words - base);
        for (uint32_t i = threadIdx.x; i < len; i += kThreads * kInFlight) {
            v4i r[kInFlight];
#pragma unroll
            for (int q = 0; q < kInFlight; ++q) {
                const uint32_t j = i + (uint32_t)q * kThreads;
                r[q] = j < len ? __builtin_nontemporal_load(p + base + j) : v4i{0, 0, 0, 0};
            }
#pragma unroll
            for (int q = 0; q < kInFlight; ++q) acc ^= (uint32_t)(r[q].x ^ r[q].y ^ r[q].z ^ r[q].w);
        }
    }
    // xor of everything this workgroup read, folded into *fold once
    for (int o = 32; o > 0; o >>= 1) acc ^= (uint32_t)__shfl_xor((int)acc, o, 64);
    if ((threadIdx.x & 63) == 0) s_fold[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t f = 0;
        for (int w = 0; w < kThreads / 64; ++w) f ^= s_fold[w];
        if (fold) __hip_atomic_fetch_xor(fold, f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // every workgroup's last claim precedes its exit count; the last one out resets
        const unsigned long long done =
            __hip_atomic_fetch_add(&rc->exits, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (done == (unsigned long long)gridDim.x - 1) {
            __hip_atomic_store(&rc->claims, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&rc->exits, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

std::mutex g_read_mu;
std::vector<ReadCounters*> g_read_counters;  // per device, kept until sssp_release_all or the process ends

int read_counters(int dev, ReadCounters** out) {
    std::lock_guard<std::mutex> lk(g_read_mu);
    if ((int)g_read_counters.size() <= dev) g_read_counters.resize(dev + 1, nullptr);
    if (!g_read_counters[dev]) {
        ReadCounters* p = nullptr;
        if (hipMalloc(&p, sizeof(ReadCounters)) != hipSuccess)
            return sssp::set_error(SSSP_ENOMEM, "hipMalloc(stream-read counters) failed");
        if (hipMemset(p, 0, sizeof(ReadCounters)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
            (void)hipFree(p);
            return sssp::set_error(SSSP_EDEVICE, "hipMemset(stream-read counters) failed");
        }
        g_read_counters[dev] = p;
    }
    *out = g_read_counters[dev];
    return SSSP_OK;
}

}  // namespace

namespace sssp {

int release_read_counters() {
    std::lock_guard<std::mutex> lk(g_read_mu);
    int cur = -1;
    (void)hipGetDevice(&cur);
    for (size_t d = 0; d < g_read_counters.size(); ++d) {
        if (!g_read_counters[d]) continue;
        // a read may still run on any stream of that device
        if (hipSetDevice((int)d) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
            return set_error(SSSP_EDEVICE, "synchronising a device before freeing its read counters failed");
        (void)hipFree(g_read_counters[d]);
        g_read_counters[d] = nullptr;
    }
    if (cur >= 0) (void)hipSetDevice(cur);
    return SSSP_OK;
}

int64_t read_counter_bytes() {
    std::lock_guard<std::mutex> lk(g_read_mu);
    int64_t b = 0;
    for (ReadCounters* p : g_read_counters) b += p ? (int64_t)sizeof(ReadCounters) : 0;
    return b;
}

}  // namespace sssp

extern "C" int sssp_stream_read(const void* buf, int64_t bytes, int64_t chunk_bytes, uint32_t* fold,
                                void* stream) {
    if (!buf || ((uintptr_t)buf & 15)) return sssp::set_error(SSSP_EINVAL, "buf is null or not 16-byte aligned");
    if (bytes < 16 || bytes % 16) return sssp::set_error(SSSP_EINVAL, "bytes must be a positive multiple of 16");
    if (chunk_bytes == 0) chunk_bytes = kDefaultChunk;
    if (chunk_bytes < 1024 || chunk_bytes > (64 << 20) || chunk_bytes % 16)
        return sssp::set_error(SSSP_EINVAL, "chunk_bytes must be 0 or a multiple of 16 in [1 KiB, 64 MiB]");
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return sssp::set_error(SSSP_EDEVICE, "device query failed");
    ReadCounters* rc = nullptr;
    if (int e = read_counters(dev, &rc)) return e;
    hipLaunchKernelGGL(k_stream_read, dim3(2 * cus), dim3(kThreads), 0, (hipStream_t)stream,
                       static_cast<const v4i*>(buf), (uint64_t)bytes / 16, (uint32_t)(chunk_bytes / 16), rc, fold);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        char msg[256];
        snprintf(msg, sizeof msg, "stream read launch: %s", hipGetErrorString(e));
        return sssp::set_error(SSSP_EDEVICE, msg);
    }
    return SSSP_OK;
}
