// Seeded, counter-based generator of dense weighted adjacency matrices (device side).
//
// Input tooling only: it holds no shortest-path arithmetic. It reproduces
// gen_host.c entry for entry (same mixer, same key, same threshold test, same
// multiply-shift weight map), so a 16 GiB matrix can be written straight into
// HBM instead of being built on the host and copied over PCIe. The two sides
// are cross-checked by the position-weighted checksum below.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GEN_INF 0x7fffffff

__device__ __forceinline__ uint64_t gdev_mix64(uint64_t x)
{
    x += 0x9e3779b97f4a7c15ULL;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
    return x ^ (x >> 31);
}

static uint64_t ghost_mix64(uint64_t x)
{
    x += 0x9e3779b97f4a7c15ULL;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
    return x ^ (x >> 31);
}

// One thread writes 4 consecutive entries of a row; grid.y walks rows.
__global__ void gdev_fill_kernel(int32_t* __restrict__ W, int64_t ld, int32_t n, int32_t r0,
                                 int32_t rows, uint64_t smix, uint64_t thresh, uint32_t lo,
                                 uint64_t span, int32_t directed)
{
    const int64_t j0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    for (int32_t r = blockIdx.y; r < rows; r += gridDim.y) {
        const uint32_t i = (uint32_t)(r0 + r);
        int32_t* row = W + (int64_t)r * ld;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t j = j0 + k;
            if (j >= n) break;
            int32_t v;
            if ((uint32_t)j == i) {
                v = 0;
            } else {
                const uint32_t jj = (uint32_t)j;
                uint64_t key;
                if (directed) key = ((uint64_t)i << 32) | jj;
                else key = i < jj ? (((uint64_t)i << 32) | jj) : (((uint64_t)jj << 32) | i);
                const uint64_t h = gdev_mix64(smix ^ key);
                v = (h >> 32) >= thresh ? GEN_INF
                                        : (int32_t)(lo + (uint32_t)(((h & 0xffffffffULL) * span) >> 32));
            }
            row[j] = v;
        }
    }
}

// Partial checksums: one 64-bit partial per block, summed on the host.
__global__ void gdev_sum_kernel(const int32_t* __restrict__ W, int64_t ld, int32_t n,
                                uint64_t* __restrict__ partial)
{
    __shared__ uint64_t red[256];
    uint64_t s = 0;
    const int64_t total = (int64_t)n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n, j = e - i * n;
        s += (uint64_t)(uint32_t)W[i * ld + j] * (2 * (uint64_t)e + 1);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

extern "C" {

// Write rows [r0, r0+rows) of the n x n matrix into Wrows (device, row stride ld >= n).
// Asynchronous on `stream`. Returns 0 or a hipError_t value.
int gen_dense_fill_device(int32_t* Wrows, int64_t ld, int32_t n, int32_t r0, int32_t rows,
                          uint64_t seed, uint64_t thresh, int32_t lo, int32_t hi,
                          int32_t directed, void* stream)
{
    if (!Wrows || n < 0 || ld < n || r0 < 0 || rows < 0 || (int64_t)r0 + rows > n || lo < 0 ||
        lo > hi || thresh > (1ULL << 32))
        return (int)hipErrorInvalidValue;
    if (n == 0 || rows == 0) return 0;
    const int threads = 256;
    const int64_t groups = ((int64_t)n + 3) / 4;
    dim3 grid((unsigned)((groups + threads - 1) / threads), (unsigned)(rows < 65535 ? rows : 65535));
    hipLaunchKernelGGL(gdev_fill_kernel, grid, dim3(threads), 0, (hipStream_t)stream, Wrows, ld, n,
                       r0, rows, ghost_mix64(seed), thresh, (uint32_t)lo,
                       (uint64_t)((int64_t)hi - lo + 1), directed);
    return (int)hipGetLastError();
}

// Checksum of an n x n device matrix; synchronises `stream`. Returns 0 or a hipError_t value.
int gen_dense_checksum_device(const int32_t* W, int64_t ld, int32_t n, uint64_t* out,
                              void* stream)
{
    if (!W || !out || n < 0 || ld < n) return (int)hipErrorInvalidValue;
    const int blocks = 4096;
    uint64_t* d = nullptr;
    hipError_t e = hipMalloc(&d, blocks * sizeof(uint64_t));
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(gdev_sum_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, W, ld, n, d);
    uint64_t h[4096];
    e = hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    hipFree(d);
    if (e != hipSuccess) return (int)e;
    uint64_t s = 0;
    for (int b = 0; b < blocks; ++b) s += h[b];
    *out = s;
    return 0;
}

}  // extern "C"
