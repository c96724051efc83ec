// GPU check of the wave-wide primitives of engine.h (wave_min64, wave_or32,
// wave_scan32) against the same operations done on the host.  Built by the
// package build (tests/native/_build/wave_ops) and run by
// tests/test_gpu_wave_ops.py.  Every wave of a 256-thread block reduces its
// own 64 inputs; the patterns cover a minimum at each lane, ties, all-ones
// keys, single set bits at each lane and random data.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "engine.h"

using namespace sssp;

__global__ void k_wave_ops(const uint64_t* __restrict__ a, const uint32_t* __restrict__ b,
                           const uint32_t* __restrict__ c, uint64_t* __restrict__ mn, uint32_t* __restrict__ orr,
                           uint32_t* __restrict__ scan) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    mn[i] = wave_min64(a[i]);
    orr[i] = wave_or32(b[i]);
    scan[i] = wave_scan32(c[i]);
}

int main() {
    const int waves = 4096;  // trials, one per wave
    const size_t N = (size_t)waves * 64;
    std::vector<uint64_t> a(N);
    std::vector<uint32_t> b(N), c(N);
    std::mt19937_64 rng(2504);
    for (int w = 0; w < waves; ++w) {
        const int kind = w % 8;
        for (int l = 0; l < 64; ++l) {
            const size_t i = (size_t)w * 64 + l;
            switch (kind) {
                case 0: a[i] = rng(); break;                                   // random keys
                case 1: a[i] = (l == w / 8 % 64) ? 5 : 1000 + rng() % 1000; break;  // minimum at one lane
                case 2: a[i] = ~0ull; break;                                   // no key anywhere
                case 3: a[i] = (rng() % 3) << 32 | (rng() % 4); break;         // many ties
                case 4: a[i] = l == 63 ? 0 : ~0ull; break;                     // minimum at the last lane
                case 5: a[i] = l == 0 ? 7 : ~0ull - l; break;                  // minimum at the first lane
                default: a[i] = (uint64_t)(rng() % 100000) << 32 | (uint32_t)rng(); break;
            }
            b[i] = kind == 1 ? (l == w / 8 % 64 ? 1u << (w % 32) : 0u) : (kind == 2 ? 0u : (uint32_t)rng() & (uint32_t)rng());
            c[i] = kind == 2 ? 0u : kind == 4 ? 1u : (uint32_t)(rng() % 65536);
        }
    }
    uint64_t *da, *dmn;
    uint32_t *db, *dc, *dor, *dsc;
    if (hipMalloc(&da, N * 8) || hipMalloc(&dmn, N * 8) || hipMalloc(&db, N * 4) || hipMalloc(&dc, N * 4) ||
        hipMalloc(&dor, N * 4) || hipMalloc(&dsc, N * 4)) {
        std::fprintf(stderr, "hipMalloc failed\n");
        return 2;
    }
    hipMemcpy(da, a.data(), N * 8, hipMemcpyHostToDevice);
    hipMemcpy(db, b.data(), N * 4, hipMemcpyHostToDevice);
    hipMemcpy(dc, c.data(), N * 4, hipMemcpyHostToDevice);
    const int threads = 256;  // four waves per block; N is a multiple of it
    hipLaunchKernelGGL(k_wave_ops, dim3((unsigned)(N / threads)), dim3(threads), 0, 0, da, db, dc, dmn, dor, dsc);
    if (hipDeviceSynchronize() != hipSuccess) {
        std::fprintf(stderr, "kernel failed\n");
        return 2;
    }
    std::vector<uint64_t> mn(N);
    std::vector<uint32_t> orr(N), sc(N);
    hipMemcpy(mn.data(), dmn, N * 8, hipMemcpyDeviceToHost);
    hipMemcpy(orr.data(), dor, N * 4, hipMemcpyDeviceToHost);
    hipMemcpy(sc.data(), dsc, N * 4, hipMemcpyDeviceToHost);
    int bad = 0;
    for (int w = 0; w < waves && bad < 10; ++w) {
        uint64_t m = ~0ull;
        uint32_t o = 0, s = 0;
        for (int l = 0; l < 64; ++l) {
            m = std::min(m, a[(size_t)w * 64 + l]);
            o |= b[(size_t)w * 64 + l];
        }
        for (int l = 0; l < 64 && bad < 10; ++l) {
            const size_t i = (size_t)w * 64 + l;
            s += c[i];
            if (mn[i] != m || orr[i] != o || sc[i] != s) {
                std::fprintf(stderr, "wave %d lane %d: min %llx/%llx or %x/%x scan %u/%u\n", w, l,
                             (unsigned long long)mn[i], (unsigned long long)m, orr[i], o, sc[i], s);
                ++bad;
            }
        }
    }
    if (bad) return 1;
    std::printf("wave ops ok (%d waves)\n", waves);
    return 0;
}
