// Declarations shared between the kernels (kernels.hip) and the C ABI (api.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sssp.h"

namespace sssp {

struct Ctl;
struct Pub;

// internal flag bits, above the public SSSP_FLAG_* bits
constexpr uint32_t kFlagLiteral = SSSP_FLAG_LITERAL;
constexpr uint32_t kFlagVec = 1u << 16;  // rows are 16-byte aligned: 128-bit loads

struct SolveArgs {
    const int32_t* W;
    int64_t ld;
    int32_t n;
    int32_t src;
    int32_t* dist;
    int32_t* pred;
    uint32_t flags;
    Ctl* ctl;
};

hipError_t launch_single(const SolveArgs& a, int threads, hipStream_t s);
int max_single_n();

// plain: ordinary launch of the same kernel, the grid already bounded by the
// occupancy query (co-resident on an otherwise idle GPU), instead of a
// cooperative launch; used for profiler runs.
hipError_t launch_grid(const SolveArgs& a, int nwg, int S, long long timeout, Pub* pubs,
                       int32_t* lists, bool plain, hipStream_t s);
int max_grid_slice();
int grid_occupancy(int slice, int* per_cu);

hipError_t launch_batch(const sssp_instance* d_inst, int32_t count, const int32_t* d_order,
                        uint32_t flags, Ctl* ctl, int threads, int nwg, hipStream_t s);
int batch_occupancy(int threads, int* per_cu);
int max_batch_n(int threads);

size_t ctl_size();
size_t pub_size();

}  // namespace sssp
