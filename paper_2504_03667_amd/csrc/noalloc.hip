// Dense solve for callers that cannot allocate device memory: the library
// scratch of a whole-GPU solve (control block, exchange records, bucket lists)
// lives in one fixed device array per GPU instead of per-stream allocations.
// The kernels are those of sssp_dense_solve_ex (kernels.hip); only where their
// scratch comes from differs.
#include <hip/hip_runtime.h>

#include <mutex>

#include "engine.h"
#include "sssp_internal.h"

namespace sssp {
int set_error(int code, const char* msg);                                      // api.cpp
int check_dense_args(const int32_t* W, int64_t ld, int32_t n, int32_t src, const int32_t* dist,
                     const int32_t* pred);                                     // api.cpp
int grid_shape(int32_t n, int workgroups, bool lc, bool one_wg, int cus, int* nwg, int* S);  // api.cpp
int device_props(int* cus, long long* clock_khz);                              // api.cpp
int single_max_default();                                                      // api.cpp
bool grid_launch_is_plain();                                                   // api.cpp
long long grid_barrier_ticks(long long clock_khz);                             // api.cpp
}  // namespace sssp

namespace {

using namespace sssp;

// Layout of the array: the control block, then the gang's exchange memory
// (records, lists and partial keys, grid_words_bytes(nwg, S) bytes: 24 bytes
// per slice column beyond the records).  With slices of S columns rounded up
// to a multiple of 4, nwg * S < n + 4 * nwg.
constexpr size_t kCtlBytes = 8192;
constexpr size_t kScratchBytes = SSSP_NOALLOC_SCRATCH_BYTES;
static_assert(sizeof(Ctl) <= kCtlBytes, "control block outgrew its place in the fixed scratch");
static_assert(kCtlBytes + grid_words_bytes(1024, 0) + 24ull * (SSSP_NOALLOC_MAX_N + 4 * 1024) <= kScratchBytes,
              "exchange memory of the largest admitted n must fit (24 bytes per slice column)");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_base[kMaxDevices];  // device address of `scratch` on each device (null until set up)

}  // namespace

// The fixed scratch.  In host code this name is only a stand-in for the
// symbol: its device address (one per GPU) comes from hipGetSymbolAddress and
// is what every launch and fill below uses.
static __device__ __align__(256) unsigned char scratch[SSSP_NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of the current device's copy of `scratch`, looked up once per
// device with that device current.
int scratch_base(char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(SSSP_EDEVICE, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices) return set_error(SSSP_EUNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_base[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return set_error(SSSP_EDEVICE, "hipGetSymbolAddress(scratch) failed");
        g_base[dev] = static_cast<char*>(p);
    }
    *out = g_base[dev];
    return SSSP_OK;
}

__global__ void k_copy_status(const Ctl* __restrict__ ctl, int32_t* __restrict__ status) {
    if (threadIdx.x == 0) *status = (int32_t)ctl->status;
}

}  // namespace

extern "C" int sssp_dense_solve_noalloc(const int32_t* W, int64_t ld, int32_t n, int32_t src, int32_t* dist,
                                        int32_t* pred, uint32_t flags, int32_t* status, void* stream) {
    int rc = check_dense_args(W, ld, n, src, dist, pred);
    if (rc) return rc;
    if ((flags & SSSP_FLAG_SINGLE) && (flags & SSSP_FLAG_GRID))
        return set_error(SSSP_EINVAL, "SSSP_FLAG_SINGLE and SSSP_FLAG_GRID are exclusive");
    if (flags & SSSP_FLAG_LABEL_CORRECTING)
        return set_error(SSSP_EUNSUPPORTED, "sssp_dense_solve_noalloc: the label-correcting method is not offered");
    if (n > SSSP_NOALLOC_MAX_N)
        return set_error(SSSP_EUNSUPPORTED, "sssp_dense_solve_noalloc: n above SSSP_NOALLOC_MAX_N (262144)");
    hipStream_t s = (hipStream_t)stream;
    char* base = nullptr;
    rc = scratch_base(&base);
    if (rc) return rc;
    int cus = 0;
    long long khz = 0;
    rc = device_props(&cus, &khz);
    if (rc) return rc;
    Ctl* ctl = reinterpret_cast<Ctl*>(base);
    SolveArgs a{W, ld, n, src, dist, pred, flags & SSSP_FLAG_LITERAL, ctl};
    if (((uintptr_t)W & 15u) == 0 && ld % 4 == 0) a.flags |= kFlagVec;
    const bool single = (flags & SSSP_FLAG_SINGLE) || (!(flags & SSSP_FLAG_GRID) && n <= single_max_default());
    hipError_t e;
    if (single) {
        if (n > max_single_n()) return set_error(SSSP_EUNSUPPORTED, "n exceeds the one-workgroup limit");
        // the one-workgroup kernel only writes the control block's status and statistics
        e = launch_single(a, n <= 1024 ? 256 : 1024, s);
        if (e != hipSuccess) return set_error(SSSP_EDEVICE, "launch of the one-workgroup solve failed");
    } else {
        int nwg = 0, S = 0;
        rc = grid_shape(n, 0, false, false, cus, &nwg, &S);
        if (rc) return rc;
        if (nwg > 1024 || kCtlBytes + grid_words_bytes(nwg, S) > kScratchBytes)
            return set_error(SSSP_EUNSUPPORTED, "sssp_dense_solve_noalloc: launch shape exceeds the fixed scratch");
        // The array keeps whatever the last call left: clear the control block
        // (barrier words, epoch, statistics) and the stamped records this launch
        // polls, with a fill kernel.  The tagged records and lists are cleared by
        // the solve itself before its first exchange.
        e = zero_fill(base, kCtlBytes + gang_recs_offset(nwg), s);
        if (e == hipSuccess)
            e = launch_grid(a, nwg, S, grid_barrier_ticks(khz), base + kCtlBytes, grid_launch_is_plain(),
                            n >= kGridBalanceMinN, s);
        if (e != hipSuccess) return set_error(SSSP_EDEVICE, "launch of the whole-GPU solve failed");
    }
    if (status) {
        hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, s, ctl, status);
        e = hipGetLastError();
        if (e != hipSuccess) return set_error(SSSP_EDEVICE, "launch of the status copy failed");
    }
    return SSSP_OK;
}
