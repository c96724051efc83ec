// C ABI of libsssp: argument validation, kernel choice, per-(device, stream)
// scratch, status readback.  No exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "engine.h"
#include "sssp_internal.h"

namespace sssp {
namespace {

thread_local std::string t_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(SSSP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

struct DeviceInfo {
    int cus = 0;
    long long clock_khz = 0;  // wall_clock64 rate
};

struct Scratch {
    int device = -1;
    hipStream_t stream = nullptr;
    Ctl* ctl = nullptr;
    char* words = nullptr;  // exchange records and lists of the whole-GPU solves (grid_words_bytes)
    size_t words_cap = 0;
    bool launched = false;
};

std::mutex g_mu;
std::vector<std::unique_ptr<Scratch>> g_scratch;
std::vector<DeviceInfo> g_dev;

int device_info(int dev, DeviceInfo& out) {
    if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
    DeviceInfo& di = g_dev[dev];
    if (di.cus == 0) {
        int cus = 0, rate = 0;
        hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute(CUs)");
        e = hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev);
        if (e != hipSuccess || rate <= 0) rate = 100000;  // 100 MHz, the gfx9 constant clock
        di.cus = cus;
        di.clock_khz = rate;
    }
    out = di;
    return SSSP_OK;
}

// Scratch of (current device, stream); created on first use.  Caller holds g_mu.
int get_scratch(hipStream_t stream, Scratch** out, DeviceInfo* info) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (info) {
        int rc = device_info(dev, *info);
        if (rc) return rc;
    }
    for (auto& s : g_scratch)
        if (s->device == dev && s->stream == stream) {
            *out = s.get();
            return SSSP_OK;
        }
    auto s = std::make_unique<Scratch>();
    s->device = dev;
    s->stream = stream;
    e = hipMalloc(&s->ctl, ctl_size());
    if (e != hipSuccess) return fail(SSSP_ENOMEM, "hipMalloc(control block): %s", hipGetErrorString(e));
    e = hipMemset(s->ctl, 0, ctl_size());
    if (e != hipSuccess) return hip_fail(e, "hipMemset(control block)");
    *out = s.get();
    g_scratch.push_back(std::move(s));
    return SSSP_OK;
}

// Grow a device buffer; waits for earlier work on the stream before freeing.
template <class X>
int ensure(Scratch* sc, X*& p, size_t& cap, size_t need, const char* what) {
    if (cap >= need && p) return SSSP_OK;
    if (p) {
        hipError_t e = hipStreamSynchronize(sc->stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    size_t n = std::max(need, cap * 2);
    hipError_t e = hipMalloc(&p, n * sizeof(X));
    if (e != hipSuccess) return fail(SSSP_ENOMEM, "hipMalloc(%s, %zu bytes): %s", what, n * sizeof(X),
                                     hipGetErrorString(e));
    // stamped records must start without stamps (see gang_exchange)
    e = hipMemset(p, 0, n * sizeof(X));
    if (e != hipSuccess) return hip_fail(e, "hipMemset(scratch)");
    cap = n;
    return SSSP_OK;
}

// Grid-barrier wait limit, SSSP_BARRIER_TIMEOUT_US microseconds (default 10 s).
// A wait that exceeds it ends the solve with SSSP_STATUS_TIMEOUT instead of
// hanging; 0 makes every wait give up at once (used to test that path).
long long barrier_timeout_ticks(const DeviceInfo& di) {
    long long us = 10000000;
    if (const char* s = getenv("SSSP_BARRIER_TIMEOUT_US")) {
        char* end = nullptr;
        long long v = strtoll(s, &end, 10);
        if (end != s && v >= 0) us = v;
    }
    return di.clock_khz * us / 1000;
}

// SSSP_GRID_LAUNCH=plain: launch the whole-GPU kernel with an ordinary launch
// (grid bounded by the occupancy query) instead of a cooperative one; profilers
// that cannot finish after cooperative launches need it.
bool plain_grid_launch() {
    const char* s = getenv("SSSP_GRID_LAUNCH");
    return s && strcmp(s, "plain") == 0;
}

int single_crossover() {
    if (const char* s = getenv("SSSP_SINGLE_MAX_N")) {
        int v = atoi(s);
        if (v > 0) return v;
    }
    return 1024;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

int check_solve_args(const int32_t* W, int64_t ld, int32_t n, int32_t src, const int32_t* dist,
                     const int32_t* pred) {
    if (!W || !dist || !pred) return fail(SSSP_EINVAL, "null buffer (W=%p dist=%p pred=%p)", (const void*)W,
                                          (const void*)dist, (const void*)pred);
    if (n < 1) return fail(SSSP_EINVAL, "n must be >= 1 (got %d)", n);
    if (ld < n) return fail(SSSP_EINVAL, "ld (%lld) must be >= n (%d)", (long long)ld, n);
    if (src < 0 || src >= n) return fail(SSSP_EINVAL, "src %d outside [0, %d)", src, n);
    return SSSP_OK;
}

// Device bytes held by one scratch block.
size_t block_bytes(const Scratch& s) {
    return (s.ctl ? ctl_size() : 0) + s.words_cap;
}

// Waits for the block's stream, then frees its device memory.  Caller holds g_mu.
void free_block(Scratch& s) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != s.device) (void)hipSetDevice(s.device);
    (void)hipStreamSynchronize(s.stream);
    (void)hipFree(s.ctl);
    (void)hipFree(s.words);
    s.ctl = nullptr;
    s.words = nullptr;
    s.words_cap = 0;
    if (cur >= 0 && cur != s.device) (void)hipSetDevice(cur);
}

}  // namespace

// Shape of a whole-GPU solve of n vertices: nwg workgroups of S columns each
// (S a multiple of 4, nwg * S >= n).  About 64 columns (256 B of each row) per
// workgroup by default, as many workgroups as are co-resident; wider slices
// when n outgrows the grid.  workgroups > 0 asks for that many; one_wg forces a
// single workgroup (the label-correcting solve on one workgroup).
int grid_shape(int32_t n, int workgroups, bool lc, bool one_wg, int cus, int* nwg_out, int* S_out) {
    int per_cu = 0;
    int want = workgroups > 0 ? workgroups : (int)std::max<int64_t>(1, ((int64_t)n + 63) / 64);
    if (one_wg) want = 1;
    int S = (int)(((int64_t)n + want - 1) / want);
    S = (S + 3) & ~3;
    if (S > max_grid_slice()) S = max_grid_slice();
    int nwg = (int)(((int64_t)n + S - 1) / S);
    hipError_t e = (hipError_t)(lc ? lc_occupancy(S, &per_cu) : grid_occupancy(S, &per_cu));
    if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    const int cap = std::min(1024, per_cu * cus);
    if (nwg > cap) {
        nwg = cap;
        S = (int)(((int64_t)n + nwg - 1) / nwg);
        S = (S + 3) & ~3;
        if (S > max_grid_slice())
            return fail(SSSP_EUNSUPPORTED, "n=%d needs more than %d co-resident workgroups", n, cap);
        nwg = (int)(((int64_t)n + S - 1) / S);
    }
    *nwg_out = nwg;
    *S_out = S;
    return SSSP_OK;
}

// Compute units and wall-clock rate of the current device (cached; allocates nothing).
int device_props(int* cus, long long* clock_khz) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceInfo di;
    int rc = device_info(dev, di);
    if (rc) return rc;
    *cus = di.cus;
    *clock_khz = di.clock_khz;
    return SSSP_OK;
}

// The one-workgroup / whole-GPU crossover of the default solve.
int single_max_default() { return single_crossover(); }

// Argument checks shared by every dense entry point (message set on failure).
int check_dense_args(const int32_t* W, int64_t ld, int32_t n, int32_t src, const int32_t* dist,
                     const int32_t* pred) {
    return check_solve_args(W, ld, n, src, dist, pred);
}

namespace {

int solve(const int32_t* W, int64_t ld, int32_t n, int32_t src, int32_t* dist, int32_t* pred,
          uint32_t flags, const sssp_tuning* tuning, hipStream_t stream) {
    int rc = check_solve_args(W, ld, n, src, dist, pred);
    if (rc) return rc;
    if ((flags & SSSP_FLAG_SINGLE) && (flags & SSSP_FLAG_GRID))
        return fail(SSSP_EINVAL, "SSSP_FLAG_SINGLE and SSSP_FLAG_GRID are exclusive");
    if ((flags & SSSP_FLAG_LABEL_CORRECTING) && (flags & SSSP_FLAG_LITERAL))
        return fail(SSSP_EINVAL, "SSSP_FLAG_LABEL_CORRECTING and SSSP_FLAG_LITERAL are exclusive");
    const bool lc = (flags & SSSP_FLAG_LABEL_CORRECTING) != 0;
    std::lock_guard<std::mutex> lk(g_mu);
    Scratch* sc = nullptr;
    DeviceInfo di;
    rc = get_scratch(stream, &sc, &di);
    if (rc) return rc;
    SolveArgs a{W, ld, n, src, dist, pred, flags & SSSP_FLAG_LITERAL, sc->ctl};
    if (aligned16(W) && ld % 4 == 0) a.flags |= kFlagVec;
    const bool single = !lc && ((flags & SSSP_FLAG_SINGLE) ||
                                (!(flags & SSSP_FLAG_GRID) && n <= single_crossover()));
    hipError_t e;
    if (single) {
        if (n > max_single_n())
            return fail(SSSP_EUNSUPPORTED, "n=%d exceeds the one-workgroup limit %d", n, max_single_n());
        int threads = tuning && tuning->threads ? tuning->threads : (n <= 1024 ? 256 : 1024);
        e = launch_single(a, threads, stream);
        if (e != hipSuccess) return hip_fail(e, "launch(one-workgroup solve)");
    } else {
        int nwg = 0, S = 0;
        rc = grid_shape(n, tuning && tuning->workgroups ? tuning->workgroups : 0, lc, lc && (flags & SSSP_FLAG_SINGLE),
                        di.cus, &nwg, &S);
        if (rc) return rc;
        rc = ensure(sc, sc->words, sc->words_cap, grid_words_bytes(nwg, S), "exchange records and lists");
        if (rc) return rc;
        if (lc) {
            e = launch_lc(a, nwg, S, barrier_timeout_ticks(di), sc->words, plain_grid_launch(), stream);
            if (e != hipSuccess) return hip_fail(e, "cooperative launch(label-correcting solve)");
        } else {
            const int32_t bal = tuning ? tuning->balance : 0;
            const bool balance = bal > 0 || (bal == 0 && n >= kGridBalanceMinN);
            e = launch_grid(a, nwg, S, barrier_timeout_ticks(di), sc->words, plain_grid_launch(), balance, stream);
            if (e != hipSuccess) return hip_fail(e, "cooperative launch(whole-GPU solve)");
        }
    }
    sc->launched = true;
    return SSSP_OK;
}

}  // namespace

// Records an error message for sssp_last_error() (used by the other sources).
int set_error(int code, const char* msg) {
    t_err = msg;
    return code;
}

const char* last_error_text() { return t_err.c_str(); }

// Control block of (current device, stream), marked as used by a launch that
// the caller is about to enqueue; its stats are what sssp_last_status reports.
// Launch mode and barrier wait limit of the other persistent grids (the CSR
// solve), from the same environment settings as the dense whole-GPU solve.
bool grid_launch_is_plain() { return plain_grid_launch(); }
long long grid_barrier_ticks(long long clock_khz) {
    DeviceInfo di;
    di.clock_khz = clock_khz;
    return barrier_timeout_ticks(di);
}

int stream_ctl(hipStream_t stream, Ctl** out, int* cus, long long* clock_khz) {
    std::lock_guard<std::mutex> lk(g_mu);
    Scratch* sc = nullptr;
    DeviceInfo di;
    int rc = get_scratch(stream, &sc, &di);
    if (rc) return rc;
    sc->launched = true;
    *out = sc->ctl;
    if (cus) *cus = di.cus;
    if (clock_khz) *clock_khz = di.clock_khz;
    return SSSP_OK;
}

int check_instance(const sssp_instance& I, int idx) {
    int rc = check_solve_args(I.W, I.ld, I.n, I.src, I.dist, I.pred);
    if (rc) return fail(rc, "instance %d: %s", idx, t_err.c_str());
    return SSSP_OK;
}

}  // namespace sssp

using namespace sssp;

extern "C" {

int sssp_version(void) { return 1; }

const char* sssp_last_error(void) { return t_err.c_str(); }

const char* sssp_strerror(int code) {
    switch (code) {
        case SSSP_OK: return "ok";
        case SSSP_EINVAL: return "invalid argument";
        case SSSP_EDEVICE: return "HIP runtime error";
        case SSSP_ENOMEM: return "out of device memory";
        case SSSP_EAGAIN: return "try again";
        case SSSP_ENOGRAPH: return "unknown graph";
        case SSSP_ETIMEDOUT: return "timed out";
        case SSSP_EUNSUPPORTED: return "unsupported size or shape";
        default: return "unknown error";
    }
}

int sssp_dense_solve(const int32_t* W, int32_t n, int32_t src, int32_t* dist, int32_t* pred, void* stream) {
    return solve(W, n, n, src, dist, pred, 0u, nullptr, (hipStream_t)stream);
}

int sssp_dense_solve_ex(const int32_t* W, int64_t ld, int32_t n, int32_t src, int32_t* dist, int32_t* pred,
                        uint32_t flags, const sssp_tuning* tuning, void* stream) {
    return solve(W, ld, n, src, dist, pred, flags, tuning, (hipStream_t)stream);
}

int sssp_last_status(void* stream, int32_t* status, int64_t* stats) {
    if (!status) return fail(SSSP_EINVAL, "status is NULL");
    Ctl c;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        Scratch* sc = nullptr;
        int rc = get_scratch((hipStream_t)stream, &sc, nullptr);
        if (rc) return rc;
        if (!sc->launched) return fail(SSSP_EINVAL, "nothing was launched on this stream");
        hipError_t e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        e = hipMemcpy(&c, sc->ctl, sizeof c, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(control block)");
    }
    *status = (int32_t)c.status;
    if (stats)
        for (int i = 0; i < kStatCount; ++i) stats[i] = (int64_t)c.last[i];
    return SSSP_OK;
}

int sssp_last_trace(void* stream, int64_t* t_ns, int32_t* rows, int32_t cap, int32_t* count) {
    if (!count || cap < 0 || (cap > 0 && (!t_ns || !rows))) return fail(SSSP_EINVAL, "bad trace buffers");
    Ctl c;
    DeviceInfo di;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        Scratch* sc = nullptr;
        int rc = get_scratch((hipStream_t)stream, &sc, &di);
        if (rc) return rc;
        if (!sc->launched) return fail(SSSP_EINVAL, "nothing was launched on this stream");
        hipError_t e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        e = hipMemcpy(&c, sc->ctl, sizeof c, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(control block)");
    }
    const int32_t nr = (int32_t)std::min<uint32_t>(c.trace_n, kTraceCap);
    const int32_t k = std::min(nr + 1, cap);
    for (int32_t i = 0; i < k; ++i) {
        t_ns[i] = (int64_t)((c.trace_t[i] - c.trace_t[0]) * 1000000.0 / (double)di.clock_khz);
        rows[i] = i < nr ? (int32_t)c.trace_m[i] : -1;
    }
    *count = nr;
    return SSSP_OK;
}


int32_t sssp_single_max_n(void) { return max_single_n(); }

int sssp_stream_release(void* stream) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_mu);
    for (size_t i = 0; i < g_scratch.size(); ++i)
        if (g_scratch[i]->device == dev && g_scratch[i]->stream == (hipStream_t)stream) {
            free_block(*g_scratch[i]);
            g_scratch.erase(g_scratch.begin() + (std::ptrdiff_t)i);
            break;
        }
    return SSSP_OK;
}

int sssp_release_all(void) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (auto& s : g_scratch) free_block(*s);
        g_scratch.clear();
    }
    return release_read_counters();
}

int sssp_scratch_bytes(int64_t* bytes) {
    if (!bytes) return fail(SSSP_EINVAL, "bytes is NULL");
    int64_t total = 0;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (auto& s : g_scratch) total += (int64_t)block_bytes(*s);
    }
    *bytes = total + read_counter_bytes();
    return SSSP_OK;
}

}  // extern "C"
