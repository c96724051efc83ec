// Continuous-batching server around the persistent serving kernel (k_serve).
//
// The host side of the serving path: graphs stay resident in HBM (borrowed
// device pointers), submitted (graph, source) queries wait in a FIFO until
// they fit — a free query slot, room in the descriptor ring and, for queries
// solved by a gang of workgroups, room for the gang's exchange records in the
// scratch arena (memory-footprint admission) — and are then published into the
// ring that the running kernel's idle workgroups poll.  Queries that arrive
// while others run are admitted as slots and memory free up and run
// concurrently on the GPU.  A host thread admits, collects completion records
// written by the GPU into pinned memory, timestamps them, and keeps a
// heartbeat that the kernel watches so it leaves if the host goes away.  A
// gang query's split follows the queue: narrower slices when nothing waits
// behind it (latency), wider ones behind a backlog (throughput).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "engine.h"
#include "sssp_internal.h"

namespace sssp {
int set_error(int code, const char* msg);  // api.cpp
}

using namespace sssp;

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

int err(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return set_error(code, buf);
}

struct Graph {
    const int32_t* W;  // the caller's matrix
    int64_t ld;
    int32_t n;
    const void* Ws;    // what is streamed: W, or the server's compact copy
    int64_t lds;
    int32_t elem;
    void* owned;       // compact copy to free on destroy
    int32_t lc_forced = 0;   // every query label-correcting
    int32_t max_rounds = 0;  // most rounds a completed Dijkstra query of it took
    int32_t lc_cheaper = -1; // cost model on its first completed Dijkstra query (-1: none yet)
};

enum { kPending = 0, kRunning = 1, kDone = 2 };

struct Query {
    int32_t graph, src;
    int32_t* dist;
    int32_t* pred;
    int32_t state = kPending;
    int32_t parts = 1, S = 0;
    int32_t method = kMethodDijkstra;
    int32_t qslot = -1;
    uint64_t off = 0, bytes = 0;
    int64_t t_submit = 0, t_admit = 0, t_done = 0;
    int32_t status = 0, rounds = 0;
    int64_t settled = 0;
    bool replanned = false;  // admission has considered the latency-mode split
};

// First-fit allocator over the scratch arena.
struct Arena {
    std::map<uint64_t, uint64_t> free_;  // offset -> size
    void reset(uint64_t bytes) {
        free_.clear();
        if (bytes) free_[0] = bytes;
    }
    bool alloc(uint64_t bytes, uint64_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const uint64_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

}  // namespace

// Host policy of the server, free of any device state (so that it can be
// queried and tested without a GPU): configuration defaults, the gang shape of
// a query, and the latency-mode and throughput-mode splits at admission.
namespace {

int normalize(sssp_server_config& c) {
    if (c.ring_slots <= 0) c.ring_slots = 4096;
    if (c.max_inflight <= 0) c.max_inflight = 1024;
    if (c.single_max_n <= 0) c.single_max_n = 4096;
    if (c.gang_columns <= 0) c.gang_columns = 2048;
    if (c.scratch_bytes <= 0) c.scratch_bytes = 256ll << 20;
    if (c.watchdog_ms <= 0) c.watchdog_ms = 2000;
    if (c.idle_park_ms <= 0) c.idle_park_ms = 20;
    if (c.idle_wait_us <= 0) c.idle_wait_us = 1000;
    if (c.lc_rounds == 0) c.lc_rounds = 64;
    if (c.lc_gang_columns <= 0) c.lc_gang_columns = 1024;
    c.lc_gang_columns = (c.lc_gang_columns + 3) & ~3;
    if (c.idle_gang_columns == 0) c.idle_gang_columns = std::max(256, c.gang_columns / 4);
    if (c.idle_gang_columns > 0) c.idle_gang_columns = (c.idle_gang_columns + 3) & ~3;
    if (c.busy_queue <= 0) c.busy_queue = 128;
    if (c.busy_gang_columns > max_serve_slice() || (c.busy_gang_columns > 0 && c.busy_gang_columns % 4))
        return err(SSSP_EINVAL, "busy_gang_columns <= %d (multiple of 4) required", max_serve_slice());
    if (c.single_max_n > max_serve_single_n() || c.gang_columns > max_serve_slice() || c.gang_columns % 4)
        return err(SSSP_EINVAL, "single_max_n <= %d and gang_columns <= %d (multiple of 4) required",
                   max_serve_single_n(), max_serve_slice());
    return SSSP_OK;
}

// Columns per gang member and number of members for an n-vertex query on a
// kernel of nwg workgroups; label-correcting queries are spread over narrow
// slices (their sweeps read several times the rows of a Dijkstra solve).
// `columns` > 0 overrides the configured width.
void gang_shape(const sssp_server_config& cfg, int nwg, int32_t n, int32_t method, int32_t* parts, int32_t* S,
                int32_t columns = 0) {
    const bool lc = method == kMethodLabelCorrecting;
    if (!lc && n <= cfg.single_max_n) {
        *parts = 1;
        *S = n;
        return;
    }
    const int32_t cols = columns > 0 ? columns : lc ? cfg.lc_gang_columns : cfg.gang_columns;
    int64_t p = ((int64_t)n + cols - 1) / cols;
    const int64_t pmin = ((int64_t)n + max_serve_slice() - 1) / max_serve_slice();
    p = std::max<int64_t>(p, std::max<int64_t>(lc ? 1 : 2, pmin));
    p = std::min<int64_t>(p, std::max(2, nwg / 2));
    int64_t s = ((int64_t)n + p - 1) / p;
    s = (s + 3) & ~int64_t(3);
    *parts = (int32_t)(((int64_t)n + s - 1) / s);
    *S = (int32_t)s;
}

uint64_t footprint(int32_t method, int32_t parts, int32_t S) {
    return item_scratch_bytes(method, parts, S);
}

// Latency mode: a gang query that nothing waits behind is split into narrower
// slices (more members, shorter rounds), as narrow as idle_gang_columns allows
// within three quarters of the workgroups minus `busy` (those of the queries in
// flight); under load the wide split keeps the workgroup time per query, and so
// the throughput, lower.  Updates parts / S / bytes when it narrows the split.
void latency_split(const sssp_server_config& cfg, int nwg, int64_t busy, int32_t n, int32_t method, int32_t* parts,
                   int32_t* S, uint64_t* bytes) {
    if (*parts <= 1 || cfg.idle_gang_columns <= 0) return;
    const int64_t budget = (int64_t)nwg * 3 / 4 - busy;
    const int32_t wide = method == kMethodLabelCorrecting ? cfg.lc_gang_columns : cfg.gang_columns;
    int32_t cols = std::min(cfg.idle_gang_columns, wide);
    if (budget > *parts && ((int64_t)n + cols - 1) / cols > budget)
        cols = (int32_t)((((int64_t)n + budget - 1) / budget + 3) & ~int64_t(3));
    int32_t p2 = 0, S2 = 0;
    gang_shape(cfg, nwg, n, method, &p2, &S2, cols);
    const uint64_t b2 = footprint(method, p2, S2);
    if (budget > *parts && p2 > *parts && p2 <= budget && b2 <= (uint64_t)cfg.scratch_bytes) {
        *parts = p2;
        *S = S2;
        *bytes = b2;
    }
}

// Throughput mode: a Dijkstra gang query admitted with at least busy_queue
// queries waiting behind it is split into wider slices (fewer members).  Under
// a backlog the workgroup time per query, not the query's latency, sets the
// throughput, and wider slices cut the per-member cost of every round (the
// exchange and the spread of finish times).  Default width: twice gang_columns
// for the caller's int32 matrices, four times for compact copies (the widths
// that served the most queries per second on the served workload).  Updates
// parts / S / bytes when it widens the split.
void throughput_split(const sssp_server_config& cfg, int nwg, int32_t n, int32_t method, int32_t elem,
                      int32_t* parts, int32_t* S, uint64_t* bytes) {
    if (*parts <= 1 || method != kMethodDijkstra || cfg.busy_gang_columns < 0) return;
    int64_t cols = cfg.busy_gang_columns > 0 ? cfg.busy_gang_columns : (int64_t)cfg.gang_columns * (elem < 4 ? 4 : 2);
    cols = std::min<int64_t>(cols, max_serve_slice()) & ~int64_t(3);
    int32_t p2 = 0, S2 = 0;
    gang_shape(cfg, nwg, n, method, &p2, &S2, (int32_t)cols);
    if (p2 < *parts) {
        *parts = p2;
        *S = S2;
        *bytes = footprint(method, p2, S2);
    }
}

}  // namespace

struct sssp_server {
    int device = 0;
    sssp_server_config cfg{};
    hipStream_t stream = nullptr;
    int nwg = 0;
    long long clock_khz = 100000;
    // pinned host memory shared with the kernel
    ServeControl* ctl = nullptr;
    ServeDesc* ring = nullptr;
    ServeDone* done = nullptr;
    // device memory
    ServeSlot* slots = nullptr;
    Bar* bars = nullptr;
    unsigned long long* head = nullptr;
    char* arena = nullptr;
    // host state, guarded by mu
    std::mutex mu;
    std::condition_variable cv;       // completions
    std::condition_variable wake;     // submissions
    std::vector<Graph> graphs;
    std::vector<Query> queries;       // ticket t is queries[t - 1]
    std::deque<uint64_t> pending;
    std::vector<int32_t> free_slots;
    std::vector<uint64_t> slot_ticket;
    std::vector<int32_t> running;     // query slots in flight
    std::deque<uint64_t> unpolled;
    Arena arena_alloc;
    uint64_t tail = 0;
    int64_t ring_used = 0;            // ring entries of queries in flight
    int64_t launches = 0;
    int64_t completed = 0;
    bool live = false;       // the kernel is (or may still be) running
    bool parking = false;    // park requested; waiting for the kernel to leave
    int64_t last_busy = 0;   // last time work was pending or in flight
    bool quit = false;
    int64_t quit_deadline = 0;  // destroy stops waiting for in-flight queries after this
    bool failed = false;
    std::thread th;

    ServeArgs args() const {
        ServeArgs a;
        a.ctl = ctl;
        a.ring = ring;
        a.ring_slots = cfg.ring_slots;
        a.done = done;
        a.slots = slots;
        a.bars = bars;
        a.head = head;
        a.arena = arena;
        a.timeout = clock_khz * 10000;  // 10 s per gang barrier wait
        a.watchdog = clock_khz * cfg.watchdog_ms;
        return a;
    }

    void plan(int32_t n, int32_t method, int32_t* parts, int32_t* S) const {
        gang_shape(cfg, nwg, n, method, parts, S);
    }

    // Workgroup time of a query of g, from a completed Dijkstra query q: the
    // rounds' exchanges (about 5 us per round for one workgroup, 8 us per member
    // and round for a gang) plus its rows at about 25 GB/s per workgroup; a
    // label-correcting solve is taken as 24 sweeps and 5x the rows (repeated
    // relaxations and the pred pass).  True when label-correcting is clearly
    // cheaper, which also keeps saturation throughput from dropping.
    bool lc_cheaper(const Graph& g, const Query& q) const {
        // both methods priced at their default (wide) split: the query may have
        // run narrower in latency mode, which costs more workgroup time
        int32_t parts = 1, S = 0;
        plan(g.n, kMethodDijkstra, &parts, &S);
        const double row_us = (double)g.n * g.elem / 25e3;  // bytes / (25 GB/s) in us
        const double round_us = parts > 1 ? 8.0 : 5.0;
        const double t_dij = (double)parts * q.rounds * round_us + (double)q.settled * row_us;
        int32_t parts_lc = 1, S_lc = 0;
        plan(g.n, kMethodLabelCorrecting, &parts_lc, &S_lc);
        const double t_lc = (double)parts_lc * 24 * 8.0 + 5.0 * (double)q.settled * row_us;
        return t_lc < 0.8 * t_dij;
    }


    // publish as many pending queries as fit; caller holds mu
    void admit() {
        bool published = false;
        while (!pending.empty()) {
            Query& q = queries[pending.front() - 1];
            if (free_slots.empty()) break;
            if (!q.replanned && pending.size() == 1) {
                q.replanned = true;
                latency_split(cfg, nwg, ring_used, graphs[q.graph].n, q.method, &q.parts, &q.S, &q.bytes);
            } else if (!q.replanned && (int64_t)pending.size() - 1 >= cfg.busy_queue) {
                q.replanned = true;
                throughput_split(cfg, nwg, graphs[q.graph].n, q.method, graphs[q.graph].elem, &q.parts, &q.S,
                                 &q.bytes);
            }
            if (ring_used + q.parts > cfg.ring_slots) break;
            uint64_t off = 0;
            if (q.bytes && !arena_alloc.alloc(q.bytes, &off)) break;
            const int32_t qs = free_slots.back();
            free_slots.pop_back();
            q.qslot = qs;
            q.off = off;
            q.state = kRunning;
            q.t_admit = now_ns();
            slot_ticket[qs] = pending.front();
            const Graph& g = graphs[q.graph];
            for (int32_t j = 0; j < q.parts; ++j) {
                ServeDesc d;
                memset(&d, 0, sizeof d);
                BatchItem& it = d.item;
                it.W = g.Ws;
                it.ld = g.lds;
                it.elem = g.elem;
                it.vec = ((uintptr_t)g.Ws % (4 * (uintptr_t)g.elem)) == 0 && g.lds % 4 == 0;
                it.dist = q.dist;
                it.pred = q.pred;
                it.n = g.n;
                it.src = q.src;
                it.parts = q.parts;
                it.S = q.S;
                it.method = q.method;
                it.scratch_off = off;
                d.part = j;
                d.qslot = (uint32_t)qs;
                d.ticket = pending.front();
                ring[(tail + j) % (uint64_t)cfg.ring_slots] = d;
            }
            tail += (uint64_t)q.parts;
            ring_used += q.parts;
            running.push_back(qs);
            pending.pop_front();
            published = true;
        }
        if (published) __atomic_store_n(&ctl->tail, tail, __ATOMIC_RELEASE);
    }

    // collect completion records; caller holds mu
    bool collect() {
        bool any = false;
        for (size_t i = 0; i < running.size();) {
            const int32_t qs = running[i];
            const uint64_t t = slot_ticket[qs];
            if (__atomic_load_n(&done[qs].ticket, __ATOMIC_ACQUIRE) != t) {
                ++i;
                continue;
            }
            Query& q = queries[t - 1];
            q.t_done = now_ns();
            q.status = (int32_t)done[qs].status;
            q.rounds = (int32_t)done[qs].rounds;
            q.settled = (int64_t)done[qs].settled;
            if (q.method == kMethodDijkstra) {
                Graph& g = graphs[q.graph];
                g.max_rounds = std::max(g.max_rounds, q.rounds);
                if (g.lc_cheaper < 0) g.lc_cheaper = lc_cheaper(g, q) ? 1 : 0;
            }
            q.state = kDone;
            if (q.bytes) arena_alloc.release(q.off, q.bytes);
            ring_used -= q.parts;
            free_slots.push_back(qs);
            unpolled.push_back(t);
            ++completed;
            running[i] = running.back();
            running.pop_back();
            any = true;
        }
        return any;
    }

    bool launch() {
        if (launch_serve(args(), nwg, stream) != hipSuccess) {
            failed = true;
            return false;
        }
        ++launches;
        live = true;
        return true;
    }

    // The server thread.  Keeps the heartbeat, admits, collects completions.
    // After idle_park_ms with nothing pending or in flight it asks the kernel
    // to leave (park) so the device is free for device-wide synchronisation
    // and other work, and launches it again when queries arrive.
    void loop() {
        (void)hipSetDevice(device);
        int64_t last_probe = now_ns();
        last_busy = now_ns();
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            __atomic_add_fetch(&ctl->heartbeat, 1ull, __ATOMIC_RELAXED);
            const int64_t t = now_ns();
            if (parking && hipStreamQuery(stream) == hipSuccess) {
                parking = false;
                live = false;
                __atomic_store_n(&ctl->park, 0u, __ATOMIC_RELEASE);
            }
            if (!pending.empty() || !running.empty()) last_busy = t;
            if (live && !parking && !pending.empty() && running.empty() && hipStreamQuery(stream) == hipSuccess)
                live = false;  // the kernel left (its heartbeat watchdog fired while the server was idle)
            if (!live && !parking && !pending.empty()) launch();
            if (live && !parking) admit();
            if (collect()) {
                cv.notify_all();
                if (live && !parking) admit();
            }
            if (quit && ((pending.empty() && running.empty()) || t > quit_deadline)) break;
            if (live && !parking && pending.empty() && running.empty() &&
                t - last_busy > (int64_t)cfg.idle_park_ms * 1000000) {
                __atomic_store_n(&ctl->park, 1u, __ATOMIC_RELEASE);
                parking = true;
            }
            if (!running.empty() && t - last_probe > 100000000) {
                // the kernel leaves only on stop, park or a stalled heartbeat; if it is
                // gone while queries are in flight, launch it again (claims resume at head)
                last_probe = t;
                if (hipStreamQuery(stream) == hipSuccess) launch();
            }
            if (running.empty() && pending.empty()) {
                wake.wait_for(lk, std::chrono::microseconds(cfg.idle_wait_us));
            } else {
                lk.unlock();
                const int64_t until = now_ns() + 2000;  // poll completions every ~2 us
                while (now_ns() < until) __builtin_ia32_pause();
                lk.lock();
            }
        }
    }
};

namespace {

template <class X>
int dev_alloc(X** p, size_t count, const char* what) {
    hipError_t e = hipMalloc(p, std::max<size_t>(1, count) * sizeof(X));
    if (e != hipSuccess) return err(SSSP_ENOMEM, "hipMalloc(%s): %s", what, hipGetErrorString(e));
    e = hipMemset(*p, 0, std::max<size_t>(1, count) * sizeof(X));
    if (e != hipSuccess) return err(SSSP_EDEVICE, "hipMemset(%s): %s", what, hipGetErrorString(e));
    return SSSP_OK;
}

template <class X>
int host_alloc(X** p, size_t count, const char* what) {
    hipError_t e = hipHostMalloc(p, count * sizeof(X), hipHostMallocCoherent | hipHostMallocMapped);
    if (e != hipSuccess) return err(SSSP_ENOMEM, "hipHostMalloc(%s): %s", what, hipGetErrorString(e));
    memset(*p, 0, count * sizeof(X));
    return SSSP_OK;
}

void release_all(sssp_server* s) {
    for (auto& g : s->graphs)
        if (g.owned) (void)hipFree(g.owned);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    (void)hipHostFree(s->ctl);
    (void)hipHostFree(s->ring);
    (void)hipHostFree(s->done);
    (void)hipFree(s->slots);
    (void)hipFree(s->bars);
    (void)hipFree(s->head);
    (void)hipFree(s->arena);
    delete s;
}

}  // namespace

extern "C" {

int64_t sssp_server_now_ns(void) { return now_ns(); }

int sssp_server_shape(const sssp_server_config* cfg, int32_t workgroups, int32_t n, int32_t method, int32_t elem,
                      int32_t busy, int32_t waiting, int32_t* parts, int32_t* columns, int64_t* scratch_bytes) {
    if (!parts || !columns || workgroups < 1 || n < 1 || (method != kMethodDijkstra && method != kMethodLabelCorrecting) ||
        (elem != 1 && elem != 2 && elem != 4) || busy < 0 || waiting < 0)
        return err(SSSP_EINVAL, "bad arguments (workgroups=%d n=%d method=%d elem=%d busy=%d waiting=%d)", workgroups,
                   n, method, elem, busy, waiting);
    sssp_server_config c{};
    if (cfg) c = *cfg;
    if (int rc = normalize(c)) return rc;
    int32_t p = 0, S = 0;
    gang_shape(c, workgroups, n, method, &p, &S);
    uint64_t bytes = footprint(method, p, S);
    if (bytes > (uint64_t)c.scratch_bytes)
        return err(SSSP_ENOMEM, "query needs %llu scratch bytes, arena has %lld", (unsigned long long)bytes,
                   (long long)c.scratch_bytes);
    if (waiting == 0) latency_split(c, workgroups, busy, n, method, &p, &S, &bytes);
    else if (waiting >= c.busy_queue) throughput_split(c, workgroups, n, method, elem, &p, &S, &bytes);
    *parts = p;
    *columns = S;
    if (scratch_bytes) *scratch_bytes = (int64_t)bytes;
    return SSSP_OK;
}

int sssp_server_create(const sssp_server_config* cfg_in, sssp_server** out) {
    if (!out) return err(SSSP_EINVAL, "out is NULL");
    *out = nullptr;
    sssp_server* s = new sssp_server();
    if (cfg_in) s->cfg = *cfg_in;
    sssp_server_config& c = s->cfg;
    if (int rc = normalize(c)) return release_all(s), rc;
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) return release_all(s), err(SSSP_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    int cus = 0, rate = 0, per_cu = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device);
    if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, s->device) == hipSuccess && rate > 0)
        s->clock_khz = rate;
    if (serve_occupancy(&per_cu) != 0 || per_cu < 1)
        return release_all(s), err(SSSP_EDEVICE, "serving kernel does not fit on a compute unit");
    // by default leave a few compute units to other kernels (the caller's own work,
    // copies done by kernels) so they can run while the server's kernel is resident
    const int reserve = std::max(4, cus / 32);
    s->nwg = c.workgroups > 0 ? std::min(c.workgroups, per_cu * cus) : per_cu * std::max(1, cus - reserve);
    int rc;
    if ((rc = host_alloc(&s->ctl, 1, "control")) || (rc = host_alloc(&s->ring, c.ring_slots, "ring")) ||
        (rc = host_alloc(&s->done, c.max_inflight, "completions")) ||
        (rc = dev_alloc(&s->slots, c.max_inflight, "slots")) ||
        (rc = dev_alloc(&s->bars, (size_t)c.max_inflight, "barriers")) ||
        (rc = dev_alloc(&s->head, 1, "head")) || (rc = dev_alloc(&s->arena, (size_t)c.scratch_bytes, "arena")))
        return release_all(s), rc;
    s->arena_alloc.reset((uint64_t)c.scratch_bytes);
    s->slot_ticket.assign(c.max_inflight, 0);
    for (int32_t i = c.max_inflight - 1; i >= 0; --i) s->free_slots.push_back(i);
    e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return release_all(s), err(SSSP_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    e = hipDeviceSynchronize();  // scratch initialised before the kernel starts
    if (e != hipSuccess) return release_all(s), err(SSSP_EDEVICE, "hipDeviceSynchronize: %s", hipGetErrorString(e));
    if (!s->launch()) return release_all(s), err(SSSP_EDEVICE, "launching the serving kernel failed");
    s->th = std::thread([s] { s->loop(); });
    *out = s;
    return SSSP_OK;
}

int sssp_server_add_graph_ex(sssp_server* s, const int32_t* W, int64_t ld, int32_t n, uint32_t flags,
                             int32_t* graph_id) {
    if (!s || !W || !graph_id) return err(SSSP_EINVAL, "null argument");
    if (n < 1 || ld < n) return err(SSSP_EINVAL, "need n >= 1 and ld >= n (n=%d ld=%lld)", n, (long long)ld);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        int32_t parts, S;
        s->plan(n, kMethodDijkstra, &parts, &S);
        if (S > max_serve_slice()) return err(SSSP_EUNSUPPORTED, "n=%d is too large for this server", n);
    }
    Graph g{W, ld, n, W, ld, 4, nullptr};
    if (flags & SSSP_FLAG_COMPACT) {
        // built on a stream of its own: the server's stream holds the resident kernel
        hipStream_t cs = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e != hipSuccess) return err(SSSP_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        CompactCopy c;
        const int rc = make_compact(W, ld, n, cs, &c);
        (void)hipStreamDestroy(cs);
        if (rc) return rc;
        if (c.elem < 4) g = Graph{W, ld, n, c.data, c.ld, c.elem, c.data};
    }
    g.lc_forced = (flags & SSSP_FLAG_LABEL_CORRECTING) ? 1 : 0;
    std::lock_guard<std::mutex> lk(s->mu);
    s->graphs.push_back(g);
    *graph_id = (int32_t)s->graphs.size() - 1;
    return SSSP_OK;
}

int sssp_server_add_graph(sssp_server* s, const int32_t* W, int64_t ld, int32_t n, int32_t* graph_id) {
    return sssp_server_add_graph_ex(s, W, ld, n, 0u, graph_id);
}

int sssp_server_graph_elem(sssp_server* s, int32_t graph_id, int32_t* elem_bytes) {
    if (!s || !elem_bytes) return err(SSSP_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size()) return err(SSSP_ENOGRAPH, "unknown graph %d", graph_id);
    *elem_bytes = s->graphs[graph_id].elem;
    return SSSP_OK;
}

int sssp_server_submit(sssp_server* s, int32_t graph_id, int32_t src, int32_t* dist, int32_t* pred,
                       uint64_t* ticket) {
    if (!s || !dist || !pred || !ticket) return err(SSSP_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size()) return err(SSSP_ENOGRAPH, "unknown graph %d", graph_id);
    const Graph& g = s->graphs[graph_id];
    if (src < 0 || src >= g.n) return err(SSSP_EINVAL, "src %d outside [0, %d)", src, g.n);
    if (s->quit) return err(SSSP_EINVAL, "server is shutting down");
    if (s->cfg.max_pending > 0 && (int64_t)s->pending.size() >= s->cfg.max_pending)
        return err(SSSP_EAGAIN, "admission queue full (%lld queries)", (long long)s->pending.size());
    Query q;
    q.graph = graph_id;
    q.src = src;
    q.dist = dist;
    q.pred = pred;
    // label-correcting: forced for the graph, or its solves take many rounds and
    // the cost model (unless switched off) finds it cheaper
    const bool lc = g.lc_forced ||
                    (s->cfg.lc_rounds > 0 && g.max_rounds >= s->cfg.lc_rounds && (s->cfg.lc_model < 0 || g.lc_cheaper == 1));
    q.method = lc ? kMethodLabelCorrecting : kMethodDijkstra;
    s->plan(g.n, q.method, &q.parts, &q.S);
    q.bytes = footprint(q.method, q.parts, q.S);
    if (q.bytes > (uint64_t)s->cfg.scratch_bytes)
        return err(SSSP_ENOMEM, "query needs %llu scratch bytes, arena has %lld", (unsigned long long)q.bytes,
                   (long long)s->cfg.scratch_bytes);
    q.t_submit = now_ns();
    s->queries.push_back(q);
    *ticket = s->queries.size();
    s->pending.push_back(*ticket);
    s->wake.notify_one();
    return SSSP_OK;
}

int sssp_server_poll(sssp_server* s, uint64_t* tickets, int32_t cap, int32_t* count) {
    if (!s || !count || cap < 0 || (cap > 0 && !tickets)) return err(SSSP_EINVAL, "bad arguments");
    std::lock_guard<std::mutex> lk(s->mu);
    int32_t k = 0;
    while (k < cap && !s->unpolled.empty()) {
        tickets[k++] = s->unpolled.front();
        s->unpolled.pop_front();
    }
    *count = k;
    return SSSP_OK;
}

int sssp_server_wait(sssp_server* s, uint64_t ticket, int64_t timeout_ns) {
    if (!s) return err(SSSP_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    if (ticket < 1 || ticket > s->queries.size()) return err(SSSP_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::nanoseconds(timeout_ns < 0 ? 0 : timeout_ns);
    while (s->queries[ticket - 1].state != kDone) {
        if (timeout_ns >= 0 && s->cv.wait_until(lk, deadline) == std::cv_status::timeout &&
            s->queries[ticket - 1].state != kDone)
            return err(SSSP_ETIMEDOUT, "query %llu not done", (unsigned long long)ticket);
        if (timeout_ns < 0) s->cv.wait(lk);
    }
    return SSSP_OK;
}

int sssp_server_query_info(sssp_server* s, uint64_t ticket, sssp_query_info* info) {
    if (!s || !info) return err(SSSP_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (ticket < 1 || ticket > s->queries.size()) return err(SSSP_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    const Query& q = s->queries[ticket - 1];
    info->state = q.state;
    info->status = q.status;
    info->parts = q.parts;
    info->rounds = q.rounds;
    info->settled = q.settled;
    info->t_submit_ns = q.t_submit;
    info->t_admit_ns = q.t_admit;
    info->t_done_ns = q.t_done;
    info->method = q.method;
    info->reserved = 0;
    return SSSP_OK;
}

int sssp_server_get_stats(sssp_server* s, sssp_server_stats* st) {
    if (!s || !st) return err(SSSP_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    st->submitted = (int64_t)s->queries.size();
    st->completed = s->completed;
    st->running = (int64_t)s->running.size();
    st->pending = (int64_t)s->pending.size();
    st->kernel_launches = s->launches;
    st->workgroups = s->nwg;
    st->failed = s->failed ? 1 : 0;
    return SSSP_OK;
}

int sssp_server_destroy(sssp_server* s) {
    if (!s) return SSSP_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->quit = true;
        s->quit_deadline = now_ns() + 120ll * 1000000000;  // drain for at most 2 minutes
        s->wake.notify_all();
    }
    if (s->th.joinable()) s->th.join();  // drains: every admitted and pending query completes
    __atomic_store_n(&s->ctl->stop, 1u, __ATOMIC_RELEASE);
    hipError_t e = hipStreamSynchronize(s->stream);
    release_all(s);
    if (e != hipSuccess) return err(SSSP_EDEVICE, "serving kernel: %s", hipGetErrorString(e));
    return SSSP_OK;
}

}  // extern "C"
