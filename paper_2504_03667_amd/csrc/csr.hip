// Graphs stored as adjacency lists (CSR): the paper's sparse family (m = 3n
// edges, Section IV-A) without the n x n matrix whose memory the paper names as
// a weakness (the third point of Section V, the conclusion).  G[u][v] is the
// smallest weight of the edges u -> v; self-loops and weights outside
// [0, INT32_MAX) play no part, exactly as for a matrix built from the same edge
// list.
//
// Such graphs have many distinct distances and few edges, so the solve uses the
// label-correcting method (the paper's CUDA design, Algorithms 3 and 4, made
// deterministic in its results) over edges:
//   * a persistent cooperative grid; sweep k relaxes the edge lists of the
//     vertices whose dist dropped in sweep k-1 (the first frontier is the
//     source) with an agent-scope atomic minimum on the head's running dist;
//     the first lowering of a vertex in a sweep appends it to the next
//     frontier (three frontier lists rotate, so a list is cleared one sweep
//     before it is filled again); a sweep reads each tail's current dist, so
//     the sweep count can vary from run to run, the distances cannot;
//   * every word shared between workgroups is read and written with
//     agent-scope atomics (coherent across XCDs), so the barrier between
//     sweeps needs no cache writeback or invalidate;
//   * once no dist changes, one pass over all edges sets pred[v] to the tail u
//     of smallest (dist[u], u) among tight edges u -> v, u != v: Algorithm 1's
//     pred unless a tight edge has weight 0.  When one does, the order in
//     which Algorithm 1 settles equal distances decides pred, and a pass over
//     the vertices that tight zero-weight edges touch recovers that order
//     exactly (zero_tie_pred below), for any n.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>

#include "engine.h"
#include "sssp.h"
#include "sssp_internal.h"

namespace sssp {
int set_error(int code, const char* msg);                                     // api.cpp
int stream_ctl(hipStream_t stream, Ctl** out, int* cus, long long* clock_khz);  // api.cpp
bool grid_launch_is_plain();                                                    // api.cpp
long long grid_barrier_ticks(long long clock_khz);                              // api.cpp

namespace {

int err(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return set_error(code, buf);
}

constexpr int kCsrThreads = 256;

// Control words of one CSR solve (device memory, zeroed by k_csr_init).
struct CsrCtl {
    uint32_t bar;  // barrier arrivals
    uint32_t pad0[31];
    uint64_t gen;  // (last completed barrier << 32) | the value it hands over
    uint32_t pad1[30];
    uint32_t count[3];    // frontier list sizes of the distance sweeps
    uint32_t zero;        // a tight zero-weight edge was seen
    uint32_t neg;         // a negative weight was seen
    uint32_t nlev;        // zero_tie_pred: levels holding non-plain vertices
    uint32_t next_level;  // zero_tie_pred: levels claimed by workgroups
    uint32_t pad2[24];
};

// Scratch of zero_tie_pred (device memory; n = vertices, H = 2^hbits >= 2n).
struct ZeroTie {
    uint32_t* flags;   // per vertex: kNonPlain | kSeed | kAvail | kDone
    uint32_t* lev;     // per non-plain vertex: the number of its level
    uint32_t* seg;     // the non-plain vertices, grouped by level
    uint32_t* cnt;     // per level: its non-plain vertices
    uint32_t* off;     // per level: where its group starts in seg
    uint32_t* fill;    // per level: vertices placed in its group so far
    uint32_t* md;      // per vertex: smallest dist of a tail of a tight edge into it
    uint64_t* ht_key;  // open-addressing table of the levels' distances (H entries)
    uint32_t* ht_lvl;  // level number of each occupied table entry
    uint32_t hbits;
};

__device__ __forceinline__ bool edge_ok(int32_t u, int32_t v, int32_t w, int32_t n) {
    return v >= 0 && v < n && v != u && w >= 0 && w != (int32_t)kInf;
}

// ---------------------------------------------------------------------------
// Edge list -> CSR.
// ---------------------------------------------------------------------------

// Edges kept: endpoints in [0, n), weight in [0, INT32_MAX), not a self-loop.
__device__ __forceinline__ bool keep_edge(int32_t u, int32_t v, int32_t w, int32_t n) {
    return u >= 0 && u < n && v >= 0 && v < n && u != v && w >= 0 && w != (int32_t)kInf;
}

__global__ void k_csr_degree(const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                             const int32_t* __restrict__ ew, int64_t m, int32_t n, int32_t directed,
                             uint32_t* __restrict__ deg, unsigned long long* __restrict__ bad) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = eu[e], v = ev[e], w = ew[e];
        const bool self = u == v && u >= 0 && u < n && w >= 0 && w != (int32_t)kInf;
        if (!keep_edge(u, v, w, n)) {
            if (!self) atomicAdd(bad, 1ull);  // a valid self-loop is ignored, not an error
            continue;
        }
        atomicAdd(&deg[u], 1u);
        if (!directed) atomicAdd(&deg[v], 1u);
    }
}

// row_ptr[0] = 0, row_ptr[i + 1] = row_ptr[i] + deg[i], in three passes over
// chunks of 1024 vertices: each chunk's total, an exclusive scan of the totals
// (one workgroup), then each chunk's scan plus its offset.
constexpr int kScanChunk = 1024;

// Inclusive scan of one value per thread over a workgroup of kScanChunk
// threads; *total gets the workgroup's sum.
__device__ __forceinline__ unsigned long long wg_inclusive_scan(unsigned long long x, unsigned long long* wsum,
                                                                unsigned long long* total) {
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long y = __shfl_up(x, (unsigned)o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[threadIdx.x >> 6] = x;
    __syncthreads();
    unsigned long long before = 0, sum = 0;
    for (int k = 0; k < kScanChunk / 64; ++k) {
        if (k < (int)(threadIdx.x >> 6)) before += wsum[k];
        sum += wsum[k];
    }
    __syncthreads();  // wsum is reused by the next call
    *total = sum;
    return before + x;
}

__global__ __launch_bounds__(kScanChunk) void k_csr_chunk_sums(const uint32_t* __restrict__ deg, int32_t n,
                                                               unsigned long long* __restrict__ sums) {
    __shared__ unsigned long long wsum[kScanChunk / 64];
    const int64_t i = (int64_t)blockIdx.x * kScanChunk + threadIdx.x;
    unsigned long long total = 0;
    (void)wg_inclusive_scan(i < n ? deg[i] : 0ull, wsum, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of the chunk totals in place; row_ptr[0] = 0.
__global__ __launch_bounds__(kScanChunk) void k_csr_scan_sums(unsigned long long* __restrict__ sums, int32_t chunks,
                                                              int64_t* __restrict__ row_ptr) {
    __shared__ unsigned long long wsum[kScanChunk / 64];
    unsigned long long carry = 0;
    if (threadIdx.x == 0) row_ptr[0] = 0;
    for (int32_t base = 0; base < chunks; base += kScanChunk) {
        const int32_t i = base + (int32_t)threadIdx.x;
        const unsigned long long x = i < chunks ? sums[i] : 0ull;
        unsigned long long total = 0;
        const unsigned long long incl = wg_inclusive_scan(x, wsum, &total);
        if (i < chunks) sums[i] = carry + incl - x;
        carry += total;
    }
}

__global__ __launch_bounds__(kScanChunk) void k_csr_scan_chunks(const uint32_t* __restrict__ deg, int32_t n,
                                                                const unsigned long long* __restrict__ sums,
                                                                int64_t* __restrict__ row_ptr) {
    __shared__ unsigned long long wsum[kScanChunk / 64];
    const int64_t i = (int64_t)blockIdx.x * kScanChunk + threadIdx.x;
    unsigned long long total = 0;
    const unsigned long long incl = wg_inclusive_scan(i < n ? deg[i] : 0ull, wsum, &total);
    if (i < n) row_ptr[i + 1] = (int64_t)(sums[blockIdx.x] + incl);
}

__global__ void k_csr_fill(const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                           const int32_t* __restrict__ ew, int64_t m, int32_t n, int32_t directed,
                           const int64_t* __restrict__ row_ptr, uint32_t* __restrict__ cursor,
                           int32_t* __restrict__ col, int32_t* __restrict__ w) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = eu[e], v = ev[e], wt = ew[e];
        if (!keep_edge(u, v, wt, n)) continue;
        int64_t p = row_ptr[u] + atomicAdd(&cursor[u], 1u);
        col[p] = v;
        w[p] = wt;
        if (!directed) {
            p = row_ptr[v] + atomicAdd(&cursor[v], 1u);
            col[p] = u;
            w[p] = wt;
        }
    }
}

// Sort each row by (head, weight) so that the lists do not depend on the order
// the atomics above took (one thread per row: the rows of the sparse graphs
// this serves are short).
__global__ void k_csr_sort_rows(const int64_t* __restrict__ row_ptr, int32_t n, int32_t* __restrict__ col,
                                int32_t* __restrict__ w) {
    for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
        const int64_t a = row_ptr[u], b = row_ptr[u + 1];
        for (int64_t i = a + 1; i < b; ++i) {
            const int32_t cv = col[i], cw = w[i];
            int64_t j = i - 1;
            while (j >= a && (col[j] > cv || (col[j] == cv && w[j] > cw))) {
                col[j + 1] = col[j];
                w[j + 1] = w[j];
                --j;
            }
            col[j + 1] = cv;
            w[j + 1] = cw;
        }
    }
}

// ---------------------------------------------------------------------------
// Solve.
//
// Labels: a running value (dist) and the sweep that last
// lowered it, packed as (value << 32) | sweep into one 64-bit word.  Sweep
// numbers grow, so an atomic minimum with (c << 32) | k lowers the value
// exactly when c is smaller (a tie keeps the older word), and the word it
// returns tells whether sweep k had already lowered it: only the first
// lowering of a vertex in a sweep appends it to the next frontier.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t label_value(uint64_t x) { return (uint32_t)(x >> 32); }

__global__ void k_csr_init(int32_t n, int32_t src, uint64_t* __restrict__ lab, uint64_t* __restrict__ pkey,
                           uint32_t* __restrict__ lists, CsrCtl* __restrict__ cc) {
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t v = gtid; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        lab[v] = v == src ? 0ull : (uint64_t)kInf << 32;
        pkey[v] = kNoKey;
    }
    if (gtid == 0) {
        lists[0] = (uint32_t)src;
        cc->bar = 0;
        cc->gen = 0ull;
        for (int i = 0; i < 3; ++i) cc->count[i] = i == 0 ? 1u : 0u;
        cc->zero = 0;
        cc->neg = 0;
        cc->nlev = 0;
        cc->next_level = 0;
    }
}

// Grid barrier b of nwg workgroups.  Everything shared goes through agent-scope
// atomics, whose completion each wave waits for before the workgroup barrier,
// so an arrival counter and a release word suffice.  The last workgroup to
// arrive reads *carry (when given: by then every other workgroup's atomics on
// it have completed) and hands it to all in the release word, saving each
// workgroup that read.  false: a wait gave up.
__device__ __forceinline__ bool csr_barrier(CsrCtl* cc, uint32_t b, uint32_t nwg, long long timeout,
                                            const uint32_t* carry = nullptr, uint32_t* value = nullptr) {
    __shared__ uint32_t handed;
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    int late = 0;
    if (threadIdx.x == 0) {
        uint32_t val = 0;
        if (nwg == 1) {
            if (carry) val = ld_agent(carry);
        } else {
            stress_delay(b);
            const uint32_t old = __hip_atomic_fetch_add(&cc->bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (old == b * nwg - 1) {
                if (carry) val = ld_agent(carry);
                st_agent(&cc->gen, ((uint64_t)b << 32) | val);
            } else {
                const long long t0 = wall_clock64();
                unsigned naps = 1;
                uint64_t g = ld_agent(&cc->gen);
                while ((uint32_t)(g >> 32) < b) {
                    for (unsigned i = 0; i < naps; ++i) __builtin_amdgcn_s_sleep(1);
                    if (naps < 8) naps <<= 1;
                    if (wall_clock64() - t0 > timeout) {
                        late = 1;
                        break;
                    }
                    g = ld_agent(&cc->gen);
                }
                val = (uint32_t)g;
            }
        }
        handed = val;
    }
    const bool ok = __syncthreads_or(late) == 0;
    if (value) *value = handed;
    return ok;
}

// Does tail u (dist du) reach head v (dist dv) over an edge of weight wt on a
// shortest path?  Both finite, du + wt == dv (both below 2^31: no wrap).
__device__ __forceinline__ bool tight(uint32_t du, uint32_t dv, int32_t wt) {
    return du < kInf && dv < kInf && du + (uint32_t)wt == dv;
}

// Frontier sweeps over three rotating lists whose sizes are count[0..2]; the
// first frontier (F vertices) is in list 0.  A group of G lanes takes one
// frontier vertex u and walks its edge list G * B edges per step, every load
// and atomic of a step in flight together: value(tail(u), u, v, w, c) says
// whether edge u -> v takes part and gives its candidate c, and an atomic
// minimum of (c << 32) | sweep on lab[v] lowers v; its first lowering in the
// sweep appends v to the next frontier, one counter update per wave and step.
// A list therefore holds a vertex at most once; the list read in one sweep is
// cleared in the next and filled in the one after.  Small frontiers are bound
// by latency: 4 lanes share a vertex so that more waves have work.  Large ones
// are bound by memory operations: a lane walks a whole list, 8 edges per step,
// and first reads each head, skipping the atomic when the edge cannot lower it.
constexpr uint32_t kLargeFrontier = 32768;

template <int G, int B, bool Filter, class Tail, class Value>
__device__ __forceinline__ void sweep_frontier(const uint32_t* __restrict__ list, uint32_t F,
                                               uint32_t* __restrict__ next, uint32_t* __restrict__ next_count,
                                               uint64_t* __restrict__ lab, const int64_t* __restrict__ row_ptr,
                                               const int32_t* __restrict__ col, const int32_t* __restrict__ w,
                                               uint32_t tag, Tail& tail, Value& value) {
    const int lane = threadIdx.x & (kWave - 1);
    const int sub = lane % G;
    const int64_t per_wave = kWave / G;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x / kWave) * per_wave;
    for (int64_t i0 = wave * per_wave; i0 < (int64_t)F; i0 += stride) {  // the same trip count in a wave
        const int64_t i = i0 + lane / G;
        int32_t u = 0;
        decltype(tail(0)) tv{};
        int64_t e = 0, e1 = 0;
        if (i < (int64_t)F) {
            u = (int32_t)ld_agent(&list[i]);
            tv = tail(u);
            e = row_ptr[u] + sub;
            e1 = row_ptr[u + 1];
        }
        while (__ballot(e < e1)) {
            int32_t v[B];
            uint32_t c[B];
            uint64_t before[B];
            bool part[B];
#pragma unroll
            for (int j = 0; j < B; ++j) {
                const int64_t ej = e + (int64_t)j * G;
                part[j] = false;
                v[j] = 0;
                c[j] = 0;
                if (ej < e1) {
                    v[j] = col[ej];
                    part[j] = value(tv, u, v[j], w[ej], c[j]);
                }
            }
            if (Filter) {
                uint64_t now[B];
#pragma unroll
                for (int j = 0; j < B; ++j) now[j] = part[j] ? ld_agent(&lab[v[j]]) : 0ull;
#pragma unroll
                for (int j = 0; j < B; ++j) part[j] = part[j] && c[j] < label_value(now[j]);
            }
#pragma unroll
            for (int j = 0; j < B; ++j)
                before[j] = part[j] ? __hip_atomic_fetch_min(&lab[v[j]], ((uint64_t)c[j] << 32) | tag, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT)
                                    : 0ull;
            uint32_t want = 0;
#pragma unroll
            for (int j = 0; j < B; ++j)
                want |= (part[j] && c[j] < label_value(before[j]) && (uint32_t)before[j] != tag ? 1u : 0u) << j;
            const uint32_t mine = (uint32_t)__popc(want);
            const uint32_t incl = wave_scan32(mine);
            const uint32_t total = __shfl(incl, kWave - 1, kWave);
            if (total) {
                uint32_t base = 0;
                if (lane == kWave - 1)
                    base = __hip_atomic_fetch_add(next_count, total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                uint32_t pos = __shfl(base, kWave - 1, kWave) + incl - mine;
#pragma unroll
                for (int j = 0; j < B; ++j)
                    if (want >> j & 1u) st_agent(&next[pos++], (uint32_t)v[j]);
            }
            e += (int64_t)G * B;
        }
    }
}

// The barrier that ends a sweep hands over the next frontier's size.  Stops at
// an empty frontier; false if a barrier wait gave up.
template <class Tail, class Value>
__device__ bool frontier_sweeps(uint32_t* __restrict__ count, uint32_t* __restrict__ lists,
                                uint64_t* __restrict__ lab, const int64_t* __restrict__ row_ptr,
                                const int32_t* __restrict__ col, const int32_t* __restrict__ w, int32_t n, CsrCtl* cc,
                                uint32_t& b, long long timeout, uint32_t F, unsigned long long& sweeps,
                                unsigned long long& rows, Tail tail, Value value) {
    const uint32_t nwg = gridDim.x;
    for (uint32_t k = 0; F != 0; ++k) {
        const uint32_t cur = k % 3, nxt = (k + 1) % 3, old = (k + 2) % 3;
        ++sweeps;
        rows += F;
        if (blockIdx.x == 0 && threadIdx.x == 0) st_agent(&count[old], 0u);
        const uint32_t tag = k + 1;
        const uint32_t* list = lists + (size_t)cur * n;
        uint32_t* next = lists + (size_t)nxt * n;
        if (F >= kLargeFrontier)
            sweep_frontier<1, 8, true>(list, F, next, &count[nxt], lab, row_ptr, col, w, tag, tail, value);
        else
            sweep_frontier<4, 2, false>(list, F, next, &count[nxt], lab, row_ptr, col, w, tag, tail, value);
        if (!csr_barrier(cc, ++b, nwg, timeout, &count[nxt], &F)) return false;
    }
    return true;
}

// Calls f(v[], w[], ok[]) for the edges of u, kBatch at a time, after loading
// them together; ok marks the edges that take part (edge_ok).
constexpr int kBatch = 4;
template <class F>
__device__ __forceinline__ void for_edges(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                          const int32_t* __restrict__ w, int32_t n, int32_t u, F f) {
    const int64_t e1 = row_ptr[u + 1];
    for (int64_t e = row_ptr[u]; e < e1; e += kBatch) {
        int32_t v[kBatch], wt[kBatch];
        bool ok[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            v[j] = 0;
            wt[j] = -1;
            if (e + j < e1) {
                v[j] = col[e + j];
                wt[j] = w[e + j];
            }
            ok[j] = e + j < e1 && edge_ok(u, v[j], wt[j], n);
        }
        f(v, wt, ok);
    }
}

// pred when tight zero-weight edges exist, from the exact distances alone
// (every workgroup of the grid calls it; b counts the grid barriers).
//
// Algorithm 1 settles vertices in order of distance, and within one distance
// (a level) it settles the lowest-index vertex whose dist already equals that
// distance: the seeds (the source, and heads of tight edges of positive weight,
// whose tails lie in lower levels) from the start, and the heads of tight
// zero-weight edges once their tail has settled.  pred[v] is the tail of the
// tight edge into v that settled first.  Vertices touched by no tight
// zero-weight edge inside their level ("plain") are seeds that make nothing
// available, so only the others ("non-plain") need a sequential pass, one
// level per workgroup: it settles them one at a time as Algorithm 1 would,
// y_1, y_2, ..., and a plain vertex p settles before y_i exactly when
// p < max(y_1 .. y_i).  Hence within a level the settle order is the order of
// the 64-bit keys p << 32 for plain p and (max(y_1 .. y_i) << 32) | i for y_i,
// and pred[v] is the tail u of smallest (dist[u], key[u]) over tight edges
// u -> v, u != v: found by a minimum of dist[u], then of key[u] among those
// tails, then the tail whose key won.  The non-plain vertices are grouped by
// level through an open-addressing table of the levels' distances.
constexpr uint32_t kNonPlain = 1u, kSeed = 2u, kAvail = 4u, kDone = 8u;
constexpr uint64_t kEmpty = ~0ull;

__device__ __forceinline__ uint32_t level_slot(uint32_t d, uint32_t hbits) {
    return (d * 2654435761u) >> (32 - hbits);
}

template <int T>
__device__ bool zero_tie_pred(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                              const int32_t* __restrict__ w, int32_t n, int32_t src, const uint64_t* __restrict__ lab,
                              uint64_t* __restrict__ rk, uint64_t* __restrict__ pk, const ZeroTie& zt, CsrCtl* cc,
                              uint32_t& b, long long timeout, int32_t* __restrict__ dist,
                              int32_t* __restrict__ pred, Red<T>& red) {
    __shared__ uint32_t claim;
    const uint32_t nwg = gridDim.x;
    const int64_t gtid = (int64_t)blockIdx.x * T + threadIdx.x;
    const int64_t gsz = (int64_t)nwg * T;
    const uint32_t hmask = (uint32_t)((1ull << zt.hbits) - 1ull);
    auto D = [&](int64_t v) { return label_value(ld_agent(&lab[v])); };
    auto set_flag = [&](int64_t v, uint32_t f) {
        __hip_atomic_fetch_or(&zt.flags[v], f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    // every vertex starts plain with its own index as settle key; the table starts empty
    for (int64_t v = gtid; v < n; v += gsz) {
        st_agent(&zt.flags[v], v == src ? kSeed : 0u);
        st_agent(&zt.cnt[v], 0u);
        st_agent(&zt.fill[v], 0u);
        st_agent(&zt.md[v], kInf);
        st_agent(&rk[v], (uint64_t)v << 32);
        st_agent(&pk[v], kNoKey);
    }
    for (int64_t h = gtid; h <= (int64_t)hmask; h += gsz) st_agent(&zt.ht_key[h], kEmpty);
    if (!csr_barrier(cc, ++b, nwg, timeout)) return false;
    // tight zero-weight edges make both ends non-plain; positive ones make the head a seed
    for (int64_t u = gtid; u < n; u += gsz) {
        const uint32_t du = D(u);
        if (du >= kInf) continue;
        for_edges(row_ptr, col, w, n, (int32_t)u, [&](const int32_t* v, const int32_t* wt, const bool* eok) {
            uint32_t dv[kBatch];
#pragma unroll
            for (int j = 0; j < kBatch; ++j) dv[j] = eok[j] ? D(v[j]) : kInf;
#pragma unroll
            for (int j = 0; j < kBatch; ++j) {
                if (!tight(du, dv[j], wt[j])) continue;
                if (wt[j] == 0) {
                    set_flag(u, kNonPlain);
                    set_flag(v[j], kNonPlain);
                } else {
                    set_flag(v[j], kSeed);
                }
            }
        });
    }
    if (!csr_barrier(cc, ++b, nwg, timeout)) return false;
    // the distance of every non-plain vertex enters the table (one entry per level)
    for (int64_t v = gtid; v < n; v += gsz) {
        if (!(ld_agent(&zt.flags[v]) & kNonPlain)) continue;
        const uint64_t d = D(v);
        for (uint32_t h = level_slot((uint32_t)d, zt.hbits);; h = (h + 1) & hmask) {
            uint64_t expect = kEmpty;
            if (__hip_atomic_compare_exchange_strong(&zt.ht_key[h], &expect, d, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT) ||
                expect == d)
                break;
        }
    }
    if (!csr_barrier(cc, ++b, nwg, timeout)) return false;
    // number the levels
    for (int64_t h = gtid; h <= (int64_t)hmask; h += gsz)
        if (ld_agent(&zt.ht_key[h]) != kEmpty)
            st_agent(&zt.ht_lvl[h], __hip_atomic_fetch_add(&cc->nlev, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (!csr_barrier(cc, ++b, nwg, timeout)) return false;
    // each non-plain vertex finds its level and counts itself in
    for (int64_t v = gtid; v < n; v += gsz) {
        if (!(ld_agent(&zt.flags[v]) & kNonPlain)) continue;
        const uint64_t d = D(v);
        uint32_t h = level_slot((uint32_t)d, zt.hbits);
        while (ld_agent(&zt.ht_key[h]) != d) h = (h + 1) & hmask;
        const uint32_t L = ld_agent(&zt.ht_lvl[h]);
        st_agent(&zt.lev[v], L);
        __hip_atomic_fetch_add(&zt.cnt[L], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!csr_barrier(cc, ++b, nwg, timeout)) return false;
    const uint32_t nl = ld_agent(&cc->nlev);
    // where each level's group starts: an exclusive scan of the counts, by workgroup 0
    if (blockIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t base = 0; base < nl; base += T) {
            const uint32_t i = base + threadIdx.x;
            const uint32_t c = i < nl ? ld_agent(&zt.cnt[i]) : 0u;
            uint32_t total = 0;
            const uint32_t ex = block_excl_scan<T>(c, total, red);
            if (i < nl) st_agent(&zt.off[i], run + ex);
            run += total;
        }
    }
    if (!csr_barrier(cc, ++b, nwg, timeout)) return false;
    // place each non-plain vertex in its level's group
    for (int64_t v = gtid; v < n; v += gsz) {
        if (!(ld_agent(&zt.flags[v]) & kNonPlain)) continue;
        const uint32_t L = ld_agent(&zt.lev[v]);
        const uint32_t pos = ld_agent(&zt.off[L]) +
                             __hip_atomic_fetch_add(&zt.fill[L], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        st_agent(&zt.seg[pos], (uint32_t)v);
    }
    if (!csr_barrier(cc, ++b, nwg, timeout)) return false;
    // the sequential pass of each level, a workgroup per level: settle the
    // lowest-index available vertex, make the heads of its tight zero-weight
    // edges available, repeat
    for (;;) {
        if (threadIdx.x == 0)
            claim = __hip_atomic_fetch_add(&cc->next_level, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint32_t L = claim;
        __syncthreads();
        if (L >= nl) break;
        const uint32_t o = ld_agent(&zt.off[L]), cntL = ld_agent(&zt.cnt[L]);
        uint32_t pm = 0, step = 0;
        for (;;) {
            uint64_t best = kNoKey;
            for (uint32_t i = threadIdx.x; i < cntL; i += T) {
                const uint32_t v = ld_agent(&zt.seg[o + i]);
                const uint32_t f = ld_agent(&zt.flags[v]);
                if ((f & (kSeed | kAvail)) && !(f & kDone)) best = umin64(best, v);
            }
            uint32_t none = 0;
            block_min_or<T>(best, none, red);
            if (best == kNoKey) break;
            const uint32_t x = (uint32_t)best;
            pm = max(pm, x);
            ++step;
            if (threadIdx.x == 0) {
                set_flag(x, kDone);
                st_agent(&rk[x], ((uint64_t)pm << 32) | step);
            }
            const uint32_t dx = D(x);
            for (int64_t e = row_ptr[x] + threadIdx.x; e < row_ptr[x + 1]; e += T) {
                const int32_t y = col[e];
                if (w[e] == 0 && edge_ok((int32_t)x, y, 0, n) && D(y) == dx) set_flag(y, kAvail);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
    }
    if (!csr_barrier(cc, ++b, nwg, timeout)) return false;
    // the smallest tail dist of a tight edge into each vertex ...
    for (int64_t u = gtid; u < n; u += gsz) {
        const uint32_t du = D(u);
        if (du >= kInf) continue;
        for_edges(row_ptr, col, w, n, (int32_t)u, [&](const int32_t* v, const int32_t* wt, const bool* eok) {
#pragma unroll
            for (int j = 0; j < kBatch; ++j)
                if (eok[j] && v[j] != src && tight(du, D(v[j]), wt[j]))
                    __hip_atomic_fetch_min(&zt.md[v[j]], du, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        });
    }
    if (!csr_barrier(cc, ++b, nwg, timeout)) return false;
    // ... the smallest settle key among those tails ...
    for (int64_t u = gtid; u < n; u += gsz) {
        const uint32_t du = D(u);
        if (du >= kInf) continue;
        const uint64_t ku = ld_agent(&rk[u]);
        for_edges(row_ptr, col, w, n, (int32_t)u, [&](const int32_t* v, const int32_t* wt, const bool* eok) {
#pragma unroll
            for (int j = 0; j < kBatch; ++j)
                if (eok[j] && v[j] != src && tight(du, D(v[j]), wt[j]) && ld_agent(&zt.md[v[j]]) == du)
                    __hip_atomic_fetch_min(&pk[v[j]], ku, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        });
    }
    if (!csr_barrier(cc, ++b, nwg, timeout)) return false;
    // ... and the tail whose key won is pred (one tail per vertex: keys differ within
    // a level); vertices without such a tail (the source, unreachable ones) get -1
    for (int64_t u = gtid; u < n; u += gsz) {
        const uint32_t du = D(u);
        if (du < kInf) {
            const uint64_t ku = ld_agent(&rk[u]);
            for_edges(row_ptr, col, w, n, (int32_t)u, [&](const int32_t* v, const int32_t* wt, const bool* eok) {
#pragma unroll
                for (int j = 0; j < kBatch; ++j)
                    if (eok[j] && v[j] != src && tight(du, D(v[j]), wt[j]) && ld_agent(&zt.md[v[j]]) == du &&
                        ld_agent(&pk[v[j]]) == ku)
                        pred[v[j]] = (int32_t)u;
            });
        }
        dist[u] = (int32_t)du;
        if (u == src || du >= kInf || ld_agent(&pk[u]) == kNoKey) pred[u] = -1;
    }
    return true;
}

template <int T>
__global__ __launch_bounds__(T) void k_csr_lc(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                              const int32_t* __restrict__ w, int32_t n, int32_t src,
                                              int32_t* __restrict__ dist, int32_t* __restrict__ pred,
                                              uint64_t* __restrict__ lab, uint64_t* __restrict__ pkey,
                                              uint64_t* __restrict__ rk, uint32_t* __restrict__ lists,
                                              CsrCtl* __restrict__ cc, ZeroTie zt, long long timeout,
                                              Ctl* __restrict__ ctl) {
    __shared__ Red<T> red;
    const uint32_t nwg = gridDim.x;
    const int64_t gtid = (int64_t)blockIdx.x * T + threadIdx.x;
    const int64_t gsz = (int64_t)nwg * T;
    uint32_t b = 0;
    unsigned long long sweeps = 0, rows = 0;
    uint32_t neg = 0;
    // distances: label-correcting sweeps from the source (the first frontier)
    bool ok = frontier_sweeps(
        cc->count, lists, lab, row_ptr, col, w, n, cc, b, timeout, 1u, sweeps, rows,
        [&](int32_t u) { return label_value(ld_agent(&lab[u])); },
        [&](uint32_t du, int32_t u, int32_t v, int32_t wt, uint32_t& c) {
            if (!edge_ok(u, v, wt, n)) {
                neg |= wt < 0 ? 1u : 0u;
                return false;
            }
            c = du + (uint32_t)wt;  // both < 2^31: no wrap
            return c < kInf;        // longer than INT32_MAX - 1: not representable
        });
    uint32_t zero = 0;
    if (ok) {
        // pred pass: the tight edge of smallest (dist[u], u) into each vertex
        for (int64_t u = gtid; u < n; u += gsz) {
            const uint32_t du = label_value(ld_agent(&lab[u]));
            if (du >= kInf) continue;
            for_edges(row_ptr, col, w, n, (int32_t)u, [&](const int32_t* v, const int32_t* wt, const bool* eok) {
                uint32_t dv[kBatch];
#pragma unroll
                for (int j = 0; j < kBatch; ++j) dv[j] = eok[j] ? label_value(ld_agent(&lab[v[j]])) : kInf;
#pragma unroll
                for (int j = 0; j < kBatch; ++j) {
                    // unreachable heads have no pred
                    if (dv[j] >= kInf || du + (uint32_t)wt[j] != dv[j]) continue;
                    __hip_atomic_fetch_min(&pkey[v[j]], make_key(du, (uint32_t)u), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    zero |= wt[j] == 0 ? 1u : 0u;
                }
            });
        }
        if (zero) __hip_atomic_fetch_or(&cc->zero, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (neg) __hip_atomic_fetch_or(&cc->neg, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = csr_barrier(cc, ++b, nwg, timeout);
    }
    uint32_t status = ok ? 0u : kStatusTimeout;
    const uint32_t Z = ok ? ld_agent(&cc->zero) : 0u;
    if (ok && Z) {
        // tight zero-weight edges: the settle order of equal distances decides pred
        ok = zero_tie_pred<T>(row_ptr, col, w, n, src, lab, rk, pkey, zt, cc, b, timeout, dist, pred, red);
        status |= ok ? kStatusZeroFallback : kStatusTimeout;
    } else if (ok) {
        for (int64_t v = gtid; v < n; v += gsz) {
            const uint32_t d = label_value(ld_agent(&lab[v]));
            const uint64_t kk = ld_agent(&pkey[v]);
            dist[v] = (int32_t)d;
            pred[v] = (v == src || d >= kInf || kk == kNoKey) ? -1 : (int32_t)(uint32_t)kk;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (ok && ld_agent(&cc->neg)) status |= kStatusNegWeight;
        ctl->last[kStatRounds] = sweeps;
        ctl->last[kStatSettled] = rows;
        ctl->last[kStatFallbacks] = (status & kStatusZeroFallback) ? 1 : 0;
        ctl->last[kStatBarriers] = b;
        ctl->status = status;
    }
}

}  // namespace

int csr_occupancy(int* per_cu) {
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(
        per_cu, reinterpret_cast<const void*>(&k_csr_lc<kCsrThreads>), kCsrThreads, 0);
}

}  // namespace sssp

using namespace sssp;

namespace {

// Workgroups of a CSR solve: about 256 vertices each, at most 1024 and at most
// the occupancy query times the compute units.  The 1024 cap is measured, not
// derived: at 2048 workgroups (8 per CU, the query's maximum for this kernel)
// grid barriers of the n = 10^6 solve waited out their time limit, so not every
// workgroup was resident, while 1024 on the same graph runs to the end.
constexpr int kCsrMaxGrid = 1024;

int csr_grid(int32_t n, const sssp_tuning* tuning, int cus, int* nwg, int* per_cu_out) {
    int per_cu = 0;
    if (csr_occupancy(&per_cu) != 0 || per_cu < 1) return err(SSSP_EDEVICE, "CSR kernel does not fit a CU");
    int g = tuning && tuning->workgroups ? tuning->workgroups : (int)std::max<int64_t>(1, (n + 255) / 256);
    *nwg = std::max(1, std::min({g, per_cu * cus, kCsrMaxGrid}));
    if (per_cu_out) *per_cu_out = per_cu;
    return SSSP_OK;
}

}  // namespace

extern "C" {

int sssp_csr_grid(int32_t n, const sssp_tuning* tuning, void* stream, int32_t* workgroups, int32_t* per_cu,
                  int32_t* cus) {
    if (n < 1 || !workgroups) return err(SSSP_EINVAL, "bad arguments (n=%d)", n);
    Ctl* ctl = nullptr;
    int c = 0;
    long long khz = 0;
    int rc = stream_ctl((hipStream_t)stream, &ctl, &c, &khz);
    if (rc) return rc;
    int g = 0, pc = 0;
    if ((rc = csr_grid(n, tuning, c, &g, &pc))) return rc;
    *workgroups = g;
    if (per_cu) *per_cu = pc;
    if (cus) *cus = c;
    return SSSP_OK;
}

int sssp_edges_to_csr(const int32_t* eu, const int32_t* ev, const int32_t* ew, int64_t m, int32_t n,
                      int32_t directed, int64_t* row_ptr, int32_t* col, int32_t* w, int64_t* m_out,
                      int64_t* bad_edges, void* stream) {
    if (!row_ptr || n < 1 || m < 0 || (m > 0 && (!eu || !ev || !ew || !col || !w)))
        return err(SSSP_EINVAL, "bad arguments (n=%d m=%lld)", n, (long long)m);
    hipStream_t s = (hipStream_t)stream;
    // scratch: degrees, then cursors (n words each), the bad-edge counter and the
    // per-chunk totals of the scan
    const int32_t chunks = (int32_t)(((int64_t)n + kScanChunk - 1) / kScanChunk);
    char* buf = nullptr;
    const size_t bytes = 2 * sizeof(uint32_t) * (size_t)n + sizeof(unsigned long long) * (1 + (size_t)chunks);
    hipError_t e = hipMallocAsync((void**)&buf, bytes, s);
    if (e != hipSuccess) return err(SSSP_ENOMEM, "hipMallocAsync: %s", hipGetErrorString(e));
    uint32_t* deg = reinterpret_cast<uint32_t*>(buf);
    uint32_t* cursor = deg + n;
    unsigned long long* bad = reinterpret_cast<unsigned long long*>(cursor + n);
    unsigned long long* sums = bad + 1;
    e = zero_fill(buf, (bytes + 3) & ~size_t(3), s);
    const unsigned eb = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (m + 255) / 256), 8192);
    const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    if (e == hipSuccess && m > 0) {
        hipLaunchKernelGGL(k_csr_degree, dim3(eb), dim3(256), 0, s, eu, ev, ew, m, n, directed, deg, bad);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_csr_chunk_sums, dim3(chunks), dim3(kScanChunk), 0, s, deg, n, sums);
        hipLaunchKernelGGL(k_csr_scan_sums, dim3(1), dim3(kScanChunk), 0, s, sums, chunks, row_ptr);
        hipLaunchKernelGGL(k_csr_scan_chunks, dim3(chunks), dim3(kScanChunk), 0, s, deg, n, sums, row_ptr);
        e = hipGetLastError();
    }
    if (e == hipSuccess && m > 0) {
        hipLaunchKernelGGL(k_csr_fill, dim3(eb), dim3(256), 0, s, eu, ev, ew, m, n, directed, row_ptr, cursor, col, w);
        e = hipGetLastError();
    }
    if (e == hipSuccess && m > 0) {
        hipLaunchKernelGGL(k_csr_sort_rows, dim3(nb), dim3(256), 0, s, row_ptr, n, col, w);
        e = hipGetLastError();
    }
    int64_t total = 0;
    unsigned long long nbad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&total, row_ptr + n, sizeof total, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&nbad, bad, sizeof nbad, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFreeAsync(buf, s);
    if (e != hipSuccess) return err(SSSP_EDEVICE, "edge list conversion: %s", hipGetErrorString(e));
    if (m_out) *m_out = total;
    if (bad_edges) *bad_edges = (int64_t)nbad;
    return SSSP_OK;
}

int sssp_csr_solve(const int64_t* row_ptr, const int32_t* col, const int32_t* w, int32_t n, int32_t src,
                   int32_t* dist, int32_t* pred, const sssp_tuning* tuning, void* stream) {
    if (!row_ptr || !dist || !pred || n < 1) return err(SSSP_EINVAL, "bad arguments (n=%d)", n);
    if (src < 0 || src >= n) return err(SSSP_EINVAL, "src %d outside [0, %d)", src, n);
    hipStream_t s = (hipStream_t)stream;
    Ctl* ctl = nullptr;
    int cus = 0;
    long long khz = 100000;
    int rc = stream_ctl(s, &ctl, &cus, &khz);
    if (rc) return rc;
    int nwg = 0;
    if ((rc = csr_grid(n, tuning, cus, &nwg, nullptr))) return rc;
    // scratch: dist labels, pred keys, settle keys (n x 8 B each), 3 frontier lists
    // (3n words), control, and the tables of the zero-weight tie pass (7n words,
    // 12 B per entry of a table of the smallest power of two >= 2n entries)
    const size_t words = (size_t)n;
    uint32_t hbits = 1;
    while ((1ull << hbits) < 2ull * words) ++hbits;
    const size_t H = (size_t)1 << hbits;
    const size_t bytes = 3 * words * 8 + 3 * words * 4 + sizeof(CsrCtl) + 256 + H * 8 + 7 * words * 4 + H * 4 + 256;
    char* buf = nullptr;
    hipError_t e = hipMallocAsync((void**)&buf, bytes, s);
    if (e != hipSuccess) return err(SSSP_ENOMEM, "hipMallocAsync(%zu bytes): %s", bytes, hipGetErrorString(e));
    uint64_t* lab = reinterpret_cast<uint64_t*>(buf);
    uint64_t* pkey = lab + words;
    uint64_t* rk = pkey + words;
    uint32_t* lists = reinterpret_cast<uint32_t*>(rk + words);
    CsrCtl* cc = reinterpret_cast<CsrCtl*>(((uintptr_t)(lists + 3 * words) + 255) & ~(uintptr_t)255);
    ZeroTie zt;
    zt.ht_key = reinterpret_cast<uint64_t*>(((uintptr_t)(cc + 1) + 255) & ~(uintptr_t)255);
    zt.ht_lvl = reinterpret_cast<uint32_t*>(zt.ht_key + H);
    zt.flags = zt.ht_lvl + H;
    zt.lev = zt.flags + words;
    zt.seg = zt.lev + words;
    zt.cnt = zt.seg + words;
    zt.off = zt.cnt + words;
    zt.fill = zt.off + words;
    zt.md = zt.fill + words;
    zt.hbits = hbits;
    const unsigned ib = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_csr_init, dim3(ib), dim3(256), 0, s, n, src, lab, pkey, lists, cc);
    e = hipGetLastError();
    if (e == hipSuccess) {
        long long timeout = grid_barrier_ticks(khz);
        if (grid_launch_is_plain()) {
            // ordinary launch of the same grid (co-resident by its size), for profilers
            hipLaunchKernelGGL(k_csr_lc<kCsrThreads>, dim3(nwg), dim3(kCsrThreads), 0, s, row_ptr, col, w, n, src,
                               dist, pred, lab, pkey, rk, lists, cc, zt, timeout, ctl);
            e = hipGetLastError();
        } else {
            void* args[] = {(void*)&row_ptr, (void*)&col, (void*)&w, &n, &src, &dist, &pred, &lab, &pkey,
                            &rk, &lists, &cc, &zt, &timeout, &ctl};
            e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_csr_lc<kCsrThreads>), dim3(nwg),
                                           dim3(kCsrThreads), args, 0, s);
        }
    }
    (void)hipFreeAsync(buf, s);
    if (e != hipSuccess) return err(SSSP_EDEVICE, "CSR solve launch: %s", hipGetErrorString(e));
    return SSSP_OK;
}

}  // extern "C"
