// Dense-matrix Dijkstra kernels for gfx950.
//
//   k_single  one workgroup solves one instance; the whole row is its slice.
//   k_grid    persistent cooperative grid: every workgroup owns a column slice,
//             one grid barrier per round (the single-GPU form of the paper's
//             per-iteration MPI_Allreduce of the global minimum, Section III-B).
//   k_batch   persistent grid of independent workgroups that pull instances
//             from a ticket counter and solve each with the k_single engine.
//
// Every kernel runs the paper's Algorithm 1 (Section III-A) in rounds.  A round
// takes the global minimum d of dist over unvisited vertices and the bucket B of
// all unvisited vertices at d.  In the default ("fused") mode the whole bucket is
// settled in one round: for each unvisited v outside B the round computes the
// lowest (d + W[u][v], u) over u in B and applies it when strictly below
// dist[v].  With every off-diagonal weight >= 1 this reproduces Algorithm 1 bit
// for bit: relaxations from B produce distances > d, so B's members neither
// change nor gain new members while Algorithm 1 settles them one by one in
// index order, and the lexicographic minimum is exactly what its strict '<'
// keeps.  A zero-weight edge from B to an unvisited vertex outside B breaks that
// argument, so such a round is discarded and only the lowest-index vertex of B
// is settled (one literal step of Algorithm 1).  In "literal" mode every round
// is one such step, i.e. the paper's loop as printed.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "engine.h"
#include "lc.h"
#include "multi.h"
#include "solve.h"
#include "sssp_internal.h"

namespace sssp {

template <int T, int G, int U>
__global__ __launch_bounds__(T) void k_single(const int32_t* __restrict__ W, int64_t ld, int32_t n,
                                              int32_t src, int32_t* __restrict__ dist,
                                              int32_t* __restrict__ pred, uint32_t flags,
                                              Ctl* __restrict__ ctl) {
    SharedSolve<T>& sh = g_sh<T>;
    SolveStats st = {0, 0, 0, 0, 0};
    const bool vec = (flags & kFlagVec) != 0;
    solve_single<T, G, U, int32_t>(W, ld, n, src, dist, pred, vec, (flags & kFlagLiteral) != 0, sh, st, ctl);
    uint32_t s = st.status;
    uint64_t dummy = kNoKey;
    block_min_or<T>(dummy, s, sh.red);
    if (threadIdx.x == 0) {
        ctl->last[kStatRounds] = st.rounds;
        ctl->last[kStatSettled] = st.settled;
        ctl->last[kStatFallbacks] = st.fallbacks;
        ctl->last[kStatBarriers] = 0;
        ctl->status = s;
    }
}

// BAL: pair balancing of large rounds (solve_gang); chosen by the launcher for
// graphs large enough to have them, since its code costs the small rounds a few
// registers.
template <int T, int G, int U, bool BAL>
__global__ __launch_bounds__(T) void k_grid(const int32_t* __restrict__ W, int64_t ld, int32_t n,
                                            int32_t src, int32_t* __restrict__ dist,
                                            int32_t* __restrict__ pred, uint32_t flags, int32_t S,
                                            long long timeout, Ctl* __restrict__ ctl, char* __restrict__ words) {
    SharedSolve<T>& sh = g_sh<T>;
    SolveStats st = {0, 0, 0, 0, 0};
    const uint32_t epoch = ld_agent(&ctl->epoch);
    solve_gang<T, G, U, int32_t, true, BAL>(W, ld, n, src, dist, pred, (flags & kFlagVec) != 0, (flags & kFlagLiteral) != 0, S,
                        blockIdx.x, gridDim.x, timeout, grid_words(words, gridDim.x, S), sh, st, ctl, epoch);
    finish_launch(ctl, st, blockIdx.x == 0);
}

// ---------------------------------------------------------------------------
// One item (a batched instance or a served query) solved by the workgroup that
// claimed it alone, or by rank `part` of a gang of item.parts workgroups.
// ---------------------------------------------------------------------------
// Each (matrix type, columns-per-thread) variant is compiled as a function of
// its own, so that its register allocation does not pay for the others.
// Rows in flight per thread.  More rows keep more bytes in flight for compact
// entries, but a thread pads the last batch of a bucket with copies of its last
// row, and the small buckets of sparse graphs made 16 rows slower overall
// (batched workload 3.6 -> 4.1 ms, served saturation -14%): 8 for every type.
template <typename E>
constexpr int rows_in_flight() { return 8; }

template <int T, int G, typename E>
__device__ __attribute__((noinline)) SolveStats single_variant(BatchItem I, bool literal) {
    SolveStats st = {0, 0, 0, 0, 0};
    solve_single<T, G, rows_in_flight<E>(), E>(static_cast<const E*>(I.W), I.ld, I.n, I.src, I.dist, I.pred,
                                              I.vec != 0, literal,
                             g_sh<T>, st, nullptr);
    uint32_t s = st.status;
    uint64_t dummy = kNoKey;
    block_min_or<T>(dummy, s, g_sh<T>.red);
    st.status = s;
    return st;
}

template <int T, int G, typename E>
__device__ __attribute__((noinline)) SolveStats gang_variant(BatchItem I, int part, bool literal, long long timeout,
                                                             Bar* bw, char* arena, uint32_t epoch) {
    SolveStats st = {0, 0, 0, 0, 0};
    solve_gang<T, G, rows_in_flight<E>(), E>(static_cast<const E*>(I.W), I.ld, I.n, I.src, I.dist, I.pred,
                                            I.vec != 0, literal, I.S, part, I.parts, timeout,
                                            gang_words(arena + I.scratch_off, I.parts, I.S), g_sh<T>, st, nullptr, epoch);
    if (threadIdx.x == 0) gang_leave(bw, (uint32_t)I.parts);
    return st;
}

// A label-correcting item (rank `part` of a gang of I.parts, possibly one): the
// sweeps, then the pred pass; a tight zero-weight edge sends the whole gang to
// the Dijkstra rounds on the same records (numbering continued).
template <int T, int G, typename E>
__device__ __attribute__((noinline)) SolveStats lc_variant(BatchItem I, int part, long long timeout, Bar* bw,
                                                           char* arena, uint32_t epoch) {
    SolveStats st = {0, 0, 0, 0, 0};
    const GangWords gw = gang_words(arena + I.scratch_off, I.parts, I.S);
    uint32_t b = 0;
    const int r = solve_lc<T, G, 8, E, false>(static_cast<const E*>(I.W), I.ld, I.n, I.src, I.dist, I.pred,
                                              I.vec != 0, I.S, part, I.parts, timeout, bw, gw.pubs, gw.lists, g_sh<T>,
                                              g_lc<T>, st, b, epoch, nullptr);
    if (r == kLcFallback) {
        ++st.fallbacks;
        st.status |= kStatusZeroFallback;
        solve_gang<T, G, 8, E>(static_cast<const E*>(I.W), I.ld, I.n, I.src, I.dist, I.pred, I.vec != 0, false,
                               I.S, part, I.parts, timeout, gw, g_sh<T>, st, nullptr, epoch, b);
    } else {
        if (r == kLcTimeout) st.status |= kStatusTimeout;
        st.barriers += b;
    }
    if (threadIdx.x == 0) gang_leave(bw, (uint32_t)I.parts);
    uint32_t s = st.status;
    uint64_t dummy = kNoKey;
    block_min_or<T>(dummy, s, g_sh<T>.red);
    st.status = s;
    return st;
}

// A group of I.K sources of one matrix in lockstep (rank `part` of a gang of
// I.parts, possibly one).
template <int T, int KP, typename E>
__device__ __attribute__((noinline)) SolveStats group_variant(BatchItem I, int part, long long timeout, Bar* bw,
                                                              char* arena, uint32_t epoch) {
    SolveStats st = {0, 0, 0, 0, 0};
    const int rw = multi_rec_words(I.K);
    uint64_t* recs = reinterpret_cast<uint64_t*>(arena + I.scratch_off);
    uint32_t* lists = reinterpret_cast<uint32_t*>(recs + 2 * (size_t)I.parts * rw);
    solve_multi<T, KP, E>(static_cast<const E*>(I.W), I.ld, I.n, static_cast<const MultiSrc*>(I.group), I.K,
                          I.vec != 0, I.S, part, I.parts, timeout, recs, lists, g_sh<T>, g_mh<T>, st, epoch);
    if (threadIdx.x == 0) gang_leave(bw, (uint32_t)I.parts);
    return st;
}

// Sources per thread of a group: the K sources spread over the P = T / L row
// partitions of a slice of I.S columns (the host keeps K <= 4P).
template <int T, typename E>
__device__ __forceinline__ SolveStats group_by_shape(const BatchItem& I, int part, long long timeout, Bar* bw,
                                                     char* arena, uint32_t epoch) {
    int L = 1;
    while (L < (I.S + 3) / 4 && L < T) L <<= 1;
    const int P = T / L;
    const int kp = (I.K + P - 1) / P;
    if (kp <= 1) return group_variant<T, 1, E>(I, part, timeout, bw, arena, epoch);
    if (kp <= 2) return group_variant<T, 2, E>(I, part, timeout, bw, arena, epoch);
    return group_variant<T, 4, E>(I, part, timeout, bw, arena, epoch);
}

template <int T, typename E>
__device__ __forceinline__ SolveStats lc_by_size(const BatchItem& I, int part, long long timeout, Bar* bw,
                                                 char* arena, uint32_t epoch) {
    const int groups = (I.S + 3) / 4;
    if (groups <= T) return lc_variant<T, 1, E>(I, part, timeout, bw, arena, epoch);
    if (groups <= 2 * T) return lc_variant<T, 2, E>(I, part, timeout, bw, arena, epoch);
    return lc_variant<T, 4, E>(I, part, timeout, bw, arena, epoch);
}

template <int T, typename E>
__device__ __forceinline__ SolveStats single_by_size(const BatchItem& I, bool literal) {
    const int groups = (I.n + 3) / 4;
    if (groups <= T) return single_variant<T, 1, E>(I, literal);
    if (groups <= 2 * T) return single_variant<T, 2, E>(I, literal);
    return single_variant<T, 4, E>(I, literal);
}

template <int T, typename E>
__device__ __forceinline__ SolveStats gang_by_size(const BatchItem& I, int part, bool literal, long long timeout,
                                                   Bar* bw, char* arena, uint32_t epoch) {
    const int groups = (I.S + 3) / 4;
    if (groups <= T) return gang_variant<T, 1, E>(I, part, literal, timeout, bw, arena, epoch);
    if (groups <= 2 * T) return gang_variant<T, 2, E>(I, part, literal, timeout, bw, arena, epoch);
    return gang_variant<T, 4, E>(I, part, literal, timeout, bw, arena, epoch);
}

template <int T>
// epoch: unique to this use of the item's exchange records (see gang_exchange).
__device__ __forceinline__ SolveStats solve_item(const BatchItem& I, int part, bool literal, long long timeout,
                                                 Bar* bw, char* arena, uint32_t epoch) {
    if (I.method == kMethodGroup) {
        if (I.elem == 1) return group_by_shape<T, uint8_t>(I, part, timeout, bw, arena, epoch);
        if (I.elem == 2) return group_by_shape<T, uint16_t>(I, part, timeout, bw, arena, epoch);
        return group_by_shape<T, int32_t>(I, part, timeout, bw, arena, epoch);
    }
    if (I.method == kMethodLabelCorrecting && !literal) {
        if (I.elem == 1) return lc_by_size<T, uint8_t>(I, part, timeout, bw, arena, epoch);
        if (I.elem == 2) return lc_by_size<T, uint16_t>(I, part, timeout, bw, arena, epoch);
        return lc_by_size<T, int32_t>(I, part, timeout, bw, arena, epoch);
    }
    if (I.parts <= 1) {
        if (I.elem == 1) return single_by_size<T, uint8_t>(I, literal);
        if (I.elem == 2) return single_by_size<T, uint16_t>(I, literal);
        return single_by_size<T, int32_t>(I, literal);
    }
    if (I.elem == 1) return gang_by_size<T, uint8_t>(I, part, literal, timeout, bw, arena, epoch);
    if (I.elem == 2) return gang_by_size<T, uint16_t>(I, part, literal, timeout, bw, arena, epoch);
    return gang_by_size<T, int32_t>(I, part, literal, timeout, bw, arena, epoch);
}

// ---------------------------------------------------------------------------
// Batched: a grid of workgroups pulls tickets from a counter; each ticket is one
// part of one item (items are ordered largest first, an item's parts are
// consecutive tickets, so at most the newest gang is incomplete at a time).
// ---------------------------------------------------------------------------
template <int T>
__global__ __launch_bounds__(T) void k_batch(const BatchItem* __restrict__ items, const BatchPart* __restrict__ parts,
                                             int32_t nparts, Bar* __restrict__ bars, char* __restrict__ arena,
                                             uint32_t flags, long long timeout, Ctl* __restrict__ ctl) {
    SharedSolve<T>& sh = g_sh<T>;
    SolveStats total = {0, 0, 0, 0, 0};
    const bool literal = (flags & kFlagLiteral) != 0;
    const uint32_t epoch = ld_agent(&ctl->epoch);
    for (;;) {
        if (threadIdx.x == 0)
            sh.item = (int32_t)__hip_atomic_fetch_add(&ctl->next_item, 1ull, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int32_t t = sh.item;
        __syncthreads();
        if (t >= nparts) break;
        const BatchPart pt = parts[t];
        const BatchItem I = items[pt.item];
        const SolveStats st = solve_item<T>(I, pt.part, literal, timeout, bars ? &bars[pt.item] : nullptr, arena, epoch);
        total.status |= st.status;
        if (pt.part == 0) {  // every gang member computes the same counts; count them once
            total.rounds += st.rounds;
            total.settled += st.settled;
            total.fallbacks += st.fallbacks;
            total.barriers += st.barriers;
        }
    }
    finish_launch(ctl, total, true);
}

// Weight range of a matrix: out[0] = min over all entries, out[1] = max over
// entries other than INT32_MAX (no edge), out[2] = min over the off-diagonal
// entries.  out must hold {INT32_MAX, INT32_MIN, INT32_MAX}.
__global__ void k_weight_range(const int32_t* __restrict__ W, int64_t ld, int32_t n, int32_t* __restrict__ out) {
    __shared__ int32_t smin[256], smax[256], soff[256];
    int32_t mn = 0x7fffffff, mx = (int32_t)0x80000000, off = 0x7fffffff;
    const int64_t total = (int64_t)n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n, j = e - i * n;
        const int32_t w = W[i * ld + j];
        mn = min(mn, w);
        if (w != 0x7fffffff) mx = max(mx, w);
        if (i != j) off = min(off, w);
    }
    smin[threadIdx.x] = mn;
    smax[threadIdx.x] = mx;
    soff[threadIdx.x] = off;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            smin[threadIdx.x] = min(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = max(smax[threadIdx.x], smax[threadIdx.x + s]);
            soff[threadIdx.x] = min(soff[threadIdx.x], soff[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMin(&out[0], smin[0]);
        atomicMax(&out[1], smax[0]);
        atomicMin(&out[2], soff[0]);
    }
}

// Clears `words` 32-bit words (scratch that a launch expects zeroed; a kernel
// rather than a memset node, so that the call can be captured into a graph).
__global__ void k_zero(uint32_t* __restrict__ p, size_t words) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Exact compact copy: INT32_MAX -> the all-ones code of E, other entries as is
// (the caller has checked that they fit below it).  Row stride ldc entries.
template <typename E>
__global__ void k_compact(const int32_t* __restrict__ W, int64_t ld, int32_t n, E* __restrict__ C, int64_t ldc) {
    const E none = (E)~(E)0;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y)
        for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < ldc; j += (int64_t)gridDim.x * blockDim.x) {
            const int32_t w = j < n ? W[i * ld + j] : 0x7fffffff;
            C[i * ldc + j] = w == 0x7fffffff ? none : (E)w;
        }
}

// ---------------------------------------------------------------------------
// Serving: a persistent grid whose workgroups claim query parts from a ring
// that the host fills in pinned memory.  A query with parts == 1 is solved by
// the claiming workgroup alone (k_single's engine); a larger one is split into
// `parts` column slices claimed by as many workgroups, which form a gang with
// its own barrier words (k_grid's engine).  Gang members claim consecutive
// ring entries, so at most the newest gang is incomplete at any time and it
// completes as soon as enough workgroups are free: parts <= gridDim.x keeps
// this deadlock-free.
// ---------------------------------------------------------------------------

// Claim the next published ring entry (copied into *out) or decide to leave:
// returns true to leave (nothing published and the host set stop or park, or
// the host's heartbeat stalled for `watchdog` ticks).  The host publishes
// nothing while park is set, so no gang can be left half claimed.  Ring and control words live in
// host memory that the host writes while the kernel runs, so they are read
// with system-scope atomic loads (never through the scalar cache).
__device__ __forceinline__ bool serve_claim(const ServeArgs& a, ServeDesc* out) {
    unsigned long long hb = __hip_atomic_load(&a.ctl->heartbeat, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    long long hb_t = wall_clock64();
    unsigned naps = 1;
    for (unsigned poll = 0;; ++poll) {
        const unsigned long long t = __hip_atomic_load(&a.ctl->tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
        unsigned long long h = __hip_atomic_load(a.head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (h < t) {
            if (__hip_atomic_compare_exchange_strong(a.head, &h, h + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)) {
                const unsigned long long* src =
                    reinterpret_cast<const unsigned long long*>(&a.ring[h % (unsigned long long)a.ring_slots]);
                unsigned long long* dst = reinterpret_cast<unsigned long long*>(out);
                for (unsigned i = 0; i < sizeof(ServeDesc) / 8; ++i)
                    dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                return false;
            }
            naps = 1;
            continue;
        }
        if ((poll & 15) == 0) {
            if (__hip_atomic_load(&a.ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) ||
                __hip_atomic_load(&a.ctl->park, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM))
                return true;
            const unsigned long long hb2 =
                __hip_atomic_load(&a.ctl->heartbeat, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            const long long now = wall_clock64();
            if (hb2 != hb) {
                hb = hb2;
                hb_t = now;
            } else if (now - hb_t > a.watchdog) {
                return true;
            }
        }
        for (unsigned i = 0; i < naps; ++i) __builtin_amdgcn_s_sleep(127);
        if (naps < 4) naps <<= 1;
    }
}

template <int T>
__global__ __launch_bounds__(T) void k_serve(ServeArgs a) {
    __shared__ ServeDesc q;
    __shared__ int32_t leave;
    for (;;) {
        if (threadIdx.x == 0) leave = serve_claim(a, &q) ? 1 : 0;
        __syncthreads();
        if (leave) break;
        // a query's ticket is unique to it: the epoch of its gang's records
        const SolveStats st = solve_item<T>(q.item, q.part, false, a.timeout, &a.bars[q.qslot], a.arena,
                                            (uint32_t)q.ticket);
        // completion: the last part to finish writes the slot's record to host memory
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) {
            ServeSlot* sl = &a.slots[q.qslot];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (st.status) __hip_atomic_fetch_or(&sl->status, st.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t prev = __hip_atomic_fetch_add(&sl->done_parts, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (prev == (uint32_t)q.item.parts - 1) {
                const uint32_t status = __hip_atomic_exchange(&sl->status, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&sl->done_parts, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ServeDone* dn = &a.done[q.qslot];
                __hip_atomic_store(&dn->status, status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&dn->rounds, (uint32_t)st.rounds, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&dn->settled, st.settled, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&dn->t_done, wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                // every part's dist/pred writes are in memory before the host sees the ticket
                __hip_atomic_store(&dn->ticket, q.ticket, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called by the C ABI in api.cpp).
// ---------------------------------------------------------------------------
template <int T, int G, int U>
static hipError_t launch_single_t(const SolveArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_single<T, G, U>), dim3(1), dim3(T), 0, s, a.W, a.ld, a.n, a.src, a.dist,
                       a.pred, a.flags, a.ctl);
    return hipGetLastError();
}

hipError_t launch_single(const SolveArgs& a, int threads, hipStream_t s) {
    const int groups = (a.n + 3) / 4;
    if (threads <= 256) {
        if (groups <= 256) return launch_single_t<256, 1, 8>(a, s);
        if (groups <= 512) return launch_single_t<256, 2, 8>(a, s);
        if (groups <= 1024) return launch_single_t<256, 4, 8>(a, s);
    }
    if (groups <= 1024) return launch_single_t<1024, 1, 8>(a, s);
    if (groups <= 2048) return launch_single_t<1024, 2, 8>(a, s);
    if (groups <= 4096) return launch_single_t<1024, 4, 8>(a, s);
    return hipErrorInvalidValue;
}

int max_single_n() { return 4 * 4 * 1024; }

template <int T, int G, int U, bool BAL>
static hipError_t launch_grid_t(const SolveArgs& a, int nwg, int S, long long timeout, char* words, bool plain,
                                hipStream_t s) {
    const int32_t* W = a.W;
    int64_t ld = a.ld;
    int32_t n = a.n, src = a.src;
    int32_t* dist = a.dist;
    int32_t* pred = a.pred;
    uint32_t flags = a.flags;
    Ctl* ctl = a.ctl;
    if (plain) {
        hipLaunchKernelGGL((k_grid<T, G, U, BAL>), dim3(nwg), dim3(T), 0, s, W, ld, n, src, dist, pred, flags, S,
                           timeout, ctl, words);
        return hipGetLastError();
    }
    void* args[] = {&W, &ld, &n, &src, &dist, &pred, &flags, &S, &timeout, &ctl, &words};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_grid<T, G, U, BAL>), dim3(nwg),
                                      dim3(T), args, 0, s);
}

hipError_t launch_grid(const SolveArgs& a, int nwg, int S, long long timeout, char* words, bool plain, bool balance,
                       hipStream_t s) {
    const int groups = (S + 3) / 4;
    if (!balance) {
        if (groups <= 1024) return launch_grid_t<1024, 1, 8, false>(a, nwg, S, timeout, words, plain, s);
        if (groups <= 2048) return launch_grid_t<1024, 2, 8, false>(a, nwg, S, timeout, words, plain, s);
        if (groups <= 4096) return launch_grid_t<1024, 4, 8, false>(a, nwg, S, timeout, words, plain, s);
        return hipErrorInvalidValue;
    }
    if (groups <= 1024) return launch_grid_t<1024, 1, 8, true>(a, nwg, S, timeout, words, plain, s);
    if (groups <= 2048) return launch_grid_t<1024, 2, 8, true>(a, nwg, S, timeout, words, plain, s);
    if (groups <= 4096) return launch_grid_t<1024, 4, 8, true>(a, nwg, S, timeout, words, plain, s);
    return hipErrorInvalidValue;
}

int max_grid_slice() { return 4 * 4 * 1024; }

int grid_occupancy(int slice, int* per_cu) {
    const int groups = (slice + 3) / 4;
    // both balancing variants have the same launch bounds and LDS
    const void* f = groups <= 1024 ? reinterpret_cast<const void*>(&k_grid<1024, 1, 8, true>)
                  : groups <= 2048 ? reinterpret_cast<const void*>(&k_grid<1024, 2, 8, true>)
                                   : reinterpret_cast<const void*>(&k_grid<1024, 4, 8, true>);
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, f, 1024, 0);
}

hipError_t launch_batch(const BatchItem* items, const BatchPart* parts, int32_t nparts, Bar* bars, char* arena,
                        uint32_t flags, long long timeout, Ctl* ctl, int nwg, hipStream_t s) {
    hipLaunchKernelGGL((k_batch<1024>), dim3(nwg), dim3(1024), 0, s, items, parts, nparts, bars, arena, flags,
                       timeout, ctl);
    return hipGetLastError();
}

int batch_occupancy(int* per_cu) {
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, reinterpret_cast<const void*>(&k_batch<1024>),
                                                             1024, 0);
}

int max_batch_single_n() { return 4 * 4 * 1024; }
int max_batch_slice() { return 4 * 4 * 1024; }

hipError_t weight_range(const int32_t* W, int64_t ld, int32_t n, int32_t* d_out3, hipStream_t s) {
    hipLaunchKernelGGL(k_weight_range, dim3(2048), dim3(256), 0, s, W, ld, n, d_out3);
    return hipGetLastError();
}

hipError_t compact_copy(const int32_t* W, int64_t ld, int32_t n, void* C, int64_t ldc, int elem, hipStream_t s) {
    dim3 grid((unsigned)((ldc + 255) / 256 < 64 ? (ldc + 255) / 256 : 64), (unsigned)(n < 65535 ? n : 65535));
    if (elem == 1)
        hipLaunchKernelGGL((k_compact<uint8_t>), grid, dim3(256), 0, s, W, ld, n, static_cast<uint8_t*>(C), ldc);
    else if (elem == 2)
        hipLaunchKernelGGL((k_compact<uint16_t>), grid, dim3(256), 0, s, W, ld, n, static_cast<uint16_t*>(C), ldc);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t zero_fill(void* p, size_t bytes, hipStream_t s) {
    if (bytes % 4) return hipErrorInvalidValue;
    const size_t words = bytes / 4;
    if (words == 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<size_t>((words + 255) / 256, 1024);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, static_cast<uint32_t*>(p), words);
    return hipGetLastError();
}

hipError_t launch_serve(const ServeArgs& a, int nwg, hipStream_t s) {
    hipLaunchKernelGGL((k_serve<1024>), dim3(nwg), dim3(1024), 0, s, a);
    return hipGetLastError();
}

int serve_occupancy(int* per_cu) {
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, reinterpret_cast<const void*>(&k_serve<1024>),
                                                             1024, 0);
}

int max_serve_single_n() { return 4 * 4 * 1024; }
int max_serve_slice() { return 4 * 4 * 1024; }

}  // namespace sssp

namespace sssp {
size_t ctl_size() { return sizeof(Ctl); }
size_t bar_size() { return sizeof(Bar); }
}  // namespace sssp
