// Device engine shared by the dense-matrix Dijkstra kernels (gfx950, wave64).
//
// Vocabulary follows Algorithm 1 of the paper (Section III-A): dist[], pred[],
// visited[], the argmin vertex u, its distance d, and row u of the weight
// matrix W relaxed into dist/pred.
//
// A workgroup owns a contiguous slice of S columns (vertices) of the matrix —
// the single-GPU form of the paper's 1-D column division (Section III-B): it
// keeps dist[], pred[] and visited[] of those vertices in registers and writes
// dist and pred out at the end, so every column has exactly one writer and no
// atomics are needed on dist or pred.
//
// Thread layout inside a workgroup of T threads.  The slice is cut into
// NG = ceil(S/4) column groups of 4 (one 128-bit load each).  L lanes cover the
// groups of one row (lane c owns groups c, c+L, ..., G of them), and the
// T/L = P row partitions stream different rows of the current bucket at the
// same time; partition 0 holds the slice state ("owner" threads).  After a
// round the P partial minima are merged through LDS into the owners.
//
// Per-column candidate of a round: the lexicographic minimum, over the rows u
// streamed, of the packed key (W[u][v] << 32 | u) compared as uint64.  Every
// row of one round has the same dist d, so this equals the minimum of
// (d + W[u][v], u): the lowest-index u wins a tie, which is what the strict
// '<' of Algorithm 1 yields when equal-distance rows are relaxed in index
// order.  Weights are read as uint32; INT32_MAX (no edge) then never improves
// anything, because d + INT32_MAX >= INT32_MAX >= dist[v].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sssp {

constexpr uint32_t kInf = 0x7fffffffu;
constexpr uint64_t kNoKey = ~0ull;
constexpr int kWave = 64;

// status bits (Ctl::status)
constexpr uint32_t kStatusTimeout = 1u;       // a grid barrier wait gave up
constexpr uint32_t kStatusNegWeight = 2u;     // a negative weight was the best candidate of a column
constexpr uint32_t kStatusZeroFallback = 4u;  // a zero-weight edge forced single-vertex steps

// statistics slots (Ctl::acc / Ctl::last)
enum { kStatRounds = 0, kStatSettled = 1, kStatFallbacks = 2, kStatBarriers = 3, kStatCount = 4 };

constexpr int kTraceCap = 256;  // rounds recorded per launch (round start time, bucket size)

// Barrier words of one group of workgroups (the whole grid, or a gang of a
// served query).  The arrival counter, the release word that waiters poll and
// the exit counter sit on separate 128-byte lines so that polling does not
// contend with arrivals.  All zero between uses: the last member to leave
// resets them.
struct Bar {
    uint32_t bar;  // arrivals
    uint32_t pad0[31];
    uint32_t gen;  // number of the last completed barrier
    uint32_t pad1[31];
    uint32_t exit;  // members that have left
    uint32_t pad2[31];
};

// Per-launch control block in device memory.  Zeroed once when allocated;
// every launch leaves it ready for the next (the last workgroup to finish
// resets the barrier words and moves the accumulators into `last`).
struct Ctl {
    Bar b;
    uint32_t status_acc;  // status bits OR-ed during the current launch
    uint32_t status;      // status of the last finished launch
    uint32_t trace_n;     // rounds recorded in trace_t / trace_m by the last launch
    uint32_t epoch;       // launches finished; stamps the exchange records of the next one
    unsigned long long acc[kStatCount];
    unsigned long long last[kStatCount];
    unsigned long long next_item;  // work-queue ticket counter (batched kernels)
    long long trace_t[kTraceCap + 1];  // wall-clock ticks at the start of each round, then the end
    uint32_t trace_m[kTraceCap];       // rows streamed in each round
};

// Stamp of exchange number b during use `epoch` of a gang's record memory.
// Bit 63 is always set, and nothing else ever stored in record or list memory
// has it: list entries are vertex indices below 2^31 (two per 64-bit word) or
// (dist << 32) | vertex with dist below INT32_MAX, and a record's key (which
// can be all ones) sits 8 bytes into its 32-byte record, while records always
// start at 32-byte offsets of the memory they share with earlier uses.  So a
// word left in the same memory by an earlier query or launch can never pass
// for the stamp a member is waiting for.
__host__ __device__ constexpr uint64_t exchange_stamp(uint32_t epoch, uint32_t b) {
    return (1ull << 63) | ((uint64_t)(epoch & 0x7fffffffu) << 32) | b;
}

// One workgroup's contribution to a round.  Written and read only with
// agent-scope atomic accesses, which are coherent across XCDs without cache
// writebacks or invalidates; `stamp` is stored last and tells the readers that
// the rest (and the workgroup's list entries) is in place.
struct alignas(32) Pub {
    uint64_t stamp;  // exchange_stamp(epoch, barrier number of the exchange it belongs to)
    uint64_t key;    // (would-be local min dist << 32) | lowest vertex at that dist; kNoKey if none
    uint32_t count;  // vertices of the slice at that dist, listed in the slot's list region
    uint32_t flags;  // bit 0: a zero-weight edge from the bucket to an unvisited vertex was seen
    uint64_t pad;
};
static_assert(sizeof(Pub) == 32, "stamped records are 32 bytes");

// Tagged exchange words.  After the first exchange of a gang's solve, every
// word a member publishes carries the number b of its exchange in the high 32
// bits (the word's tag) and a 32-bit value in the low ones, so a reader takes
// each word as soon as it shows the tag it waits for: a member neither waits
// for its own stores to complete nor orders them behind a stamp.  Each member
// clears its tagged words (tag 0) before the solve's first exchange, which
// uses stamps and so completes every member's earlier stores before anyone
// passes it; from then on a tagged word holds 0, a tag of an earlier exchange
// of the same solve (b - 2, b - 4, ... in the same slot) or the awaited one,
// and the tag of exchange b is b >= 1, below 2^32 because a solve of n < 2^31
// vertices has at most 2n + 1 exchanges.
__host__ __device__ constexpr uint64_t tag_word(uint32_t tag, uint32_t value) {
    return ((uint64_t)tag << 32) | value;
}
__host__ __device__ constexpr uint32_t word_tag(uint64_t w) { return (uint32_t)(w >> 32); }

// A gang's tagged records of the Dijkstra rounds, as a structure of arrays:
// for each slot (exchange parity) and field, nwg consecutive words (member g at
// index g), so that a wave reading the words of 64 consecutive members touches
// four cache lines instead of one per member.  Fields: the dist of the
// member's key (0xffffffff: no key), the key's vertex, and (count << 1) | the
// zero-weight hazard flag; each word tagged.  The fourth field is unused
// (32 bytes per member and slot).
enum { kRecDist = 0, kRecVert = 1, kRecCnt = 2, kRecFields = 4 };
__host__ __device__ inline uint64_t* rec_word(uint64_t* recs, int nwg, uint32_t slot, int field, int g) {
    return recs + ((size_t)slot * kRecFields + (size_t)field) * (size_t)nwg + (size_t)g;
}

template <typename X>
__device__ __forceinline__ X ld_agent(const X* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename X>
__device__ __forceinline__ void st_agent(X* p, X v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier stress (the separately built libsssp_stress.so only): before it
// arrives at an exchange (its stamp or barrier arrival; in a tagged exchange,
// its list entries and, separately, its record), a workgroup pauses for a
// pseudo-random 0 to ~25 us chosen by (workgroup, key), so that tests see many
// arrival orders, late members and entries that arrive after their record.
// Compiled out of the product library.
__device__ __forceinline__ void stress_delay(uint32_t key) {
#ifdef SSSP_STRESS_DELAYS
    uint32_t h = (blockIdx.x + 1u) * 0x9E3779B9u ^ (key * 0x85EBCA6Bu);
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    if ((h & 3u) == 0u)
        for (uint32_t i = 0, k = (h >> 8) & 7u; i < k; ++i) __builtin_amdgcn_s_sleep(127);
#else
    (void)key;
#endif
}

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return b < a ? b : a; }
__host__ __device__ __forceinline__ uint64_t make_key(uint32_t d, uint32_t v) {
    return ((uint64_t)d << 32) | v;
}

// Lane index within the wave, recomputed where it is used: the empty asm keeps
// the compiler from hoisting the shuffle addresses derived from it out of the
// round loops, where they would stay live (and spill) across the row streams.
__device__ __forceinline__ int wave_lane() {
    int l = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    asm volatile("" : "+v"(l));
    return l;
}
// x of lane (lane ^ o); o < 64
__device__ __forceinline__ uint32_t xor_lane32(uint32_t x, int lane, int o) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute((lane ^ o) << 2, (int)x);
}

// Wave-wide reductions and scans, which every caller runs with all 64 lanes
// active.  Inside each row of 16 lanes they use DPP row shifts (a VALU operand
// read from the lane k below, no LDS round trip: ds_bpermute chains made the
// per-round reductions cost about 1 us each); the four row results are then
// combined from lanes 15, 31, 47 and 63 with v_readlane (scalar registers).
// row_shr:k; a lane with no source lane in its row gets `old`.
template <int K>
__device__ __forceinline__ uint32_t row_shr(uint32_t old, uint32_t x) {
    static_assert(K >= 1 && K <= 15, "row_shr:1..15");
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)x, 0x110 + K, 0xf, 0xf, false);
}
template <int K>
__device__ __forceinline__ uint64_t row_shr64(uint64_t x) {  // a lane with no source keeps x
    return ((uint64_t)row_shr<K>((uint32_t)(x >> 32), (uint32_t)(x >> 32)) << 32) |
           row_shr<K>((uint32_t)x, (uint32_t)x);
}
__device__ __forceinline__ uint32_t lane_value(uint32_t x, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, l);
}
__device__ __forceinline__ uint64_t lane_value64(uint64_t x, int l) {
    return ((uint64_t)lane_value((uint32_t)(x >> 32), l) << 32) | lane_value((uint32_t)x, l);
}

// minimum over the wave, in every lane
__device__ __forceinline__ uint64_t wave_min64(uint64_t x) {
    x = umin64(x, row_shr64<1>(x));
    x = umin64(x, row_shr64<2>(x));
    x = umin64(x, row_shr64<4>(x));
    x = umin64(x, row_shr64<8>(x));  // lane 15 of each row: the row's minimum
    return umin64(umin64(lane_value64(x, 15), lane_value64(x, 31)), umin64(lane_value64(x, 47), lane_value64(x, 63)));
}
// OR over the wave, in every lane
__device__ __forceinline__ uint32_t wave_or32(uint32_t x) {
    x |= row_shr<1>(0u, x);
    x |= row_shr<2>(0u, x);
    x |= row_shr<4>(0u, x);
    x |= row_shr<8>(0u, x);
    return lane_value(x, 15) | lane_value(x, 31) | lane_value(x, 47) | lane_value(x, 63);
}
// inclusive prefix sum over the wave
__device__ __forceinline__ uint32_t wave_scan32(uint32_t x) {
    x += row_shr<1>(0u, x);
    x += row_shr<2>(0u, x);
    x += row_shr<4>(0u, x);
    x += row_shr<8>(0u, x);  // prefix within the row
    const uint32_t r0 = lane_value(x, 15), r1 = lane_value(x, 31), r2 = lane_value(x, 47);
    const int row = wave_lane() >> 4;
    return x + (row >= 1 ? r0 : 0u) + (row >= 2 ? r1 : 0u) + (row >= 3 ? r2 : 0u);
}

// LDS scratch for block-wide reductions (one slot per wave).
template <int T>
struct Red {
    uint64_t k[T / kWave];
    uint32_t a[T / kWave];
    uint32_t b[T / kWave];
};

// Block-wide min of a 64-bit key and OR of 32-bit flags; every thread gets both.
template <int T>
__device__ __forceinline__ void block_min_or(uint64_t& key, uint32_t& flags, Red<T>& red) {
    key = wave_min64(key);
    flags = wave_or32(flags);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        red.k[w] = key;
        red.a[w] = flags;
    }
    __syncthreads();
    key = red.k[0];
    flags = red.a[0];
#pragma unroll
    for (int i = 1; i < T / kWave; ++i) {
        key = umin64(key, red.k[i]);
        flags |= red.a[i];
    }
    __syncthreads();
}

// Block-wide "any": true in every thread if pred is non-zero in some thread.
// Also a workgroup barrier.
template <int T>
__device__ __forceinline__ bool block_any(int pred, Red<T>& red) {
    const bool w = __builtin_amdgcn_ballot_w64(pred != 0) != 0;
    if ((threadIdx.x & (kWave - 1)) == 0) red.a[threadIdx.x / kWave] = w ? 1u : 0u;
    __syncthreads();
    uint32_t any = 0;
#pragma unroll
    for (int i = 0; i < T / kWave; ++i) any |= red.a[i];
    __syncthreads();
    return any != 0;
}

// Block-wide exclusive prefix sum; returns this thread's offset and the total.
template <int T>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t& total, Red<T>& red) {
    const uint32_t inc = wave_scan32(x);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == kWave - 1) red.b[w] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < T / kWave; ++i) {
        const uint32_t s = red.b[i];
        if (i < w) before += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return before + inc - x;
}

// Thread -> (row partition, lane) layout for a slice of S columns.
struct Layout {
    int L;   // lanes per row (power of two, <= T)
    int P;   // row partitions (T / L)
    int r;   // this thread's partition
    int c;   // this thread's lane
    int NG;  // column groups of 4 in the slice
};

template <int T>
__device__ __forceinline__ Layout make_layout(int S) {
    Layout lo;
    lo.NG = (S + 3) >> 2;
    int L = 1;
    while (L < lo.NG && L < T) L <<= 1;
    lo.L = L;
    lo.P = T / L;
    lo.r = threadIdx.x / L;
    lo.c = threadIdx.x % L;
    return lo;
}


// Matrix entries as stored.  int32_t is the caller's matrix (INT32_MAX = no
// edge).  uint16_t / uint8_t are exact compact copies that the library builds
// of a graph it will stream many times, when every finite weight fits below
// the type's all-ones code, which stands for "no edge".  Four consecutive
// entries (one column group) are read with one 16-, 8- or 4-byte load and
// widened to uint32 with the no-edge code mapped back to INT32_MAX.
template <typename E>
__device__ __forceinline__ uint32_t widen(uint32_t v);
template <>
__device__ __forceinline__ uint32_t widen<int32_t>(uint32_t v) { return v; }
template <>
__device__ __forceinline__ uint32_t widen<uint16_t>(uint32_t v) { return v == 0xffffu ? kInf : v; }
template <>
__device__ __forceinline__ uint32_t widen<uint8_t>(uint32_t v) { return v == 0xffu ? kInf : v; }

// Per-column candidate key of a round: the lexicographic minimum over the
// streamed rows u of (weight, u).  For the caller's int32 matrix a 64-bit key
// (W[u][v] << 32) | u.  For compact copies (n <= 65536) a 32-bit key
// (code << 16) | u built from the stored code itself: the no-edge code (all
// ones) sorts above every weight, so nothing is widened while streaming (3
// vector operations per entry: extract, shift-or, 32-bit minimum, instead of
// about 8 with widened 64-bit keys) and a lane's keys take half the registers.
template <typename E>
struct KeyOf {
    typedef uint64_t type;
};
template <>
struct KeyOf<uint16_t> {
    typedef uint32_t type;
};
template <>
struct KeyOf<uint8_t> {
    typedef uint32_t type;
};
template <typename E>
using key_t = typename KeyOf<E>::type;

template <typename E>
__device__ __forceinline__ key_t<E> key_none() {
    return (key_t<E>)~(key_t<E>)0;
}
// Key of an entry as read (the int32 bits, or the compact code) in row u.
template <typename E>
__device__ __forceinline__ key_t<E> key_make(uint32_t raw, uint32_t u) {
    if constexpr (sizeof(E) == 4) return ((uint64_t)raw << 32) | u;
    else return (raw << 16) | u;
}
// Weight of a key: INT32_MAX for no edge (and for the no-key value of compact
// keys); an int32 key above INT32_MAX holds a negative weight (or is no key).
template <typename E>
__device__ __forceinline__ uint32_t key_weight(key_t<E> k) {
    if constexpr (sizeof(E) == 4) {
        return (uint32_t)(k >> 32);
    } else {
        const uint32_t code = k >> 16;
        return code >= (uint32_t)(E)~(E)0 ? kInf : code;
    }
}
template <typename E>
__device__ __forceinline__ uint32_t key_row(key_t<E> k) {
    if constexpr (sizeof(E) == 4) return (uint32_t)k;
    else return k & 0xffffu;
}
// Entry value standing for "no column here" when a partial group is read.
template <typename E>
__device__ __forceinline__ uint32_t absent_code() {
    return sizeof(E) == 4 ? kInf : 0xffffu;
}
template <typename X>
__device__ __forceinline__ X key_min(X a, X b) {
    return b < a ? b : a;
}

// Columns of the slice held by one thread: G groups of 4.  dist and pred stay in
// registers for the whole solve and are written out once at the end (a8), so no
// per-column output address is kept live across the rounds.
template <int G, typename E = int32_t>
struct Cols {
    uint32_t dist[G][4];
    int32_t pred[G][4];
    key_t<E> best[G][4];
    uint32_t vis;  // bit 4k+j: visited, or not a column of the slice/matrix
};

// The matrix always lives in global memory (device or pinned host memory).
// Descriptors loaded from memory carry generic pointers, which the compiler
// would access with FLAT instructions; casting to the global address space
// makes the row loads plain global loads.
// (The host pass of the same source has no address spaces.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using global_ptr = const __attribute__((address_space(1))) T*;
#else
template <typename T>
using global_ptr = const T*;
#endif

// One column group as loaded (16, 8 or 4 bytes) and its widening to uint32.
template <typename E>
struct Raw;
typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned v2u __attribute__((ext_vector_type(2)));
template <>
struct Raw<int32_t> {
    typedef v4i type;
};
template <>
struct Raw<uint16_t> {
    typedef v2u type;
};
template <>
struct Raw<uint8_t> {
    typedef uint32_t type;
};

template <typename E>
__device__ __forceinline__ void unpack(const typename Raw<E>::type& x, uint32_t (&w)[4]);
template <>
__device__ __forceinline__ void unpack<int32_t>(const v4i& x, uint32_t (&w)[4]) {
    w[0] = (uint32_t)x.x;
    w[1] = (uint32_t)x.y;
    w[2] = (uint32_t)x.z;
    w[3] = (uint32_t)x.w;
}
// Compact entries stay as codes (see key_make).
template <>
__device__ __forceinline__ void unpack<uint16_t>(const v2u& x, uint32_t (&w)[4]) {
    w[0] = x.x & 0xffffu;
    w[1] = x.x >> 16;
    w[2] = x.y & 0xffffu;
    w[3] = x.y >> 16;
}
template <>
__device__ __forceinline__ void unpack<uint8_t>(const uint32_t& x, uint32_t (&w)[4]) {
    w[0] = x & 0xffu;
    w[1] = (x >> 8) & 0xffu;
    w[2] = (x >> 16) & 0xffu;
    w[3] = x >> 24;
}

// Rows list[r], list[r + P], ... of one column group (4 columns starting at p0
// within each row) into `best`.  FULL: the 4 entries exist and are aligned for
// one load; otherwise only the first `valid` are read, one by one.  NT: the
// loads carry the nontemporal hint, for matrices streamed once per solve (the
// whole-GPU solve) rather than reused from the caches across instances.
template <int U, bool FULL, typename E, bool NT>
__device__ __forceinline__ void stream_group(key_t<E> (&best)[4], const E* __restrict__ p0, int64_t ld,
                                             int valid, const int32_t* list, int m, int first, int step) {
    for (int i = first; i < m; i += step * U) {
        // past the end of the list, repeat its last row: a duplicate cannot change a minimum
        uint32_t uu[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int idx = i + q * step;
            uu[q] = (uint32_t)list[idx < m ? idx : m - 1];
        }
        uint32_t w[U][4];
        if (FULL) {
            // issue all U loads before using any of them: keeps U rows in flight per thread
            typename Raw<E>::type raw[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const global_ptr<typename Raw<E>::type> a =
                    reinterpret_cast<global_ptr<typename Raw<E>::type>>((global_ptr<E>)p0 + (int64_t)uu[q] * ld);
                raw[q] = NT ? __builtin_nontemporal_load(a) : *a;
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < U; ++q) unpack<E>(raw[q], w[q]);
        } else {
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const global_ptr<E> p = (global_ptr<E>)p0 + (int64_t)uu[q] * ld;
#pragma unroll
                for (int j = 0; j < 4; ++j) w[q][j] = j < valid ? (uint32_t)p[j] : absent_code<E>();
            }
        }
#pragma unroll
        for (int q = 0; q < U; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) best[j] = key_min(best[j], key_make<E>(w[q][j], uu[q]));
    }
}

// Stream rows list[r], list[r + P], ... (m entries in `list`, partition r) of
// the matrix restricted to the slice into the running per-column minima, U rows
// in flight per thread.  `width` = columns of the slice that exist in the
// matrix (<= S).  `vec`: row segments are aligned for whole-group loads (W
// aligned, ld and the slice start multiples of 4); otherwise, and for a
// partial last group, entries are read one by one.
template <int G, int U, typename E, bool NT = false>
__device__ __forceinline__ void stream_rows(Cols<G, E>& cs, const Layout& lo, const E* __restrict__ W,
                                            int64_t ld, int64_t col0, int width, bool vec,
                                            const int32_t* list, int m) {
    // One column group at a time keeps only U x 4 weights live per thread.
#pragma unroll
    for (int k = 0; k < G; ++k) {
        const int v0 = 4 * (lo.c + k * lo.L);
        if (v0 >= width) continue;
        const E* p0 = W + col0 + v0;
        if (vec && v0 + 3 < width)
            stream_group<U, true, E, NT>(cs.best[k], p0, ld, 4, list, m, lo.r, lo.P);
        else
            stream_group<U, false, E, NT>(cs.best[k], p0, ld, min(4, width - v0), list, m, lo.r, lo.P);
    }
}

// Merge the P partitions' minima into the owner threads (partition 0): every
// partition takes an LDS atomic minimum into one key per column, then the
// owners read the result and put the all-ones key back.  `mrg` (4 * L keys or
// more) is all ones between merges (clear_merge at the start of a solve).
// Only used when P > 1, which implies G == 1.
template <int T, int G, typename E>
__device__ __forceinline__ void merge_partitions(Cols<G, E>& cs, const Layout& lo, uint64_t* mrg) {
    if (lo.P == 1) return;
    key_t<E>* m = reinterpret_cast<key_t<E>*>(mrg);  // all-ones keys of either width
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (cs.best[0][j] != key_none<E>())
            __hip_atomic_fetch_min(&m[j * lo.L + lo.c], cs.best[0][j], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();
    if (lo.r == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            cs.best[0][j] = m[j * lo.L + lo.c];
            m[j * lo.L + lo.c] = key_none<E>();
        }
    }
}

// Fill the partition-merge area (n64 keys) with all ones; ordered before its
// first use by the workgroup barriers that precede any merge.
template <int T>
__device__ __forceinline__ void clear_merge(uint64_t* mrg, int n64) {
    for (int i = threadIdx.x; i < n64; i += T) mrg[i] = kNoKey;
}

// Minimum of key and OR of flags over the slice owners (the first L threads,
// partition 0); valid in the owners.  Threads that are not owners must pass
// kNoKey / 0.  When the owners fit in wave 0 this is a wave reduction with no
// workgroup barrier (and only wave 0 takes part); otherwise a block reduction
// that every thread must enter.
template <int T>
__device__ __forceinline__ void owner_min_or(uint64_t& key, uint32_t& flags, int L, Red<T>& red) {
    if (L <= kWave) {
        if (threadIdx.x < kWave) {
            key = wave_min64(key);
            flags = wave_or32(flags);
        }
        return;
    }
    block_min_or<T>(key, flags, red);
}

// Exclusive prefix sum over the owners (same rules as owner_min_or); `total`
// gets the sum.
template <int T>
__device__ __forceinline__ uint32_t owner_excl_scan(uint32_t x, uint32_t& total, int L, Red<T>& red) {
    if (L <= kWave) {
        uint32_t inc = 0;
        if (threadIdx.x < kWave) {
            inc = wave_scan32(x);
            total = (uint32_t)__builtin_amdgcn_readlane((int)inc, kWave - 1);
        }
        return inc - x;
    }
    return block_excl_scan<T>(x, total, red);
}

template <int G, typename E>
__device__ __forceinline__ void reset_best(Cols<G, E>& cs) {
#pragma unroll
    for (int k = 0; k < G; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) cs.best[k][j] = key_none<E>();
}

// Local vertex index of (k, j) for this thread.
__device__ __forceinline__ int local_col(const Layout& lo, int k, int j) {
    return 4 * (lo.c + k * lo.L) + j;
}

// Initialise the owned columns: dist = inf (0 at the source), pred = -1, not
// visited; columns past the slice/matrix are flagged visited so they never take part.
template <int G, typename E>
__device__ __forceinline__ void init_cols(Cols<G, E>& cs, const Layout& lo, int64_t col0, int width,
                                          int32_t src) {
    cs.vis = 0;
#pragma unroll
    for (int k = 0; k < G; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int v = local_col(lo, k, j);
            const bool mine = lo.r == 0 && k * lo.L + lo.c < lo.NG && v < width;
            cs.dist[k][j] = (mine && col0 + v == src) ? 0u : kInf;
            cs.pred[k][j] = -1;
            if (!mine) cs.vis |= 1u << (4 * k + j);
        }
    reset_best(cs);
}

// Lowest (dist, vertex) key among unvisited owned columns.
template <int G, typename E>
__device__ __forceinline__ uint64_t local_argmin(const Cols<G, E>& cs, const Layout& lo, int64_t col0) {
    uint64_t key = kNoKey;
#pragma unroll
    for (int k = 0; k < G; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (!(cs.vis >> (4 * k + j) & 1u))
                key = umin64(key, make_key(cs.dist[k][j], (uint32_t)(col0 + local_col(lo, k, j))));
    return key;
}

// Bitmask of unvisited owned columns whose dist equals d (the round's bucket).
template <int G, typename E>
__device__ __forceinline__ uint32_t bucket_mask(const Cols<G, E>& cs, uint32_t d) {
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < G; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (!(cs.vis >> (4 * k + j) & 1u) && cs.dist[k][j] == d) m |= 1u << (4 * k + j);
    return m;
}

// Candidate dist of a column from the round's minimum key (d + min weight);
// returns kInf + something >= dist when there is no usable edge.  Sets *neg if
// the minimum weight read as uint32 exceeds INT32_MAX (a negative weight).
template <typename E>
__device__ __forceinline__ uint32_t candidate(key_t<E> best, uint32_t d, uint32_t& neg) {
    const uint32_t w = key_weight<E>(best);
    if (w > kInf) {
        neg |= best != key_none<E>() ? kStatusNegWeight : 0u;
        return 0xffffffffu;
    }
    return d + w;  // d < 2^31-1 and w <= 2^31-1: no wrap
}

// Zero-weight hazard of a fused round: an unvisited vertex outside the bucket
// (dist > d) reachable from the bucket by a weight-0 edge would join the bucket
// during the round and change the order Algorithm 1 settles it in.
template <int G, typename E>
__device__ __forceinline__ uint32_t zero_hazard(const Cols<G, E>& cs, uint32_t d) {
    uint32_t z = 0;
#pragma unroll
    for (int k = 0; k < G; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (!(cs.vis >> (4 * k + j) & 1u) && cs.dist[k][j] > d &&
                key_weight<E>(cs.best[k][j]) == 0u)
                z = 1;
    return z;
}

// Apply a fused round: the bucket (mask) becomes visited; every other unvisited
// column takes its candidate if strictly smaller (pred = the candidate's row).
template <int G, typename E>
__device__ __forceinline__ uint32_t commit_fused(Cols<G, E>& cs, uint32_t d, uint32_t bucket) {
    uint32_t neg = 0;
    cs.vis |= bucket;
#pragma unroll
    for (int k = 0; k < G; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (cs.vis >> (4 * k + j) & 1u) continue;
            const uint32_t c = candidate<E>(cs.best[k][j], d, neg);
            if (c < cs.dist[k][j]) {
                cs.dist[k][j] = c;
                cs.pred[k][j] = (int32_t)key_row<E>(cs.best[k][j]);
            }
        }
    reset_best(cs);
    return neg;
}

// Would-be dist of a column if the pending fused round were applied (kNoKey-style
// sentinel 0xffffffff for columns that are visited or in the bucket).
template <int G, typename E>
__device__ __forceinline__ uint32_t would_be(const Cols<G, E>& cs, int k, int j, uint32_t d,
                                             uint32_t bucket, uint32_t& neg) {
    const uint32_t bit = 1u << (4 * k + j);
    if ((cs.vis | bucket) & bit) return 0xffffffffu;
    const uint32_t c = candidate<E>(cs.best[k][j], d, neg);
    return c < cs.dist[k][j] ? c : cs.dist[k][j];
}

// Write the owned dist and pred values out (a8: writeback): one 16-byte store
// per column group and array where the group is whole and aligned.
template <int G, typename E>
__device__ __forceinline__ void write_out(const Cols<G, E>& cs, const Layout& lo, int64_t col0, int width,
                                          int32_t* __restrict__ dist, int32_t* __restrict__ pred) {
    if (lo.r != 0) return;
#pragma unroll
    for (int k = 0; k < G; ++k) {
        if (k * lo.L + lo.c >= lo.NG) continue;
        const int v0 = local_col(lo, k, 0);
        int32_t* dp = dist + col0 + v0;
        int32_t* pp = pred + col0 + v0;
        if (v0 + 3 < width && (((uintptr_t)dp | (uintptr_t)pp) & 15u) == 0) {
            *reinterpret_cast<v4i*>(dp) = v4i{(int)cs.dist[k][0], (int)cs.dist[k][1], (int)cs.dist[k][2],
                                              (int)cs.dist[k][3]};
            *reinterpret_cast<v4i*>(pp) = v4i{cs.pred[k][0], cs.pred[k][1], cs.pred[k][2], cs.pred[k][3]};
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (v0 + j < width) {
                    dp[j] = (int32_t)cs.dist[k][j];
                    pp[j] = cs.pred[k][j];
                }
        }
    }
}

}  // namespace sssp
