// Several sources on one matrix, solved in lockstep by one gang: each row is
// read once per round for every source whose bucket holds it.
//
// Algorithm 1 (Section III-A) relaxes the row of every settled vertex into
// dist[]; a fused round (kernels.hip) settles a source's whole bucket, all
// unvisited vertices at its minimal dist, at once.  K sources of one matrix
// run their fused rounds side by side: in round r, source k settles its r-th
// bucket B_k.  The union of the K buckets is streamed once, each row with the
// mask of the sources whose bucket holds it, and each source applies only the
// rows of its own bucket, so every source computes exactly what it computes
// alone.  Only matrices whose off-diagonal weights are all >= 1 are solved
// this way: then a fused round never meets a zero-weight hazard and never has
// to fall back to a single-vertex step, so the sources stay in lockstep.
//
// Mapping.  A gang of `nwg` workgroups; member g owns columns [g*S, g*S + S) of
// every source.  Its T threads form P partitions of L lanes (make_layout); lane
// c holds columns 4c..4c+3 (S <= 4L), and partition r holds the sources
// r, r + P, ..., r + (KP-1)P, so each thread keeps dist, pred and the round's
// best key of its 4 columns for its KP sources in registers.  Every partition
// streams the whole union list (rows that hold none of its sources are
// skipped); partitions read the same rows, from the caches after the first.
//
// Exchange per round (records in the arena, stamped as in solve.h): member m
// publishes, per source k, the lowest (dist, vertex) key among its unvisited
// columns and how many of its columns sit at that dist, plus one list of its
// columns at their local minimum for any source: (local column << 16) | mask.
// After the exchange every member takes, per source, the global minimum d_k;
// a member qualifies for source k when its local minimum is d_k, and an entry
// of its list counts for source k when bit k is set and the member qualifies.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "engine.h"
#include "solve.h"

namespace sssp {

constexpr int kMultiMax = 16;  // sources per group (16 mask bits per list entry)

// One source of a group: its vertex and its outputs.
struct MultiSrc {
    int32_t src;
    int32_t pad;
    int32_t* dist;
    int32_t* pred;
};

// Record of a member, in 64-bit words: [0] stamp, [1] entries in the member's
// list, [2, 2 + K) the member's lowest key per source (kRecNone: none), then the
// number of its columns at that key's dist, two 32-bit counts per word.  Every
// word but the stamp has bit 63 clear, so no stale word passes for a stamp.
constexpr uint64_t kRecNone = 0x7fffffffffffffffull;
__host__ __device__ constexpr int multi_rec_words(int K) { return ((2 + K + (K + 1) / 2) + 3) & ~3; }

// Arena bytes of a group's records and lists (double-buffered by exchange parity).
__host__ __device__ inline unsigned long long multi_scratch_bytes(int K, int parts, int S) {
    const unsigned long long b =
        2ull * parts * multi_rec_words(K) * 8ull + 2ull * parts * (unsigned long long)S * 4ull;
    return (b + 255) & ~255ull;
}

template <int T>
struct SharedMulti {
    uint64_t key[kMultiMax];   // this member's lowest key per source, being reduced
    uint64_t gkey[kMultiMax];  // the gang's lowest key per source (after an exchange)
    uint32_t cnt[kMultiMax];   // this member's columns at its lowest dist, per source
    uint32_t qual[T];          // per member: the sources it qualifies for (after an exchange)
    uint32_t emask[kCap];      // staged union entries: source mask (rows in SharedSolve::list)
    uint32_t settled;          // vertices the round settles, over all sources
};

template <int T>
__shared__ SharedMulti<T> g_mh;

// Minimum of a 64-bit key over the L lanes of this thread's partition (L a
// power of two); valid in every lane of the partition when L <= 64, and in the
// first lane of each wave when L > 64 (the caller then combines waves).
__device__ __forceinline__ uint64_t segment_min64(uint64_t x, int L) {
    const int lane = wave_lane();
    const int span = L < kWave ? L : kWave;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        if (o < span) {
            const uint64_t y = ((uint64_t)xor_lane32((uint32_t)(x >> 32), lane, o) << 32) |
                               xor_lane32((uint32_t)x, lane, o);
            x = umin64(x, y);
        }
    return x;
}
__device__ __forceinline__ uint32_t segment_sum32(uint32_t x, int L) {
    const int lane = wave_lane();
    const int span = L < kWave ? L : kWave;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        if (o < span) x += xor_lane32(x, lane, o);
    return x;
}

// Rank g of a gang of nwg workgroups solving the K sources of srcs on W
// (n x n, row stride ld, entries of type E).  recs: 2 * nwg * multi_rec_words(K)
// words; lists: 2 * nwg * S entries.  Returns false if an exchange timed out.
template <int T, int KP, typename E>
__device__ __forceinline__ bool solve_multi(const E* __restrict__ W, int64_t ld, int32_t n,
                                            const MultiSrc* __restrict__ srcs, int K, bool vec, int S, int g, int nwg,
                                            long long timeout, uint64_t* __restrict__ recs,
                                            uint32_t* __restrict__ lists, SharedSolve<T>& sh, SharedMulti<T>& mh,
                                            SolveStats& st, uint32_t epoch) {
    static_assert(T == kCap, "one staged entry per thread");
    const int64_t col0 = (int64_t)g * S;
    const int width = (int)max((int64_t)0, min((int64_t)S, (int64_t)n - col0));
    const Layout lo = make_layout<T>(S);
    const int rw = multi_rec_words(K);
    uint32_t* colmask = reinterpret_cast<uint32_t*>(sh.mrg);  // S <= 4T <= 8T words
    const bool mycols = lo.c < lo.NG;
    // this partition's sources, as a mask
    uint32_t mine = 0;
#pragma unroll
    for (int i = 0; i < KP; ++i)
        if (lo.r + i * lo.P < K) mine |= 1u << (lo.r + i * lo.P);

    uint32_t dist[KP][4];
    int32_t pred[KP][4];
    key_t<E> best[KP][4];
    uint32_t vis = 0;  // bit 4i + j: column j of source slot i visited, or absent
#pragma unroll
    for (int i = 0; i < KP; ++i) {
        const int k = lo.r + i * lo.P;
        const int32_t sk = k < K ? srcs[k].src : -1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int v = 4 * lo.c + j;
            const bool ok = k < K && mycols && v < width;
            dist[i][j] = (ok && col0 + v == sk) ? 0u : kInf;
            pred[i][j] = -1;
            best[i][j] = key_none<E>();
            if (!ok) vis |= 1u << (4 * i + j);
        }
    }
    for (int i = threadIdx.x; i < S; i += T) colmask[i] = 0;
    if (threadIdx.x < kMultiMax) {
        mh.key[threadIdx.x] = kRecNone;
        mh.cnt[threadIdx.x] = 0;
    }
    __syncthreads();

    uint32_t b = 0;  // exchanges passed
    auto rec = [&](uint32_t slot, int m) { return recs + ((size_t)slot * nwg + m) * rw; };
    auto lst = [&](uint32_t slot, int m) { return lists + ((size_t)slot * nwg + m) * S; };

    // Publish this member's committed state into record slot (b & 1), then exchange.
    auto publish_exchange = [&]() -> bool {
        // per source: the lowest (dist, vertex) key over the member's unvisited columns
#pragma unroll
        for (int i = 0; i < KP; ++i) {
            uint64_t key = kRecNone;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (!(vis >> (4 * i + j) & 1u))
                    key = umin64(key, make_key(dist[i][j], (uint32_t)(col0 + 4 * lo.c + j)));
            key = segment_min64(key, lo.L);
            const int k = lo.r + i * lo.P;
            if (k < K && (threadIdx.x & (kWave - 1) & (lo.L - 1)) == 0 && key != kRecNone)
                __hip_atomic_fetch_min(&mh.key[k], key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __syncthreads();
        // mark the columns at each source's local minimum, and count them
#pragma unroll
        for (int i = 0; i < KP; ++i) {
            const int k = lo.r + i * lo.P;
            uint32_t c = 0;
            if (k < K) {
                const uint64_t key = mh.key[k];
                const uint32_t dl = (uint32_t)(key >> 32);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (dl < kInf && !(vis >> (4 * i + j) & 1u) && dist[i][j] == dl) {
                        __hip_atomic_fetch_or(&colmask[4 * lo.c + j], 1u << k, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_WORKGROUP);
                        ++c;
                    }
            }
            c = segment_sum32(c, lo.L);
            if (k < K && (threadIdx.x & (kWave - 1) & (lo.L - 1)) == 0 && c)
                __hip_atomic_fetch_add(&mh.cnt[k], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __syncthreads();
        // the member's list: its marked columns in order, (column << 16) | mask
        const uint32_t slot = b & 1;
        uint32_t* out = lst(slot, g);
        uint32_t m4[4];
        uint32_t here = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int v = threadIdx.x * 4 + q;
            m4[q] = v < S ? colmask[v] : 0u;
            here += m4[q] != 0;
        }
        uint32_t total = 0;
        uint32_t pos = block_excl_scan<T>(here, total, sh.red);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int v = threadIdx.x * 4 + q;
            if (m4[q]) st_agent(&out[pos++], ((uint32_t)v << 16) | m4[q]);
            if (v < S) colmask[v] = 0;
        }
        uint64_t* r = rec(slot, g);
        if (threadIdx.x == 0) st_agent(&r[1], (uint64_t)total);
        if (threadIdx.x < K) {
            st_agent(&r[2 + threadIdx.x], mh.key[threadIdx.x]);
            mh.key[threadIdx.x] = kRecNone;
        }
        if (threadIdx.x < (K + 1) / 2) {
            const uint32_t lo32 = mh.cnt[2 * threadIdx.x];
            const uint32_t hi32 = 2 * threadIdx.x + 1 < K ? mh.cnt[2 * threadIdx.x + 1] : 0u;
            st_agent(&r[2 + K + threadIdx.x], ((uint64_t)hi32 << 32) | lo32);
        }
        __syncthreads();
        if (threadIdx.x < kMultiMax) mh.cnt[threadIdx.x] = 0;
        ++b;
        return stamp_exchange<T>(rec((b - 1) & 1, 0), (size_t)rw, g, exchange_stamp(epoch, b), (uint32_t)nwg,
                                 timeout, sh.red);
    };

    bool ok = publish_exchange();
    while (ok) {
        // the gang's records: per source the lowest key; per member the sources it
        // qualifies for and the length of its list if it qualifies for any
        const uint32_t slot = (b - 1) & 1;
        if (threadIdx.x < kMultiMax) mh.gkey[threadIdx.x] = kRecNone;
        if (threadIdx.x == 0) mh.settled = 0;
        __syncthreads();
        uint64_t mk[kMultiMax];
        if ((int)threadIdx.x < nwg) {
            const uint64_t* r = rec(slot, threadIdx.x);
#pragma unroll
            for (int k = 0; k < kMultiMax; ++k) {
                mk[k] = k < K ? ld_agent(&r[2 + k]) : kRecNone;
                if (mk[k] != kRecNone)
                    __hip_atomic_fetch_min(&mh.gkey[k], mk[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        __syncthreads();
        uint32_t q = 0, len = 0;
        if ((int)threadIdx.x < nwg) {
            const uint64_t* r = rec(slot, threadIdx.x);
            // the count words and the list length loaded together (a load per
            // qualifying source would be waited for before the next)
            uint64_t cwv[kMultiMax / 2];
#pragma unroll
            for (int k2 = 0; k2 < kMultiMax / 2; ++k2) cwv[k2] = 2 * k2 < K ? ld_agent(&r[2 + K + k2]) : 0ull;
            const uint32_t lenv = (uint32_t)ld_agent(&r[1]);
            uint32_t settled = 0;
#pragma unroll
            for (int k = 0; k < kMultiMax; ++k)
                if (k < K && mk[k] != kRecNone && (uint32_t)(mk[k] >> 32) == (uint32_t)(mh.gkey[k] >> 32) &&
                    (uint32_t)(mh.gkey[k] >> 32) < kInf) {
                    q |= 1u << k;
                    settled += (uint32_t)(k & 1 ? cwv[k / 2] >> 32 : cwv[k / 2]);
                }
            if (q) {
                len = lenv;
                __hip_atomic_fetch_add(&mh.settled, settled, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            mh.qual[threadIdx.x] = q;
        }
        uint32_t M = 0;
        const uint32_t pre = block_excl_scan<T>(len, M, sh.red);
        if ((int)threadIdx.x < nwg) {
            sh.pre[threadIdx.x] = pre;
            sh.cnt[threadIdx.x] = len;
        }
        __syncthreads();
        if (M == 0) break;  // no source has a reachable unvisited vertex left
        ++st.rounds;
        st.settled += mh.settled;
        uint32_t dk[KP];
#pragma unroll
        for (int i = 0; i < KP; ++i) {
            const int k = lo.r + i * lo.P;
            dk[i] = k < K ? (uint32_t)(mh.gkey[k] >> 32) : kInf;
        }

        // stream the union, chunk by chunk
        const uint32_t* rl = lists + (size_t)slot * nwg * S;
        for (uint32_t e0 = 0; e0 < M; e0 += kCap) {
            const uint32_t e = e0 + threadIdx.x;
            if (e < M) {
                int lo_i = 0, hi_i = nwg - 1;  // last member whose prefix is <= e
                while (lo_i < hi_i) {
                    const int mid = (lo_i + hi_i + 1) >> 1;
                    if (sh.pre[mid] <= e) lo_i = mid;
                    else hi_i = mid - 1;
                }
                const uint32_t x = ld_agent(&rl[(size_t)lo_i * S + (e - sh.pre[lo_i])]);
                sh.list[threadIdx.x] = (int32_t)((int64_t)lo_i * S + (x >> 16));
                mh.emask[threadIdx.x] = x & 0xffffu & mh.qual[lo_i];
            }
            __syncthreads();
            const int m = (int)min((uint32_t)kCap, M - e0);
            constexpr int U = KP <= 2 ? 8 : 4;  // rows in flight (fewer when a thread holds 4 sources)
            if (mycols && mine) {
                const int v0 = 4 * lo.c;
                const bool full = vec && v0 + 3 < width;
                for (int i0 = 0; i0 < m; i0 += U) {
                    uint32_t row[U], msk[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int idx = i0 + u;
                        msk[u] = idx < m ? mh.emask[idx] & mine : 0u;
                        row[u] = idx < m ? (uint32_t)sh.list[idx] : 0u;
                    }
                    uint32_t w[U][4];
                    if (full) {
                        typename Raw<E>::type raw[U];
#pragma unroll
                        for (int u = 0; u < U; ++u)
                            if (msk[u]) {
                                const global_ptr<typename Raw<E>::type> a = reinterpret_cast<global_ptr<typename Raw<E>::type>>(
                                    (global_ptr<E>)W + (int64_t)row[u] * ld + col0 + v0);
                                raw[u] = *a;
                            }
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int u = 0; u < U; ++u)
                            if (msk[u]) unpack<E>(raw[u], w[u]);
                    } else {
#pragma unroll
                        for (int u = 0; u < U; ++u)
                            if (msk[u]) {
                                const global_ptr<E> p = (global_ptr<E>)W + (int64_t)row[u] * ld + col0 + v0;
#pragma unroll
                                for (int j = 0; j < 4; ++j) w[u][j] = v0 + j < width ? (uint32_t)p[j] : absent_code<E>();
                            }
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u)
#pragma unroll
                        for (int i = 0; i < KP; ++i)
                            if (msk[u] >> (lo.r + i * lo.P) & 1u)
#pragma unroll
                                for (int j = 0; j < 4; ++j) best[i][j] = key_min(best[i][j], key_make<E>(w[u][j], row[u]));
                }
            }
            __syncthreads();
        }

        // commit: each source settles its bucket and takes the candidates of its rows
        uint32_t neg = 0;
#pragma unroll
        for (int i = 0; i < KP; ++i) {
            if (dk[i] >= kInf) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t bit = 1u << (4 * i + j);
                if (vis & bit) continue;
                if (dist[i][j] == dk[i]) {
                    vis |= bit;
                    continue;
                }
                const uint32_t c = candidate<E>(best[i][j], dk[i], neg);
                if (c < dist[i][j]) {
                    dist[i][j] = c;
                    pred[i][j] = (int32_t)key_row<E>(best[i][j]);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < KP; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) best[i][j] = key_none<E>();
        st.status |= neg;
        ok = publish_exchange();
    }
    if (!ok) st.status |= kStatusTimeout;
    // a8: dist and pred of every source's owned columns
#pragma unroll
    for (int i = 0; i < KP; ++i) {
        const int k = lo.r + i * lo.P;
        if (k >= K || !mycols) continue;
        const int v0 = 4 * lo.c;
        int32_t* dp = srcs[k].dist + col0 + v0;
        int32_t* pp = srcs[k].pred + col0 + v0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (v0 + j < width) {
                dp[j] = (int32_t)dist[i][j];
                pp[j] = pred[i][j];
            }
    }
    st.barriers += b;
    uint32_t s = st.status;
    uint64_t dummy = kNoKey;
    block_min_or<T>(dummy, s, sh.red);
    st.status = s;
    return ok;
}

}  // namespace sssp
