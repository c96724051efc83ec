// Round engines shared by the kernels: one workgroup solving a whole instance
// (solve_single) and a gang of workgroups that each own a column slice and
// meet at one barrier per round (solve_gang), with the barrier, the per-round
// records and the bucket gather they use.  See kernels.hip for the method.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "engine.h"
#include "sssp_internal.h"

namespace sssp {

constexpr int kCap = 1024;  // bucket rows staged in LDS per chunk
constexpr uint32_t kPairChunks = 8;  // chunks from which a round is balanced within pairs (solve_gang)
constexpr uint32_t kPairUnit = 256;  // rows per claim unit of a balanced round

template <int T>
struct SharedSolve {
    Red<T> red;
    int32_t list[kCap];
    uint64_t mrg[4 * T];
    uint32_t pre[T];
    uint32_t cnt[T];
    uint64_t rk;  // read_records results for the whole workgroup
    uint32_t rz, rm;
    uint32_t claim[2];    // chunk claims of a balanced round, broadcast by thread 0
    uint32_t late;        // a member's record did not arrive in time (read_records)
    uint32_t stage_late;  // a bucket entry did not arrive in time (set once; the solve then ends)
    int32_t item;
    uint32_t flag;
};

struct SolveStats {
    unsigned long long rounds, settled, fallbacks, barriers;
    uint32_t status;
};

// The workgroup's LDS state, at namespace scope so that solver variants compiled
// as separate functions still address it as LDS.
template <int T>
__shared__ SharedSolve<T> g_sh;

// bit of local column v (0 <= v < width) if this thread owns it, else 0
__device__ __forceinline__ uint32_t owner_bit(const Layout& lo, int64_t v, int width) {
    if (v < 0 || v >= width || lo.r != 0) return 0;
    const int64_t gi = v >> 2;
    if (gi % lo.L != lo.c) return 0;
    const int k = (int)(gi / lo.L);
    return 1u << (4 * k + (int)(v & 3));
}

// ---------------------------------------------------------------------------
// One workgroup, whole row.
// ---------------------------------------------------------------------------
template <int T, int G, int U, typename E>
__device__ __forceinline__ void solve_single(const E* __restrict__ W, int64_t ld, int32_t n, int32_t src,
                             int32_t* __restrict__ dist, int32_t* __restrict__ pred, bool vec,
                             bool literal, SharedSolve<T>& sh, SolveStats& st, Ctl* trace) {
    const Layout lo = make_layout<T>(n);
    Cols<G, E> cs;
    init_cols(cs, lo, 0, n, src);
    clear_merge<T>(sh.mrg, 4 * T);
    for (;;) {
        // a2/a3: argmin over unvisited vertices, lowest index on ties
        uint64_t key = local_argmin(cs, lo, 0);
        uint32_t none = 0;
        block_min_or<T>(key, none, sh.red);
        const uint32_t d = (uint32_t)(key >> 32);
        if (key == kNoKey || d >= kInf) break;  // a4: nothing reachable is left
        const uint32_t u0 = (uint32_t)key;
        const long long t_round = wall_clock64();
        uint32_t bucket;
        uint32_t M;
        if (literal) {
            bucket = owner_bit(lo, u0, n);
            M = 1;
            if (threadIdx.x == 0) sh.list[0] = (int32_t)u0;
            __syncthreads();
            stream_rows<G, U, E>(cs, lo, W, ld, 0, n, vec, sh.list, 1);
        } else {
            bucket = bucket_mask(cs, d);
            const uint32_t base = block_excl_scan<T>(__popc(bucket), M, sh.red);
            for (uint32_t e0 = 0; e0 < M; e0 += kCap) {
                uint32_t rank = base;
#pragma unroll
                for (int k = 0; k < G; ++k)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (bucket >> (4 * k + j) & 1u) {
                            if (rank >= e0 && rank < e0 + kCap)
                                sh.list[rank - e0] = local_col(lo, k, j);
                            ++rank;
                        }
                __syncthreads();
                stream_rows<G, U, E>(cs, lo, W, ld, 0, n, vec, sh.list, (int)min((uint32_t)kCap, M - e0));
                __syncthreads();
            }
        }
        merge_partitions<T, G>(cs, lo, sh.mrg);
        ++st.rounds;
        if (trace && threadIdx.x == 0 && st.rounds <= (unsigned long long)kTraceCap) {
            trace->trace_t[st.rounds - 1] = t_round;
            trace->trace_m[st.rounds - 1] = M;
        }
        if (!literal) {
            uint32_t z = lo.r == 0 ? zero_hazard(cs, d) : 0u;
            uint64_t dummy = kNoKey;
            block_min_or<T>(dummy, z, sh.red);
            if (z) {
                // discard the fused round; settle only u0 (one literal step)
                ++st.fallbacks;
                st.status |= kStatusZeroFallback;
                reset_best(cs);
                if (threadIdx.x == 0) sh.list[0] = (int32_t)u0;
                __syncthreads();
                stream_rows<G, U, E>(cs, lo, W, ld, 0, n, vec, sh.list, 1);
                merge_partitions<T, G>(cs, lo, sh.mrg);
                bucket = owner_bit(lo, u0, n);
                M = 1;
            }
        }
        // a5/a6: settle the bucket and relax
        if (lo.r == 0) st.status |= commit_fused(cs, d, bucket);
        else reset_best(cs);
        st.settled += M;
    }
    write_out(cs, lo, 0, n, dist, pred);  // a8
    if (trace && threadIdx.x == 0) {
        const unsigned long long nr = st.rounds < (unsigned long long)kTraceCap ? st.rounds : kTraceCap;
        trace->trace_t[nr] = wall_clock64();
        trace->trace_n = (uint32_t)nr;
    }
}
// ---------------------------------------------------------------------------
// Gang solve: `nwg` workgroups (ranks 0..nwg-1) each own a column slice of S
// columns and meet at one barrier per round.  Used by the whole-GPU kernel
// (the gang is the grid) and by the serving kernel (a gang per large query).
// ---------------------------------------------------------------------------

// Exchange number b of a gang of `members` workgroups, rank g: publishes this
// member's record in `slot` (filled before; records `stride` 64-bit words apart,
// the stamp in the first) and waits until every member's record there carries
// the same stamp.  Records and list entries are
// written and read with agent-scope atomic accesses (coherent across XCDs
// without cache writebacks or invalidates), so the only ordering needed is that
// a member's other stores are complete before its stamp: every wave waits for
// its stores (s_waitcnt 0) before the workgroup barrier, and thread 0 stores the
// stamp after it.  A reader reads a record's other fields only after seeing its
// stamp.  Thread t < members polls record t; nothing is counted in a shared
// word.  Gives up after `timeout` wall-clock ticks (returns false) so that a
// gang that is not co-resident cannot hang.  stamp = exchange_stamp(epoch, b)
// with an epoch unique to this use of the records' memory, so neither a record
// nor any other word left there by an earlier use ever matches.
template <int T>
__device__ __forceinline__ bool stamp_exchange(uint64_t* slot, size_t stride, int g, uint64_t stamp,
                                               uint32_t members, long long timeout, Red<T>& red) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (members == 1) return true;  // one workgroup: its own barrier orders everything
    if (threadIdx.x == 0) {
        stress_delay((uint32_t)(stamp ^ (stamp >> 29)));
        __builtin_amdgcn_s_waitcnt(0);
        st_agent(&slot[(size_t)g * stride], stamp);
    }
    int late = 0;
    if (threadIdx.x < members) {
        // polls back off (up to ~1 us apart) so that members waiting through a
        // long round do not load the memory system the others are streaming from
        const long long t0 = wall_clock64();
        unsigned naps = 1;
        while (ld_agent(&slot[(size_t)threadIdx.x * stride]) != stamp) {
            for (unsigned i = 0; i < naps; ++i) __builtin_amdgcn_s_sleep(1);
            if (naps < 32) naps <<= 1;
            if (wall_clock64() - t0 > timeout) {
                late = 1;
                break;
            }
        }
    }
    return !block_any<T>(late, red);
}

// The exchange over 32-byte Pub records (stamp first).
template <int T>
__device__ __forceinline__ bool gang_exchange(Pub* slot, int g, uint64_t stamp, uint32_t members, long long timeout,
                                              Red<T>& red) {
    return stamp_exchange<T>(&slot->stamp, sizeof(Pub) / sizeof(uint64_t), g, stamp, members, timeout, red);
}

// Thread 0 of each member calls this once when it is done with the gang's
// words; the last of `members` resets them for the next use.  Returns true in
// the last member.
__device__ __forceinline__ bool gang_leave(Bar* bw, uint32_t members) {
    stress_delay(0xfffffffeu);
    const uint32_t prev = __hip_atomic_fetch_add(&bw->exit, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (prev != members - 1) return false;
    __hip_atomic_store(&bw->bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&bw->gen, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&bw->exit, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// The last workgroup of a launch publishes the launch's statistics and resets
// the barrier words, the ticket counter and the accumulators for the next launch.
__device__ __forceinline__ void finish_launch(Ctl* ctl, const SolveStats& st, bool add_stats) {
    if (threadIdx.x != 0) return;
    if (st.status) __hip_atomic_fetch_or(&ctl->status_acc, st.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (add_stats) {
        __hip_atomic_fetch_add(&ctl->acc[kStatRounds], st.rounds, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&ctl->acc[kStatSettled], st.settled, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&ctl->acc[kStatFallbacks], st.fallbacks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&ctl->acc[kStatBarriers], st.barriers, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    stress_delay(0xffffffffu);
    const uint32_t prev = __hip_atomic_fetch_add(&ctl->b.exit, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == gridDim.x - 1) {
        for (int i = 0; i < kStatCount; ++i) {
            ctl->last[i] = __hip_atomic_load(&ctl->acc[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->acc[i], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        ctl->status = __hip_atomic_exchange(&ctl->status_acc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // a new epoch for the next launch's exchange records
        __hip_atomic_fetch_add(&ctl->epoch, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->next_item, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->b.bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->b.gen, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->b.exit, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Clear this member's tagged words (both slots of its record and of its list
// region) before the solve's first exchange; see tag_word.
template <int T>
__device__ __forceinline__ void clear_tagged(uint64_t* __restrict__ recs, uint64_t* __restrict__ lists,
                                             uint32_t* __restrict__ ctr, uint64_t* __restrict__ done, int g, int nwg,
                                             int S) {
    if (threadIdx.x < 2 * kRecFields)
        st_agent(rec_word(recs, nwg, threadIdx.x / kRecFields, threadIdx.x % kRecFields, g), (uint64_t)0);
    if (threadIdx.x == 2 * kRecFields) st_agent(&done[2 * g], (uint64_t)0);
    if (threadIdx.x == 2 * kRecFields + 1) st_agent(&ctr[4 * g], 0u);
    if (threadIdx.x == 2 * kRecFields + 2) st_agent(&ctr[4 * g + 1], 0u);
    for (int i = threadIdx.x; i < 2 * S; i += T) {
        const int s = i >= S ? 1 : 0;
        st_agent(&lists[((size_t)s * nwg + g) * S + (i - s * S)], (uint64_t)0);
    }
}

// Publish this workgroup's record for exchange `tag`: the lowest (dist, vertex)
// key among `cand` (one would-be dist per owned column, 0xffffffff = excluded),
// the vertices of the slice at that dist (list entries; none if `entries` is
// false) and the zero-weight hazard flag, every word tagged.  Nothing waits for
// the stores: readers check each word's tag.
template <int T, int G>
__device__ __forceinline__ void publish(const uint32_t (&cand)[G][4], const Layout& lo, int64_t col0,
                                        uint32_t zero, bool entries, uint32_t tag, uint64_t* __restrict__ recs,
                                        int nwg, int g, uint64_t* __restrict__ list, SharedSolve<T>& sh) {
    uint64_t key = kNoKey;
    if (lo.r == 0) {
#pragma unroll
        for (int k = 0; k < G; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (cand[k][j] != 0xffffffffu)
                    key = umin64(key, make_key(cand[k][j], (uint32_t)(col0 + local_col(lo, k, j))));
    }
    owner_min_or<T>(key, zero, lo.L, sh.red);
    const uint32_t dmin = (uint32_t)(key >> 32);
    uint32_t mask = 0;
    if (lo.r == 0 && key != kNoKey && dmin < kInf) {
#pragma unroll
        for (int k = 0; k < G; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (cand[k][j] == dmin) mask |= 1u << (4 * k + j);
    }
    uint32_t total = 0;
    uint32_t rank = owner_excl_scan<T>(__popc(mask), total, lo.L, sh.red);
    if (entries) {
        stress_delay(2u * tag + 1u);
#pragma unroll
        for (int k = 0; k < G; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (mask >> (4 * k + j) & 1u)
                    st_agent(&list[rank++], tag_word(tag, (uint32_t)(col0 + local_col(lo, k, j))));
    }
    if (threadIdx.x == 0) {
        stress_delay(2u * tag);
        const uint32_t slot = (tag - 1) & 1;
        st_agent(rec_word(recs, nwg, slot, kRecVert, g), tag_word(tag, (uint32_t)key));
        st_agent(rec_word(recs, nwg, slot, kRecCnt, g), tag_word(tag, (total << 1) | (zero ? 1u : 0u)));
        st_agent(rec_word(recs, nwg, slot, kRecDist, g), tag_word(tag, (uint32_t)(key >> 32)));
    }
}

// Bounded wait for a tagged word: returns it once it carries `tag`; on time-out
// sets `late` and returns the last value read.
__device__ __forceinline__ uint64_t wait_tag(const uint64_t* p, uint64_t w, uint32_t tag, long long timeout,
                                             uint32_t& late) {
    if (word_tag(w) == tag) return w;
    const long long t0 = wall_clock64();
    for (;;) {
        __builtin_amdgcn_s_sleep(1);
        w = ld_agent(p);
        if (word_tag(w) == tag) return w;
        if (wall_clock64() - t0 > timeout) {
            late = 1;
            return w;
        }
    }
}

// Exchange `tag` from the reader's side: waits for the gang's nwg tagged records
// of its slot and reduces them.  `stamps` (the solve's first exchange only):
// each member's tagged words are read only after its stamp, which it stored
// once its cleared words were in place, has been seen (in an earlier poll, so
// the tagged loads are issued after the stamp load returned).
// K = the lowest key, Z = the OR of the hazard flags; for the round's bucket
// (records whose key has dist d = K >> 32) each record's count and offset go to
// sh.cnt / sh.pre and their sum to M.  Wave 0 polls and reduces (lane l takes
// members l, l + 64, l + 128, l + 192, so that each load instruction reads 64
// consecutive words) and shares the results through LDS after one workgroup
// barrier; gangs of more than 256 members take a block-wide path.  Returns
// false (K = no key, M = 0) if a member's record did not arrive within
// `timeout` ticks.
template <int T>
__device__ __forceinline__ bool read_records(uint64_t* recs, int nwg, uint32_t tag, long long timeout,
                                             SharedSolve<T>& sh, uint64_t& K, uint32_t& Z, uint32_t& M,
                                             const Pub* stamps, uint64_t stamp) {
    const uint32_t slot = (tag - 1) & 1;
    const uint64_t* rd = rec_word(recs, nwg, slot, kRecDist, 0);
    const uint64_t* rv = rec_word(recs, nwg, slot, kRecVert, 0);
    const uint64_t* rc = rec_word(recs, nwg, slot, kRecCnt, 0);
    if (nwg <= 4 * kWave) {
        if (threadIdx.x < kWave) {
            const int l = (int)threadIdx.x;
            uint64_t key[4];
            uint32_t cnt[4];
            uint32_t want = 0, f = 0, late = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                key[k] = kNoKey;
                cnt[k] = 0;
                if (l + kWave * k < nwg) want |= 1u << k;
            }
            // Every poll issues all of its loads before it checks any (member indexes
            // clamped to the last member): a load per branch would be waited for
            // before the next one, four round trips per poll instead of one.  Polls
            // back off (up to ~0.1 us apart) so that members waiting through a long
            // round do not load the memory system the others are streaming from.
            const long long t0 = wall_clock64();
            unsigned naps = 0;
            if (stamps) {
                uint32_t need = want;
                for (;;) {
                    uint64_t sv[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) sv[k] = ld_agent(&stamps[min(l + kWave * k, nwg - 1)].stamp);
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (sv[k] == stamp) need &= ~(1u << k);
                    if (!need) break;
                    if (wall_clock64() - t0 > timeout) {
                        late = 1;
                        want = 0;
                        break;
                    }
                    for (unsigned i = 0; i < naps; ++i) __builtin_amdgcn_s_sleep(1);
                    naps = naps ? (naps < 4 ? naps << 1 : naps) : 1;
                }
            }
            while (want) {
                uint64_t a[4], b[4], c[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int m = min(l + kWave * k, nwg - 1);
                    a[k] = ld_agent(&rd[m]);
                    b[k] = ld_agent(&rv[m]);
                    c[k] = ld_agent(&rc[m]);
                }
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if ((want >> k & 1u) && word_tag(a[k]) == tag && word_tag(b[k]) == tag && word_tag(c[k]) == tag) {
                        key[k] = make_key((uint32_t)a[k], (uint32_t)b[k]);
                        cnt[k] = (uint32_t)c[k] >> 1;
                        f |= (uint32_t)c[k] & 1u;
                        want &= ~(1u << k);
                    }
                if (!want) break;
                if (wall_clock64() - t0 > timeout) {
                    late = 1;
                    break;
                }
                for (unsigned i = 0; i < naps; ++i) __builtin_amdgcn_s_sleep(1);
                naps = naps ? (naps < 4 ? naps << 1 : naps) : 1;
            }
            uint64_t kmin = kNoKey;
#pragma unroll
            for (int k = 0; k < 4; ++k) kmin = umin64(kmin, key[k]);
            kmin = wave_min64(kmin);
            f = wave_or32(f);
            late = wave_or32(late);
            const uint32_t d = (uint32_t)(kmin >> 32);
            // The bucket is the concatenation of the bucket records' lists in
            // position order, position 4 l + k holding member l + 64 k (see
            // entry_addr): one scan over the lanes' sums.
            uint32_t c[4], local = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                c[k] = (key[k] == kNoKey || (uint32_t)(key[k] >> 32) != d) ? 0u : cnt[k];
                local += c[k];
            }
            const uint32_t inc = wave_scan32(local);
            uint32_t run = inc - local;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                sh.pre[4 * l + k] = run;
                sh.cnt[4 * l + k] = c[k];
                run += c[k];
            }
            if (l == 0) {
                sh.rk = late ? kNoKey : kmin;
                sh.rz = f;
                sh.rm = late ? 0u : lane_value(inc, kWave - 1);
                sh.late = late;
            }
        }
        __syncthreads();
        // the same in every thread: scalar registers
        K = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(sh.rk >> 32)) << 32) |
            (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)sh.rk);
        Z = (uint32_t)__builtin_amdgcn_readfirstlane((int)sh.rz);
        M = (uint32_t)__builtin_amdgcn_readfirstlane((int)sh.rm);
        return __builtin_amdgcn_readfirstlane((int)sh.late) == 0;
    }
    uint64_t key = kNoKey;
    uint32_t c = 0, f = 0, late = 0;
    if ((int)threadIdx.x < nwg) {
        const int m = (int)threadIdx.x;
        if (stamps) {
            const long long t0 = wall_clock64();
            while (ld_agent(&stamps[m].stamp) != stamp)
                if (wall_clock64() - t0 > timeout) {
                    late = 1;
                    break;
                }
        }
        const uint64_t a = wait_tag(&rd[m], ld_agent(&rd[m]), tag, timeout, late);
        const uint64_t b = wait_tag(&rv[m], ld_agent(&rv[m]), tag, timeout, late);
        const uint64_t w = wait_tag(&rc[m], ld_agent(&rc[m]), tag, timeout, late);
        key = make_key((uint32_t)a, (uint32_t)b);
        c = (uint32_t)w >> 1;
        f = ((uint32_t)w & 1u) | (late << 1);
    }
    K = key;
    Z = f;
    block_min_or<T>(K, Z, sh.red);
    if (key == kNoKey || (uint32_t)(key >> 32) != (uint32_t)(K >> 32)) c = 0;
    const uint32_t pre = block_excl_scan<T>(c, M, sh.red);
    if ((int)threadIdx.x < nwg) {
        sh.pre[threadIdx.x] = pre;
        sh.cnt[threadIdx.x] = c;
    }
    if (threadIdx.x == 0) sh.late = (Z >> 1) & 1u;
    __syncthreads();
    if (Z & 2u) {
        K = kNoKey;
        M = 0;
        return false;
    }
    Z &= 1u;
    return true;
}

// Address of entry e of the round's bucket, the concatenation of the lists of
// the records whose minimum equals d.  sh.pre / sh.cnt hold each position's
// prefix offset and count; with at most 256 members (read_records' wave path)
// position 4 l + k holds member l + 64 k (positions of absent members count 0),
// otherwise position m holds member m.
template <int T>
__device__ __forceinline__ const uint64_t* entry_addr(const SharedSolve<T>& sh, const uint64_t* __restrict__ rl,
                                                      int nwg, int S, uint32_t e) {
    const bool packed = nwg <= 4 * kWave;
    int lo_i = 0, hi_i = packed ? 4 * kWave - 1 : nwg - 1;  // last position whose prefix is <= e
    while (lo_i < hi_i) {
        const int mid = (lo_i + hi_i + 1) >> 1;
        if (sh.pre[mid] <= e) lo_i = mid;
        else hi_i = mid - 1;
    }
    const int m = packed ? (lo_i & 3) * kWave + (lo_i >> 2) : lo_i;
    return &rl[(size_t)m * S + (e - sh.pre[lo_i])];
}

// Rank g of a gang of nwg workgroups.  gw: the gang's exchange memory (see
// gang_words_bytes).  Returns false if a wait timed out.  `trace` (may be null)
// receives rank 0's round trace.  b0: exchanges the gang's words have already
// counted in this use (a solve that follows another one on the same words
// continues the numbering); epoch: unique to this use of the words (stamps of
// the first exchange).
//
// BAL: pair balancing of large rounds.  Equal slices do not take equal time
// (workgroups on some XCDs stream measurably slower), and a round lasts as long
// as its slowest member.  In a round of at least kPairChunks chunks, members g
// and g ^ 1 claim the rows of their own slice from the front of a counter, a
// staging chunk (kCap rows) at a time; one that runs out claims the partner's
// remaining rows from the back, kPairUnit rows at a time, streams them over the
// partner's columns, then hands the partial minima over (partial keys, then a
// tagged done word once they are in memory).  The counter word counts units of
// kPairUnit rows, front claims in its low 16 bits and back claims in its high
// 16 bits; the atomic adds serialise the claims, a claim made when front +
// back < units is valid, a front claim stops at the back claims made before it,
// and later back claims see its whole increment, so no row is taken twice or
// left out.  Claims are made two ahead so that their latency hides behind the
// streaming; the helper's claims from the back do not wait for the rows the
// owner has reserved at the front.  Each member has two
// counters (round parity) and resets one only after reading the exchange that
// follows the round that used it, when both members' claims on it have
// returned, and before its next publish (the partner claims on it again only
// after that publish).
template <int T, int G, int U, typename E, bool NT = false, bool BAL = false>
__device__ __forceinline__ bool solve_gang(const E* __restrict__ W, int64_t ld, int32_t n, int32_t src,
                           int32_t* __restrict__ dist, int32_t* __restrict__ pred, bool vec, bool literal,
                           int S, int g, int nwg, long long timeout, GangWords gw, SharedSolve<T>& sh,
                           SolveStats& st, Ctl* trace, uint32_t epoch, uint32_t b0 = 0) {
    static_assert(T == kCap, "one staged bucket entry per thread");
    static_assert(!BAL || sizeof(E) == 4, "pair balancing keeps 64-bit keys");
    const int64_t col0 = (int64_t)g * S;
    const int width = (int)max((int64_t)0, min((int64_t)S, (int64_t)n - col0));
    const Layout lo = make_layout<T>(S);
    Cols<G, E> cs;
    init_cols(cs, lo, col0, width, src);
    clear_merge<T>(sh.mrg, 4 * T);
    auto list_of = [&](uint32_t x, int m) { return gw.lists + ((size_t)((x - 1) & 1) * nwg + m) * S; };

    uint32_t b = b0;  // exchanges passed
    bool ok = true;
    // Clear this member's tagged words, then stamp its record for the first
    // exchange (b0 + 1) once they are in place: readers take its tagged words
    // only after seeing that stamp (read_records).
    clear_tagged<T>(gw.recs, gw.lists, gw.ctr, gw.done, g, nwg, S);
    // pair balancing: the partner, counter slots that a round has used and not
    // yet reset, and the value of the last reset (used before the next publish)
    const int pg = g ^ 1;
    const bool paired = BAL && pg < nwg && lo.P > 1;
    uint32_t used = 0, reset_old = 0;
    // the same in every thread (it comes from a load): a scalar register
    const uint64_t stamp1 = exchange_stamp((uint32_t)__builtin_amdgcn_readfirstlane((int)epoch), b0 + 1);
    const Pub* stamps1 = gw.pubs + (size_t)(b0 & 1) * nwg;
    if (threadIdx.x == 0) sh.stage_late = 0u;
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        stress_delay((uint32_t)(stamp1 ^ (stamp1 >> 29)));
        __builtin_amdgcn_s_waitcnt(0);
        st_agent(&gw.pubs[(size_t)(b0 & 1) * nwg + g].stamp, stamp1);
    }
    // The first round's bucket, {src} at distance 0, is the same in every
    // member's view: no exchange precedes it.
    uint32_t d = 0, u0 = (uint32_t)src, M = 1;
    bool first = true;
    uint32_t cand[G][4];
    for (;;) {
        ++st.rounds;
        const long long t_round = wall_clock64();
        uint32_t bucket;
        if (literal) {
            M = 1;
            bucket = owner_bit(lo, (int64_t)u0 - col0, width);
            if (threadIdx.x == 0) sh.list[0] = (int32_t)u0;
            __syncthreads();
            stream_rows<G, U, E, NT>(cs, lo, W, ld, col0, width, vec, sh.list, 1);
        } else {
            bucket = bucket_mask(cs, d);
            const uint64_t* rl = list_of(b, 0);
            // entry e of the bucket into sh.list[threadIdx.x]; w: its word as loaded
            auto stage = [&](uint32_t e, uint64_t w) {
                uint32_t late = 0;
                if (word_tag(w) != b) w = wait_tag(entry_addr<T>(sh, rl, nwg, S, e), w, b, timeout, late);
                // a time-out stages a valid row; the solve then ends with the time-out status
                sh.list[threadIdx.x] = late ? (int32_t)u0 : (int32_t)(uint32_t)w;
                if (late) sh.stage_late = 1u;
            };
            const uint32_t C = (M + kCap - 1) / kCap;
            if (paired && C >= kPairChunks) {
                const uint32_t slot = b & 1;
                const uint32_t tag = b + 1;  // the exchange this round publishes
                key_t<E>* keep = reinterpret_cast<key_t<E>*>(sh.mrg + 2 * T);
                uint32_t own = 0;
                for (int side = 0; side < 2; ++side) {
                    const int m = side ? pg : g;
                    const int64_t c0 = (int64_t)m * S;
                    const int wd = (int)max((int64_t)0, min((int64_t)S, (int64_t)n - c0));
                    uint32_t* ctr = &gw.ctr[4 * m + slot];
                    // claims count units of kPairUnit rows: the owner takes a staging
                    // chunk (kCap rows) at a time from the front, the helper one unit at
                    // a time from the back
                    constexpr uint32_t kChunkUnits = (uint32_t)kCap / kPairUnit;
                    const uint32_t units = (M + kPairUnit - 1) / kPairUnit;
                    uint32_t left = units;  // units unclaimed when the last decoded claim was made
                    // rows [begin, begin + count) of a claim of `n` units (the counter
                    // before it in `old`); count 0 if it came too late.  A front claim stops
                    // at the back claims made before it; later back claims see its whole
                    // increment and stay clear.
                    auto rows_of = [&](uint32_t old, uint32_t nu, uint32_t& begin) -> uint32_t {
                        const uint32_t f = old & 0xffffu, h = old >> 16;
                        begin = 0;
                        left = f + h >= units ? 0u : units - f - h;
                        if (!left) return 0u;
                        const uint32_t u0 = side ? units - 1 - h : f;
                        const uint32_t u1 = side ? u0 + 1 : min(f + nu, units - h);
                        begin = u0 * kPairUnit;
                        return min(u1 * kPairUnit, M) - begin;
                    };
                    // the owner claims whole staging chunks, single units once few are
                    // left (so that it reserves little for the helper to wait behind);
                    // the helper always claims single units
                    auto units_next = [&]() { return side || left <= 3 * kChunkUnits ? 1u : kChunkUnits; };
                    auto inc_of = [&](uint32_t nu) { return side ? 0x10000u : nu; };
                    if (side == 1) {
                        // keep this member's candidates while it streams rows for the partner
                        merge_partitions<T, G>(cs, lo, sh.mrg);
                        if (lo.r == 0)
#pragma unroll
                            for (int j = 0; j < 4; ++j) keep[j * lo.L + lo.c] = cs.best[0][j];
                        reset_best(cs);
                    }
                    const uint32_t nu0 = units_next();
                    if (threadIdx.x == 0) {
                        if (side == 0) stress_delay(4u * tag + 3u);  // late starters: partners steal
                        sh.claim[0] = __hip_atomic_fetch_add(ctr, inc_of(nu0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        sh.claim[1] = __hip_atomic_fetch_add(ctr, inc_of(nu0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    __syncthreads();
                    uint32_t kb = 0, nb = 0;
                    uint32_t kcnt = rows_of((uint32_t)__builtin_amdgcn_readfirstlane((int)sh.claim[0]), nu0, kb);
                    uint32_t ncnt = rows_of((uint32_t)__builtin_amdgcn_readfirstlane((int)sh.claim[1]), nu0, nb);
                    uint32_t chunks = 0;  // rows streamed on this side
                    uint64_t w = 0;
                    if (threadIdx.x < kcnt) w = ld_agent(entry_addr<T>(sh, rl, nwg, S, kb + threadIdx.x));
                    while (kcnt) {
                        if (threadIdx.x < kcnt) stage(kb + threadIdx.x, w);
                        __syncthreads();
                        uint32_t a = 0xffffffffu;  // no further claim: nothing is left after the next one
                        const uint32_t nua = units_next();
                        if (ncnt) {
                            if (threadIdx.x < ncnt) w = ld_agent(entry_addr<T>(sh, rl, nwg, S, nb + threadIdx.x));
                            if (threadIdx.x == 0)
                                a = __hip_atomic_fetch_add(ctr, inc_of(nua), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        }
                        stream_rows<G, U, E, NT>(cs, lo, W, ld, c0, wd, vec, sh.list, (int)kcnt);
                        if (threadIdx.x == 0) sh.claim[0] = a;
                        __syncthreads();
                        chunks += kcnt;
                        kb = nb;
                        kcnt = ncnt;
                        ncnt = rows_of((uint32_t)__builtin_amdgcn_readfirstlane((int)sh.claim[0]), nua, nb);
                    }
                    if (side == 0) {
                        own = chunks;
                        continue;
                    }
                    if (chunks) {
                        // the partner's share of its own columns: partial minima, then the
                        // tagged done word once they are in memory
                        merge_partitions<T, G>(cs, lo, sh.mrg);
                        if (lo.r == 0)
#pragma unroll
                            for (int j = 0; j < 4; ++j)
                                st_agent(&gw.part[(size_t)pg * S + 4 * lo.c + j], (uint64_t)cs.best[0][j]);
                        __builtin_amdgcn_s_waitcnt(0);
                        __syncthreads();
                        if (threadIdx.x == 0) st_agent(&gw.done[2 * pg], tag_word(tag, chunks));
                    }
                    // back to this member's own candidates
                    if (lo.r == 0) {
#pragma unroll
                        for (int j = 0; j < 4; ++j) cs.best[0][j] = keep[j * lo.L + lo.c];
                    } else {
                        reset_best(cs);
                    }
                }
                if (own < M && lo.r == 0) {
                    // the partner streamed the rest of this member's chunks: its partial minima
                    uint32_t late = 0;
                    (void)wait_tag(&gw.done[2 * g], ld_agent(&gw.done[2 * g]), tag, timeout, late);
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        cs.best[0][j] = key_min(cs.best[0][j], (key_t<E>)ld_agent(&gw.part[(size_t)g * S + 4 * lo.c + j]));
                    if (late) sh.stage_late = 1u;
                }
                used |= 1u << slot;
            } else {
                // stage the bucket chunk by chunk; the next chunk's entries are loaded
                // while the current chunk's rows stream (the first round's one entry,
                // the source, is not loaded)
                uint64_t nxt = first ? tag_word(b, u0)
                             : threadIdx.x < M ? ld_agent(entry_addr<T>(sh, rl, nwg, S, threadIdx.x)) : 0;
                for (uint32_t e0 = 0; e0 < M; e0 += kCap) {
                    const uint32_t e = e0 + threadIdx.x;
                    if (e < M) stage(e, nxt);
                    __syncthreads();
                    if (e + kCap < M) nxt = ld_agent(entry_addr<T>(sh, rl, nwg, S, e + kCap));
                    stream_rows<G, U, E, NT>(cs, lo, W, ld, col0, width, vec, sh.list,
                                             (int)min((uint32_t)kCap, M - e0));
                    __syncthreads();
                }
            }
        }
        merge_partitions<T, G>(cs, lo, sh.mrg);
        if (sh.stage_late) {
            ok = false;
            break;
        }
        if (trace && g == 0 && threadIdx.x == 0 && st.rounds <= (unsigned long long)kTraceCap) {
            trace->trace_t[st.rounds - 1] = t_round;
            trace->trace_m[st.rounds - 1] = M;
        }

        // would-be state if this round is applied; publish it with the hazard flag
        uint32_t neg = 0;
#pragma unroll
        for (int k = 0; k < G; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j) cand[k][j] = would_be(cs, k, j, d, bucket, neg);
        st.status |= neg;
        const uint32_t zero = (!literal && lo.r == 0) ? zero_hazard(cs, d) : 0u;
        ++b;
        if (BAL) asm volatile("" ::"v"(reset_old));  // a counter reset has completed before this publish
        publish<T, G>(cand, lo, col0, zero, !literal, b, gw.recs, nwg, g, list_of(b, g), sh);
        uint64_t K;
        uint32_t Z, M_rec;
        ok = read_records<T>(gw.recs, nwg, b, timeout, sh, K, Z, M_rec, first ? stamps1 : nullptr, stamp1);
        first = false;
        if (!ok) break;
        if (BAL && (used >> ((b - 1) & 1) & 1u)) {
            // every claim on the counter slot of the round just published has returned
            if (threadIdx.x == 0)
                reset_old = __hip_atomic_exchange(&gw.ctr[4 * g + ((b - 1) & 1)], 0u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
            used &= ~(1u << ((b - 1) & 1));
        }
        if (Z) {
            // the fused round read a zero-weight edge out of its bucket: discard it
            // and settle only the bucket's lowest-index vertex (one literal step)
            ++st.fallbacks;
            st.status |= kStatusZeroFallback;
            reset_best(cs);
            if (threadIdx.x == 0) sh.list[0] = (int32_t)u0;
            __syncthreads();
            stream_rows<G, U, E, NT>(cs, lo, W, ld, col0, width, vec, sh.list, 1);
            merge_partitions<T, G>(cs, lo, sh.mrg);
            if (lo.r == 0) st.status |= commit_fused(cs, d, owner_bit(lo, (int64_t)u0 - col0, width));
            else reset_best(cs);
            st.settled += 1;
#pragma unroll
            for (int k = 0; k < G; ++k)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    cand[k][j] = (cs.vis >> (4 * k + j) & 1u) ? 0xffffffffu : cs.dist[k][j];
            ++b;
            if (BAL) asm volatile("" ::"v"(reset_old));
            publish<T, G>(cand, lo, col0, 0u, !literal, b, gw.recs, nwg, g, list_of(b, g), sh);
            ok = read_records<T>(gw.recs, nwg, b, timeout, sh, K, Z, M_rec, nullptr, 0);
            if (!ok) break;
        } else {
            if (lo.r == 0) st.status |= commit_fused(cs, d, bucket);
            else reset_best(cs);
            st.settled += M;
        }
        d = (uint32_t)(K >> 32);
        if (K == kNoKey || d >= kInf) break;
        u0 = (uint32_t)K;
        M = M_rec;
    }
    if (!ok) st.status |= kStatusTimeout;
    write_out(cs, lo, col0, width, dist, pred);
    st.barriers += b;
    if (trace && g == 0 && threadIdx.x == 0) {
        const unsigned long long nr = st.rounds < (unsigned long long)kTraceCap ? st.rounds : kTraceCap;
        trace->trace_t[nr] = wall_clock64();
        trace->trace_n = (uint32_t)nr;
    }
    uint32_t s = st.status;
    uint64_t dummy = kNoKey;
    block_min_or<T>(dummy, s, sh.red);
    st.status = s;
    return ok;
}

}  // namespace sssp
