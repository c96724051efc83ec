// Label-correcting solve: the paper's CUDA design (Section III-C, Algorithms 3
// and 4) made deterministic and coalesced.  The single-solve call offers it as
// an alternative to the Dijkstra rounds; batched plans and servers use it for
// graphs whose solves need many rounds (sparse graphs with many distinct
// distances), where it replaces hundreds of exchanges by a few sweeps.
//
// Algorithm 4 lets every vertex relax its whole row in each sweep, with an
// atomicMin on dist and a separate, racy store of pred, and Algorithm 3 repeats
// sweeps until no dist changes.  Here:
//   * a sweep relaxes only the rows of the vertices whose dist changed in the
//     previous sweep (the frontier; the first frontier is the source), each row
//     with the dist its vertex had when the sweep started;
//   * every workgroup owns a column slice, as in the whole-GPU Dijkstra solve,
//     so the per-column minimum needs no atomics and the rows are read by
//     consecutive lanes (coalesced) rather than one row per thread;
//   * the convergence test is on the device: a sweep whose frontier is empty
//     ends the loop, with no host round trip;
//   * pred is not written during the sweeps.  Once dist is final, one more pass
//     over the rows of all reachable vertices sets pred[v] to the u with the
//     lexicographically smallest (dist[u], u) among u != v with
//     dist[u] + W[u][v] == dist[v].  When no such tight edge has weight 0,
//     Algorithm 1 settles vertices in (dist, index) order, and that u is the
//     first settled vertex to offer dist[v] — exactly the pred its strict '<'
//     keeps.  If the pass finds a tight zero-weight edge (u != v), the order of
//     Algorithm 1 is no longer (dist, index), so the launch re-solves with the
//     Dijkstra rounds instead (status bit ZERO_FALLBACK).
// dist is exact in every case: it is the unique shortest-path distance, which
// any label-correcting order reaches.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "engine.h"
#include "solve.h"

namespace sssp {

// LDS beyond SharedSolve: dist of the staged frontier rows, and the column
// dist of the owners for the other row partitions during the pred pass.
template <int T>
struct SharedLC {
    uint32_t dl[kCap];
    uint32_t dcol[4 * T];
};
template <int T>
__shared__ SharedLC<T> g_lc;

// Frontier entries are (dist << 32 | vertex) in 64-bit list slots.
__host__ __device__ constexpr uint64_t lc_entry(uint32_t d, uint32_t v) { return ((uint64_t)d << 32) | v; }

// Loads of U rows (list[i], list[i + step], ...) of one column group, widened;
// past the end of the list the last row repeats (harmless for a minimum).
template <int U, bool FULL, typename E, bool NT>
__device__ __forceinline__ void lc_load(uint32_t (&w)[U][4], uint32_t (&uu)[U], uint32_t (&du)[U],
                                        const E* __restrict__ p0, int64_t ld, int valid, const int32_t* list,
                                        const uint32_t* dl, int m, int i, int step) {
#pragma unroll
    for (int q = 0; q < U; ++q) {
        const int idx = i + q * step;
        const int ii = idx < m ? idx : m - 1;
        uu[q] = (uint32_t)list[ii];
        du[q] = dl[ii];
    }
    if (FULL) {
        typename Raw<E>::type raw[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const global_ptr<typename Raw<E>::type> a =
                reinterpret_cast<global_ptr<typename Raw<E>::type>>((global_ptr<E>)p0 + (int64_t)uu[q] * ld);
            raw[q] = NT ? __builtin_nontemporal_load(a) : *a;
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < U; ++q) {
            unpack<E>(raw[q], w[q]);
#pragma unroll
            for (int j = 0; j < 4; ++j) w[q][j] = widen<E>(w[q][j]);  // compact codes -> weights
        }
    } else {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const global_ptr<E> p = (global_ptr<E>)p0 + (int64_t)uu[q] * ld;
#pragma unroll
            for (int j = 0; j < 4; ++j) w[q][j] = j < valid ? widen<E>((uint32_t)p[j]) : kInf;
        }
    }
}

// Sweep: best[j] = min over the rows u of dist(u) + W[u][v].  No edge
// (INT32_MAX) and negative weights (> INT32_MAX as uint32) offer nothing; a
// negative weight sets *neg.  dist(u) < INT32_MAX and W < INT32_MAX: no wrap.
template <int U, bool FULL, typename E, bool NT>
__device__ __forceinline__ void lc_sweep_group(uint32_t (&best)[4], const E* __restrict__ p0, int64_t ld,
                                               int valid, const int32_t* list, const uint32_t* dl, int m,
                                               int first, int step, uint32_t& neg) {
    for (int i = first; i < m; i += step * U) {
        uint32_t w[U][4], uu[U], du[U];
        lc_load<U, FULL, E, NT>(w, uu, du, p0, ld, valid, list, dl, m, i, step);
#pragma unroll
        for (int q = 0; q < U; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                neg |= w[q][j] > kInf ? kStatusNegWeight : 0u;
                const uint32_t c = w[q][j] >= kInf ? 0xffffffffu : du[q] + w[q][j];
                best[j] = min(best[j], c);
            }
    }
}

// Pred pass: key[j] = lowest (dist(u) << 32 | u) over rows u tight at column
// v0 + j (dist(u) + W[u][v] == dv[j]; dv = 0xffffffff for unreachable columns,
// which no sum reaches).  Row v itself is tight when W[v][v] = 0; its key
// (dist[v], v) loses to any tight u with a positive weight (dist(u) < dist[v]),
// and a tight u with weight 0 sets *zero, so it never decides a pred.
template <int U, bool FULL, typename E, bool NT>
__device__ __forceinline__ void lc_pred_group(uint64_t (&key)[4], const uint32_t (&dv)[4], uint32_t v0,
                                              const E* __restrict__ p0, int64_t ld, int valid, const int32_t* list,
                                              const uint32_t* dl, int m, int first, int step, uint32_t& zero) {
    for (int i = first; i < m; i += step * U) {
        uint32_t w[U][4], uu[U], du[U];
        lc_load<U, FULL, E, NT>(w, uu, du, p0, ld, valid, list, dl, m, i, step);
#pragma unroll
        for (int q = 0; q < U; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool tight = w[q][j] < kInf && du[q] + w[q][j] == dv[j];
                if (tight) {
                    key[j] = umin64(key[j], lc_entry(du[q], uu[q]));
                    if (w[q][j] == 0u && uu[q] != v0 + (uint32_t)j) zero = 1u;
                }
            }
    }
}

// One pass of the staged rows over this thread's column groups.
template <int G, int U, typename E, bool NT>
__device__ __forceinline__ void lc_sweep_rows(uint32_t (&best)[G][4], const Layout& lo, const E* __restrict__ W,
                                              int64_t ld, int64_t col0, int width, bool vec, const int32_t* list,
                                              const uint32_t* dl, int m, uint32_t& neg) {
#pragma unroll
    for (int k = 0; k < G; ++k) {
        const int v0 = 4 * (lo.c + k * lo.L);
        if (v0 >= width) continue;
        const E* p0 = W + col0 + v0;
        if (vec && v0 + 3 < width)
            lc_sweep_group<U, true, E, NT>(best[k], p0, ld, 4, list, dl, m, lo.r, lo.P, neg);
        else
            lc_sweep_group<U, false, E, NT>(best[k], p0, ld, min(4, width - v0), list, dl, m, lo.r, lo.P, neg);
    }
}

template <int G, int U, typename E, bool NT>
__device__ __forceinline__ void lc_pred_rows(uint64_t (&key)[G][4], const uint32_t (&dv)[G][4], const Layout& lo,
                                             const E* __restrict__ W, int64_t ld, int64_t col0, int width, bool vec,
                                             const int32_t* list, const uint32_t* dl, int m, uint32_t& zero) {
#pragma unroll
    for (int k = 0; k < G; ++k) {
        const int v0 = 4 * (lo.c + k * lo.L);
        if (v0 >= width) continue;
        const E* p0 = W + col0 + v0;
        if (vec && v0 + 3 < width)
            lc_pred_group<U, true, E, NT>(key[k], dv[k], (uint32_t)(col0 + v0), p0, ld, 4, list, dl, m, lo.r, lo.P,
                                          zero);
        else
            lc_pred_group<U, false, E, NT>(key[k], dv[k], (uint32_t)(col0 + v0), p0, ld, min(4, width - v0), list,
                                           dl, m, lo.r, lo.P, zero);
    }
}

// Merge the P row partitions' results into the owners (partition 0) with LDS
// atomic minima, as merge_partitions does (P > 1 implies G == 1; the merge area
// is all ones between merges: the 32-bit view of the all-ones 64-bit key).
template <int T, int G>
__device__ __forceinline__ void lc_merge32(uint32_t (&best)[G][4], const Layout& lo, uint64_t* mrg) {
    if (lo.P == 1) return;
    uint32_t* m32 = reinterpret_cast<uint32_t*>(mrg);
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (best[0][j] != 0xffffffffu)
            __hip_atomic_fetch_min(&m32[j * lo.L + lo.c], best[0][j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();
    if (lo.r == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            best[0][j] = m32[j * lo.L + lo.c];
            m32[j * lo.L + lo.c] = 0xffffffffu;
        }
    }
}

template <int T, int G>
__device__ __forceinline__ void lc_merge64(uint64_t (&key)[G][4], const Layout& lo, uint64_t* mrg) {
    if (lo.P == 1) return;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (key[0][j] != kNoKey)
            __hip_atomic_fetch_min(&mrg[j * lo.L + lo.c], key[0][j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();
    if (lo.r == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            key[0][j] = mrg[j * lo.L + lo.c];
            mrg[j * lo.L + lo.c] = kNoKey;
        }
    }
}

// Publish the owned columns selected by `mask` as (dist, vertex) entries of
// this workgroup's list, with their count and `flags` in its record.
template <int T, int G>
__device__ __forceinline__ void lc_publish(uint32_t mask, const uint32_t (&dv)[G][4], const Layout& lo, int64_t col0,
                                           uint32_t flags, Pub* __restrict__ pub, uint64_t* __restrict__ list,
                                           SharedSolve<T>& sh) {
    uint32_t total = 0;
    uint32_t rank = owner_excl_scan<T>(__popc(mask), total, lo.L, sh.red);
#pragma unroll
    for (int k = 0; k < G; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (mask >> (4 * k + j) & 1u)
                st_agent(&list[rank++], lc_entry(dv[k][j], (uint32_t)(col0 + local_col(lo, k, j))));
    if (threadIdx.x == 0) {
        st_agent(&pub->key, (uint64_t)total);
        st_agent(&pub->count, total);
        st_agent(&pub->flags, flags);
    }
}

// Read the records of the last exchange: per-record prefix offsets and counts
// into sh.pre / sh.cnt; returns the total and ORs the records' flags into
// *flags.  Wave 0 does it for gangs of up to 256 members (one workgroup
// barrier), as read_records does.
template <int T>
__device__ __forceinline__ uint32_t lc_records(const Pub* rp, int nwg, SharedSolve<T>& sh, uint32_t& flags) {
    if (nwg <= 4 * kWave) {
        if (threadIdx.x < kWave) {
            const int q = (nwg + kWave - 1) / kWave;
            const int i0 = (int)threadIdx.x * q;
            uint32_t cnt[4], fl[4];
            uint32_t f = 0, local = 0;
            // all loads issued before any is used (record indexes clamped to the
            // last member): a load per branch would be waited for before the next
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int m = min(i0 + k, nwg - 1);
                cnt[k] = ld_agent(&rp[m].count);
                fl[k] = ld_agent(&rp[m].flags);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!(k < q && i0 + k < nwg)) cnt[k] = fl[k] = 0;
                f |= fl[k];
                local += cnt[k];
            }
            f = wave_or32(f);
            const uint32_t inc = wave_scan32(local);
            uint32_t run = inc - local;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k < q && i0 + k < nwg) {
                    sh.pre[i0 + k] = run;
                    sh.cnt[i0 + k] = cnt[k];
                    run += cnt[k];
                }
            if (threadIdx.x == kWave - 1) {
                sh.rz = f;
                sh.rm = inc;
            }
        }
        __syncthreads();
        flags = sh.rz;
        return sh.rm;
    }
    uint32_t c = 0, f = 0;
    if ((int)threadIdx.x < nwg) {
        c = ld_agent(&rp[threadIdx.x].count);
        f = ld_agent(&rp[threadIdx.x].flags);
    }
    uint32_t M;
    const uint32_t pre = block_excl_scan<T>(c, M, sh.red);
    if ((int)threadIdx.x < nwg) {
        sh.pre[threadIdx.x] = pre;
        sh.cnt[threadIdx.x] = c;
    }
    uint64_t dummy = kNoKey;
    block_min_or<T>(dummy, f, sh.red);  // also makes sh.pre / sh.cnt visible
    flags = f;
    return M;
}

// Entry e0 + threadIdx.x of the concatenated lists (as gather_entry).
template <int T>
__device__ __forceinline__ uint64_t lc_gather(const SharedSolve<T>& sh, const uint64_t* __restrict__ rl, int nwg,
                                              int S, uint32_t e0, uint32_t M) {
    const uint32_t e = e0 + threadIdx.x;
    if (e >= M) return 0;
    int lo_i = 0, hi_i = nwg - 1;
    while (lo_i < hi_i) {
        const int mid = (lo_i + hi_i + 1) >> 1;
        if (sh.pre[mid] <= e) lo_i = mid;
        else hi_i = mid - 1;
    }
    return ld_agent(&rl[(size_t)lo_i * S + (e - sh.pre[lo_i])]);
}

// Stage the M listed rows chunk by chunk into LDS and run `pass` over each
// chunk; the next chunk's entries load while the current one streams.
template <int T, class Pass>
__device__ __forceinline__ void lc_stream(const uint64_t* rl, int nwg, int S, uint32_t M, SharedSolve<T>& sh,
                                          SharedLC<T>& lc, Pass pass) {
    uint64_t nxt = lc_gather<T>(sh, rl, nwg, S, 0, M);
    for (uint32_t e0 = 0; e0 < M; e0 += kCap) {
        sh.list[threadIdx.x] = (int32_t)(uint32_t)nxt;
        lc.dl[threadIdx.x] = (uint32_t)(nxt >> 32);
        __syncthreads();
        if (e0 + kCap < M) nxt = lc_gather<T>(sh, rl, nwg, S, e0 + kCap, M);
        pass((int)min((uint32_t)kCap, M - e0));
        __syncthreads();
    }
}

enum LcResult { kLcDone = 0, kLcTimeout = 1, kLcFallback = 2 };

// Rank g of a gang of nwg workgroups (the whole grid).  pubs: 2 * nwg records;
// lists: 2 * nwg * S 64-bit entries, double-buffered by exchange parity.  b
// counts the exchanges passed (a fallback solve continues the numbering);
// epoch stamps this launch's records (see gang_exchange).
template <int T, int G, int U, typename E, bool NT>
__device__ __forceinline__ int solve_lc(const E* __restrict__ W, int64_t ld, int32_t n, int32_t src,
                                        int32_t* __restrict__ dist, int32_t* __restrict__ pred, bool vec, int S,
                                        int g, int nwg, long long timeout, Bar* bw, Pub* __restrict__ pubs,
                                        uint64_t* __restrict__ lists, SharedSolve<T>& sh, SharedLC<T>& lc,
                                        SolveStats& st, uint32_t& b, uint32_t epoch, Ctl* trace) {
    static_assert(T == kCap, "one staged entry per thread");
    const int64_t col0 = (int64_t)g * S;
    const int width = (int)max((int64_t)0, min((int64_t)S, (int64_t)n - col0));
    const Layout lo = make_layout<T>(S);
    uint32_t dv[G][4];
    uint32_t own = 0, chg = 0;
#pragma unroll
    for (int k = 0; k < G; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int v = local_col(lo, k, j);
            const bool mine = lo.r == 0 && k * lo.L + lo.c < lo.NG && v < width;
            const bool is_src = mine && col0 + v == src;
            dv[k][j] = is_src ? 0u : kInf;
            own |= mine ? 1u << (4 * k + j) : 0u;
            chg |= is_src ? 1u << (4 * k + j) : 0u;
        }
    clear_merge<T>(sh.mrg, 4 * T);
    auto slot_pub = [&](uint32_t s) { return pubs + (size_t)s * nwg; };
    auto slot_list = [&](uint32_t s) { return lists + (size_t)s * nwg * S; };
    // the next exchange: members' records of slot (b & 1) carry stamp b + 1
    auto exchange = [&]() {
        ++b;
        return gang_exchange<T>(slot_pub((b - 1) & 1), g, exchange_stamp(epoch, b), (uint32_t)nwg, timeout, sh.red);
    };

    // sweep 1 relaxes the source's row
    lc_publish<T, G>(chg, dv, lo, col0, 0u, &slot_pub(b & 1)[g], slot_list(b & 1) + (size_t)g * S, sh);
    bool ok = exchange();
    uint32_t neg = 0;
    while (ok) {
        const uint32_t s = (b - 1) & 1;
        uint32_t f;
        const uint32_t M = lc_records<T>(slot_pub(s), nwg, sh, f);
        if (M == 0) break;
        ++st.rounds;
        st.settled += M;
        const long long t_round = wall_clock64();
        uint32_t best[G][4];
#pragma unroll
        for (int k = 0; k < G; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j) best[k][j] = 0xffffffffu;
        lc_stream<T>(slot_list(s), nwg, S, M, sh, lc, [&](int m) {
            lc_sweep_rows<G, U, E, NT>(best, lo, W, ld, col0, width, vec, sh.list, lc.dl, m, neg);
        });
        lc_merge32<T, G>(best, lo, sh.mrg);
        if (trace && g == 0 && threadIdx.x == 0 && st.rounds <= (unsigned long long)kTraceCap) {
            trace->trace_t[st.rounds - 1] = t_round;
            trace->trace_m[st.rounds - 1] = M;
        }
        chg = 0;
        if (lo.r == 0) {
#pragma unroll
            for (int k = 0; k < G; ++k)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if ((own >> (4 * k + j) & 1u) && best[k][j] < dv[k][j]) {
                        dv[k][j] = best[k][j];
                        chg |= 1u << (4 * k + j);
                    }
        }
        lc_publish<T, G>(chg, dv, lo, col0, 0u, &slot_pub(b & 1)[g], slot_list(b & 1) + (size_t)g * S, sh);
        ok = exchange();
    }
    st.status |= neg;
    if (!ok) return kLcTimeout;

    // pred pass over the rows of every reachable vertex
    uint32_t reach = 0;
#pragma unroll
    for (int k = 0; k < G; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if ((own >> (4 * k + j) & 1u) && dv[k][j] < kInf) reach |= 1u << (4 * k + j);
    lc_publish<T, G>(reach, dv, lo, col0, 0u, &slot_pub(b & 1)[g], slot_list(b & 1) + (size_t)g * S, sh);
    if (!exchange()) return kLcTimeout;
    uint32_t f;
    const uint32_t R = lc_records<T>(slot_pub((b - 1) & 1), nwg, sh, f);
    st.settled += R;
    // every row partition needs its columns' dist: owners broadcast them
    uint32_t dt[G][4];
    if (lo.P > 1) {
        if (lo.r == 0)
#pragma unroll
            for (int j = 0; j < 4; ++j) lc.dcol[4 * lo.c + j] = dv[0][j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 4; ++j) dt[0][j] = lc.dcol[4 * lo.c + j];
        __syncthreads();
    } else {
#pragma unroll
        for (int k = 0; k < G; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j) dt[k][j] = dv[k][j];
    }
#pragma unroll
    for (int k = 0; k < G; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (dt[k][j] >= kInf) dt[k][j] = 0xffffffffu;
    uint64_t key[G][4];
#pragma unroll
    for (int k = 0; k < G; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) key[k][j] = kNoKey;
    uint32_t zero = 0;
    lc_stream<T>(slot_list((b - 1) & 1), nwg, S, R, sh, lc, [&](int m) {
        lc_pred_rows<G, U, E, NT>(key, dt, lo, W, ld, col0, width, vec, sh.list, lc.dl, m, zero);
    });
    lc_merge64<T, G>(key, lo, sh.mrg);
    // agree on the tight-zero-edge verdict before writing anything
    uint64_t dummy = kNoKey;
    block_min_or<T>(dummy, zero, sh.red);
    if (threadIdx.x == 0) {
        Pub* p = &slot_pub(b & 1)[g];
        st_agent(&p->key, (uint64_t)0);
        st_agent(&p->count, 0u);
        st_agent(&p->flags, zero);
    }
    if (!exchange()) return kLcTimeout;
    uint32_t Z;
    (void)lc_records<T>(slot_pub((b - 1) & 1), nwg, sh, Z);
    if (Z) return kLcFallback;
    if (lo.r == 0) {
#pragma unroll
        for (int k = 0; k < G; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (!(own >> (4 * k + j) & 1u)) continue;
                const int64_t v = col0 + local_col(lo, k, j);
                dist[v] = (int32_t)dv[k][j];
                pred[v] = (v == src || dv[k][j] >= kInf || key[k][j] == kNoKey) ? -1 : (int32_t)(uint32_t)key[k][j];
            }
    }
    return kLcDone;
}

}  // namespace sssp
