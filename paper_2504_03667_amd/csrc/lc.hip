// The whole-GPU label-correcting kernel and its launcher; the method is
// described in lc.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "engine.h"
#include "lc.h"
#include "solve.h"
#include "sssp_internal.h"

namespace sssp {

template <int T, int G, int U>
__global__ __launch_bounds__(T) void k_lc(const int32_t* __restrict__ W, int64_t ld, int32_t n, int32_t src,
                                          int32_t* __restrict__ dist, int32_t* __restrict__ pred, uint32_t flags,
                                          int32_t S, long long timeout, Ctl* __restrict__ ctl,
                                          char* __restrict__ words) {
    SharedSolve<T>& sh = g_sh<T>;
    SolveStats st = {0, 0, 0, 0, 0};
    uint32_t b = 0;
    const bool vec = (flags & kFlagVec) != 0;
    const uint32_t epoch = ld_agent(&ctl->epoch);
    const GangWords gw = grid_words(words, gridDim.x, S);
    const int r = solve_lc<T, G, U, int32_t, true>(W, ld, n, src, dist, pred, vec, S, blockIdx.x, gridDim.x, timeout,
                                                   &ctl->b, gw.pubs, gw.lists, sh, g_lc<T>, st, b, epoch, ctl);
    if (r == kLcTimeout) {
        st.status |= kStatusTimeout;
        st.barriers += b;
    } else if (r == kLcFallback) {
        // a tight zero-weight edge: Algorithm 1's settle order is not (dist, index),
        // so solve again with the Dijkstra rounds (which handle zero weights)
        ++st.fallbacks;
        st.status |= kStatusZeroFallback;
        solve_gang<T, G, U, int32_t, true>(W, ld, n, src, dist, pred, vec, false, S, blockIdx.x, gridDim.x, timeout,
                                           gw, sh, st, ctl, epoch, b);
    } else {
        st.barriers += b;
    }
    if (r != kLcFallback && blockIdx.x == 0 && threadIdx.x == 0) {
        const unsigned long long nr = st.rounds < (unsigned long long)kTraceCap ? st.rounds : kTraceCap;
        ctl->trace_t[nr] = wall_clock64();
        ctl->trace_n = (uint32_t)nr;
    }
    uint32_t s = st.status;
    uint64_t dummy = kNoKey;
    block_min_or<T>(dummy, s, sh.red);
    st.status = s;
    finish_launch(ctl, st, blockIdx.x == 0);
}

template <int T, int G, int U>
static hipError_t launch_lc_t(const SolveArgs& a, int nwg, int S, long long timeout, char* words, bool plain,
                              hipStream_t s) {
    const int32_t* W = a.W;
    int64_t ld = a.ld;
    int32_t n = a.n, src = a.src;
    int32_t* dist = a.dist;
    int32_t* pred = a.pred;
    uint32_t flags = a.flags;
    Ctl* ctl = a.ctl;
    if (plain) {
        hipLaunchKernelGGL((k_lc<T, G, U>), dim3(nwg), dim3(T), 0, s, W, ld, n, src, dist, pred, flags, S, timeout,
                           ctl, words);
        return hipGetLastError();
    }
    void* args[] = {&W, &ld, &n, &src, &dist, &pred, &flags, &S, &timeout, &ctl, &words};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_lc<T, G, U>), dim3(nwg), dim3(T), args, 0, s);
}

hipError_t launch_lc(const SolveArgs& a, int nwg, int S, long long timeout, char* words, bool plain,
                     hipStream_t s) {
    const int groups = (S + 3) / 4;
    if (groups <= 1024) return launch_lc_t<1024, 1, 8>(a, nwg, S, timeout, words, plain, s);
    if (groups <= 2048) return launch_lc_t<1024, 2, 8>(a, nwg, S, timeout, words, plain, s);
    if (groups <= 4096) return launch_lc_t<1024, 4, 8>(a, nwg, S, timeout, words, plain, s);
    return hipErrorInvalidValue;
}

int lc_occupancy(int slice, int* per_cu) {
    const int groups = (slice + 3) / 4;
    const void* f = groups <= 1024 ? reinterpret_cast<const void*>(&k_lc<1024, 1, 8>)
                  : groups <= 2048 ? reinterpret_cast<const void*>(&k_lc<1024, 2, 8>)
                                   : reinterpret_cast<const void*>(&k_lc<1024, 4, 8>);
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, f, 1024, 0);
}

}  // namespace sssp
