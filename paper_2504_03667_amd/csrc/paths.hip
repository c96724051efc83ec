// The steps on either side of the solve: building the dense matrix from an edge
// list (Section III: the program writes the input edge list into the adjacency
// matrix, both orientations unless the graph is directed), and reading paths
// back out of pred (Algorithm 1 records pred[v] = u for the edge that last
// improved dist[v]).
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>

#include "sssp.h"

namespace sssp {
int set_error(int code, const char* msg);
}

namespace {

constexpr int32_t kInf = 0x7fffffff;

int err(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return sssp::set_error(code, buf);
}

// W[i][j] = 0 on the diagonal, INT32_MAX (no edge) elsewhere.
__global__ void k_fill_empty(int32_t* __restrict__ W, int64_t ld, int32_t n) {
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y)
        for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
            W[i * ld + j] = i == j ? 0 : kInf;
}

// Scatter the edges with an atomic minimum, so a duplicated edge keeps its
// smallest weight; a self-loop leaves the diagonal at 0.  Edges with an
// endpoint outside [0, n) or a weight outside [0, INT32_MAX) are skipped and
// counted in *bad.
__global__ void k_scatter_edges(const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                                const int32_t* __restrict__ ew, int64_t m, int32_t n, int32_t directed,
                                int32_t* __restrict__ W, int64_t ld, unsigned long long* __restrict__ bad) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = eu[e], v = ev[e], w = ew[e];
        if (u < 0 || u >= n || v < 0 || v >= n || w < 0 || w == kInf) {
            atomicAdd(bad, 1ull);
            continue;
        }
        if (u == v) continue;
        atomicMin(&W[(int64_t)u * ld + v], w);
        if (!directed) atomicMin(&W[(int64_t)v * ld + u], w);
    }
}

// Pointer jumping over the pred forest: after the last step hops[v] is the
// number of edges on v's pred chain to the source (0 at the source, -1 when v
// is unreachable).  a/b hold (ancestor, hops so far) and are double-buffered.
__global__ void k_hops_init(const int32_t* __restrict__ pred, const int32_t* __restrict__ dist, int32_t n,
                            int32_t* __restrict__ anc, int32_t* __restrict__ hop) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const bool reach = dist[v] != kInf;
        anc[v] = reach ? pred[v] : -1;
        hop[v] = reach ? (pred[v] >= 0 ? 1 : 0) : -1;
    }
}

__global__ void k_hops_step(const int32_t* __restrict__ anc_in, const int32_t* __restrict__ hop_in, int32_t n,
                            int32_t* __restrict__ anc_out, int32_t* __restrict__ hop_out) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int32_t a = anc_in[v];
        if (a >= 0 && a < n) {
            anc_out[v] = anc_in[a];
            hop_out[v] = hop_in[v] + hop_in[a];
        } else {
            anc_out[v] = a;
            hop_out[v] = hop_in[v];
        }
    }
}

// One thread per target: walk pred back from the target and write the path
// source ... target into out[off[i] .. off[i] + hops[t]].
__global__ void k_paths(const int32_t* __restrict__ pred, const int32_t* __restrict__ hops, int32_t n,
                        const int32_t* __restrict__ targets, int32_t count, const int64_t* __restrict__ off,
                        int32_t* __restrict__ out) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        int32_t v = targets[i];
        if (v < 0 || v >= n) continue;
        const int32_t h = hops[v];
        if (h < 0) continue;
        for (int32_t k = h; k >= 0 && v >= 0 && v < n; --k) {
            out[off[i] + k] = v;
            v = pred[v];
        }
    }
}

}  // namespace

extern "C" {

int sssp_edges_to_dense(const int32_t* eu, const int32_t* ev, const int32_t* ew, int64_t m, int32_t n,
                        int32_t directed, int32_t* W, int64_t ld, int64_t* bad_edges, void* stream) {
    if (!W || n < 1 || ld < n || m < 0 || (m > 0 && (!eu || !ev || !ew)))
        return err(SSSP_EINVAL, "bad arguments (n=%d ld=%lld m=%lld)", n, (long long)ld, (long long)m);
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* d_bad = nullptr;
    hipError_t e = hipMallocAsync((void**)&d_bad, sizeof(unsigned long long), s);
    if (e != hipSuccess) return err(SSSP_ENOMEM, "hipMallocAsync: %s", hipGetErrorString(e));
    e = hipMemsetAsync(d_bad, 0, sizeof(unsigned long long), s);
    dim3 fg((unsigned)((n + 255) / 256 < 64 ? (n + 255) / 256 : 64), (unsigned)(n < 65535 ? n : 65535));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_fill_empty, fg, dim3(256), 0, s, W, ld, n);
        e = hipGetLastError();
    }
    if (e == hipSuccess && m > 0) {
        const int64_t blocks = (m + 255) / 256 < 8192 ? (m + 255) / 256 : 8192;
        hipLaunchKernelGGL(k_scatter_edges, dim3((unsigned)blocks), dim3(256), 0, s, eu, ev, ew, m, n, directed, W, ld,
                           d_bad);
        e = hipGetLastError();
    }
    unsigned long long bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, d_bad, sizeof bad, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFreeAsync(d_bad, s);
    if (e != hipSuccess) return err(SSSP_EDEVICE, "edge list conversion: %s", hipGetErrorString(e));
    if (bad_edges) *bad_edges = (int64_t)bad;
    return SSSP_OK;
}

int sssp_hops(const int32_t* pred, const int32_t* dist, int32_t n, int32_t* hops, void* stream) {
    if (!pred || !dist || !hops || n < 1) return err(SSSP_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    int32_t* buf = nullptr;
    hipError_t e = hipMallocAsync((void**)&buf, 3 * sizeof(int32_t) * (size_t)n, s);
    if (e != hipSuccess) return err(SSSP_ENOMEM, "hipMallocAsync: %s", hipGetErrorString(e));
    int32_t* a0 = buf;
    int32_t* a1 = buf + n;
    int32_t* h1 = buf + 2 * (size_t)n;
    const unsigned blocks = (unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_hops_init, dim3(blocks), dim3(256), 0, s, pred, dist, n, a0, hops);
    // ceil(log2 n) + 1 doublings reach the root of every chain
    int steps = 1;
    while ((1ll << (steps - 1)) < n) ++steps;
    int32_t *ai = a0, *hi = hops, *ao = a1, *ho = h1;
    for (int k = 0; k < steps; ++k) {
        hipLaunchKernelGGL(k_hops_step, dim3(blocks), dim3(256), 0, s, ai, hi, n, ao, ho);
        int32_t* t = ai;
        ai = ao;
        ao = t;
        t = hi;
        hi = ho;
        ho = t;
    }
    e = hipGetLastError();
    if (e == hipSuccess && hi != hops) e = hipMemcpyAsync(hops, hi, sizeof(int32_t) * (size_t)n,
                                                          hipMemcpyDeviceToDevice, s);
    (void)hipFreeAsync(buf, s);
    if (e != hipSuccess) return err(SSSP_EDEVICE, "hops: %s", hipGetErrorString(e));
    return SSSP_OK;
}

int sssp_paths(const int32_t* pred, const int32_t* hops, int32_t n, const int32_t* targets, int32_t count,
               const int64_t* offsets, int32_t* out, void* stream) {
    if (!pred || !hops || n < 1 || count < 0 || (count > 0 && (!targets || !offsets || !out)))
        return err(SSSP_EINVAL, "bad arguments");
    if (count == 0) return SSSP_OK;
    const unsigned blocks = (unsigned)((count + 255) / 256 < 4096 ? (count + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_paths, dim3(blocks), dim3(256), 0, (hipStream_t)stream, pred, hops, n, targets, count,
                       offsets, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return err(SSSP_EDEVICE, "paths: %s", hipGetErrorString(e));
    return SSSP_OK;
}

}  // extern "C"
