/*
 * Seeded, counter-based generator of dense weighted adjacency matrices (host side).
 *
 * This is input tooling shared by the oracle side and the GPU side: it holds no
 * shortest-path arithmetic.  Every matrix entry is a pure function of
 * (seed, i, j), so any row or tile can be produced independently and the
 * device generator in gen_device.hip reproduces it exactly.
 *
 * Entry (i, j), i != j:
 *   key  = undirected ? (min(i,j) << 32 | max(i,j)) : (i << 32 | j)
 *   h    = mix(mix(seed) ^ key)          mix = SplitMix64 finaliser
 *                                         (Steele, Lea & Flood, OOPSLA 2014)
 *   edge iff (h >> 32) < thresh          thresh = floor(p * 2^32), 0..2^32
 *   w    = lo + (((h & 0xffffffff) * (hi - lo + 1)) >> 32)
 *                                         (Lemire's multiply-shift range map)
 *   W[i][j] = edge ? w : INT32_MAX ; W[i][i] = 0
 *
 * The matrix is the one the paper builds from an edge list (Section III-A):
 * row = tail vertex, column = head vertex, infinity for a missing edge, zero
 * diagonal; an undirected graph stores each edge in both orientations.
 */
#include <stdint.h>
#include <stdlib.h>
#include <pthread.h>

#define GEN_INF 0x7fffffff

static inline uint64_t gen_mix64(uint64_t x)
{
    x += 0x9e3779b97f4a7c15ULL;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
    return x ^ (x >> 31);
}

uint64_t gen_mix64_c(uint64_t x) { return gen_mix64(x); }

static inline int32_t gen_entry(uint64_t smix, uint64_t thresh, uint32_t lo,
                                uint64_t span, int directed, uint32_t i, uint32_t j)
{
    if (i == j) return 0;
    uint64_t key;
    if (directed) key = ((uint64_t)i << 32) | j;
    else key = i < j ? (((uint64_t)i << 32) | j) : (((uint64_t)j << 32) | i);
    uint64_t h = gen_mix64(smix ^ key);
    if ((h >> 32) >= thresh) return GEN_INF;
    return (int32_t)(lo + (uint32_t)(((h & 0xffffffffULL) * span) >> 32));
}

int32_t gen_entry_c(uint64_t seed, uint64_t thresh, int32_t lo, int32_t hi,
                    int32_t directed, int32_t i, int32_t j)
{
    return gen_entry(gen_mix64(seed), thresh, (uint32_t)lo,
                     (uint64_t)((int64_t)hi - lo + 1), directed, (uint32_t)i, (uint32_t)j);
}

typedef struct {
    int32_t* W; int64_t ld; int32_t n; uint64_t smix; uint64_t thresh;
    uint32_t lo; uint64_t span; int directed; int32_t r0, r1;
    uint64_t sum;
    const int32_t* Wc;
} gen_job;

static void* gen_fill_worker(void* arg)
{
    gen_job* jb = (gen_job*)arg;
    for (int32_t i = jb->r0; i < jb->r1; ++i) {
        int32_t* row = jb->W + (int64_t)i * jb->ld;
        for (int32_t j = 0; j < jb->n; ++j)
            row[j] = gen_entry(jb->smix, jb->thresh, jb->lo, jb->span, jb->directed,
                               (uint32_t)i, (uint32_t)j);
    }
    return NULL;
}

/* Position-weighted checksum: sum over entries of (uint32)W[i][j] * (2*(i*n+j)+1), mod 2^64.
 * Order independent, so host and device reductions agree exactly. */
static void* gen_sum_worker(void* arg)
{
    gen_job* jb = (gen_job*)arg;
    uint64_t s = 0;
    for (int32_t i = jb->r0; i < jb->r1; ++i) {
        const int32_t* row = jb->Wc + (int64_t)i * jb->ld;
        uint64_t base = (uint64_t)i * (uint64_t)jb->n;
        for (int32_t j = 0; j < jb->n; ++j)
            s += (uint64_t)(uint32_t)row[j] * (2 * (base + (uint64_t)j) + 1);
    }
    jb->sum = s;
    return NULL;
}

static int gen_run(gen_job* proto, int threads, void* (*fn)(void*), uint64_t* sum_out)
{
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    int32_t rows = proto->r1 - proto->r0;
    if (threads > rows) threads = rows > 0 ? rows : 1;
    gen_job jobs[256];
    pthread_t tid[256];
    int32_t per = (rows + threads - 1) / threads;
    for (int t = 0; t < threads; ++t) {
        jobs[t] = *proto;
        jobs[t].r0 = proto->r0 + t * per;
        jobs[t].r1 = jobs[t].r0 + per;
        if (jobs[t].r1 > proto->r1) jobs[t].r1 = proto->r1;
        if (jobs[t].r0 >= jobs[t].r1) { jobs[t].sum = 0; continue; }
        if (pthread_create(&tid[t], NULL, fn, &jobs[t]) != 0) {
            fn(&jobs[t]);
            tid[t] = 0;
        }
    }
    uint64_t s = 0;
    for (int t = 0; t < threads; ++t) {
        if (jobs[t].r0 >= jobs[t].r1) continue;
        if (tid[t]) pthread_join(tid[t], NULL);
        s += jobs[t].sum;
    }
    if (sum_out) *sum_out = s;
    return 0;
}

/* Fill rows [0, n) of W (row stride ld >= n, int32 entries). Returns 0, or -1 on bad arguments. */
int gen_dense_fill(int32_t* W, int64_t ld, int32_t n, uint64_t seed, uint64_t thresh,
                   int32_t lo, int32_t hi, int32_t directed, int32_t threads)
{
    if (!W || n < 0 || ld < n || lo > hi || lo < 0 || thresh > (1ULL << 32)) return -1;
    gen_job jb = {0};
    jb.W = W; jb.ld = ld; jb.n = n; jb.smix = gen_mix64(seed); jb.thresh = thresh;
    jb.lo = (uint32_t)lo; jb.span = (uint64_t)((int64_t)hi - lo + 1); jb.directed = directed;
    jb.r0 = 0; jb.r1 = n;
    return gen_run(&jb, threads, gen_fill_worker, NULL);
}

/* Fill rows [r0, r0+rows) into a buffer that holds only those rows (row stride ld). */
int gen_dense_fill_rows(int32_t* Wrows, int64_t ld, int32_t n, int32_t r0, int32_t rows,
                        uint64_t seed, uint64_t thresh, int32_t lo, int32_t hi,
                        int32_t directed)
{
    if (!Wrows || n < 0 || ld < n || r0 < 0 || rows < 0 || r0 + rows > n || lo > hi || lo < 0)
        return -1;
    uint64_t smix = gen_mix64(seed), span = (uint64_t)((int64_t)hi - lo + 1);
    for (int32_t r = 0; r < rows; ++r)
        for (int32_t j = 0; j < n; ++j)
            Wrows[(int64_t)r * ld + j] = gen_entry(smix, thresh, (uint32_t)lo, span, directed,
                                                   (uint32_t)(r0 + r), (uint32_t)j);
    return 0;
}

uint64_t gen_dense_checksum(const int32_t* W, int64_t ld, int32_t n, int32_t threads)
{
    gen_job jb = {0};
    jb.Wc = W; jb.ld = ld; jb.n = n; jb.r0 = 0; jb.r1 = n;
    uint64_t s = 0;
    gen_run(&jb, threads, gen_sum_worker, &s);
    return s;
}

/*
 * Seeded edge list of a sparse graph (the paper's sparse family, Section IV-A:
 * m edges among n vertices).  Edge e, 0 <= e < m, is a pure function of
 * (seed, e):
 *   h = mix(mix(seed) ^ (e | 2^63)),  u = (hi32(h) * n) >> 32,  v = (lo32(h) * n) >> 32,
 *   w = lo + ((lo32(mix(h)) * (hi - lo + 1)) >> 32).
 * A pair may repeat and u may equal v; the conversion to a matrix or to CSR
 * keeps a repeated pair's smallest weight and ignores self-loops.
 */
int gen_sparse_edges(int32_t n, int64_t m, int32_t lo, int32_t hi, uint64_t seed,
                     int32_t* eu, int32_t* ev, int32_t* ew)
{
    if (n < 1 || m < 0 || hi < lo || !eu || !ev || !ew) return -1;
    const uint64_t smix = gen_mix64(seed), span = (uint64_t)((int64_t)hi - lo + 1);
    for (int64_t e = 0; e < m; ++e) {
        const uint64_t h = gen_mix64(smix ^ ((uint64_t)e | (1ULL << 63)));
        eu[e] = (int32_t)(((h >> 32) * (uint64_t)n) >> 32);
        ev[e] = (int32_t)(((h & 0xffffffffULL) * (uint64_t)n) >> 32);
        const uint64_t h2 = gen_mix64(h);
        ew[e] = (int32_t)(lo + (uint32_t)(((h2 & 0xffffffffULL) * span) >> 32));
    }
    return 0;
}
