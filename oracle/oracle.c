/*
 * CPU oracle for single-source shortest paths on a dense adjacency matrix.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source with the GPU library.
 *
 * Conventions (the paper's matrix of Section III-A): W is row-major int32 with
 * row stride ld; W[u][v] is the weight of edge u -> v; INT32_MAX means "no
 * edge" (the paper's infinity); the diagonal is 0.  dist[v] = INT32_MAX means
 * unreachable; pred[v] = -1 for the source and for unreachable vertices.
 *
 * Functions
 *   oracle_dijkstra        Algorithm 1 of the paper, step by step (serial).
 *   oracle_dijkstra_every_source  the same from every source of many tiny
 *                          matrices (a loop, for exhaustive pins).
 *   oracle_floyd_warshall  textbook all-pairs distances (dist only).
 *   oracle_bellman_ford    textbook single-source distances (dist only).
 *   oracle_certificate     shortest-path certificate of (dist, pred), O(n^2).
 *   oracle_closed_form_pred  pred characterised without running the loop;
 *                          equals Algorithm 1's pred whenever every
 *                          off-diagonal weight is >= 1.
 *   oracle_label_correcting  the paper's CUDA method (Algorithms 3 and 4) as
 *                          synchronous sweeps over the changed vertices:
 *                          dist, the number of sweeps and the rows relaxed.
 *   oracle_dijkstra_csr, oracle_certificate_csr, oracle_closed_form_pred_csr
 *                          the same on a graph stored as adjacency lists
 *                          (CSR): G[u][v] is the smallest weight of the edges
 *                          u -> v, self-loops and weights outside
 *                          [0, INT32_MAX) play no part.
 * All arithmetic on path lengths is exact (int64).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define OR_INF 0x7fffffff
#define OR_INF64 ((int64_t)1 << 62)

/*
 * Algorithm 1 (Section III-A): n iterations; each takes the unvisited vertex
 * with minimal dist (scanning indices upward with a strict '<', so the lowest
 * index wins a tie), marks it visited, then for every v that is unvisited,
 * has G[u][v] != inf and dist[u] + G[u][v] < dist[v] (strict), sets dist[v]
 * and pred[v] = u.
 *
 * Readings where the paper is silent: pred starts at -1; infinity is
 * INT32_MAX; the sum is formed in int64 so it never wraps.  When the minimal
 * unvisited dist is infinity every later iteration relaxes nothing (inf + w
 * is never < dist[v]), so with early_exit != 0 the loop stops there; the
 * outputs are identical either way.
 *
 * order (optional, n entries): settle order, -1 past the last settled vertex.
 * max_iters > 0 stops after that many iterations (a timing sample of the same
 * loop; the outputs are then partial).
 * Returns the number of settled vertices whose dist was finite (rows relaxed),
 * or -1 on bad arguments.
 */
int64_t oracle_dijkstra_iters(const int32_t* W, int64_t ld, int32_t n, int32_t src, int32_t* dist,
                              int32_t* pred, int32_t* order, int32_t early_exit, int32_t max_iters)
{
    if (!W || !dist || !pred || n < 1 || ld < n || src < 0 || src >= n) return -1;
    unsigned char* visited = (unsigned char*)calloc((size_t)n, 1);
    if (!visited) return -1;
    for (int32_t i = 0; i < n; ++i) {
        dist[i] = OR_INF;
        pred[i] = -1;
        if (order) order[i] = -1;
    }
    dist[src] = 0;
    int64_t relaxed = 0;
    const int32_t iters = (max_iters > 0 && max_iters < n) ? max_iters : n;
    for (int32_t i = 0; i < iters; ++i) {
        int32_t u = -1;
        for (int32_t v = 0; v < n; ++v)
            if (!visited[v] && (u < 0 || dist[v] < dist[u])) u = v;
        if (dist[u] == OR_INF && early_exit) break;
        visited[u] = 1;
        if (order) order[i] = u;
        if (dist[u] == OR_INF) continue; /* inf + w < dist[v] never holds */
        ++relaxed;
        const int32_t* row = W + (int64_t)u * ld;
        for (int32_t v = 0; v < n; ++v) {
            int32_t w = row[v];
            if (!visited[v] && w != OR_INF && (int64_t)dist[u] + (int64_t)w < (int64_t)dist[v]) {
                dist[v] = (int32_t)((int64_t)dist[u] + w);
                pred[v] = u;
            }
        }
    }
    free(visited);
    return relaxed;
}

int64_t oracle_dijkstra(const int32_t* W, int64_t ld, int32_t n, int32_t src, int32_t* dist,
                        int32_t* pred, int32_t* order, int32_t early_exit)
{
    return oracle_dijkstra_iters(W, ld, n, src, dist, pred, order, early_exit, 0);
}

/* Algorithm 1 from every source of each of `count` n x n matrices stored one
 * after another (row stride n): dist and pred get count x n x n entries, [g][s][v].
 * A loop over oracle_dijkstra for exhaustive pins over many tiny graphs.
 * Returns 0, or -1 on bad arguments. */
int oracle_dijkstra_every_source(const int32_t* Ws, int64_t count, int32_t n, int32_t* dist, int32_t* pred)
{
    if (!Ws || !dist || !pred || count < 0 || n < 1) return -1;
    const int64_t nn = (int64_t)n * n;
    for (int64_t g = 0; g < count; ++g)
        for (int32_t s = 0; s < n; ++s)
            if (oracle_dijkstra(Ws + g * nn, n, n, s, dist + g * nn + (int64_t)s * n, pred + g * nn + (int64_t)s * n,
                                0, 1) < 0)
                return -1;
    return 0;
}

/* Textbook Floyd-Warshall over the matrix; D is n x n int64, OR_INF64 = no path.
 * Path lengths >= INT32_MAX are reported as OR_INF64 (not representable as dist). */
int oracle_floyd_warshall(const int32_t* W, int64_t ld, int32_t n, int64_t* D)
{
    if (!W || !D || n < 1 || ld < n) return -1;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n; ++j) {
            int32_t w = W[(int64_t)i * ld + j];
            D[(int64_t)i * n + j] = (i == j) ? 0 : (w == OR_INF ? OR_INF64 : (int64_t)w);
        }
    for (int32_t k = 0; k < n; ++k)
        for (int32_t i = 0; i < n; ++i) {
            int64_t dik = D[(int64_t)i * n + k];
            if (dik >= OR_INF64) continue;
            for (int32_t j = 0; j < n; ++j) {
                int64_t dkj = D[(int64_t)k * n + j];
                if (dkj < OR_INF64 && dik + dkj < D[(int64_t)i * n + j])
                    D[(int64_t)i * n + j] = dik + dkj;
            }
        }
    for (int64_t e = 0; e < (int64_t)n * n; ++e)
        if (D[e] >= OR_INF) D[e] = OR_INF64;
    return 0;
}

/* Textbook Bellman-Ford from src: up to n-1 passes relaxing every finite edge. */
int oracle_bellman_ford(const int32_t* W, int64_t ld, int32_t n, int32_t src, int64_t* dist)
{
    if (!W || !dist || n < 1 || ld < n || src < 0 || src >= n) return -1;
    for (int32_t i = 0; i < n; ++i) dist[i] = OR_INF64;
    dist[src] = 0;
    for (int32_t pass = 0; pass < n - 1; ++pass) {
        int changed = 0;
        for (int32_t u = 0; u < n; ++u) {
            if (dist[u] >= OR_INF64) continue;
            for (int32_t v = 0; v < n; ++v) {
                int32_t w = W[(int64_t)u * ld + v];
                if (w != OR_INF && dist[u] + w < dist[v]) {
                    dist[v] = dist[u] + w;
                    changed = 1;
                }
            }
        }
        if (!changed) break;
    }
    for (int32_t i = 0; i < n; ++i)
        if (dist[i] >= OR_INF) dist[i] = OR_INF64;
    return 0;
}

/* ---------------- certificate: O(n^2), row-parallel ---------------- */

typedef struct {
    const int32_t* W; int64_t ld; int32_t n; const int32_t* dist;
    int32_t r0, r1; int64_t bad;
    const int32_t* order; int32_t* pred_out; int32_t c0, c1;
} or_job;

/* Feasibility: every finite edge u -> v out of a reachable u has dist[u] + w >= dist[v]. */
static void* or_feasible_worker(void* a)
{
    or_job* j = (or_job*)a;
    j->bad = -1;
    for (int32_t u = j->r0; u < j->r1 && j->bad < 0; ++u) {
        if (j->dist[u] == OR_INF) continue;
        const int32_t* row = j->W + (int64_t)u * j->ld;
        const int64_t du = j->dist[u];
        for (int32_t v = 0; v < j->n; ++v) {
            int32_t w = row[v];
            if (w != OR_INF && du + w < (int64_t)j->dist[v]) { j->bad = (int64_t)u * j->n + v; break; }
        }
    }
    return NULL;
}

static int or_threads(int32_t t, int32_t rows)
{
    if (t < 1) t = 1;
    if (t > 64) t = 64;
    if (t > rows) t = rows;
    return t < 1 ? 1 : t;
}

/*
 * Checks that (dist, pred) is a shortest-path tree from src:
 *   1  dist[src] != 0 or pred[src] != -1
 *   2  an edge u -> v with dist[u] + W[u][v] < dist[v]        (infeasible)
 *   3  a reachable v != src whose pred edge is not tight, or pred out of range
 *   4  an unreachable v with pred[v] != -1
 *   5  a pred chain that does not reach src (cycle)
 * Feasibility and tightness together pin dist to the true distances: tight pred
 * edges give a path of length dist[v], feasibility bounds every path below.
 * Returns 0 if valid; *where receives the offending vertex (or u*n+v for 2).
 */
int oracle_certificate(const int32_t* W, int64_t ld, int32_t n, int32_t src, const int32_t* dist,
                       const int32_t* pred, int32_t threads, int64_t* where)
{
    if (!W || !dist || !pred || n < 1 || ld < n || src < 0 || src >= n) return -1;
    if (where) *where = -1;
    if (dist[src] != 0 || pred[src] != -1) { if (where) *where = src; return 1; }
    int nt = or_threads(threads, n);
    or_job jobs[64];
    pthread_t tid[64];
    int32_t per = (n + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
        jobs[t].W = W; jobs[t].ld = ld; jobs[t].n = n; jobs[t].dist = dist;
        jobs[t].r0 = t * per; jobs[t].r1 = (t + 1) * per < n ? (t + 1) * per : n;
        if (pthread_create(&tid[t], NULL, or_feasible_worker, &jobs[t]) != 0) {
            or_feasible_worker(&jobs[t]);
            tid[t] = 0;
        }
    }
    int64_t bad = -1;
    for (int t = 0; t < nt; ++t) {
        if (tid[t]) pthread_join(tid[t], NULL);
        if (bad < 0 && jobs[t].bad >= 0) bad = jobs[t].bad;
    }
    if (bad >= 0) { if (where) *where = bad; return 2; }
    for (int32_t v = 0; v < n; ++v) {
        if (v == src) continue;
        if (dist[v] == OR_INF) {
            if (pred[v] != -1) { if (where) *where = v; return 4; }
            continue;
        }
        int32_t p = pred[v];
        if (p < 0 || p >= n || p == v || dist[p] == OR_INF) { if (where) *where = v; return 3; }
        int32_t w = W[(int64_t)p * ld + v];
        if (w == OR_INF || (int64_t)dist[p] + w != (int64_t)dist[v]) { if (where) *where = v; return 3; }
    }
    /* every pred chain must end at src: colour 0 = unseen, 1 = on stack, 2 = reaches src */
    unsigned char* col = (unsigned char*)calloc((size_t)n, 1);
    int32_t* stack = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!col || !stack) { free(col); free(stack); return -1; }
    col[src] = 2;
    for (int32_t v = 0; v < n; ++v) {
        if (dist[v] == OR_INF || col[v] == 2) continue;
        int32_t sp = 0, x = v;
        while (col[x] == 0) { col[x] = 1; stack[sp++] = x; x = pred[x]; }
        if (col[x] == 1) { free(col); free(stack); if (where) *where = v; return 5; }
        while (sp) col[stack[--sp]] = 2;
    }
    free(col);
    free(stack);
    return 0;
}

/* ---------------- closed-form pred ---------------- */

static int or_cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y);
}

static void* or_pred_worker(void* a)
{
    or_job* j = (or_job*)a;
    for (int32_t v = j->c0; v < j->c1; ++v) j->pred_out[v] = -1;
    int32_t left = j->c1 - j->c0;
    for (int32_t k = 0; k < j->n && left > 0; ++k) {
        int32_t u = j->order[k];
        if (j->dist[u] == OR_INF) break;
        const int32_t* row = j->W + (int64_t)u * j->ld;
        const int64_t du = j->dist[u];
        for (int32_t v = j->c0; v < j->c1; ++v) {
            if (j->pred_out[v] != -1 || v == u) continue;
            int32_t w = row[v];
            if (w != OR_INF && j->dist[v] != OR_INF && du + w == (int64_t)j->dist[v]) {
                j->pred_out[v] = u;
                --left;
            }
        }
    }
    return NULL;
}

/*
 * pred[v] = the u != v minimising (dist[u], u) among in-neighbours with
 * dist[u] + W[u][v] == dist[v]; -1 if there is none.
 *
 * Why it equals Algorithm 1's pred when every off-diagonal weight is >= 1:
 * then a vertex is settled only after every vertex of smaller dist, and
 * equal-dist vertices are settled by index, so the settle order is sorted by
 * (dist, index).  pred[v] is written by the first settled u whose relaxation
 * reaches the final dist[v]; later u with the same sum fail the strict '<'.
 * Rows are visited in (dist, index) order, columns split over threads.
 */
int oracle_closed_form_pred(const int32_t* W, int64_t ld, int32_t n, const int32_t* dist,
                            int32_t* pred, int32_t threads)
{
    if (!W || !dist || !pred || n < 1 || ld < n) return -1;
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
    if (!order || !keys) { free(order); free(keys); return -1; }
    for (int32_t i = 0; i < n; ++i) keys[i] = ((uint64_t)(uint32_t)dist[i] << 32) | (uint32_t)i;
    qsort(keys, (size_t)n, sizeof(uint64_t), or_cmp_u64);
    for (int32_t i = 0; i < n; ++i) order[i] = (int32_t)(keys[i] & 0xffffffffu);
    free(keys);
    int nt = or_threads(threads, n);
    or_job jobs[64];
    pthread_t tid[64];
    int32_t per = (n + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
        jobs[t].W = W; jobs[t].ld = ld; jobs[t].n = n; jobs[t].dist = dist;
        jobs[t].order = order; jobs[t].pred_out = pred;
        jobs[t].c0 = t * per; jobs[t].c1 = (t + 1) * per < n ? (t + 1) * per : n;
        if (jobs[t].c0 > n) jobs[t].c0 = n;
        if (pthread_create(&tid[t], NULL, or_pred_worker, &jobs[t]) != 0) {
            or_pred_worker(&jobs[t]);
            tid[t] = 0;
        }
    }
    for (int t = 0; t < nt; ++t)
        if (tid[t]) pthread_join(tid[t], NULL);
    free(order);
    return 0;
}

/*
 * Label-correcting sweeps (Section III-C: Algorithm 3 repeats the kernel of
 * Algorithm 4 until no dist changes; each kernel thread relaxes the row of its
 * vertex with dist[tid] + Adj[tid][v] < dist[v]).  Taken here in synchronous
 * form: a sweep relaxes the row of every vertex whose dist changed in the
 * previous sweep (the source in the first), each with the dist it had when
 * the sweep began, and all improvements take effect when the sweep ends.
 * Rows of vertices whose dist did not change cannot improve anything, which is
 * why Algorithm 4's full sweep can be narrowed to them.  Stops after a sweep
 * that changes nothing.  dist only (pred is not part of this method's steps);
 * *sweeps and *rows (both may be NULL) get the number of sweeps and the total
 * of rows relaxed.  Returns 0, or -1 on bad arguments / no memory.
 */
int oracle_label_correcting(const int32_t* W, int64_t ld, int32_t n, int32_t src, int32_t* dist,
                            int64_t* sweeps, int64_t* rows)
{
    if (!W || !dist || n < 1 || ld < n || src < 0 || src >= n) return -1;
    int64_t* d = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* next = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    unsigned char* changed = (unsigned char*)malloc((size_t)n);
    if (!d || !next || !changed) { free(d); free(next); free(changed); return -1; }
    for (int32_t v = 0; v < n; ++v) { d[v] = OR_INF; changed[v] = 0; }
    d[src] = 0;
    changed[src] = 1;
    int64_t nsweeps = 0, nrows = 0;
    for (;;) {
        int any = 0;
        for (int32_t v = 0; v < n; ++v) any |= changed[v];
        if (!any) break;
        ++nsweeps;
        memcpy(next, d, sizeof(int64_t) * (size_t)n);
        for (int32_t u = 0; u < n; ++u) {
            if (!changed[u]) continue;
            ++nrows;
            const int32_t* row = W + (int64_t)u * ld;
            for (int32_t v = 0; v < n; ++v) {
                if (row[v] == OR_INF) continue;
                int64_t c = d[u] + (int64_t)row[v];
                if (c < next[v]) next[v] = c;
            }
        }
        for (int32_t v = 0; v < n; ++v) {
            changed[v] = next[v] < d[v];
            d[v] = next[v];
        }
    }
    for (int32_t v = 0; v < n; ++v) dist[v] = d[v] >= OR_INF ? OR_INF : (int32_t)d[v];
    if (sweeps) *sweeps = nsweeps;
    if (rows) *rows = nrows;
    free(d);
    free(next);
    free(changed);
    return 0;
}

/* ---------------- input and output steps ---------------- */

/*
 * The input step of Section III: an edge list written into the adjacency
 * matrix.  Diagonal 0, INT32_MAX elsewhere, then each edge (u, v, w) at
 * W[u][v] and, for an undirected graph, at W[v][u]; a repeated edge keeps its
 * smallest weight and a self-loop leaves the diagonal at 0 (readings: the
 * paper does not say).  Edges with an endpoint outside [0, n) or a weight
 * outside [0, INT32_MAX) are skipped; returns how many, or -1 on bad arguments.
 */
int64_t oracle_edges_to_dense(const int32_t* eu, const int32_t* ev, const int32_t* ew, int64_t m, int32_t n,
                              int32_t directed, int32_t* W, int64_t ld)
{
    if (!W || n < 1 || ld < n || m < 0) return -1;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n; ++j) W[(int64_t)i * ld + j] = (i == j) ? 0 : OR_INF;
    int64_t bad = 0;
    for (int64_t e = 0; e < m; ++e) {
        int32_t u = eu[e], v = ev[e], w = ew[e];
        if (u < 0 || u >= n || v < 0 || v >= n || w < 0 || w == OR_INF) { ++bad; continue; }
        if (u == v) continue;
        if (w < W[(int64_t)u * ld + v]) W[(int64_t)u * ld + v] = w;
        if (!directed && w < W[(int64_t)v * ld + u]) W[(int64_t)v * ld + u] = w;
    }
    return bad;
}

/* Edges on the pred chain from the source to v, by walking it; -1 if unreachable. */
int oracle_hops(const int32_t* pred, const int32_t* dist, int32_t n, int32_t* hops)
{
    if (!pred || !dist || !hops || n < 1) return -1;
    for (int32_t v = 0; v < n; ++v) {
        if (dist[v] == OR_INF) { hops[v] = -1; continue; }
        int32_t h = 0, x = v;
        while (pred[x] >= 0 && h <= n) { x = pred[x]; ++h; }
        hops[v] = h;
    }
    return 0;
}

/* ---------------- graphs stored as adjacency lists (CSR) ---------------- */

/* Edge e of row u (row_ptr[u] <= e < row_ptr[u+1]) is u -> col[e] of weight w[e]. */
static int or_csr_edge_ok(int32_t u, int32_t v, int32_t w, int32_t n)
{
    return v >= 0 && v < n && v != u && w >= 0 && w != OR_INF;
}

/*
 * Algorithm 1 (Section III-A) with the relaxation of row u running over u's
 * edge list instead of a matrix row: identical argmin, strict '<' and int64
 * sums.  Several edges u -> v are relaxed in list order; the strict '<' makes
 * the smallest weight win, as G[u][v] = that weight would.
 * Returns the rows (edge lists) relaxed, or -1 on bad arguments.
 */
int64_t oracle_dijkstra_csr(const int64_t* row_ptr, const int32_t* col, const int32_t* w, int32_t n,
                            int32_t src, int32_t* dist, int32_t* pred)
{
    if (!row_ptr || !dist || !pred || n < 1 || src < 0 || src >= n) return -1;
    unsigned char* vis = (unsigned char*)calloc((size_t)n, 1);
    int64_t* d = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!vis || !d) { free(vis); free(d); return -1; }
    for (int32_t i = 0; i < n; ++i) { d[i] = OR_INF; pred[i] = -1; }
    d[src] = 0;
    int64_t relaxed = 0;
    for (int32_t it = 0; it < n; ++it) {
        int32_t u = -1;
        int64_t best = OR_INF;
        for (int32_t i = 0; i < n; ++i)
            if (!vis[i] && d[i] < best) { best = d[i]; u = i; }
        if (u < 0) break;  /* every unvisited dist is infinite */
        vis[u] = 1;
        ++relaxed;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            const int32_t v = col[e], wt = w[e];
            if (!or_csr_edge_ok(u, v, wt, n) || vis[v]) continue;
            const int64_t c = d[u] + wt;
            if (c < d[v]) { d[v] = c; pred[v] = u; }
        }
    }
    for (int32_t i = 0; i < n; ++i) dist[i] = d[i] >= OR_INF ? OR_INF : (int32_t)d[i];
    free(vis);
    free(d);
    return relaxed;
}

/*
 * The shortest-path certificate of (dist, pred) over edge lists; same codes as
 * oracle_certificate (1 source, 2 infeasible edge, 3 pred edge not tight,
 * 4 unreachable vertex with a pred, 5 pred chain not reaching the source).
 * O(n + m).
 */
int oracle_certificate_csr(const int64_t* row_ptr, const int32_t* col, const int32_t* w, int32_t n,
                           int32_t src, const int32_t* dist, const int32_t* pred, int64_t* where)
{
    if (!row_ptr || !dist || !pred || n < 1 || src < 0 || src >= n) return -1;
    if (where) *where = -1;
    if (dist[src] != 0 || pred[src] != -1) { if (where) *where = src; return 1; }
    /* smallest weight of the edge pred[v] -> v, to check tightness */
    int64_t* wp = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!wp) return -1;
    for (int32_t v = 0; v < n; ++v) wp[v] = OR_INF;
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            const int32_t v = col[e], wt = w[e];
            if (!or_csr_edge_ok(u, v, wt, n)) continue;
            if (dist[u] != OR_INF && (int64_t)dist[u] + wt < (int64_t)dist[v]) {
                free(wp);
                if (where) *where = v;
                return 2;
            }
            if (pred[v] == u && wt < wp[v]) wp[v] = wt;
        }
    for (int32_t v = 0; v < n; ++v) {
        if (v == src) continue;
        if (dist[v] == OR_INF) {
            if (pred[v] != -1) { free(wp); if (where) *where = v; return 4; }
            continue;
        }
        const int32_t p = pred[v];
        if (p < 0 || p >= n || p == v || dist[p] == OR_INF || wp[v] == OR_INF ||
            (int64_t)dist[p] + wp[v] != (int64_t)dist[v]) {
            free(wp);
            if (where) *where = v;
            return 3;
        }
    }
    free(wp);
    unsigned char* cl = (unsigned char*)calloc((size_t)n, 1);
    int32_t* stack = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!cl || !stack) { free(cl); free(stack); return -1; }
    cl[src] = 2;
    for (int32_t v = 0; v < n; ++v) {
        if (dist[v] == OR_INF || cl[v] == 2) continue;
        int32_t sp = 0, x = v;
        while (cl[x] == 0) { cl[x] = 1; stack[sp++] = x; x = pred[x]; }
        if (cl[x] == 1) { free(cl); free(stack); if (where) *where = v; return 5; }
        while (sp) cl[stack[--sp]] = 2;
    }
    free(cl);
    free(stack);
    return 0;
}

/*
 * pred[v] = the u != v of smallest (dist[u], u) with an edge u -> v such that
 * dist[u] + weight == dist[v] (-1 if none), over edge lists: Algorithm 1's pred
 * whenever no such tight edge has weight 0 (see oracle_closed_form_pred).
 */
int oracle_closed_form_pred_csr(const int64_t* row_ptr, const int32_t* col, const int32_t* w, int32_t n,
                                const int32_t* dist, int32_t* pred)
{
    if (!row_ptr || !dist || !pred || n < 1) return -1;
    uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
    if (!key) return -1;
    for (int32_t v = 0; v < n; ++v) key[v] = ~0ULL;
    for (int32_t u = 0; u < n; ++u) {
        if (dist[u] == OR_INF) continue;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            const int32_t v = col[e], wt = w[e];
            if (!or_csr_edge_ok(u, v, wt, n)) continue;
            if ((int64_t)dist[u] + wt != (int64_t)dist[v]) continue;
            const uint64_t k = ((uint64_t)(uint32_t)dist[u] << 32) | (uint32_t)u;
            if (k < key[v]) key[v] = k;
        }
    }
    for (int32_t v = 0; v < n; ++v) pred[v] = key[v] == ~0ULL ? -1 : (int32_t)(key[v] & 0xffffffffu);
    free(key);
    return 0;
}
