/*
 * sssp.h — C ABI of libsssp: single-source shortest paths on a dense n x n
 * int32 adjacency matrix, by Dijkstra's algorithm as given in Algorithm 1 of
 * "High-Performance Parallelization of Dijkstra's Algorithm Using MPI and CUDA"
 * (Section III-A), on AMD Instinct MI355X (gfx950).
 *
 * Data conventions (Section III-A's adjacency matrix):
 *   W      device pointer, row-major int32, n rows of `ld` entries (ld >= n).
 *          W[u*ld + v] is the weight of edge u -> v; INT32_MAX means "no edge"
 *          (the paper's infinity); the diagonal should be 0.  Weights must lie
 *          in [0, INT32_MAX-1]; a negative weight violates the precondition of
 *          Dijkstra's algorithm (its result is then unspecified; the kernels
 *          raise SSSP_STATUS_NEG_WEIGHT when they notice one).
 *   dist   device pointer, n int32 outputs: shortest distance from src, or
 *          INT32_MAX when unreachable.
 *   pred   device pointer, n int32 outputs: predecessor on the shortest path
 *          that Algorithm 1 finds (argmin ties go to the lowest vertex index,
 *          relaxation uses a strict '<'); -1 for src and unreachable vertices.
 * All buffers belong to the caller and must stay valid until the work that
 * uses them has finished on the stream.  The library owns only its internal
 * scratch (barrier words, exchange records), cached per (device, stream) until
 * sssp_stream_release / sssp_release_all.
 *
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Solves are
 * asynchronous; synchronise the stream before reading dist/pred.  Calls that
 * share a stream are ordered; solves issued on different streams use separate
 * scratch and may overlap, except whole-GPU solves (cooperative grids that
 * occupy every compute unit): one issued while another runs on a different
 * stream fails to launch (SSSP_EDEVICE); issue those on one stream.
 *
 * Errors: every entry point returns SSSP_OK (0) or a negative SSSP_E* code and
 * never throws.  sssp_last_error() returns a message for the calling thread's
 * most recent failure.  Faults detected inside a kernel (a barrier that timed
 * out, a negative weight) are reported asynchronously through
 * sssp_last_status().
 */
#ifndef SSSP_H
#define SSSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define SSSP_OK 0
#define SSSP_EINVAL (-1)     /* bad argument: null pointer, n < 1, src outside [0, n), ld < n, ... */
#define SSSP_EDEVICE (-2)    /* a HIP runtime call failed */
#define SSSP_ENOMEM (-3)     /* scratch allocation failed */
#define SSSP_EAGAIN (-4)     /* server admission full; retry later */
#define SSSP_ENOGRAPH (-5)   /* unknown server graph id */
#define SSSP_ETIMEDOUT (-6)  /* a wait expired */
#define SSSP_EUNSUPPORTED (-7)  /* size or shape not handled by the requested kernel */

/* asynchronous status bits (sssp_last_status) */
#define SSSP_STATUS_TIMEOUT 1         /* a grid barrier gave up waiting: results invalid */
#define SSSP_STATUS_NEG_WEIGHT 2      /* a negative weight was seen: precondition violated */
#define SSSP_STATUS_ZERO_FALLBACK 4   /* zero-weight edges forced single-vertex steps, sent a label-correcting
                                         solve back to the Dijkstra rounds, or made sssp_csr_solve order
                                         equal distances by a pass over them (informational) */

/* flags for sssp_dense_solve_ex / batched calls */
#define SSSP_FLAG_LITERAL 1u  /* settle one vertex per round: Algorithm 1 exactly as printed */
#define SSSP_FLAG_SINGLE 2u   /* force the one-workgroup kernel */
#define SSSP_FLAG_GRID 4u     /* force the persistent whole-GPU kernel */
#define SSSP_FLAG_COMPACT 8u  /* plans and servers: stream an exact uint8/uint16 copy of each graph
                                 whose weights all fit (built once, owned by the plan or server) */
#define SSSP_FLAG_LABEL_CORRECTING 16u
/* sssp_dense_solve_ex: the label-correcting method of the paper's CUDA design
 * (Section III-C, Algorithms 3 and 4), made deterministic: sweeps relax the rows
 * of the vertices whose dist changed in the previous sweep until none changes,
 * then one pass over the reachable rows sets pred[v] to the u of smallest
 * (dist[u], u) with dist[u] + W[u][v] == dist[v].  Same dist and pred as
 * Algorithm 1: when that pass finds a tight zero-weight edge the launch solves
 * again with the Dijkstra rounds (SSSP_STATUS_ZERO_FALLBACK).  Runs on the
 * whole-GPU grid (SSSP_FLAG_SINGLE: one workgroup); not with SSSP_FLAG_LITERAL.
 * Stats: ROUNDS = sweeps, SETTLED = rows streamed (frontiers plus the pred pass). */

/* statistics of a finished launch (sssp_last_status `stats`, 4 entries) */
#define SSSP_STAT_ROUNDS 0     /* rounds (one bucket of equal-dist vertices, or one vertex, each) */
#define SSSP_STAT_SETTLED 1    /* vertices settled with finite dist = matrix rows relaxed */
#define SSSP_STAT_FALLBACKS 2  /* rounds redone as one literal step because of zero weights */
#define SSSP_STAT_BARRIERS 3   /* grid barriers passed (whole-GPU kernel) */

/* Tuning knobs; pass NULL for the library's choice.  A zero field means "choose". */
typedef struct sssp_tuning {
    int32_t threads;       /* one-workgroup solve: workgroup size, 256 or 1024 */
    int32_t workgroups;    /* workgroups of the whole-GPU kernel, or of a batched launch */
    int32_t single_max_n;  /* batched plans: largest n solved by one workgroup (0 = autotune) */
    int32_t gang_columns;  /* batched plans: columns per gang member above that */
    int32_t group_sources; /* batched plans: sources of one shared matrix solved in lockstep by one
                              gang, 2..16 (0 = autotune, 1 = never; see sssp_batch_plan_create) */
    int32_t group_columns; /* batched plans: columns per member of such a gang, 512..4096, a multiple
                              of 4 (0 = with group_sources: 1024) */
    int32_t balance;       /* whole-GPU solve: pairs of workgroups share the rows of rounds of at
                              least 8192 rows (0 = from n >= 32768, 1 = always, -1 = never); dist
                              and pred do not depend on it */
    int32_t reserved[1];
} sssp_tuning;

/* One solve of a batch: same meaning as the arguments of sssp_dense_solve_ex. */
typedef struct sssp_instance {
    const int32_t* W;
    int64_t ld;
    int32_t n;
    int32_t src;
    int32_t* dist;
    int32_t* pred;
} sssp_instance;

int sssp_version(void);
const char* sssp_last_error(void);
const char* sssp_strerror(int code);

/*
 * Single-source solve, Algorithm 1 (Section III-A) on an n x n matrix with
 * ld = n.  Picks the one-workgroup kernel for small n and the persistent
 * whole-GPU kernel (one column slice per workgroup, the one-GPU form of the
 * column division of Section III-B) otherwise.  Returns after enqueueing.
 */
int sssp_dense_solve(const int32_t* W, int32_t n, int32_t src, int32_t* dist, int32_t* pred,
                     void* stream);

/* As sssp_dense_solve with a row stride, SSSP_FLAG_* flags and tuning (NULL = default). */
int sssp_dense_solve_ex(const int32_t* W, int64_t ld, int32_t n, int32_t src, int32_t* dist,
                        int32_t* pred, uint32_t flags, const sssp_tuning* tuning, void* stream);

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * solve as sssp_dense_solve_ex (same kernels, same dist/pred; flags LITERAL,
 * SINGLE, GRID; no tuning), but it allocates nothing: the library scratch of
 * the whole-GPU kernel (control block, exchange records, bucket lists) lives
 * in one fixed array of SSSP_NOALLOC_SCRATCH_BYTES per GPU, held from the
 * first call on that GPU until the process ends.  n <= SSSP_NOALLOC_MAX_N
 * (larger n: SSSP_EUNSUPPORTED, nothing launched); SSSP_FLAG_LABEL_CORRECTING
 * is refused with SSSP_EUNSUPPORTED.  `status` (device pointer to one int32,
 * may be NULL) receives the solve's SSSP_STATUS_* bits when it finishes, in
 * stream order; sssp_last_status() does not see these solves.
 * Every call on one GPU shares that GPU's array: calls whose work overlaps on
 * one GPU (other streams, other host threads, the same call issued again
 * before the previous one finished on another stream) race and give wrong
 * results; calls on one stream are ordered and safe.  Each call clears what
 * must start at zero with a fill kernel, so no call depends on the previous
 * one's leftovers.  Asynchronous, like sssp_dense_solve.
 */
#define SSSP_NOALLOC_SCRATCH_BYTES (8u << 20)
#define SSSP_NOALLOC_MAX_N 262144
int sssp_dense_solve_noalloc(const int32_t* W, int64_t ld, int32_t n, int32_t src, int32_t* dist,
                             int32_t* pred, uint32_t flags, int32_t* status, void* stream);

/*
 * Synchronises `stream` and reports the last solve or batch launched on it by
 * this library: *status gets SSSP_STATUS_* bits, stats (may be NULL) gets the
 * 4 SSSP_STAT_* counters.  Returns SSSP_EINVAL if nothing was launched on it.
 */
int sssp_last_status(void* stream, int32_t* status, int64_t* stats);

/*
 * Per-round trace of the last one-workgroup or whole-GPU solve on `stream`
 * (synchronises it): t_ns[i] = start of round i in ns after the start of
 * round 0, t_ns[count] = end of the solve, rows[i] = matrix rows streamed in
 * round i (rows[count] = -1).  Writes min(count + 1, cap) entries; *count gets
 * the number of rounds recorded (at most 256).  A debugging and tuning aid.
 */
int sssp_last_trace(void* stream, int64_t* t_ns, int32_t* rows, int32_t cap, int32_t* count);

/*
 * Batched solve: `count` independent instances (host array of descriptors
 * pointing at device buffers; instances may share W) in ONE persistent launch
 * in which workgroups pull work from a ticket counter, largest instance first:
 * an instance with n <= sssp_batch_max_n() is solved by one workgroup, a
 * larger one by a gang of workgroups that split its columns.  With
 * SSSP_FLAG_LABEL_CORRECTING every instance whose matrix is not shared by 32
 * or more instances is solved with the label-correcting method (see that
 * flag) by a gang of 256-column slices.  Asynchronous.
 */
int sssp_dense_solve_batched(const sssp_instance* inst, int32_t count, uint32_t flags,
                             const sssp_tuning* tuning, void* stream);
int32_t sssp_batch_max_n(void);

/*
 * Batched plans: built once for a fixed set of instances, launched many times.
 * Creation (synchronous on `stream`) validates the instances; with
 * SSSP_FLAG_COMPACT it builds exact compact copies of the distinct matrices
 * whose weights fit (uint8 when 0 <= w <= 254, uint16 when <= 65534; the
 * all-ones code means "no edge") and whose n is at most 65536 (larger ones
 * stay int32), which cut the bytes streamed per row 4x or 2x and give
 * identical dist/pred; it then measures candidate splits of the
 * instances into workgroups (one workgroup per instance, or gangs of
 * workgroups that share an instance's columns) unless `tuning` fixes one,
 * keeps the fastest, and captures the launch into a hipGraph.  A launch
 * replays the graph on `stream`: one persistent kernel for all instances.
 * Instances of a matrix shared by 32 or more instances are solved by one
 * workgroup each, or, when that matrix has n <= 16384 and no off-diagonal
 * weight below 1, in groups of `group_sources` sources run in lockstep by a
 * gang (shared-row relaxation: each round reads a row once for every source
 * of the group whose current bucket holds it; same dist/pred as alone); the
 * plan measures group sizes and keeps them only if the launch is faster, unless
 * `tuning` fixes group_sources (1 = never).  When it measures splits, it also solves each other
 * distinct matrix once (from its first instance's source, into scratch
 * buffers): a matrix whose solve takes 64 or more rounds (many distinct
 * distances) is a candidate for the label-correcting method, which is kept
 * for those instances if the whole launch is faster with it;
 * SSSP_FLAG_LABEL_CORRECTING uses it for all of them without measuring.
 * Results are the same either way.  The instance buffers must stay valid
 * while the plan exists.
 */
typedef struct sssp_batch_plan sssp_batch_plan;

typedef struct sssp_plan_info {
    int32_t threads, workgroups;
    int32_t single_max_n, gang_columns;  /* the chosen split */
    int32_t max_parts;                   /* largest gang */
    int32_t candidates;                  /* configurations measured */
    int32_t compact_graphs;              /* matrices streamed from a compact copy */
    int32_t graph;                       /* 1: launches replay a captured hipGraph */
    int64_t compact_bytes;               /* device bytes held by the compact copies */
    double tuned_ms;                     /* time of the chosen configuration, -1 if not measured */
    double build_ms;                     /* wall time of sssp_batch_plan_create */
    int32_t lc_instances;                /* instances solved with the label-correcting method */
    int32_t lc_candidates;               /* instances whose matrix qualified for it */
    int32_t group_sources, group_columns; /* the chosen lockstep groups (0: none) */
    int32_t group_items;                 /* groups in the launch */
    int32_t group_candidates;            /* instances whose matrix qualified for them */
} sssp_plan_info;

/* How a batched launch splits its instances (the item order and gang shapes of
 * sssp_dense_solve_batched / sssp_batch_plan_create for the given shape
 * parameters), computed on the host: it touches no device and reads none of the
 * buffers, only checks the instances' arguments as those calls do.  Entry k of
 * out (count entries) is the k-th item of the launch: largest n first, then the
 * instances of a matrix shared by at least 32 of them (each solved by one
 * workgroup).  An instance with n <= single_max_n (0 = the batch limit) is one
 * workgroup; a larger one a gang of `parts` workgroups of `columns` columns each
 * (a multiple of 4; parts = ceil(n / columns), at least 2), sized from
 * gang_columns (0 = 4096; a multiple of 4) and at most max_parts (0 = 512)
 * members.  With SSSP_FLAG_LABEL_CORRECTING every unshared instance is a
 * label-correcting gang (possibly of one) of at most 256 columns per member.
 * scratch_offset / scratch_bytes: its exchange records and lists in the launch's
 * arena (-1 / 0 when it has none); *arena_bytes (may be NULL) gets the total.
 * SSSP_EUNSUPPORTED if an instance would need columns above the batch limit. */
typedef struct sssp_layout_entry {
    int32_t instance;        /* index into inst */
    int32_t parts;           /* workgroups that solve it */
    int32_t columns;         /* columns per workgroup (n for one workgroup) */
    int32_t method;          /* 0: Dijkstra rounds, 1: label-correcting */
    int64_t scratch_offset;  /* byte offset in the arena, -1 if none */
    int64_t scratch_bytes;
} sssp_layout_entry;
int sssp_batch_layout(const sssp_instance* inst, int32_t count, uint32_t flags, int32_t single_max_n,
                      int32_t gang_columns, int32_t max_parts, sssp_layout_entry* out, int64_t* arena_bytes);

int sssp_batch_plan_create(const sssp_instance* inst, int32_t count, uint32_t flags, const sssp_tuning* tuning,
                           void* stream, sssp_batch_plan** out);
int sssp_batch_plan_launch(sssp_batch_plan* plan, void* stream);
int sssp_batch_plan_info(const sssp_batch_plan* plan, sssp_plan_info* info);
/* Synchronises `stream`; status and SSSP_STAT_* counters of the plan's last launch. */
int sssp_batch_plan_status(sssp_batch_plan* plan, void* stream, int32_t* status, int64_t* stats);
/* Waits for the plan's last launch, then frees it and its compact copies. */
int sssp_batch_plan_destroy(sssp_batch_plan* plan);

/*
 * Edge list -> dense matrix (the input step of Section III): W (device, n rows
 * of stride ld) is set to 0 on the diagonal and INT32_MAX elsewhere, then each
 * edge (eu[e], ev[e], ew[e]) (device arrays of m entries) is written at
 * W[u][v], and also at W[v][u] unless `directed`.  A repeated edge keeps its
 * smallest weight; a self-loop leaves the diagonal at 0; an edge with an
 * endpoint outside [0, n) or a weight outside [0, INT32_MAX) is skipped and
 * counted in *bad_edges (may be NULL).  Synchronises `stream`.
 */
int sssp_edges_to_dense(const int32_t* eu, const int32_t* ev, const int32_t* ew, int64_t m, int32_t n,
                        int32_t directed, int32_t* W, int64_t ld, int64_t* bad_edges, void* stream);

/*
 * Hop counts of the shortest-path tree a solve returned (device arrays of n):
 * hops[v] = edges on the pred chain from the source to v, 0 at the source,
 * -1 where dist[v] is INT32_MAX.  Pointer jumping, O(log n) passes;
 * asynchronous.  pred must come from a solve (a forest rooted at the source).
 */
int sssp_hops(const int32_t* pred, const int32_t* dist, int32_t n, int32_t* hops, void* stream);

/*
 * Paths out of pred: for each of `count` targets (device array), writes the
 * hops[t] + 1 vertices source ... t into out[offsets[i] ...] (device arrays;
 * offsets are the caller's, e.g. an exclusive prefix sum of hops[t] + 1).
 * Unreachable or out-of-range targets write nothing.  Asynchronous.
 */
int sssp_paths(const int32_t* pred, const int32_t* hops, int32_t n, const int32_t* targets, int32_t count,
               const int64_t* offsets, int32_t* out, void* stream);

/* Weight range of a device matrix (synchronous): *min_w over all entries, *max_finite_w
 * over entries other than INT32_MAX.  This checks the precondition of Dijkstra's
 * algorithm (the 1959 method Section II names as the basis assumes non-negative
 * weights): *min_w < 0 means the input violates it. */
int sssp_dense_validate(const int32_t* W, int64_t ld, int32_t n, int32_t* min_w, int32_t* max_finite_w,
                        void* stream);

/* Largest n the one-workgroup kernel accepts. */
int32_t sssp_single_max_n(void);

/*
 * Library scratch.  The solve, batched and adjacency-list calls keep a small
 * scratch block per (device, stream): a control block, exchange records and
 * bucket lists, about 8 bytes per vertex of the largest solve issued there,
 * plus a few counters per device for sssp_stream_read.  It is allocated on
 * first use and grows as needed; it is released here, not at process exit
 * (the runtime reclaims it with the process).
 * sssp_stream_release: waits for `stream` (on the current device), frees its
 * scratch and forgets it, so that a stream about to be destroyed leaves no
 * entry behind; call it before hipStreamDestroy on a stream the library has
 * used.  A later call on the stream allocates again; sssp_last_status then
 * reports nothing launched.  SSSP_OK also when nothing was held.
 * sssp_release_all: the same for every stream of every device, then frees the
 * stream-read counters after a device synchronisation of each device that has
 * them (so it also waits for other work on those devices).  Call it before
 * unloading the library (dlclose); servers and batch plans own their memory
 * and are released by their destroy calls, not here.
 * sssp_scratch_bytes: device bytes of scratch currently held, all devices.
 */
int sssp_stream_release(void* stream);
int sssp_release_all(void);
int sssp_scratch_bytes(int64_t* bytes);

/* Diagnostic: launches (asynchronously, on `stream`) a plain kernel that reads
 * the first `bytes` (a positive multiple of 16) of the device buffer `buf`
 * (16-byte aligned) exactly once with nontemporal 16-byte loads and does
 * nothing else; time it to obtain the read bandwidth the device delivers in
 * practice, the ceiling for the row-streaming solves.  Workgroups claim
 * chunks of `chunk_bytes` (0: 256 KiB; else a multiple of 16 in [1 KiB,
 * 64 MiB]) from a counter, so faster XCDs take more of them.  If `fold`
 * (device uint32, may be NULL) is given, the xor of every 32-bit word read is
 * xor-ed into it (zero it first to obtain the buffer's xor).  The claim
 * counter is the library's, one per device, reset by each launch at its end:
 * calls on one device must not overlap (issue them on one stream).
 * SSSP_EINVAL on bad arguments, SSSP_ENOMEM / SSSP_EDEVICE on runtime errors. */
int sssp_stream_read(const void* buf, int64_t bytes, int64_t chunk_bytes, uint32_t* fold, void* stream);

/* ------------------------------------------------------------------------
 * Graphs stored as adjacency lists (CSR), for sparse graphs (the paper's m = 3n
 * family, Section IV-A) whose n x n matrix would waste memory (the third point
 * of Section V, the conclusion).  Row u lists edges u -> col[e] with weight
 * w[e] for row_ptr[u] <= e < row_ptr[u+1] (row_ptr: n + 1 int64; col, w:
 * int32; device pointers).  The
 * graph means what the matrix built from the same edges means: G[u][v] is the
 * smallest weight of the edges u -> v; self-loops and weights outside
 * [0, INT32_MAX) play no part.
 * ------------------------------------------------------------------------ */

/* Edge list (eu, ev, ew: m device int32 each) -> CSR on the device: both
 * orientations of each edge unless `directed`; self-loops dropped; edges with an
 * endpoint outside [0, n) or a weight outside [0, INT32_MAX) skipped and counted
 * in *bad_edges.  col and w must hold (directed ? m : 2m) entries; *m_out gets
 * the number used (row_ptr[n]).  Each row is sorted by (head, weight).
 * Synchronous (returns after the conversion). */
int sssp_edges_to_csr(const int32_t* eu, const int32_t* ev, const int32_t* ew, int64_t m, int32_t n,
                      int32_t directed, int64_t* row_ptr, int32_t* col, int32_t* w, int64_t* m_out,
                      int64_t* bad_edges, void* stream);

/* Single-source solve on a CSR graph: dist and pred as Algorithm 1 computes them
 * on the equivalent matrix (Section III-A), at any n.  The label-correcting
 * method over edges (see SSSP_FLAG_LABEL_CORRECTING) on a persistent
 * cooperative grid, then pred from the exact distances: the tail of smallest
 * (dist[u], u) among tight edges into v, or, when tight zero-weight edges make
 * the order in which Algorithm 1 settles equal distances matter, the tail that
 * order settles first, recovered by a pass over the vertices those edges touch
 * (one workgroup per distance; SSSP_STATUS_ZERO_FALLBACK, informational).
 * tuning->workgroups (may be NULL) sets the grid (default about n / 256; never
 * above 1024 nor the co-resident count).  Stats: ROUNDS = sweeps, SETTLED = edge
 * lists relaxed (the sweep count may differ between runs; dist and pred do not).
 * Allocates stream-ordered scratch of about 100 n bytes.  Asynchronous. */
int sssp_csr_solve(const int64_t* row_ptr, const int32_t* col, const int32_t* w, int32_t n, int32_t src,
                   int32_t* dist, int32_t* pred, const sssp_tuning* tuning, void* stream);

/* The grid sssp_csr_solve would launch for n vertices on the stream's device:
 * *workgroups, and (each may be NULL) the co-resident workgroups per compute unit
 * and the compute units that bound it. */
int sssp_csr_grid(int32_t n, const sssp_tuning* tuning, void* stream, int32_t* workgroups, int32_t* per_cu,
                  int32_t* cus);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of (graph, source) queries on a persistent
 * kernel.  Graphs stay resident in HBM; each query is solved exactly as
 * sssp_dense_solve would solve it (same dist and pred).  A query is solved by
 * one workgroup when n <= single_max_n, otherwise by a gang of workgroups
 * that split its columns (the column division of Section III-B inside the
 * running kernel).  Submitted queries wait in a FIFO until a query slot, ring
 * space and (for gangs) arena memory for their exchange records are free,
 * then run concurrently with those already on the GPU.  While queries are
 * pending or running the server's kernel stays resident on the compute units
 * it was given (all but a few by default; other kernels run on the rest), so a
 * device-wide synchronisation (hipDeviceSynchronize) returns only after the
 * server has been idle for idle_park_ms and its kernel has left; prefer
 * stream synchronisation.  Buffers passed to submit must already hold their
 * final contents on the device (no pending writes).
 * ---------------------------------------------------------------------- */
typedef struct sssp_server sssp_server;

typedef struct sssp_server_config {
    int32_t workgroups;     /* persistent workgroups (0 = one per CU, leaving max(4, CUs/32) CUs free) */
    int32_t ring_slots;     /* descriptor ring entries (0 = 4096) */
    int32_t max_inflight;   /* queries admitted to the GPU at once (0 = 1024) */
    int32_t single_max_n;   /* largest n solved by one workgroup (0 = 4096; at most 16384) */
    int32_t gang_columns;   /* columns per gang member for larger n (0 = 2048; multiple of 4) */
    int32_t watchdog_ms;    /* kernel leaves if the host heartbeat stalls this long (0 = 2000) */
    int64_t scratch_bytes;  /* device arena for gang exchange records (0 = 256 MiB) */
    int64_t max_pending;    /* submissions waiting for admission before SSSP_EAGAIN (0 = no limit) */
    int32_t idle_park_ms;   /* kernel leaves after this long with no query; relaunched on demand (0 = 20) */
    int32_t lc_rounds;      /* once a query of a graph took this many rounds, later queries of that graph
                               use the label-correcting method if a cost model of the first such query
                               (exchanges per round vs rows streamed) finds it cheaper (0 = 64; < 0 = never) */
    int32_t lc_gang_columns;  /* columns per gang member of label-correcting queries (0 = 1024) */
    int32_t lc_model;       /* < 0: switch on lc_rounds alone, without the cost model (0 = use it) */
    int32_t idle_gang_columns;  /* latency mode: a gang query admitted while no other query waits is
                                   split into slices of this many columns (or wider, to fit in three
                                   quarters of the workgroups minus those in flight), for lower
                                   latency when the server is not saturated; Dijkstra and
                                   label-correcting gangs alike (0 = max(256, gang_columns / 4);
                                   < 0 = off: always gang_columns / lc_gang_columns) */
    int32_t idle_wait_us;   /* with nothing pending or in flight, the server thread beats the heartbeat
                               and looks for work this often (0 = 1000); above watchdog_ms the kernel
                               leaves whenever the server is idle and is relaunched on the next query */
    int32_t busy_gang_columns;  /* throughput mode: a Dijkstra gang query admitted with at least
                                   busy_queue queries waiting behind it is split into slices of this
                                   many columns (fewer members: less exchange cost per query, higher
                                   throughput under a backlog); 0 = 2 x gang_columns for int32
                                   graphs, 4 x for compact copies (at most 16384); < 0 = off;
                                   otherwise a multiple of 4, at most 16384 */
    int32_t busy_queue;     /* queries waiting behind a query that switch it to throughput mode
                               (0 = 128) */
} sssp_server_config;

/* query states */
#define SSSP_QUERY_PENDING 0
#define SSSP_QUERY_RUNNING 1
#define SSSP_QUERY_DONE 2

typedef struct sssp_query_info {
    int32_t state;        /* SSSP_QUERY_* */
    int32_t status;       /* SSSP_STATUS_* bits of its solve */
    int32_t parts;        /* workgroups that solved it */
    int32_t rounds;
    int64_t settled;      /* rows relaxed */
    int64_t t_submit_ns;  /* sssp_server_now_ns() clock */
    int64_t t_admit_ns;
    int64_t t_done_ns;    /* when the host saw the completion record */
    int32_t method;       /* 0: Dijkstra rounds, 1: label-correcting (rounds = sweeps) */
    int32_t reserved;
} sssp_query_info;

typedef struct sssp_server_stats {
    int64_t submitted, completed, running, pending, kernel_launches;
    int32_t workgroups;
    int32_t failed;  /* a relaunch of the kernel failed */
} sssp_server_stats;

/* Host monotonic clock (ns) used for all server timestamps. */
int64_t sssp_server_now_ns(void);

/* The split the server gives an n-vertex query, computed on the host (no
 * device, no server): with configuration *cfg (NULL = all defaults; filled in as
 * sssp_server_create does) on a kernel of `workgroups` workgroups, for the
 * Dijkstra rounds (method 0) or the label-correcting method (1) on a graph
 * stored with `elem` bytes per entry (4: the caller's int32 matrix; 2 / 1: a
 * compact copy), when `busy` workgroups already hold queries in flight and
 * `waiting` queries are queued behind it (the latency-mode split of
 * idle_gang_columns applies when waiting == 0, the throughput-mode split of
 * busy_gang_columns when waiting >= busy_queue).  *parts: workgroups that
 * solve it (1 = one workgroup); *columns: columns per member (n for a
 * Dijkstra query solved by one workgroup alone; otherwise a multiple of 4, also
 * for a label-correcting gang of one); *scratch_bytes (may be NULL): arena
 * bytes for its exchange records.  SSSP_ENOMEM if the query could never fit the
 * arena (sssp_server_submit refuses it the same way). */
int sssp_server_shape(const sssp_server_config* cfg, int32_t workgroups, int32_t n, int32_t method, int32_t elem,
                      int32_t busy, int32_t waiting, int32_t* parts, int32_t* columns, int64_t* scratch_bytes);

/* Creates a server on the current device and launches its kernel; cfg may be NULL. */
int sssp_server_create(const sssp_server_config* cfg, sssp_server** out);

/* Registers a device-resident n x n matrix (row stride ld); the server borrows
 * W until sssp_server_destroy.  *graph_id receives its id. */
int sssp_server_add_graph(sssp_server* s, const int32_t* W, int64_t ld, int32_t n, int32_t* graph_id);

/* As sssp_server_add_graph; with SSSP_FLAG_COMPACT the server builds and keeps an
 * exact uint8/uint16 copy of W when its weights fit (see sssp_batch_plan_create)
 * and streams that copy; with SSSP_FLAG_LABEL_CORRECTING every query of the graph
 * uses the label-correcting method (otherwise only after one took lc_rounds
 * rounds).  Same dist/pred either way.  Synchronous. */
int sssp_server_add_graph_ex(sssp_server* s, const int32_t* W, int64_t ld, int32_t n, uint32_t flags,
                             int32_t* graph_id);

/* Bytes per matrix entry the server streams for a graph: 4, 2 or 1. */
int sssp_server_graph_elem(sssp_server* s, int32_t graph_id, int32_t* elem_bytes);

/* Queues a query; dist and pred are caller-owned device buffers of n int32
 * that must stay valid until the query is done.  Never blocks; returns
 * SSSP_EAGAIN when max_pending queries already wait, SSSP_ENOGRAPH for an
 * unknown graph.  *ticket (1, 2, ...) names the query. */
int sssp_server_submit(sssp_server* s, int32_t graph_id, int32_t src, int32_t* dist, int32_t* pred,
                       uint64_t* ticket);

/* Moves up to cap tickets of completed, not yet polled queries into tickets[]. */
int sssp_server_poll(sssp_server* s, uint64_t* tickets, int32_t cap, int32_t* count);

/* Waits until the query is done (timeout_ns < 0: no limit); SSSP_ETIMEDOUT otherwise.
 * dist/pred are then complete in device memory. */
int sssp_server_wait(sssp_server* s, uint64_t ticket, int64_t timeout_ns);

int sssp_server_query_info(sssp_server* s, uint64_t ticket, sssp_query_info* info);
int sssp_server_get_stats(sssp_server* s, sssp_server_stats* stats);

/* Drains (every submitted query completes), stops the kernel, frees the server. */
int sssp_server_destroy(sssp_server* s);

#ifdef __cplusplus
}
#endif

#endif /* SSSP_H */
