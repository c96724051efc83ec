// Batched solves: the one-shot call, and plans that are built once (exact
// compact copies of reused graphs, autotuned workgroups per instance, one
// captured hipGraph) and launched many times.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <vector>

#include "engine.h"
#include "multi.h"
#include "sssp_internal.h"

namespace sssp {
int set_error(int code, const char* msg);
const char* last_error_text();
int stream_ctl(hipStream_t stream, Ctl** out, int* cus, long long* clock_khz);
int check_instance(const sssp_instance& I, int idx);
}  // namespace sssp

using namespace sssp;

namespace {

int err(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return set_error(code, buf);
}

int hip_err(hipError_t e, const char* what) { return err(SSSP_EDEVICE, "%s: %s", what, hipGetErrorString(e)); }

// The matrix an instance is streamed from: the caller's, or a compact copy.
struct Source {
    const void* W;
    int64_t ld;
    int elem;
};

struct Build {
    std::vector<BatchItem> items;  // largest first
    std::vector<BatchPart> parts;
    std::vector<MultiSrc> groups;  // sources of the lockstep groups; an item's `group` holds its first index
    uint64_t arena_bytes = 0;
    int32_t max_parts = 1;
    int32_t group_items = 0;
};

bool aligned(const void* p, int64_t ld, int elem) {
    return ((uintptr_t)p % (4 * (uintptr_t)elem)) == 0 && ld % 4 == 0;
}

// Instances of one matrix shared by at least this many sources fill the GPU by
// themselves: each is solved by one workgroup (no gang exchange), and they are
// queued after the other instances, whose gangs are bound by their chains of
// rounds and start first; the shared ones fill the workgroups the gangs leave.
constexpr int32_t kSharedSources = 32;

// Columns per gang member of a label-correcting instance: its sweeps read 3-5
// times the rows of a Dijkstra solve, so it is spread over many workgroups.
constexpr int32_t kLcColumns = 256;

// Lockstep groups (multi.h): matrices up to this n; slices of 512..4096 columns.
constexpr int32_t kGroupMaxN = 16384;

// Shape of a group of up to `want` sources on an n-vertex matrix with slices of
// `cols` columns: *S columns per member, *parts members, and the sources per
// group (at most 4 per thread: 4 times the row partitions of a 1024-thread
// workgroup over S columns, and at most kMultiMax).
void group_shape(int32_t n, int32_t want, int32_t cols, int32_t* S, int32_t* parts, int32_t* K) {
    int32_t s = std::min<int32_t>(cols, (n + 3) & ~3);
    int32_t L = 1;
    while (L < (s + 3) / 4 && L < 1024) L <<= 1;
    const int32_t P = 1024 / L;
    *S = s;
    *parts = (n + s - 1) / s;
    *K = std::max<int32_t>(1, std::min<int32_t>({want, kMultiMax, 4 * P}));
}

// Items in largest-first order (instances of shared matrices last); an instance
// with n > single_max_n is split into parts of at most gang_columns columns
// solved by a gang of workgroups.  lc (may be null): per instance, solve it
// with the label-correcting method (never for shared matrices).
// group_k > 1 (with group_ok marking the eligible instances): instances of a
// shared matrix are solved group_k at a time in lockstep by gangs of group_cols
// columns per member (kMethodGroup items, queued between the other instances
// and the remaining shared ones).
int build(const sssp_instance* inst, const Source* src, int32_t count, int32_t single_max_n,
          int32_t gang_columns, int32_t max_parts, Build* out, const char* lc = nullptr,
          std::vector<int32_t>* order_out = nullptr, int32_t group_k = 0, int32_t group_cols = 0,
          const char* group_ok = nullptr) {
    std::vector<int32_t> order(count);
    for (int32_t i = 0; i < count; ++i) order[i] = i;
    std::map<std::pair<const void*, int64_t>, int32_t> uses;
    for (int32_t i = 0; i < count; ++i) ++uses[{src[i].W, src[i].ld}];
    std::vector<char> shared(count);
    for (int32_t i = 0; i < count; ++i)
        shared[i] = uses[{src[i].W, src[i].ld}] >= kSharedSources && inst[i].n <= max_batch_single_n();
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        if (shared[x] != shared[y]) return shared[x] < shared[y];
        return inst[x].n > inst[y].n;
    });
    out->items.clear();
    out->parts.clear();
    out->groups.clear();
    out->arena_bytes = 0;
    out->max_parts = 1;
    out->group_items = 0;
    std::vector<char> grouped(count, 0);
    bool groups_done = false;
    auto emit_groups = [&]() {
        groups_done = true;
        if (group_k < 2 || !group_ok) return;
        // eligible shared instances by matrix, in instance order
        std::map<std::pair<const void*, int64_t>, std::vector<int32_t>> by_matrix;
        for (int32_t i = 0; i < count; ++i)
            if (shared[i] && group_ok[i] && inst[i].n <= kGroupMaxN) by_matrix[{src[i].W, src[i].ld}].push_back(i);
        for (const auto& kv : by_matrix) {
            const std::vector<int32_t>& ids = kv.second;
            const sssp_instance& I0 = inst[ids.front()];
            int32_t S = 0, parts = 0, K = 0;
            group_shape(I0.n, group_k, group_cols, &S, &parts, &K);
            if (K < 2 || parts > max_parts) continue;
            for (size_t a = 0; a < ids.size(); a += (size_t)K) {
                const int32_t k = (int32_t)std::min<size_t>((size_t)K, ids.size() - a);
                BatchItem b;
                memset(&b, 0, sizeof b);
                b.W = src[ids[a]].W;
                b.ld = src[ids[a]].ld;
                b.elem = src[ids[a]].elem;
                b.n = I0.n;
                b.src = -1;
                b.vec = aligned(b.W, b.ld, b.elem) ? 1 : 0;
                b.method = kMethodGroup;
                b.K = k;
                b.S = S;
                b.parts = parts;
                b.group = reinterpret_cast<const void*>((uintptr_t)out->groups.size());
                for (int32_t j = 0; j < k; ++j) {
                    const sssp_instance& I = inst[ids[a + j]];
                    out->groups.push_back(MultiSrc{I.src, 0, I.dist, I.pred});
                    grouped[ids[a + j]] = 1;
                }
                b.scratch_off = out->arena_bytes;
                out->arena_bytes += multi_scratch_bytes(k, parts, S);
                out->max_parts = std::max(out->max_parts, parts);
                for (int32_t j = 0; j < parts; ++j) out->parts.push_back(BatchPart{(int32_t)out->items.size(), j});
                out->items.push_back(b);
                ++out->group_items;
            }
        }
    };
    for (int32_t k = 0; k < count; ++k) {
        if (!groups_done && shared[order[k]]) emit_groups();
        if (grouped[order[k]]) continue;
        const sssp_instance& I = inst[order[k]];
        BatchItem b;
        memset(&b, 0, sizeof b);
        b.W = src[order[k]].W;
        b.ld = src[order[k]].ld;
        b.elem = src[order[k]].elem;
        b.dist = I.dist;
        b.pred = I.pred;
        b.n = I.n;
        b.src = I.src;
        b.vec = aligned(b.W, b.ld, b.elem) ? 1 : 0;
        const bool use_lc = lc && lc[order[k]] && !shared[order[k]];
        b.method = use_lc ? kMethodLabelCorrecting : kMethodDijkstra;
        if (!use_lc && (I.n <= single_max_n || shared[order[k]])) {
            b.parts = 1;
            b.S = I.n;
        } else {
            const int32_t cols = use_lc ? kLcColumns : gang_columns;
            int64_t p = ((int64_t)I.n + cols - 1) / cols;
            p = std::max<int64_t>(use_lc ? 1 : 2, std::min<int64_t>(p, max_parts));
            int64_t s = ((int64_t)I.n + p - 1) / p;
            s = (s + 3) & ~int64_t(3);
            if (s > max_batch_slice())
                return err(SSSP_EUNSUPPORTED, "instance n=%d needs more than %d workgroups", I.n, max_parts);
            b.S = (int32_t)s;
            b.parts = (int32_t)(((int64_t)I.n + s - 1) / s);
            b.scratch_off = out->arena_bytes;
            out->arena_bytes += item_scratch_bytes(b.method, b.parts, b.S);
            out->max_parts = std::max(out->max_parts, b.parts);
        }
        for (int32_t j = 0; j < b.parts; ++j) out->parts.push_back(BatchPart{(int32_t)out->items.size(), j});
        out->items.push_back(b);
    }
    if (!groups_done) emit_groups();
    if (order_out) *order_out = order;
    return SSSP_OK;
}

int check_all(const sssp_instance* inst, int32_t count) {
    if (count < 0 || (count > 0 && !inst)) return err(SSSP_EINVAL, "bad instance array");
    for (int32_t i = 0; i < count; ++i) {
        int rc = check_instance(inst[i], i);
        if (rc) return rc;
    }
    return SSSP_OK;
}

}  // namespace

namespace sssp {

int matrix_range(const int32_t* W, int64_t ld, int32_t n, hipStream_t s, int32_t* wmin, int32_t* wmax, int32_t* woff) {
    int32_t* d = nullptr;
    hipError_t e = hipMalloc(&d, 3 * sizeof(int32_t));
    if (e != hipSuccess) return err(SSSP_ENOMEM, "hipMalloc(range): %s", hipGetErrorString(e));
    int32_t init[3] = {0x7fffffff, (int32_t)0x80000000, 0x7fffffff}, r[3];
    e = hipMemcpyAsync(d, init, sizeof init, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = weight_range(W, ld, n, d, s);
    if (e == hipSuccess) e = hipMemcpyAsync(r, d, sizeof r, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_err(e, "weight range");
    *wmin = r[0];
    *wmax = r[1];
    *woff = r[2];
    return SSSP_OK;
}

// Exact compact copy of W when every weight is >= 0 and every finite weight
// fits below the all-ones code of uint8 (<= 254) or uint16 (<= 65534).
// Synchronous.  out->elem == 4 (and no copy) when neither fits.
int make_compact(const int32_t* W, int64_t ld, int32_t n, hipStream_t s, CompactCopy* out) {
    out->data = nullptr;
    out->ld = ld;
    out->elem = 4;
    int32_t r[3];
    if (int rc = matrix_range(W, ld, n, s, &r[0], &r[1], &r[2])) return rc;
    out->wmin = r[0];
    out->wmax = r[1];
    out->woff = r[2];
    hipError_t e;
    // compact keys carry the row in 16 bits: copies only for n <= 65536
    int elem = 4;
    if (n > 65536) elem = 4;
    else if (r[0] >= 0 && r[1] <= 254) elem = 1;
    else if (r[0] >= 0 && r[1] <= 65534) elem = 2;
    if (elem == 4) return SSSP_OK;
    const int64_t ldc = ((int64_t)n + 15) & ~int64_t(15);
    void* c = nullptr;
    e = hipMalloc(&c, (size_t)ldc * n * elem);
    if (e != hipSuccess) return err(SSSP_ENOMEM, "hipMalloc(compact copy): %s", hipGetErrorString(e));
    e = compact_copy(W, ld, n, c, ldc, elem, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(c);
        return hip_err(e, "compact copy");
    }
    out->data = c;
    out->ld = ldc;
    out->elem = elem;
    return SSSP_OK;
}

}  // namespace sssp

struct sssp_batch_plan {
    int device = 0;
    uint32_t flags = 0;
    int nwg = 0;
    long long clock_khz = 100000;
    std::vector<sssp_instance> inst;
    std::vector<Source> src;
    std::vector<CompactCopy> copies;
    std::vector<char> lc;  // per instance: label-correcting (empty: none)
    std::vector<char> group_ok;  // per instance: its matrix may be solved in lockstep groups (empty: none)
    BatchItem* d_items = nullptr;
    MultiSrc* d_groups = nullptr;
    BatchPart* d_parts = nullptr;
    int32_t nparts = 0;
    Bar* d_bars = nullptr;
    char* d_arena = nullptr;
    Ctl* d_ctl = nullptr;
    hipStream_t cap = nullptr;
    hipEvent_t done = nullptr;  // recorded after every launch of the graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    sssp_plan_info info{};

    void free_device() {
        (void)hipFree(d_items);
        (void)hipFree(d_parts);
        (void)hipFree(d_bars);
        (void)hipFree(d_arena);
        (void)hipFree(d_groups);
        d_items = nullptr;
        d_parts = nullptr;
        d_bars = nullptr;
        d_arena = nullptr;
        d_groups = nullptr;
    }

    // Upload one configuration's items, parts and scratch (group_k < 2: no lockstep groups).
    int upload(int32_t single_max_n, int32_t gang_columns, int32_t group_k = 0, int32_t group_cols = 0) {
        Build b;
        int rc = ::build(inst.data(), src.data(), (int32_t)inst.size(), single_max_n, gang_columns,
                         std::max(2, nwg / 2), &b, lc.empty() ? nullptr : lc.data(), nullptr, group_k, group_cols,
                         group_ok.empty() ? nullptr : group_ok.data());
        if (rc) return rc;
        lc_items = 0;
        for (const BatchItem& it : b.items) lc_items += it.method == kMethodLabelCorrecting;
        group_items = b.group_items;
        free_device();
        hipError_t e = hipSuccess;
        if (!b.groups.empty()) {
            e = hipMalloc(&d_groups, sizeof(MultiSrc) * b.groups.size());
            if (e == hipSuccess)
                e = hipMemcpy(d_groups, b.groups.data(), sizeof(MultiSrc) * b.groups.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) return err(SSSP_ENOMEM, "group sources: %s", hipGetErrorString(e));
            for (BatchItem& it : b.items)
                if (it.method == kMethodGroup) it.group = d_groups + (uintptr_t)it.group;
        }
        e = hipMalloc(&d_items, sizeof(BatchItem) * b.items.size());
        if (e == hipSuccess) e = hipMalloc(&d_parts, sizeof(BatchPart) * b.parts.size());
        if (e == hipSuccess) e = hipMalloc(&d_bars, sizeof(Bar) * b.items.size());
        if (e == hipSuccess && b.arena_bytes) e = hipMalloc(&d_arena, b.arena_bytes);
        if (e != hipSuccess) return err(SSSP_ENOMEM, "allocating a batch plan: %s", hipGetErrorString(e));
        e = hipMemcpy(d_items, b.items.data(), sizeof(BatchItem) * b.items.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(d_parts, b.parts.data(), sizeof(BatchPart) * b.parts.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(d_bars, 0, sizeof(Bar) * b.items.size());
        // exchange records must start without stamps (see gang_exchange)
        if (e == hipSuccess && b.arena_bytes) e = hipMemset(d_arena, 0, b.arena_bytes);
        if (e != hipSuccess) return hip_err(e, "uploading a batch plan");
        nparts = (int32_t)b.parts.size();
        info.max_parts = b.max_parts;
        return SSSP_OK;
    }

    hipError_t enqueue(hipStream_t s) {
        return launch_batch(d_items, d_parts, nparts, d_bars, d_arena, flags & SSSP_FLAG_LITERAL,
                            clock_khz * 10000, d_ctl, nwg, s);
    }

    int32_t lc_items = 0;
    int32_t group_items = 0;

    // Median-free timing of the uploaded configuration: best of 2 launches after a
    // warm-up (ms), or a negative value on a launch error (e set).
    float time_launches(hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, hipError_t& e) {
        float ms = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            (void)hipEventRecord(ev0, s);
            e = enqueue(s);
            (void)hipEventRecord(ev1, s);
            if (e == hipSuccess) e = hipEventSynchronize(ev1);
            if (e != hipSuccess) return -1.0f;
            float t = 0;
            (void)hipEventElapsedTime(&t, ev0, ev1);
            if (rep > 0) ms = std::min(ms, t);  // first run warms caches
        }
        return ms;
    }
};

namespace {

// Rounds of a Dijkstra solve from which a matrix is tried with the
// label-correcting method: with that many distinct distances the rounds'
// exchanges, not the bytes, bound its instances.
constexpr int64_t kLcRounds = 64;

// Marks p->lc for every instance of a distinct matrix (used by fewer than
// kSharedSources instances) whose solve from its first instance's source takes
// kLcRounds rounds or more; the solves write into scratch buffers.  With
// SSSP_FLAG_LABEL_CORRECTING nothing is measured.
int lc_candidates(sssp_batch_plan* p, hipStream_t s) {
    p->lc.clear();
    p->info.lc_candidates = 0;
    if (p->flags & (SSSP_FLAG_LABEL_CORRECTING | SSSP_FLAG_LITERAL)) return SSSP_OK;
    const int32_t count = (int32_t)p->inst.size();
    std::map<std::pair<const int32_t*, int64_t>, std::vector<int32_t>> by_matrix;
    for (int32_t i = 0; i < count; ++i) by_matrix[{p->inst[i].W, p->inst[i].ld}].push_back(i);
    int32_t nmax = 0;
    for (const auto& I : p->inst) nmax = std::max(nmax, I.n);
    int32_t* buf = nullptr;
    hipError_t e = hipMalloc(&buf, 2 * sizeof(int32_t) * (size_t)nmax);
    if (e != hipSuccess) return err(SSSP_ENOMEM, "hipMalloc(probe buffers): %s", hipGetErrorString(e));
    std::vector<char> lc(count, 0);
    int rc = SSSP_OK;
    for (const auto& kv : by_matrix) {
        if ((int32_t)kv.second.size() >= kSharedSources) continue;
        const sssp_instance& I = p->inst[kv.second.front()];
        rc = sssp_dense_solve_ex(I.W, I.ld, I.n, I.src, buf, buf + nmax, 0u, nullptr, s);
        int32_t status = 0;
        int64_t stats[kStatCount] = {0};
        if (rc == SSSP_OK) rc = sssp_last_status(s, &status, stats);
        if (rc != SSSP_OK) break;
        if (stats[kStatRounds] >= kLcRounds)
            for (int32_t i : kv.second) lc[i] = 1;
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
    if (rc != SSSP_OK) return rc;
    for (char c : lc) p->info.lc_candidates += c;
    if (p->info.lc_candidates > 0) p->lc = lc;
    return SSSP_OK;
}

}  // namespace

extern "C" {

int32_t sssp_batch_max_n(void) { return max_batch_single_n(); }

int sssp_batch_layout(const sssp_instance* inst, int32_t count, uint32_t flags, int32_t single_max_n,
                      int32_t gang_columns, int32_t max_parts, sssp_layout_entry* out, int64_t* arena_bytes) {
    int rc = check_all(inst, count);
    if (rc) return rc;
    if (!out && count > 0) return err(SSSP_EINVAL, "out is NULL");
    if (single_max_n < 0 || gang_columns < 0 || max_parts < 0) return err(SSSP_EINVAL, "negative tuning value");
    if (single_max_n > max_batch_single_n())
        return err(SSSP_EINVAL, "single_max_n %d above the limit %d", single_max_n, max_batch_single_n());
    if (gang_columns % 4) return err(SSSP_EINVAL, "gang_columns %d is not a multiple of 4", gang_columns);
    std::vector<Source> src(count);
    for (int32_t i = 0; i < count; ++i) src[i] = Source{inst[i].W, inst[i].ld, 4};
    std::vector<char> lc;
    if (flags & SSSP_FLAG_LABEL_CORRECTING) lc.assign(count, 1);
    Build b;
    std::vector<int32_t> order;
    rc = build(inst, src.data(), count, single_max_n ? single_max_n : max_batch_single_n(),
               gang_columns ? gang_columns : 4096, max_parts ? max_parts : 512, &b, lc.empty() ? nullptr : lc.data(),
               &order);
    if (rc) return rc;
    for (int32_t k = 0; k < count; ++k) {
        const BatchItem& it = b.items[k];
        const unsigned long long bytes = item_scratch_bytes(it.method, it.parts, it.S);
        out[k] = sssp_layout_entry{order[k], it.parts, it.S, it.method,
                                   bytes ? (int64_t)it.scratch_off : -1, (int64_t)bytes};
    }
    if (arena_bytes) *arena_bytes = (int64_t)b.arena_bytes;
    return SSSP_OK;
}

int sssp_dense_validate(const int32_t* W, int64_t ld, int32_t n, int32_t* min_w, int32_t* max_finite_w,
                        void* stream) {
    if (!W || !min_w || !max_finite_w) return err(SSSP_EINVAL, "null argument");
    if (n < 1 || ld < n) return err(SSSP_EINVAL, "need n >= 1 and ld >= n");
    int32_t woff = 0;
    return matrix_range(W, ld, n, (hipStream_t)stream, min_w, max_finite_w, &woff);
}

int sssp_dense_solve_batched(const sssp_instance* inst, int32_t count, uint32_t flags, const sssp_tuning* tuning,
                             void* stream) {
    int rc = check_all(inst, count);
    if (rc) return rc;
    if (count == 0) return SSSP_OK;
    hipStream_t s = (hipStream_t)stream;
    Ctl* ctl = nullptr;
    int cus = 0;
    long long khz = 100000;
    rc = stream_ctl(s, &ctl, &cus, &khz);
    if (rc) return rc;
    int per_cu = 0;
    if (batch_occupancy(&per_cu) != 0 || per_cu < 1) return err(SSSP_EDEVICE, "batched kernel does not fit a CU");
    int nwg = tuning && tuning->workgroups ? std::min(tuning->workgroups, per_cu * cus) : per_cu * cus;
    std::vector<Source> src(count);
    for (int32_t i = 0; i < count; ++i) src[i] = Source{inst[i].W, inst[i].ld, 4};
    Build b;
    std::vector<char> lc;
    if (flags & SSSP_FLAG_LABEL_CORRECTING) lc.assign(count, 1);
    rc = build(inst, src.data(), count, max_batch_single_n(), 4096, std::max(2, nwg / 2), &b,
               lc.empty() ? nullptr : lc.data());
    if (rc) return rc;
    nwg = std::max(1, std::min<int>(nwg, (int)b.parts.size()));
    if (nwg < b.max_parts) nwg = b.max_parts;
    // stream-ordered scratch: allocated and freed in the stream's order, so the
    // call stays asynchronous (copies from pageable memory are staged at once)
    BatchItem* d_items = nullptr;
    BatchPart* d_parts = nullptr;
    Bar* d_bars = nullptr;
    char* d_arena = nullptr;
    hipError_t e = hipMallocAsync((void**)&d_items, sizeof(BatchItem) * b.items.size(), s);
    if (e == hipSuccess) e = hipMallocAsync((void**)&d_parts, sizeof(BatchPart) * b.parts.size(), s);
    if (e == hipSuccess) e = hipMallocAsync((void**)&d_bars, sizeof(Bar) * b.items.size(), s);
    if (e == hipSuccess && b.arena_bytes) e = hipMallocAsync((void**)&d_arena, b.arena_bytes, s);
    if (e != hipSuccess) return err(SSSP_ENOMEM, "hipMallocAsync(batch): %s", hipGetErrorString(e));
    e = hipMemcpyAsync(d_items, b.items.data(), sizeof(BatchItem) * b.items.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_parts, b.parts.data(), sizeof(BatchPart) * b.parts.size(), hipMemcpyHostToDevice, s);
    // barrier words and exchange records start zeroed (fill kernels, not memset
    // nodes, so that the call can be captured into a graph)
    if (e == hipSuccess) e = zero_fill(d_bars, sizeof(Bar) * b.items.size(), s);
    if (e == hipSuccess && b.arena_bytes) e = zero_fill(d_arena, b.arena_bytes, s);
    if (e == hipSuccess)
        e = launch_batch(d_items, d_parts, (int32_t)b.parts.size(), d_bars, d_arena, flags & SSSP_FLAG_LITERAL,
                         khz * 10000, ctl, nwg, s);
    (void)hipFreeAsync(d_items, s);
    (void)hipFreeAsync(d_parts, s);
    (void)hipFreeAsync(d_bars, s);
    if (d_arena) (void)hipFreeAsync(d_arena, s);
    if (e != hipSuccess) return hip_err(e, "batched launch");
    return SSSP_OK;
}

int sssp_batch_plan_create(const sssp_instance* inst, int32_t count, uint32_t flags, const sssp_tuning* tuning,
                           void* stream, sssp_batch_plan** out) {
    if (!out) return err(SSSP_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_all(inst, count);
    if (rc) return rc;
    if (count == 0) return err(SSSP_EINVAL, "empty plan");
    hipStream_t s = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    sssp_batch_plan* p = new sssp_batch_plan();
    auto fail = [&](int code) {
        p->free_device();
        for (auto& c : p->copies) (void)hipFree(c.data);
        (void)hipFree(p->d_ctl);
        if (p->exec) (void)hipGraphExecDestroy(p->exec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        if (p->cap) (void)hipStreamDestroy(p->cap);
        if (p->done) (void)hipEventDestroy(p->done);
        delete p;
        return code;
    };
    p->flags = flags;
    (void)hipGetDevice(&p->device);
    int cus = 0, rate = 0, per_cu = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, p->device) == hipSuccess && rate > 0)
        p->clock_khz = rate;
    if (batch_occupancy(&per_cu) != 0 || per_cu < 1) return fail(err(SSSP_EDEVICE, "batched kernel does not fit"));
    p->nwg = tuning && tuning->workgroups ? std::min(tuning->workgroups, per_cu * cus) : per_cu * cus;
    p->inst.assign(inst, inst + count);
    p->src.resize(count);
    // exact compact copies of the distinct matrices, when asked for and when they fit
    std::map<std::pair<const int32_t*, int64_t>, int> seen;
    for (int32_t i = 0; i < count; ++i) {
        p->src[i] = Source{inst[i].W, inst[i].ld, 4};
        if (!(flags & SSSP_FLAG_COMPACT)) continue;
        auto key = std::make_pair(inst[i].W, inst[i].ld);
        auto it = seen.find(key);
        if (it == seen.end()) {
            CompactCopy c;
            rc = make_compact(inst[i].W, inst[i].ld, inst[i].n, s, &c);
            if (rc) return fail(rc);
            p->copies.push_back(c);
            it = seen.emplace(key, (int)p->copies.size() - 1).first;
            if (c.elem < 4) {
                p->info.compact_graphs += 1;
                p->info.compact_bytes += (int64_t)c.ld * inst[i].n * c.elem;
            }
        }
        const CompactCopy& c = p->copies[it->second];
        if (c.elem < 4) p->src[i] = Source{c.data, c.ld, c.elem};
    }
    // matrices whose shared instances may run in lockstep groups: n <= kGroupMaxN and
    // every off-diagonal weight >= 1 (fused rounds then never fall back)
    const int32_t want_group = tuning ? tuning->group_sources : 0;
    if (!(flags & (SSSP_FLAG_LITERAL | SSSP_FLAG_LABEL_CORRECTING))) {
        std::map<std::pair<const int32_t*, int64_t>, std::vector<int32_t>> by_matrix;
        for (int32_t i = 0; i < count; ++i) by_matrix[{inst[i].W, inst[i].ld}].push_back(i);
        p->group_ok.assign(count, 0);
        for (const auto& kv : by_matrix) {
            const sssp_instance& I = inst[kv.second.front()];
            if ((int32_t)kv.second.size() < kSharedSources || I.n > kGroupMaxN || I.n > max_batch_single_n()) continue;
            int32_t wmin = 0, wmax = 0, woff = 0;
            auto cit = seen.find(kv.first);
            if (cit != seen.end()) {
                woff = p->copies[cit->second].woff;
            } else if ((rc = matrix_range(I.W, I.ld, I.n, s, &wmin, &wmax, &woff))) {
                return fail(rc);
            }
            if (woff < 1) continue;
            for (int32_t i : kv.second) p->group_ok[i] = 1;
            p->info.group_candidates += (int32_t)kv.second.size();
        }
        if (p->info.group_candidates == 0) p->group_ok.clear();
    }
    hipError_t e = hipMalloc(&p->d_ctl, ctl_size());
    if (e == hipSuccess) e = hipMemset(p->d_ctl, 0, ctl_size());
    if (e != hipSuccess) return fail(err(SSSP_ENOMEM, "plan control block: %s", hipGetErrorString(e)));
    // workgroups per instance: a single workgroup for n up to the single limit, or gangs
    // with a given number of columns per member; measured, fastest kept
    struct Cand {
        int32_t single_max_n, gang_columns;
    };
    std::vector<Cand> cands;
    int32_t nmax = 0;
    for (auto& I : p->inst) nmax = std::max(nmax, I.n);
    if (tuning && tuning->single_max_n > 0) {
        cands.push_back(Cand{tuning->single_max_n, tuning->gang_columns > 0 ? tuning->gang_columns : 4096});
    } else {
        if (nmax <= max_batch_single_n()) cands.push_back(Cand{max_batch_single_n(), 4096});
        for (int32_t c : {4096, 2048, 1024, 512, 256})
            if (c < nmax) cands.push_back(Cand{c, c});
    }
    double best_ms = 1e30;
    Cand best = cands.front();
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (cands.size() > 1) {
        (void)hipEventCreate(&ev0);
        (void)hipEventCreate(&ev1);
        for (const Cand& c : cands) {
            rc = p->upload(c.single_max_n, c.gang_columns);
            if (rc) continue;
            const float ms = p->time_launches(s, ev0, ev1, e);
            if (e != hipSuccess) {
                (void)hipEventDestroy(ev0);
                (void)hipEventDestroy(ev1);
                return fail(hip_err(e, "autotuning launch"));
            }
            p->info.candidates += 1;
            if (ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
        // label-correcting candidates: distinct matrices (not shared by many
        // instances) whose solve needs many rounds; kept if the launch is faster
        rc = lc_candidates(p, s);
        if (rc) {
            (void)hipEventDestroy(ev0);
            (void)hipEventDestroy(ev1);
            return fail(rc);
        }
        if (p->info.lc_candidates > 0) {
            rc = p->upload(best.single_max_n, best.gang_columns);
            float ms = rc ? -1.0f : p->time_launches(s, ev0, ev1, e);
            if (rc == 0 && e != hipSuccess) {
                (void)hipEventDestroy(ev0);
                (void)hipEventDestroy(ev1);
                return fail(hip_err(e, "autotuning launch"));
            }
            p->info.candidates += 1;
            if (ms >= 0 && ms < best_ms) best_ms = ms;
            else p->lc.clear();
        }
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
    } else if (flags & SSSP_FLAG_LABEL_CORRECTING) {
        p->lc.assign(count, 1);
    }
    if (flags & SSSP_FLAG_LABEL_CORRECTING) p->lc.assign(count, 1);
    // lockstep groups of the shared matrices' instances: fixed by the tuning, or
    // measured (group size, columns per member) and kept only if the launch is faster
    struct GroupCand {
        int32_t k, cols;
    };
    GroupCand gbest{0, 0};
    if (!p->group_ok.empty() && want_group != 1) {
        if (want_group >= 2) {
            gbest = GroupCand{std::min<int32_t>(want_group, kMultiMax),
                              tuning->group_columns > 0 ? tuning->group_columns : 1024};
        } else {
            (void)hipEventCreate(&ev0);
            (void)hipEventCreate(&ev1);
            auto measure = [&](const GroupCand& g, float* ms) -> int {
                int r = p->upload(best.single_max_n, best.gang_columns, g.k, g.cols);
                if (r) return r;
                *ms = p->time_launches(s, ev0, ev1, e);
                if (e != hipSuccess) return hip_err(e, "autotuning launch");
                p->info.candidates += 1;
                return SSSP_OK;
            };
            float ms = 0;
            if (best_ms >= 1e29) {  // the split was fixed: time it without groups first
                if ((rc = measure(GroupCand{0, 0}, &ms))) {
                    (void)hipEventDestroy(ev0);
                    (void)hipEventDestroy(ev1);
                    return fail(rc);
                }
                best_ms = ms;
            }
            // shapes with at most two sources per thread (4 per 1024-column slice, 2 per
            // 2048, 1..2 per 4096, 8 per 512 / 1024): the wider ones spill registers
            for (const GroupCand& g : {GroupCand{8, 1024}, GroupCand{4, 2048}, GroupCand{2, 4096}, GroupCand{16, 512}}) {
                if ((rc = measure(g, &ms))) {
                    (void)hipEventDestroy(ev0);
                    (void)hipEventDestroy(ev1);
                    return fail(rc);
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    gbest = g;
                }
            }
            (void)hipEventDestroy(ev0);
            (void)hipEventDestroy(ev1);
        }
    }
    if (gbest.cols % 4 || (gbest.k && (gbest.cols < 512 || gbest.cols > 4096)))
        return fail(err(SSSP_EINVAL, "group_columns %d: a multiple of 4 in [512, 4096]", gbest.cols));
    rc = p->upload(best.single_max_n, best.gang_columns, gbest.k, gbest.cols);
    if (rc) return fail(rc);
    p->info.group_sources = p->group_items ? gbest.k : 0;
    p->info.group_columns = p->group_items ? gbest.cols : 0;
    p->info.group_items = p->group_items;
    p->info.lc_instances = p->lc_items;
    p->info.threads = 1024;
    p->info.workgroups = p->nwg;
    p->info.single_max_n = best.single_max_n;
    p->info.gang_columns = best.gang_columns;
    p->info.tuned_ms = best_ms < 1e29 ? best_ms : -1.0;
    // capture the launch into a graph, replayed by sssp_batch_plan_launch
    e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = p->enqueue(p->cap);
        e = hipStreamEndCapture(p->cap, &p->graph);
        if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return fail(hip_err(e, "capturing the batched launch"));
    e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
    if (e != hipSuccess) return fail(hip_err(e, "hipEventCreate"));
    p->info.graph = 1;
    p->info.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = p;
    return SSSP_OK;
}

int sssp_batch_plan_launch(sssp_batch_plan* p, void* stream) {
    if (!p) return err(SSSP_EINVAL, "null plan");
    hipError_t e = hipGraphLaunch(p->exec, (hipStream_t)stream);
    if (e == hipSuccess) e = hipEventRecord(p->done, (hipStream_t)stream);
    if (e != hipSuccess) return hip_err(e, "hipGraphLaunch");
    return SSSP_OK;
}

int sssp_batch_plan_info(const sssp_batch_plan* p, sssp_plan_info* info) {
    if (!p || !info) return err(SSSP_EINVAL, "null argument");
    *info = p->info;
    return SSSP_OK;
}

int sssp_batch_plan_status(sssp_batch_plan* p, void* stream, int32_t* status, int64_t* stats) {
    if (!p || !status) return err(SSSP_EINVAL, "null argument");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    Ctl c;
    if (e == hipSuccess) e = hipMemcpy(&c, p->d_ctl, sizeof c, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_err(e, "reading plan status");
    *status = (int32_t)c.status;
    if (stats)
        for (int i = 0; i < kStatCount; ++i) stats[i] = (int64_t)c.last[i];
    return SSSP_OK;
}

int sssp_batch_plan_destroy(sssp_batch_plan* p) {
    if (!p) return SSSP_OK;
    if (p->done) {
        (void)hipEventSynchronize(p->done);  // the last launch of the plan has finished
        (void)hipEventDestroy(p->done);
    }
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    p->free_device();
    for (auto& c : p->copies) (void)hipFree(c.data);
    (void)hipFree(p->d_ctl);
    delete p;
    return SSSP_OK;
}

}  // extern "C"
