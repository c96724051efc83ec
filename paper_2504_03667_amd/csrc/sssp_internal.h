// Declarations shared between the kernels (kernels.hip) and the C ABI (api.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sssp.h"

namespace sssp {

struct Ctl;
struct Pub;
struct Bar;

// internal flag bits, above the public SSSP_FLAG_* bits
constexpr uint32_t kFlagLiteral = SSSP_FLAG_LITERAL;
constexpr uint32_t kFlagVec = 1u << 16;  // rows are 16-byte aligned: 128-bit loads

struct SolveArgs {
    const int32_t* W;
    int64_t ld;
    int32_t n;
    int32_t src;
    int32_t* dist;
    int32_t* pred;
    uint32_t flags;
    Ctl* ctl;
};

hipError_t launch_single(const SolveArgs& a, int threads, hipStream_t s);
int max_single_n();

// plain: ordinary launch of the same kernel, the grid already bounded by the
// occupancy query (co-resident on an otherwise idle GPU), instead of a
// cooperative launch; used for profiler runs.
// words: grid_words_bytes(nwg, S) bytes of exchange memory.  balance: pair
// balancing of large rounds (see solve_gang).
hipError_t launch_grid(const SolveArgs& a, int nwg, int S, long long timeout, char* words, bool plain, bool balance,
                       hipStream_t s);
int max_grid_slice();
int grid_occupancy(int slice, int* per_cu);
// Graphs from which the whole-GPU kernel balances large rounds within pairs
// of workgroups by default (rounds of at least 8 Ki rows become likely).
constexpr int32_t kGridBalanceMinN = 32768;

// Label-correcting solve on a cooperative grid of nwg workgroups (slices of S
// columns); words: gang_words_bytes(nwg, S) bytes of exchange memory.
hipError_t launch_lc(const SolveArgs& a, int nwg, int S, long long timeout, char* words, bool plain,
                     hipStream_t s);

// Zeroes `bytes` (a multiple of 4) of device memory with a kernel on stream s.
hipError_t zero_fill(void* p, size_t bytes, hipStream_t s);
int lc_occupancy(int slice, int* per_cu);

// One instance of a batched launch or one served query, as the kernels read it.
struct BatchItem {
    const void* W;       // int32_t, uint16_t or uint8_t entries (elem bytes each)
    int64_t ld;          // row stride in entries
    int32_t* dist;
    int32_t* pred;
    int32_t n;
    int32_t src;
    int32_t elem;        // 4: the caller's int32 matrix; 2 / 1: an exact compact copy
    int32_t vec;         // rows aligned for whole-group loads
    int32_t parts;       // workgroups that solve it (1: one workgroup alone; > 1: a gang)
    int32_t S;           // columns per gang member
    int32_t method;      // kMethodDijkstra, kMethodLabelCorrecting or kMethodGroup
    int32_t K;           // kMethodGroup: sources of the group (src, dist, pred above unused)
    unsigned long long scratch_off;  // byte offset of a gang's records and lists in the arena
    const void* group;   // kMethodGroup: device array of K MultiSrc (multi.h)
};

// BatchItem::method.  Label-correcting items always run as a gang (possibly of
// one) with exchange records and 64-bit lists in the arena.
constexpr int32_t kMethodDijkstra = 0;
constexpr int32_t kMethodLabelCorrecting = 1;
// Several sources of one matrix solved in lockstep by a gang (multi.h); only for
// matrices whose off-diagonal weights are all >= 1.
constexpr int32_t kMethodGroup = 2;

// Exchange memory of a gang of nwg workgroups with slices of S columns, one
// block: 2 * nwg stamped records (Pub, 32 bytes), the tagged records (32 bytes
// per member and slot, see rec_word), the pair words (16 bytes per member: two
// chunk-claim counters and a tagged "done" word, see solve_gang), then
// 2 * nwg * S 64-bit list words (tagged bucket entries of the Dijkstra rounds,
// or the label-correcting frontier).  Records and lists are double-buffered by
// exchange parity.  The whole-GPU layout (grid_words) adds nwg * S 64-bit
// partial keys (a pair partner's share of a member's columns).
constexpr size_t kPubBytes = 32;
constexpr size_t kTRecBytes = 32;
constexpr size_t kPairBytes = 16;
__host__ __device__ constexpr size_t gang_recs_offset(int nwg) { return 2 * (size_t)nwg * kPubBytes; }
__host__ __device__ constexpr size_t gang_pair_offset(int nwg) {
    return gang_recs_offset(nwg) + 2 * (size_t)nwg * kTRecBytes;
}
__host__ __device__ constexpr size_t gang_lists_offset(int nwg) {
    return gang_pair_offset(nwg) + (size_t)nwg * kPairBytes;
}
__host__ __device__ constexpr size_t gang_part_offset(int nwg, int S) {
    return gang_lists_offset(nwg) + 2 * (size_t)nwg * (size_t)S * sizeof(uint64_t);
}
__host__ __device__ constexpr size_t gang_words_bytes(int nwg, int S) { return gang_part_offset(nwg, S); }

struct GangWords {
    Pub* pubs;
    uint64_t* recs;
    uint32_t* ctr;    // member g: ctr[4 g + slot], slot 0 or 1
    uint64_t* done;   // member g: done[2 g] (the odd words are unused)
    uint64_t* lists;
    uint64_t* part;   // member g: part[g S + local column] (whole-GPU layout only, else null)
};
__host__ __device__ inline GangWords gang_words(char* base, int nwg, int S) {
    return GangWords{reinterpret_cast<Pub*>(base), reinterpret_cast<uint64_t*>(base + gang_recs_offset(nwg)),
                     reinterpret_cast<uint32_t*>(base + gang_pair_offset(nwg)),
                     reinterpret_cast<uint64_t*>(base + gang_pair_offset(nwg)) + 1,
                     reinterpret_cast<uint64_t*>(base + gang_lists_offset(nwg)), nullptr};
}

// The whole-GPU kernels' exchange memory (per-stream scratch, reused by
// launches of every width): the stamped records always take the first
// kGridPubBytes (room for 1024 members), so that stamps sit at the same
// addresses in every use and no other word (the partial keys of pair
// balancing can have bit 63 set) is ever left where a later launch polls a
// stamp.  The rest follows as in gang_words.
constexpr size_t kGridPubBytes = 2 * 1024 * kPubBytes;
__host__ __device__ constexpr size_t grid_words_bytes(int nwg, int S) {
    return kGridPubBytes + gang_words_bytes(nwg, S) - gang_recs_offset(nwg) +
           (size_t)nwg * (size_t)S * sizeof(uint64_t);
}
__host__ __device__ inline GangWords grid_words(char* base, int nwg, int S) {
    char* rest = base + kGridPubBytes - gang_recs_offset(nwg);  // the gang layout past its stamped records
    GangWords gw = gang_words(rest, nwg, S);
    gw.pubs = reinterpret_cast<Pub*>(base);
    gw.part = reinterpret_cast<uint64_t*>(rest + gang_part_offset(nwg, S));
    return gw;
}

// Arena bytes of an item's exchange memory (0 for a Dijkstra item solved by
// one workgroup).
inline unsigned long long item_scratch_bytes(int32_t method, int32_t parts, int32_t S) {
    if (method == kMethodDijkstra && parts <= 1) return 0;
    return ((unsigned long long)gang_words_bytes(parts, S) + 255) & ~255ull;
}

// Ticket t of a batched launch is part parts[t].part of item parts[t].item;
// the parts of one item are consecutive.
struct BatchPart {
    int32_t item;
    int32_t part;
};

hipError_t launch_batch(const BatchItem* items, const BatchPart* parts, int32_t nparts, Bar* bars, char* arena,
                        uint32_t flags, long long timeout, Ctl* ctl, int nwg, hipStream_t s);
int batch_occupancy(int* per_cu);
int max_batch_single_n();
int max_batch_slice();

// Exact compact copy of a matrix (see make_compact).
struct CompactCopy {
    void* data = nullptr;  // null when the weights do not fit a narrower type
    int64_t ld = 0;        // row stride in entries
    int elem = 4;          // 1, 2, or 4 (no copy)
    int32_t wmin = 0, wmax = 0;
    int32_t woff = 0;      // smallest off-diagonal entry
};
int make_compact(const int32_t* W, int64_t ld, int32_t n, hipStream_t s, CompactCopy* out);
// Weight range of a matrix (synchronous): min over all entries, max over finite
// ones, min over off-diagonal ones.
int matrix_range(const int32_t* W, int64_t ld, int32_t n, hipStream_t s, int32_t* wmin, int32_t* wmax, int32_t* woff);

// Exact compact copies (int32 -> uint16 / uint8) and weight ranges.
// d_out3 (device, 3 int32): min over all entries, max over finite entries, min
// over off-diagonal entries; initialised by the caller to {INT32_MAX, INT32_MIN, INT32_MAX}.
hipError_t weight_range(const int32_t* W, int64_t ld, int32_t n, int32_t* d_out3, hipStream_t s);
hipError_t compact_copy(const int32_t* W, int64_t ld, int32_t n, void* C, int64_t ldc, int elem, hipStream_t s);

size_t ctl_size();

// Per-device counters of the read-ceiling kernel (diag.hip): freed (after a
// device synchronisation) by sssp_release_all; their device bytes.
int release_read_counters();
int64_t read_counter_bytes();

}  // namespace sssp

// ---------------------------------------------------------------------------
// Serving: structures shared by the persistent kernel and the host server.
// ---------------------------------------------------------------------------
namespace sssp {

// Host-written control words, in fine-grained (coherent) pinned host memory.
struct ServeControl {
    unsigned long long tail;  // ring entries published so far
    unsigned long long pad0[15];
    unsigned long long heartbeat;  // bumped by the host server thread while it lives
    unsigned long long pad1[15];
    uint32_t stop;  // set once: workgroups leave when they find no work
    uint32_t park;  // set while the host has nothing in flight: idle workgroups leave
    uint32_t pad2[30];
};

// One part of a query: rank `part` of a gang of `parts` workgroups (parts == 1:
// the query is solved by one workgroup alone).  Written by the host into the
// ring (pinned host memory) before `tail` is advanced past it.
struct ServeDesc {
    BatchItem item;
    int32_t part;
    uint32_t qslot;  // in-flight query slot (device state, completion record)
    unsigned long long ticket;
};

// Completion record of a query slot, written by the GPU into pinned host memory.
struct ServeDone {
    unsigned long long ticket;  // ticket of the query that completed in this slot
    uint32_t status;
    uint32_t rounds;
    unsigned long long settled;
    long long t_done;  // device wall clock at completion
    unsigned long long pad[4];
};

// Per-slot device state of an in-flight query.
struct ServeSlot {
    uint32_t done_parts;  // gang members finished
    uint32_t status;      // status bits OR-ed by the members
    uint32_t pad[30];
};

struct ServeArgs {
    ServeControl* ctl;         // pinned
    const ServeDesc* ring;     // pinned
    int32_t ring_slots;
    ServeDone* done;           // pinned, one per query slot
    ServeSlot* slots;          // device, one per query slot
    Bar* bars;                 // device, one per query slot
    unsigned long long* head;  // device: ring entries claimed so far
    char* arena;               // device scratch for gang records and lists
    long long timeout;         // gang barrier wait limit (wall-clock ticks)
    long long watchdog;        // leave when the heartbeat stalls this long (ticks)
};

hipError_t launch_serve(const ServeArgs& a, int nwg, hipStream_t s);
int serve_occupancy(int* per_cu);
int max_serve_single_n();
int max_serve_slice();
size_t bar_size();

}  // namespace sssp
