// Host-only check of the exchange-record encoding (built and run by
// tests/test_encoding.py; no kernel is launched).  A gang member waits for
// exchange_stamp(epoch, b) in each member's record.  Record memory is reused
// by later queries and launches without being cleared, so no word that any
// use of that memory stores may equal a stamp: this program checks, over the
// boundary values and random samples of every field, that stamps have bit 63
// set while list entries, tagged words and records' other words at stamp
// offsets do not, and that tagged words carry their tag.  The partial keys of
// pair balancing can have bit 63 set (a negative weight); they are written only
// into the whole-GPU kernels' memory, whose stamp region is fixed (grid_words),
// so they never sit where a later launch polls a stamp.
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <random>

#include "engine.h"
#include "lc.h"
#include "multi.h"
#include "sssp_internal.h"

using namespace sssp;

static int failures = 0;
#define CHECK(c)                                                    \
    do {                                                            \
        if (!(c)) {                                                 \
            std::fprintf(stderr, "FAILED line %d: %s\n", __LINE__, #c); \
            ++failures;                                             \
        }                                                           \
    } while (0)

int main() {
    std::mt19937_64 rng(2504036670ull);
    const uint32_t epochs[] = {0u, 1u, 2u, 3u, 0x7ffffffeu, 0x7fffffffu, 0x80000000u, 0xffffffffu};
    const uint32_t bars[] = {0u, 1u, 2u, 3u, 1000u, 0x7fffffffu, 0xffffffffu};
    for (uint32_t e : epochs)
        for (uint32_t b : bars) {
            const uint64_t s = exchange_stamp(e, b);
            CHECK(s >> 63 == 1u);
            CHECK((uint32_t)s == b);
        }
    // distinct (epoch mod 2^31, b) give distinct stamps
    CHECK(exchange_stamp(5, 1) != exchange_stamp(6, 1));
    CHECK(exchange_stamp(5, 1) != exchange_stamp(5, 2));
    for (int i = 0; i < 1000000; ++i) {
        const uint32_t e = (uint32_t)rng(), b = (uint32_t)rng();
        CHECK(exchange_stamp(e, b) >> 63 == 1u);
        // label-correcting frontier entries: dist below INT32_MAX, vertex below 2^31
        const uint32_t d = (uint32_t)(rng() % kInf), v = (uint32_t)(rng() & 0x7fffffffu);
        CHECK(lc_entry(d, v) >> 63 == 0u);
        // two int32 bucket-list entries (vertex indices) read as one 64-bit word
        const uint64_t pair = ((uint64_t)(uint32_t)(rng() & 0x7fffffffu) << 32) | (uint32_t)(rng() & 0x7fffffffu);
        CHECK(pair >> 63 == 0u);
        // record keys (dist << 32 | vertex, dist up to INT32_MAX) outside their own slot
        CHECK(make_key(d, v) >> 63 == 0u);
        if (failures > 10) break;
    }
    CHECK(lc_entry(kInf - 1, 0x7fffffffu) >> 63 == 0u);
    CHECK(make_key(kInf, 0x7fffffffu) >> 63 == 0u);
    // the record layout the argument relies on: 32-byte records with the stamp first
    // and the (possibly all-ones) key 8 bytes in
    CHECK(sizeof(Pub) == 32 && alignof(Pub) == 32);
    CHECK(offsetof(Pub, stamp) == 0);
    CHECK(offsetof(Pub, key) == 8);
    // tagged words (tag_word): the tag of exchange b is b, at most 2n + 1 < 2^31 for any
    // matrix that fits in memory, so tagged words never have bit 63 either; a cleared
    // word (0) carries tag 0, which no exchange uses (b >= 1)
    CHECK(kRecFields * sizeof(uint64_t) == kTRecBytes);
    CHECK(word_tag(0) == 0u);
    for (int i = 0; i < 1000000; ++i) {
        const uint32_t tag = 1u + (uint32_t)(rng() % 0x7fffffffu), v = (uint32_t)rng();
        const uint64_t w = tag_word(tag, v);
        CHECK(w >> 63 == 0u);
        CHECK(word_tag(w) == tag && (uint32_t)w == v);
        CHECK(w != exchange_stamp((uint32_t)rng(), (uint32_t)rng()));
        if (failures > 10) break;
    }
    // a gang's exchange memory: stamped records, tagged records and lists, each region
    // at a 32-byte offset, so every use places its stamps at 32-byte offsets; arena
    // regions of batched items and served queries are multiples of 256 bytes
    for (int i = 0; i < 100000; ++i) {
        const int32_t method = (int32_t)(rng() % 3), parts = 1 + (int32_t)(rng() % 1024),
                      S = 4 * (1 + (int32_t)(rng() % 4096));
        CHECK(gang_recs_offset(parts) % 32 == 0 && gang_lists_offset(parts) % 8 == 0);
        CHECK(gang_recs_offset(parts) == 2 * (size_t)parts * sizeof(Pub));
        CHECK(gang_pair_offset(parts) == gang_recs_offset(parts) + 2 * (size_t)parts * kTRecBytes);
        CHECK(gang_lists_offset(parts) == gang_pair_offset(parts) + (size_t)parts * kPairBytes);
        CHECK(gang_pair_offset(parts) % 16 == 0 && gang_part_offset(parts, S) % 8 == 0);
        // whole-GPU layout: stamps at fixed addresses below kGridPubBytes, nothing else there
        const GangWords gg = grid_words(nullptr, parts, S);
        CHECK((char*)gg.pubs == nullptr && (size_t)((char*)gg.recs - (char*)nullptr) == kGridPubBytes);
        CHECK(grid_words_bytes(parts, S) ==
              kGridPubBytes + gang_words_bytes(parts, S) - gang_recs_offset(parts) + 8 * (size_t)parts * (size_t)S);
        CHECK((size_t)((char*)gg.lists - (char*)nullptr) + 16 * (size_t)parts * (size_t)S ==
              (size_t)((char*)gg.part - (char*)nullptr));
        CHECK((size_t)((char*)&gg.part[(size_t)parts * S - 1] - (char*)nullptr) + 8 == grid_words_bytes(parts, S));
        // the tagged words of every (slot, field, member) lie inside the tagged-record region
        uint64_t* recs = reinterpret_cast<uint64_t*>(gang_recs_offset(parts));
        const size_t last = (size_t)(rec_word(recs, parts, 1, kRecFields - 1, parts - 1) - recs);
        CHECK(last == 2 * (size_t)parts * kRecFields - 1);
        CHECK(gang_part_offset(parts, S) == gang_lists_offset(parts) + 16 * (size_t)parts * (size_t)S);
        CHECK(gang_words_bytes(parts, S) == gang_part_offset(parts, S));
        // the pair words: member g's two counters and its done word inside its 16 bytes
        char* base = nullptr;
        const GangWords gw = gang_words(base, parts, S);
        const size_t g = (size_t)(parts - 1);
        CHECK((size_t)((char*)&gw.ctr[4 * g + 1] - base) + 4 <= gang_pair_offset(parts) + 16 * g + 8);
        CHECK((size_t)((char*)&gw.done[2 * g] - base) == gang_pair_offset(parts) + 16 * g + 8);
        CHECK(gw.part == nullptr);
        if (method != kMethodGroup) {
            const unsigned long long bytes = item_scratch_bytes(method, parts, S);
            CHECK(bytes % 256 == 0);
            CHECK(bytes >= (method == kMethodDijkstra && parts <= 1 ? 0 : gang_words_bytes(parts, S)));
        }
        if (failures > 10) break;
    }
    // lockstep-group records: whole 32-byte multiples, every word but the stamp
    // below 2^63 (keys at most kRecNone, counts and lengths below 2^31), list
    // entries (column << 16 | mask) with the column below 4096, and arena regions
    // of 256-byte multiples
    CHECK(kRecNone >> 63 == 0u);
    for (int K = 1; K <= kMultiMax; ++K) {
        CHECK(multi_rec_words(K) % 4 == 0);
        CHECK(multi_rec_words(K) >= 2 + K + (K + 1) / 2);
        for (int parts = 1; parts <= 32; ++parts)
            for (int S = 512; S <= 4096; S += 4) CHECK(multi_scratch_bytes(K, parts, S) % 256 == 0);
    }
    for (int i = 0; i < 100000; ++i) {
        const uint32_t col = (uint32_t)(rng() % 4096), mask = (uint32_t)(rng() & 0xffffu);
        const uint32_t e1 = (col << 16) | mask, e2 = ((uint32_t)(rng() % 4096) << 16) | (uint32_t)(rng() & 0xffffu);
        CHECK((((uint64_t)e1 << 32) | e2) >> 63 == 0u);
        const uint64_t key = make_key((uint32_t)(rng() % kInf), (uint32_t)(rng() & 0x7fffffffu));
        CHECK(key >> 63 == 0u && key < kRecNone);
        if (failures > 10) break;
    }
    if (failures) return 1;
    std::printf("stamp encoding ok\n");
    return 0;
}
