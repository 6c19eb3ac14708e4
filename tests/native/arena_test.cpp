// CPU test of the request server's output arena: random alloc / free
// sequences checked against a brute-force occupancy map of the byte range
// (no two live regions overlap, every region inside the range and 16-byte
// aligned) and against the ring's promise (an allocation that fails could
// not have been placed at the head or, after a wrap, at offset 0).
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <map>
#include <random>
#include <vector>

#include "lc_arena.h"

static int fail(const char* what, long a, long b)
{
    fprintf(stderr, "FAIL %s (%ld, %ld)\n", what, a, b);
    return 1;
}

int main()
{
    // fixed cases
    {
        lc::Arena a(100);  // rounds down to 96
        if (a.size() != 96) return fail("size", a.size(), 96);
        if (a.alloc(97) != lc::Arena::kNone) return fail("too big", 0, 0);
        uint64_t r0 = a.alloc(40), r1 = a.alloc(40);  // 48 + 48
        if (r0 != 0 || r1 != 48) return fail("first fit", r0, r1);
        if (a.alloc(1) != lc::Arena::kNone) return fail("full", 0, 0);
        if (!a.free(r1)) return fail("free r1", 0, 0);
        if (a.alloc(16) != lc::Arena::kNone) return fail("younger freed region still reserved", 0, 0);
        if (!a.free(r0)) return fail("free r0", 0, 0);
        if (a.live_bytes() != 0 || a.live_regions() != 0) return fail("empty", a.live_bytes(), a.live_regions());
        if (a.alloc(96) != 0) return fail("whole", 0, 0);
        if (a.free(5)) return fail("free unknown", 0, 0);
    }
    {
        lc::Arena a(160);
        uint64_t r0 = a.alloc(64), r1 = a.alloc(64);  // [0,64) [64,128)
        if (!a.free(r0)) return fail("free", 0, 0);
        uint64_t r2 = a.alloc(48);                     // no room at the end (32 left): wraps to 0
        if (r2 != 0) return fail("wrap", r2, 0);
        if (a.alloc(32) != lc::Arena::kNone) return fail("wrapped: only [48,64) free", 0, 0);
        uint64_t r3 = a.alloc(16);
        if (r3 != 48) return fail("wrapped fill", r3, 48);
        if (!a.free(r1)) return fail("free r1", 0, 0);  // run is now [0,64)
        uint64_t r4 = a.alloc(96);
        if (r4 != 64) return fail("after unwrap", r4, 64);
        (void)r3;
    }
    // random sequences against an occupancy map
    std::mt19937_64 rng(12345);
    for (int trial = 0; trial < 200; trial++) {
        const uint64_t size = 16 * (1 + rng() % 200);
        lc::Arena a(size);
        std::vector<int> owner(size / 16, -1);
        std::map<uint64_t, std::pair<uint64_t, int>> live;  // off -> (bytes rounded, id)
        std::vector<uint64_t> order;                         // live offsets in allocation order
        int next_id = 0;
        for (int step = 0; step < 3000; step++) {
            const bool do_alloc = live.empty() || rng() % 100 < 55;
            if (do_alloc) {
                const uint64_t want = rng() % (size / 3 + 1);
                const uint64_t off = a.alloc(want);
                const uint64_t x = want <= 16 ? 16 : (want + 15) / 16 * 16;
                if (off == lc::Arena::kNone) continue;
                if (off % 16 || off + x > size) return fail("bounds", off, x);
                for (uint64_t c = off / 16; c < (off + x) / 16; c++) {
                    if (owner[c] != -1) return fail("overlap", off, owner[c]);
                    owner[c] = next_id;
                }
                live[off] = {x, next_id++};
                order.push_back(off);
            } else {
                // free a random live region
                auto it = live.begin();
                std::advance(it, rng() % live.size());
                const uint64_t off = it->first;
                if (!a.free(off)) return fail("free live", off, 0);
                for (uint64_t c = off / 16; c < (off + it->second.first) / 16; c++) owner[c] = -1;
                live.erase(it);
            }
            uint64_t lb = 0;
            for (auto& kv : live) lb += kv.second.first;
            if (a.live_bytes() != lb) return fail("live bytes", a.live_bytes(), lb);
            if (a.live_regions() != live.size()) return fail("live regions", a.live_regions(), live.size());
        }
        // drain: everything freed returns the arena to empty
        for (auto& kv : live) a.free(kv.first);
        if (a.live_bytes() != 0 || a.alloc(size) != 0) return fail("drain", a.live_bytes(), 0);
    }
    printf("arena ok\n");
    return 0;
}
