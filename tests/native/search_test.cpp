// CPU test of the point queries' searches (csrc/lc_search.h): find_segment
// against a linear scan over random sorted segment starts, and gallop_last
// from arbitrary guesses over non-decreasing arrays with repeats (the anchor
// search of lower_bound).
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <random>
#include <vector>

#include "lc_search.h"

int main()
{
    std::mt19937_64 rng(2);
    long checks = 0;
    for (int trial = 0; trial < 100000; trial++) {
        const uint32_t nkeys = 1 + rng() % 4096;
        const uint32_t nseg = 1 + rng() % nkeys;
        std::vector<uint16_t> st(nseg);
        st[0] = 0;
        std::vector<uint32_t> pos;
        for (uint32_t p = 1; p < nkeys; p++) pos.push_back(p);
        std::shuffle(pos.begin(), pos.end(), rng);
        std::vector<uint32_t> sel(pos.begin(), pos.begin() + (nseg - 1));
        std::sort(sel.begin(), sel.end());
        for (uint32_t t = 1; t < nseg; t++) st[t] = (uint16_t)sel[t - 1];
        for (int q = 0; q < 4; q++) {
            const uint32_t j = rng() % nkeys;
            uint32_t want = 0;
            for (uint32_t t = 0; t < nseg; t++)
                if (st[t] <= j) want = t;
            if (lc::find_segment(st.data(), nseg, nkeys, j) != want) {
                fprintf(stderr, "FAIL find_segment nkeys=%u nseg=%u j=%u\n", nkeys, nseg, j);
                return 1;
            }
            checks++;
        }
        std::vector<uint64_t> an(nseg);
        an[0] = 0;
        for (uint32_t t = 1; t < nseg; t++) an[t] = an[t - 1] + (rng() % 4 == 0 ? 0 : rng() % 1000);
        for (int q = 0; q < 4; q++) {
            const uint64_t y = 1 + rng() % (an[nseg - 1] + 2);
            uint32_t want = 0;
            for (uint32_t t = 0; t < nseg; t++)
                if (an[t] < y) want = t;
            const uint32_t guess = (uint32_t)(rng() % (nseg + 3));
            if (lc::gallop_last(nseg, guess, [&](uint32_t u) { return an[u] < y; }) != want) {
                fprintf(stderr, "FAIL gallop_last n=%u guess=%u\n", nseg, guess);
                return 1;
            }
            checks++;
        }
    }
    printf("search ok (%ld checks)\n", checks);
    return 0;
}
