// Searches shared by the point-query kernels and their host-side test:
// last index of a prefix-true predicate, started from a guess.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define LC_HD __host__ __device__ __forceinline__
#else
#define LC_HD inline
#endif

namespace lc {

// Last t in [0, n) with pred(t), for a predicate that holds on a prefix of
// [0, n) including 0: probe the guess, gallop to a bracket [lo, hi) with
// pred(lo) and !pred(hi) (hi = n standing for past the end), then halve it.
// With a good guess a handful of probes fall in one or two cache lines
// instead of log2(n) dependent ones.
template <typename Pred>
LC_HD uint32_t gallop_last(uint32_t n, uint32_t guess, Pred pred)
{
    if (n <= 1) return 0;
    uint32_t t = guess < n ? guess : n - 1;
    uint32_t lo, hi;
    if (pred(t)) {
        lo = t;
        hi = n;
        for (uint32_t step = 1; lo + step < n; step <<= 1) {
            if (pred(lo + step)) {
                lo += step;
            } else {
                hi = lo + step;
                break;
            }
        }
    } else {
        hi = t;
        lo = 0;
        for (uint32_t step = 1; step <= hi; step <<= 1) {
            if (pred(hi - step)) {
                lo = hi - step;
                break;
            }
            hi -= step;
            if (step > hi) break;
        }
    }
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pred(mid)) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Last t with start[t] <= j (start[0] = 0 <= j), from the proportional guess
// j * nseg / nkeys: segments of a block are usually of similar length.
LC_HD uint32_t find_segment(const uint16_t* st, uint32_t nseg, uint32_t nkeys, uint32_t j)
{
    return gallop_last(nseg, (uint32_t)(((uint64_t)j * nseg) / nkeys), [&](uint32_t t) { return st[t] <= j; });
}

}  // namespace lc
