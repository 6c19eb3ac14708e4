// CPU test of the fit kernels' one-round division (csrc/lc_arith.h):
// floor(x / d) and x mod d against integer division for x < 2^49 and
// d = 1 .. 4096, with 1 / d rounded and then pushed up to 4 ulps either way
// (a relative error near 2^-50, more than the kernels' refined reciprocal).
#include <math.h>
#include <stdint.h>
#include <stdio.h>

#include <random>

#include "lc_arith.h"

int main()
{
    std::mt19937_64 rng(3);
    long checks = 0;
    const uint64_t top = (1ull << 49) - 1;
    for (uint32_t d = 1; d <= 4096; d++) {
        double invs[9];
        double up = 1.0 / d, dn = 1.0 / d;
        invs[0] = up;
        for (int k = 1; k <= 4; k++) {
            up = nextafter(up, 2.0);
            dn = nextafter(dn, 0.0);
            invs[2 * k - 1] = up;
            invs[2 * k] = dn;
        }
        for (int t = 0; t < 400; t++) {
            uint64_t x;
            switch (t % 8) {
            case 0: x = top - rng() % 5000; break;                               // the top of the range
            case 1: x = (top / d - rng() % 1000) * d; break;                    // multiples of d
            case 2: x = (top / d - rng() % 1000) * d + d - 1; break;            // one below a multiple
            case 3: x = rng() % 100000; break;                                  // small
            default: x = rng() & top; break;
            }
            for (double inv : invs) {
                uint32_t rem = 0;
                const uint64_t q = lc::div_fast(x, d, inv, &rem);
                if (q != x / d || rem != x % d) {
                    printf("FAIL x=%llu d=%u inv=%.20g q=%llu rem=%u\n", (unsigned long long)x, d, inv,
                           (unsigned long long)q, rem);
                    return 1;
                }
                checks++;
            }
        }
    }
    printf("div ok (%ld checks)\n", checks);
    return 0;
}
