// Integer arithmetic shared by the fit kernels and its host-side test.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define LC_ARITH_HD __host__ __device__ __forceinline__
#else
#define LC_ARITH_HD inline
#endif

namespace lc {

// floor(x / d) (and x mod d) for x < 2^49 and 1 <= d <= 4096, given inv
// within a relative 2^-50 of 1 / d.  The FP64 product x * inv is then within
// 2^49 (2^-50 + 2^-53) < 1 of x / d, so its truncation is within 1 of the
// floor and one correction from the remainder makes it exact.
LC_ARITH_HD uint64_t div_fast(uint64_t x, uint32_t d, double inv, uint32_t* rem = nullptr)
{
    const uint64_t q0 = (uint64_t)((double)x * inv);
    const int64_t r0 = (int64_t)(x - q0 * d);
    const int64_t c = (r0 >= (int64_t)d) - (r0 < 0);
    if (rem) *rem = (uint32_t)(r0 - c * (int64_t)d);
    return q0 + c;
}

}  // namespace lc
