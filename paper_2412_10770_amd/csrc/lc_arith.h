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
// within a relative 2^-50 of 1 / d.  Both conversions go through the
// mantissa of 2^52 + v, which holds any integer v < 2^52 exactly: x as a
// double is (2^52 | x) - 2^52, and fma(x, inv, 2^52) rounds x * inv to the
// nearest integer in the mantissa.  x * inv is within 2^49 * 2^-50 = 1/2 of
// x / d, so that integer is the floor or one above; one correction from the
// remainder (either way) makes it exact.
LC_ARITH_HD uint64_t div_fast(uint64_t x, uint32_t d, double inv, uint32_t* rem = nullptr)
{
    const double two52 = 4503599627370496.0;
    const uint64_t mant = 0x4330000000000000ull;  // the bits of 2^52
    const uint64_t xb = mant | x;
    double xf;
    __builtin_memcpy(&xf, &xb, 8);
    xf -= two52;  // exact
    const double qf = __builtin_fma(xf, inv, two52);
    uint64_t qb;
    __builtin_memcpy(&qb, &qf, 8);
    const uint64_t q0 = qb - mant;
    const int64_t r0 = (int64_t)(x - q0 * d);
    const int64_t c = (r0 >= (int64_t)d) - (r0 < 0);
    if (rem) *rem = (uint32_t)(r0 - c * (int64_t)d);
    return q0 + c;
}

}  // namespace lc
