// Exact integer helpers shared by the search kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace trs {

// floor(s1^2 / n) for 0 <= s1 < 2^38 and 1 <= n < 2^27.  The quotient is at most the
// region's sum of squares (< 2^50), so a double estimate is within one unit; the exact
// remainder in wrapping 64-bit arithmetic corrects it.
__device__ __forceinline__ unsigned long long floor_sq_div(unsigned long long s1, unsigned n)
{
    const double d = (double)s1;
    unsigned long long q = (unsigned long long)((d * d) / (double)n);
    long long rem = (long long)(s1 * s1 - q * (unsigned long long)n);
    while (rem < 0) { q--; rem += n; }
    while (rem >= (long long)n) { q++; rem -= n; }
    return q;
}

}  // namespace trs
