// Per-pixel accumulation of path radiances in fixed point.
//
// A pixel's value is the mean radiance of its paths over the launch's sample range.  The
// persistent kernels finish paths in no fixed order, so a floating-point sum would depend on
// scheduling.  Each path's radiance L is instead rounded to the integer v = round(L 2^32)
// (L in [0, 2^24), so v < 2^56) and added to the pixel's two 64-bit words: the low 32 bits of
// v to word 0, the high bits to word 1 (the persistent kernels gather a wave's paths of a pixel
// in LDS first, gpss_sched.hpp).  Integer additions commute, so the sum is exact and
// independent of the order; 2^31 additions of either part cannot overflow its word.  The
// mean is then (word1 2^32 + word0) 2^-32 / samples, formed in double and rounded once to
// float.  Every form of the tracer (persistent, batch, wavefront, one thread per path) forms
// its image this way, so their images are identical.
//
// A radiance that is not a finite number in [0, 2^24) is not a valid path estimate of this
// method (every factor is non-negative): it adds 0 (NaN, infinite or negative) or 2^24
// (saturated), and is counted by the caller's event counters.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gpss {

constexpr double kAccScale = 4294967296.0;      // 2^32
constexpr float kAccMax = 16777216.0f;          // 2^24

enum AccClass : int { kAccOk = 0, kAccNonFinite = 1, kAccSaturated = 2 };

__device__ __forceinline__ int acc_class(float L) {
    if (!(L >= 0.0f) || isinf(L)) return kAccNonFinite;   // NaN, -inf, +inf, negative
    return L < kAccMax ? kAccOk : kAccSaturated;
}

__device__ __forceinline__ uint64_t acc_fixed(float L) {
    const int c = acc_class(L);
    if (c == kAccNonFinite) return 0ull;
    const float v = c == kAccSaturated ? kAccMax : L;
    return (uint64_t)__double2ull_rn((double)v * kAccScale);
}

// Mean of `ns` samples from the two words.
__device__ __forceinline__ float acc_mean(unsigned long long lo, unsigned long long hi, uint32_t ns) {
    const double sum = ((double)hi * kAccScale + (double)lo) * (1.0 / kAccScale);
    return (float)(sum / (double)ns);
}

}  // namespace gpss
