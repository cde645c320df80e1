// Small device helpers: wavefront reductions and error-free transformations.
#pragma once

#include <hip/hip_runtime.h>

namespace dfjk {

// Sum over the 64 lanes of a wavefront (butterfly; every lane gets the sum).
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Knuth's TwoSum: s + e == a + b exactly (round-to-nearest, no overflow).
__device__ inline void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// TwoProduct via fused multiply-add: p + e == a * b exactly.
__device__ inline void two_prod(float a, float b, float& p, float& e) {
    p = a * b;
    e = __builtin_fmaf(a, b, -p);
}

// One step of the compensated dot product "Dot2" of Ogita, Rump and Oishi
// (SIAM J. Sci. Comput. 26(6), 2005): (s, c) accumulates x*y with the
// rounding errors of the products and sums collected in c.
__device__ inline void dot2_step(float x, float y, float& s, float& c) {
    float p, ep, t, es;
    two_prod(x, y, p, ep);
    two_sum(s, p, t, es);
    s = t;
    c += es + ep;
}

// Narrow FP64 to FP32 rounding to odd: a later round-to-nearest-even step to a
// format with at least two fewer significand bits then equals one correct
// rounding from FP64 (Boldo & Melquiond, IEEE Trans. Computers 57(4), 2008).
__device__ inline float to_float_round_odd(double x) {
    float f = (float)x;  // round to nearest even
    if ((double)f != x && x == x) {
        uint32_t u = __float_as_uint(f);
        if (fabs((double)f) > fabs(x)) u -= 1;  // step back toward zero (also inf -> max finite)
        u |= 1u;
        f = __uint_as_float(u);
    }
    return f;
}

// FP32 -> bfloat16 bits, round to nearest even (NaN kept quiet).
__device__ inline uint16_t float_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

}  // namespace dfjk
