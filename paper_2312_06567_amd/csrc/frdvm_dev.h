// Device helpers shared by the HIP sources (included by .hip files only).
#pragma once

#include <hip/hip_runtime.h>

namespace frdvm {

// exp of an exponent held in FP64, rounded once to FP32.  E = (n + r) ln 2
// with n integer and |r| <= 1/2, reduced in FP64; 2^r = e^t, t = r ln 2
// (|t| <= 0.347), by its Taylor series to degree 8 in FP64 (error below
// 3e-10 relative), scaled by 2^n and rounded to FP32: within half an FP32
// ulp plus 3e-10, with no systematic sign.  (An FP32 exponent of a few units
// would bias every equilibrium value of a point by ~1e-7; the hardware FP32
// exp2, accurate to 1 ulp but not correctly rounded, still leaves a bias
// that shows as a mass drift of the collision over many steps.)
// a * b + c in FP64 as one three-operand instruction (all operands in VGPRs)
__device__ __forceinline__ double fma3(double a, double b, double c) {
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

__device__ __forceinline__ float exp_to_f32(double E) {
    const double e2 = E * 1.4426950408889634074;  // log2(e)
    const double n = rint(e2);
    const double t = (e2 - n) * 0.69314718055994530942;  // ln(2)
    // Horner on 1/k!, k = 8 .. 0.  The three-operand FMA is spelled out:
    // left to itself the compiler takes the accumulating two-operand form,
    // which first copies each (loop-invariant) coefficient into the result
    // register.
    double p = 1.0 / 40320.0;
    p = fma3(p, t, 1.0 / 5040.0);
    p = fma3(p, t, 1.0 / 720.0);
    p = fma3(p, t, 1.0 / 120.0);
    p = fma3(p, t, 1.0 / 24.0);
    p = fma3(p, t, 1.0 / 6.0);
    p = fma(p, t, 0.5);
    p = fma(p, t, 1.0);
    p = fma(p, t, 1.0);
    return (float)ldexp(p, (int)n);
}

// Stochastic rounding of the FP32 state.  A value computed in FP64 is stored
// in FP32 rounded up or down with probabilities that make the rounding
// unbiased: r (32 random bits) shifted to the 29 mantissa bits that the
// conversion drops is added to the magnitude and those bits are cut, so the
// stored magnitude is the next one up with probability equal to the dropped
// fraction.  Round to nearest instead leaves a rounding error that repeats
// from stage to stage on a smooth, slowly changing state and accumulates in
// the conserved moments.  (Values below the FP32 normal range are rounded
// once more by the conversion.)
__device__ __forceinline__ float round_stochastic(double x, uint32_t r) {
    unsigned long long b = (unsigned long long)__double_as_longlong(x);
    b += (unsigned long long)(r >> 3);
    b &= ~((1ull << 29) - 1ull);
    return (float)__longlong_as_double((long long)b);
}

// 32-bit integer hash "lowbias32" (C. Wellons' hash-prospector search: two
// multiply-xorshift rounds); the random bits of the stochastic rounding of
// state value k of solution point pt in a stage with seed `seed`.
__device__ __forceinline__ uint32_t hash_lowbias32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
__device__ __forceinline__ uint32_t round_bits(uint32_t seed, uint32_t pt, uint32_t k) {
    return hash_lowbias32(seed ^ hash_lowbias32(pt * 0x01000193u ^ k));
}

}  // namespace frdvm
