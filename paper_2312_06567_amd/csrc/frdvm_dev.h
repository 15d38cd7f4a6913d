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
    // (an exponent of -inf, a point without an equilibrium, gives 0 and not
    // the NaN of its reduction)
    const double e2 = fmax(E, -2000.0) * 1.4426950408889634074;  // log2(e)
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

// a * b + c in FP64 with c a wave-uniform constant (one scalar register pair
// operand): the coefficients of a polynomial then need no vector registers
__device__ __forceinline__ double fma3s(double a, double b, double c) {
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
    return d;
}

// exp of an exponent held in FP64, in FP64 to a few ulp: E = n ln 2 + t with
// n = rint(E log2 e), t = E - n ln 2 reduced with ln 2 split into its nearest
// double and the remainder (|t| <= 0.347), e^t by its Taylor series to degree
// 12 (truncation below 2e-16 relative), scaled by 2^n (0 below the FP64
// range).
__device__ __forceinline__ double exp_f64(double E) {
    E = fmax(E, -2000.0);  // -inf (no equilibrium) gives 0
    const double n = rint(E * 1.4426950408889634074);
    double t = fma(-n, 0.6931471805599453, E);
    t = fma(-n, 2.3190468138462996e-17, t);
    double p = 1.0 / 479001600.0;  // 1/12!
    p = fma3s(p, t, 1.0 / 39916800.0);
    p = fma3s(p, t, 1.0 / 3628800.0);
    p = fma3s(p, t, 1.0 / 362880.0);
    p = fma3s(p, t, 1.0 / 40320.0);
    p = fma3s(p, t, 1.0 / 5040.0);
    p = fma3s(p, t, 1.0 / 720.0);
    p = fma3s(p, t, 1.0 / 120.0);
    p = fma3s(p, t, 1.0 / 24.0);
    p = fma3s(p, t, 1.0 / 6.0);
    p = fma(p, t, 0.5);
    p = fma(p, t, 1.0);
    p = fma(p, t, 1.0);
    return ldexp(p, (int)n);
}

// The exponent polynomial of an element reference (FP32 deviation storage):
// E(u) = c0 + c1 ux + c2 uy + c3 uz + c4 ux^2 + c5 uy^2 + c6 uz^2
//        + c7 ux uy + c8 ux uz + c9 uy uz,
// in FP32 from the coefficients and the velocity rounded to FP32: one fixed
// sequence of IEEE operations wherever it is evaluated.
constexpr int kRefCoef = 10;
__device__ __forceinline__ float ref_exponent(const float *c, const float u[3]) {
    float tx = fmaf(c[4], u[0], c[1]);
    tx = fmaf(c[7], u[1], tx);
    tx = fmaf(c[8], u[2], tx);
    float ty = fmaf(c[5], u[1], c[2]);
    ty = fmaf(c[9], u[2], ty);
    const float tz = fmaf(c[6], u[2], c[3]);
    float E = fmaf(u[0], tx, c[0]);
    E = fmaf(u[1], ty, E);
    return fmaf(u[2], tz, E);
}

// Reference value at exponent E: the FP32 hardware exp2 of E log2(e).  It
// has to be close to f and the same bits wherever it is evaluated (it is
// subtracted when a value is stored and added back when it is read and its
// moments are summed separately), not accurate.  An FP32 number, so sums and
// differences of two references and of a reference and an FP32 value near
// it are exact or rounded once.
__device__ __forceinline__ float ref_value(float E) {
    return __builtin_amdgcn_exp2f(E * 1.44269504f);
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

// One step of Marsaglia's xorshift32 generator (shifts 13, 17, 5; period
// 2^32 - 1 over nonzero states): a lane that rounds several values in a row
// seeds it once with round_bits (forced odd, so never zero) and steps it per
// value, three shifts and three xors instead of two hash rounds.
__device__ __forceinline__ uint32_t xorshift32(uint32_t x) {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}

}  // namespace frdvm
