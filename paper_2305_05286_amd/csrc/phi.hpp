// FP32 device math of the check rule on gfx950.
//
// phi(x) = -ln tanh(x/2) (Sec. II-A, eq. equ_s2e5) is its own inverse.  The
// log-tanh kernels keep every LLR in log2 units (L / ln 2); there the rule
// needs g(x) = phi(x ln2) / ln2, which is again its own inverse, so one
// function maps a V2C magnitude to its phi-domain term and a phi-domain sum
// back to a C2V magnitude, and the hardware log2/exp2 need no scaling:
//
//   x <  1/ln2: -log2(x * QA(x^2)),  QA(u) ~ tanh(ln2 sqrt(u)/2) / sqrt(u)
//   x >= 1/ln2: t * UB(t^2), t = 2^-x,  UB(s) ~ (2/ln2) atanh(sqrt s) / sqrt s
//
// (the large-argument form is phi = 2 atanh(e^-x); the small-argument form
// keeps 1 - t from cancelling).  Each range takes one hardware
// transcendental (v_log_f32 / v_exp_f32) and a degree-3 polynomial, an
// iteratively reweighted least-squares fit for relative error (max 5.8e-7
// and 4.1e-7 on its interval); g stays within 8.3e-7 relative of
// phi(x ln2)/ln2 for x up to 60 (degree 4 would give 1.8e-7 for two more FMAs
// per evaluation, about 6% of the CBP kernel's instructions; the decoders'
// messages stay within 1e-4 of the FP64 oracle either way).  Large sums
// underflow to denormals / 0.
//
// Check-belief representation.  The paper keeps Omega in the LLR domain and
// recovers an excluded C2V message through psi- (eq. equ_s4e13), i.e. a
// difference of phi sums.  In FP32 that difference cancels catastrophically
// when the excluded input dominates the sum, so the kernels keep a row's
// belief in the phi domain as (max term Mx with the sign parity in its sign
// bit, S = sum of the other terms).  Excluding a term f that was folded in,
// the rest is S + (Mx - f): 0 <= f <= Mx, so Mx - f is exact whenever f is
// within a factor 2 of Mx (Sterbenz) and exactly 0 when f is the maximum, and
// the result carries one rounding relative to itself, however small the rest
// is next to the excluded term.  This is the exclusion of eq. (equ_s3e2) /
// App. A (equ_ae7) without the cancellation; f must be bit-identical to the
// folded value (cached, or recomputed from the unchanged V2C value by the
// same code).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cbp {

constexpr float kLn2 = 0.6931471805599453f;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kInvLn2 = 1.4426950408889634f;

// Both ranges are evaluated and one result selected: the lanes of a wave
// almost always straddle the split, and branching then costs more than the
// second polynomial (measured on MI355X: 10% of the CBP kernel).
__device__ __forceinline__ float phi2(float x) {
    const float uu = x * x;
    float p = -2.6695948690758087e-05f;
    p = __builtin_fmaf(p, uu, 0.0006596098537556827f);
    p = __builtin_fmaf(p, uu, -0.013873166404664516f);
    p = __builtin_fmaf(p, uu, 0.3465734124183655f);
    const float small = -__builtin_amdgcn_logf(x * p);
    const float t = __builtin_amdgcn_exp2f(-x);
    const float s = t * t;
    float u = 0.514183759689331f;
    u = __builtin_fmaf(u, s, 0.568022608757019f);
    u = __builtin_fmaf(u, s, 0.9620470404624939f);
    u = __builtin_fmaf(u, s, 2.8853890895843506f);
    return x < kInvLn2 ? small : t * u;
}

// g of a V2C magnitude (log2 units) clamped to [a2, lmax2], a2 = g(lmax2)
// (saturation of the messages entering a check).  The host keeps a2 <= lmax2,
// where the median of three is that clamp in one instruction.
__device__ __forceinline__ float clamp_mag(float q, float a2, float lmax2) {
    return __builtin_amdgcn_fmed3f(__builtin_fabsf(q), a2, lmax2);
}
__device__ __forceinline__ float phi2_clamped(float q, float a2, float lmax2) {
    return phi2(clamp_mag(q, a2, lmax2));
}

// Float carrying magnitude m >= 0 with its sign bit set iff neg.
__device__ __forceinline__ float with_sign(float m, bool neg) {
    return __int_as_float(__float_as_int(m) | (neg ? int(0x80000000u) : 0));
}
__device__ __forceinline__ bool sign_bit(float v) { return __float_as_int(v) < 0; }
__device__ __forceinline__ float abs_bits(float v) {
    return __int_as_float(__float_as_int(v) & 0x7fffffff);
}

// Sign handling on raw bits.  The register-resident kernels canonicalise the
// channel LLRs (L + 0.0f turns -0.0 into +0.0).  Then every V2C message and
// posterior is nonzero or +0.0 (a sum can only be -0.0 if both terms are, and
// x - x = +0.0), so its sign bit equals [value < 0] (sgn(0) = +1) and signs
// combine with integer XOR.  (A C2V message can be -0.0 when its magnitude
// underflows; added to anything it acts as +0.0.)
__device__ __forceinline__ uint32_t fbits(float v) { return __float_as_uint(v); }
__device__ __forceinline__ float or_sign(float mag, uint32_t sign_src) {
    return __uint_as_float(__float_as_uint(mag) | (sign_src & 0x80000000u));
}

// phi-domain magnitude of a row belief (Mx = max term, S = rest) excluding f.
__device__ __forceinline__ float excl_sum(float Mx, float S, float f) {
    return S + (Mx - f);
}

// Fold one phi-domain term into a (max, rest) accumulator.
__device__ __forceinline__ void fold(float &Mx, float &S, float f) {
    S += __builtin_fminf(Mx, f);
    Mx = __builtin_fmaxf(Mx, f);
}
// Fold two terms at once: the two smaller of (Mx, f, g) join the rest.
__device__ __forceinline__ void fold2(float &Mx, float &S, float f, float g) {
    const float lo = __builtin_fminf(__builtin_fminf(Mx, f), g);
    const float mid = __builtin_amdgcn_fmed3f(Mx, f, g);
    Mx = __builtin_fmaxf(__builtin_fmaxf(Mx, f), g);
    S = (S + lo) + mid;
}
// Two-smallest (min1 <= min2) accumulator of the min-sum rule, one term and
// two at a time (the second smallest of {m1, m2, f, g} is min(m2, med(m1, f, g))).
__device__ __forceinline__ void fold_min(float &m1, float &m2, float f) {
    m2 = __builtin_fminf(m2, __builtin_fmaxf(m1, f));
    m1 = __builtin_fminf(m1, f);
}
__device__ __forceinline__ void fold_min2(float &m1, float &m2, float f, float g) {
    m2 = __builtin_fminf(m2, __builtin_amdgcn_fmed3f(m1, f, g));
    m1 = __builtin_fminf(__builtin_fminf(m1, f), g);
}
// a ^ b ^ c in one instruction
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

}  // namespace cbp
