// FP32 device math of the check rule on gfx950.
//
// phi(x) = -ln tanh(x/2) (Sec. II-A, eq. equ_s2e5) is evaluated with one
// hardware transcendental and a degree-4 polynomial on each side of x = 1:
//   x <  1: phi = -ln(h * P(h^2)),  h = x/2,  P(y) ~ tanh(sqrt y)/sqrt y
//   x >= 1: phi = 2 t U(t^2),       t = e^-x, U(s) ~ atanh(sqrt s)/sqrt s
// (the second form is phi = ln((1+t)/(1-t)) = 2 atanh t).  The polynomials
// are weighted least-squares fits for relative error (max 1.3e-8 and 1.1e-8
// on their intervals); with v_log_f32 / v_exp_f32 the function is within
// ~1e-6 relative of phi for x <= 20 (the exp argument's rounding dominates
// near x = 20) and underflows to denormals/0 beyond x ~ 87.
//
// Check-belief representation.  The paper keeps Omega in the LLR domain and
// recovers an excluded C2V message through psi- (eq. equ_s4e13), i.e. a
// difference of phi sums.  In FP32 that difference cancels catastrophically
// when the excluded input dominates the sum, so the kernels keep a row's
// belief in the phi domain as (max term M with the sign parity in its sign
// bit, S = sum of the other terms).  Excluding a term f that was folded in:
//   f == M : the rest is S                      (no subtraction at all)
//   else   : the rest is M + (S - f)            (f <= M, so the error of the
//                                                 difference is <= eps * M)
// which is the exclusion of eq. (equ_s3e2) / App. A (equ_ae7) without the
// cancellation; the value of f must be bit-identical to the folded one, so it
// is cached per variable.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cbp {

constexpr float kLn2 = 0.6931471805599453f;
constexpr float kLog2e = 1.4426950408889634f;

__device__ __forceinline__ float phi32(float x) {
    if (x < 1.0f) {
        const float h = 0.5f * x;
        const float y = h * h;
        float p = 0.017135001718997955f;
        p = __builtin_fmaf(p, y, -0.05298607423901558f);
        p = __builtin_fmaf(p, y, 0.13324779272079468f);
        p = __builtin_fmaf(p, y, -0.3333306908607483f);
        p = __builtin_fmaf(p, y, 1.0f);
        return -kLn2 * __builtin_amdgcn_logf(h * p);
    }
    const float t = __builtin_amdgcn_exp2f(-x * kLog2e);
    const float s = t * t;
    float u = 0.1488138735294342f;
    u = __builtin_fmaf(u, s, 0.1380910724401474f);
    u = __builtin_fmaf(u, s, 0.2002381980419159f);
    u = __builtin_fmaf(u, s, 0.3333292305469513f);
    u = __builtin_fmaf(u, s, 1.0f);
    return (2.0f * t) * u;
}

// phi of a V2C magnitude clamped to [a, lmax], a = phi(lmax) (saturation of
// the messages entering a check).
__device__ __forceinline__ float phiq32(float q, float a, float lmax) {
    return phi32(__builtin_fminf(__builtin_fmaxf(__builtin_fabsf(q), a), lmax));
}

// Float carrying magnitude m >= 0 with its sign bit set iff neg.
__device__ __forceinline__ float with_sign(float m, bool neg) {
    return __int_as_float(__float_as_int(m) | (neg ? int(0x80000000u) : 0));
}
__device__ __forceinline__ bool sign_bit(float v) { return __float_as_int(v) < 0; }
__device__ __forceinline__ float abs_bits(float v) {
    return __int_as_float(__float_as_int(v) & 0x7fffffff);
}

// C2V magnitude of a row belief (Mx = max term, S = rest) excluding f.
__device__ __forceinline__ float excl_sum(float Mx, float S, float f) {
    return (f == Mx) ? S : Mx + (S - f);
}

// Fold one phi term into a (max, rest) accumulator.
__device__ __forceinline__ void fold(float &Mx, float &S, float f) {
    S += __builtin_fminf(Mx, f);
    Mx = __builtin_fmaxf(Mx, f);
}

}  // namespace cbp
