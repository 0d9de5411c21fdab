// Check rules shared by the CSR kernels (one frame per lane, and frames
// staged in LDS), so that both compute every message with the same
// instructions and give the same result bit for bit.
#pragma once
#include "internal.hpp"
#include "phi.hpp"

namespace cbp {

// C2V of a check recovered from its belief (om = max term or min1 with the
// parity in its sign bit, os = rest of the sum or min2), excluding q
// (B2V, eq. equ_s4e18; min-sum form of Sec. IV-D with kMin).
template <bool kMin>
__device__ float b2v(float om, float os, float q, const Params &p) {
    if constexpr (!kMin) {
        return with_sign(phi2(excl_sum(abs_bits(om), os, phi2_clamped(q, p.a, p.lmax))), sign_bit(om) ^ (q < 0.0f));
    } else {
        const float aq = __builtin_fminf(__builtin_fabsf(q), p.lmax);
        const float m1 = abs_bits(om);
        return with_sign(p.alpha * ((aq == m1) ? os : m1), sign_bit(om) ^ (q < 0.0f));
    }
}

// The same B2V from the excluded term itself: t is the check-rule term of q
// as the check folded it, with q's sign (|t| = phi2_clamped(q) or
// min(|q|, lmax), sign bit = q < 0), so the result is b2v's bit for bit.
template <bool kMin>
__device__ float b2v_term(float om, float os, float t, const Params &p) {
    if constexpr (!kMin) {
        return with_sign(phi2(excl_sum(abs_bits(om), os, abs_bits(t))), sign_bit(om) ^ sign_bit(t));
    } else {
        const float m1 = abs_bits(om);
        return with_sign(p.alpha * ((abs_bits(t) == m1) ? os : m1), sign_bit(om) ^ sign_bit(t));
    }
}

// Flooding posterior at the end of a sweep: channel LLR (scaled to the
// rule's units) plus the sum of the sweep's C2V messages (eq. equ_s2e6).
__device__ __forceinline__ float flood_posterior(float l, float us, float acc) { return l * us + acc; }

}  // namespace cbp
