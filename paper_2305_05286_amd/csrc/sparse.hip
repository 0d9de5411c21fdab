// One frame per lane, any parity-check matrix (CSR).
//
// Every lane of a wave runs the whole sweep of its own frame in the paper's
// row order; since all lanes share the code, the row/edge loops and the table
// reads are wave-uniform (scalar loads through the constant address space)
// and the per-frame state is stored
// frame-interleaved (index-major, frame-minor) so that each access of a wave
// is one contiguous 256-byte line.  Frames that have stopped are masked off;
// the wave leaves its loop once every lane has stopped.
#include "internal.hpp"
#include "phi.hpp"

namespace cbp {
namespace {

constexpr int kWave = 64;
constexpr int kSyndromeBlock = 256;
constexpr int kFillBlock = 256;

__device__ bool lane_syndrome_ok(const SparseDev &g, const uint8_t *xb, int64_t S, int64_t lf) {
    uint32_t bad = 0;
    for (int i = 0; i < g.M; ++i) {
        uint32_t p = 0;
        for (int e = ldc(g.row_ptr, i); e < ldc(g.row_ptr, i + 1); ++e) p ^= xb[(int64_t)ldc(g.col_idx, e) * S + lf];
        bad |= p;
    }
    return bad == 0;
}

__device__ void write_out(const SparseDev &g, const uint8_t *xb, int64_t S, int64_t lf,
                          uint8_t *bits, int32_t *iters, int64_t f, int t) {
    for (int v = 0; v < g.N; ++v) bits[f * g.N + v] = xb[(int64_t)v * S + lf];
    iters[f] = t;
}

// --------------------------------------------------------------------------
// CBP.  ws: a0 = Q[N] (latest V2C), a1 = PQ[N] (phi2 of the clamped Q folded
// into the latest check), a2 = R[E], a3 = OmM[M] (max phi2 term, sign bit =
// parity), a4 = OmS[M] (rest of the phi2 sum), xb = hard decisions [N].  The
// log-tanh rule keeps LLRs in log2 units (L / ln2), where phi2 serves both
// directions of the check rule; Params a and lmax arrive already scaled.
// --------------------------------------------------------------------------
// C2V of a check recovered from its belief (om = max term or min1 with the
// parity in its sign bit, os = rest of the sum or min2), excluding q.
template <bool kMin>
__device__ float b2v(float om, float os, float pq, float q, const Params &p) {
    if constexpr (!kMin) {
        return with_sign(phi2(excl_sum(abs_bits(om), os, pq)), sign_bit(om) ^ (q < 0.0f));
    } else {
        const float aq = __builtin_fminf(__builtin_fabsf(q), p.lmax);
        const float m1 = abs_bits(om);
        return with_sign(p.alpha * ((aq == m1) ? os : m1), sign_bit(om) ^ (q < 0.0f));
    }
}

template <bool kMin>
__device__ float cbp_flushed(const SparseDev &g, const SparseWs &w, int64_t lf, int v, const Params &p) {
    const int64_t S = w.stride;
    const int e = ldc(g.last_edge, v);
    const int j = ldc(g.edge_row, e);
    const float q = w.a0[(int64_t)v * S + lf];
    return q + b2v<kMin>(w.a3[(int64_t)j * S + lf], w.a4[(int64_t)j * S + lf], w.a1[(int64_t)v * S + lf], q, p);
}

// Flushed posterior after a stop in the middle of sweep t, right after row
// istop: v's latest check is its last row <= istop in this sweep, else (t > 1)
// its last row of the previous sweep, else none (B2V 0).  The column's edges
// are walked backwards from its last edge through pred_edge.
template <bool kMin>
__device__ float cbp_flushed_at(const SparseDev &g, const SparseWs &w, int64_t lf, int v, const Params &p,
                                int istop, int t) {
    const int64_t S = w.stride;
    const float q = w.a0[(int64_t)v * S + lf];
    int e = ldc(g.last_edge, v);
    while (ldc(g.edge_row, e) > istop) {
        if (ldc(g.first, e)) {  // no visit of v yet in this sweep
            if (t == 1) return q;
            e = ldc(g.last_edge, v);
            break;
        }
        e = ldc(g.pred_edge, e);
    }
    const int j = ldc(g.edge_row, e);
    return q + b2v<kMin>(w.a3[(int64_t)j * S + lf], w.a4[(int64_t)j * S + lf], w.a1[(int64_t)v * S + lf], q, p);
}

// kMin: the normalized min-sum check rule (OmM = min1 | parity, OmS = min2).
template <bool kMin>
__global__ __launch_bounds__(kWave) void cbp_sparse_kernel(
    SparseDev g, const float *__restrict__ llr, uint8_t *__restrict__ bits,
    int32_t *__restrict__ iters, int64_t f0, int64_t nf, int max_iter, Params p, SparseWs w,
    Dump d) {
    const int64_t lf = (int64_t)gid_x() * kWave + tid_x();
    const bool valid = lf < nf;
    const int64_t f = f0 + lf;
    const int64_t S = w.stride;
    float *Q = w.a0, *PQ = w.a1, *R = w.a2, *OmM = w.a3, *OmS = w.a4;
    const float us = kMin ? 1.0f : kLog2e;  // log2 units for the log-tanh rule
    const float un = kMin ? 1.0f : kLn2;    // dumps in natural units
    p.a *= us;
    p.lmax *= us;
    uint8_t *xb = w.xb;
    bool active = valid;
    // paper's stopping rule (stop_rule 1): check updates in a row, across
    // sweeps, whose belief is positive and that flipped no decision
    int64_t run = 0;
    // Step 1: latest V2C = channel LLR, R = 0, x = [L < 0]
    if (valid) {
        for (int v = 0; v < g.N; ++v) {
            const float l = llr[f * g.N + v] * us;
            Q[(int64_t)v * S + lf] = l;
            xb[(int64_t)v * S + lf] = l < 0.0f;
        }
        for (int e = 0; e < g.E; ++e) R[(int64_t)e * S + lf] = 0.0f;
        if (p.stop_rule == 0 && lane_syndrome_ok(g, xb, S, lf)) {
            write_out(g, xb, S, lf, bits, iters, f, 0);
            active = false;
        }
    }
    for (int t = 1; t <= max_iter; ++t) {
        if (__ballot(active) == 0) break;
        if (active) {
            // Step 2: check-nodes in index order
            bool paper_stop = false;
            int istop = 0;
            for (int i = 0; i < g.M; ++i) {
                float Mx = kMin ? __builtin_inff() : 0.0f, Sr = kMin ? __builtin_inff() : 0.0f;
                bool par = false, flip = false;
                for (int e = ldc(g.row_ptr, i); e < ldc(g.row_ptr, i + 1); ++e) {
                    const int v = ldc(g.col_idx, e);
                    const int64_t iv = (int64_t)v * S + lf;
                    const float q = Q[iv];
                    float rn = 0.0f;
                    if (!(t == 1 && ldc(g.first, e))) {
                        // B2V (eq. equ_s4e18): C2V of the latest check c_j recovered
                        // from its belief, then committed to R(c_j -> v) first.
                        const int64_t ij = (int64_t)ldc(g.pred_row, e) * S + lf;
                        rn = b2v<kMin>(OmM[ij], OmS[ij], PQ[iv], q, p);
                        R[(int64_t)ldc(g.pred_edge, e) * S + lf] = rn;
                    }
                    const float lam = q + rn;                 // eq. equ_s4e20
                    const uint8_t nx = lam < 0.0f;            // eq. equ_s2e7
                    if (p.stop_rule == 1) flip |= nx != xb[iv];
                    xb[iv] = nx;
                    const float qn = lam - R[(int64_t)e * S + lf];  // V2C, eq. equ_s4e19
                    Q[iv] = qn;
                    if constexpr (!kMin) {
                        const float fq = phi2_clamped(qn, p.a, p.lmax);
                        PQ[iv] = fq;
                        fold(Mx, Sr, fq);                     // C2B, eq. equ_s4e21
                    } else {                                  // eq. equ_s4e21xx
                        const float aq = __builtin_fminf(__builtin_fabsf(qn), p.lmax);
                        Sr = __builtin_fminf(Sr, __builtin_fmaxf(Mx, aq));
                        Mx = __builtin_fminf(Mx, aq);
                    }
                    par ^= (qn < 0.0f);
                }
                OmM[(int64_t)i * S + lf] = with_sign(Mx, par);  // eq. equ_s4e23
                OmS[(int64_t)i * S + lf] = Sr;
                if (p.stop_rule == 1) {  // Step 2(3): M updates in a row with Omega > 0, no flip
                    run = (!par && !flip) ? run + 1 : 0;
                    if (run >= g.M) {
                        paper_stop = true;
                        istop = i;
                        break;
                    }
                }
            }
            if (paper_stop) {
                if (p.hd_mode == 1)
                    for (int v = 0; v < g.N; ++v)
                        xb[(int64_t)v * S + lf] = cbp_flushed_at<kMin>(g, w, lf, v, p, istop, t) < 0.0f;
                write_out(g, xb, S, lf, bits, iters, f, t);
                active = false;
                continue;
            }
            if (p.hd_mode == 1)
                for (int v = 0; v < g.N; ++v) xb[(int64_t)v * S + lf] = cbp_flushed<kMin>(g, w, lf, v, p) < 0.0f;
            if (t == d.sweep && f < d.frames) {
                for (int v = 0; v < g.N; ++v) {
                    if (d.q) d.q[f * g.N + v] = Q[(int64_t)v * S + lf] * un;
                    if (d.lam) d.lam[f * g.N + v] = cbp_flushed<kMin>(g, w, lf, v, p) * un;
                }
                if (d.r)
                    for (int e = 0; e < g.E; ++e) d.r[f * g.E + e] = R[(int64_t)e * S + lf] * un;
                if (d.om)
                    for (int i = 0; i < g.M; ++i) {
                        const float om = OmM[(int64_t)i * S + lf];
                        d.om[f * g.M + i] =
                            kMin ? with_sign(p.alpha * abs_bits(om), sign_bit(om))
                                 : with_sign(phi2(abs_bits(om) + OmS[(int64_t)i * S + lf]) * un, sign_bit(om));
                    }
            }
            const bool stop = (p.stop_rule == 0 && lane_syndrome_ok(g, xb, S, lf)) || t == max_iter;
            if (stop) {
                write_out(g, xb, S, lf, bits, iters, f, t);
                active = false;
            }
        }
    }
    if (active) write_out(g, xb, S, lf, bits, iters, f, max_iter);  // max_iter == 0
}

// --------------------------------------------------------------------------
// Normalized min-sum baselines.  ws: a0 = Lambda[N], a1 = R[E],
// a2 = Lambda accumulator of the flooding schedule [N].
// --------------------------------------------------------------------------
template <bool kFlood>
__global__ __launch_bounds__(kWave) void nms_sparse_kernel(
    SparseDev g, const float *__restrict__ llr, uint8_t *__restrict__ bits,
    int32_t *__restrict__ iters, int64_t f0, int64_t nf, int max_iter, Params p, SparseWs w,
    Dump d) {
    const int64_t lf = (int64_t)gid_x() * kWave + tid_x();
    const bool valid = lf < nf;
    const int64_t f = f0 + lf;
    const int64_t S = w.stride;
    float *Lam = w.a0, *R = w.a1, *Acc = w.a2;
    uint8_t *xb = w.xb;
    bool active = valid;
    if (valid) {
        for (int v = 0; v < g.N; ++v) {
            const float l = llr[f * g.N + v];
            Lam[(int64_t)v * S + lf] = l;
            xb[(int64_t)v * S + lf] = l < 0.0f;
        }
        for (int e = 0; e < g.E; ++e) R[(int64_t)e * S + lf] = 0.0f;
        if (p.stop_rule == 0 && lane_syndrome_ok(g, xb, S, lf)) {
            write_out(g, xb, S, lf, bits, iters, f, 0);
            active = false;
        }
    }
    for (int t = 1; t <= max_iter; ++t) {
        if (__ballot(active) == 0) break;
        if (active) {
            if (kFlood)
                for (int v = 0; v < g.N; ++v) Acc[(int64_t)v * S + lf] = 0.0f;
            for (int i = 0; i < g.M; ++i) {
                const int e0 = ldc(g.row_ptr, i), e1 = ldc(g.row_ptr, i + 1);
                float m1 = __builtin_inff(), m2 = __builtin_inff();
                bool par = false;
                for (int e = e0; e < e1; ++e) {
                    const float q = Lam[(int64_t)ldc(g.col_idx, e) * S + lf] - R[(int64_t)e * S + lf];
                    const float aq = __builtin_fminf(__builtin_fabsf(q), p.lmax);
                    m2 = __builtin_fminf(m2, __builtin_fmaxf(m1, aq));
                    m1 = __builtin_fminf(m1, aq);
                    par ^= (q < 0.0f);
                }
                for (int e = e0; e < e1; ++e) {
                    const int64_t iv = (int64_t)ldc(g.col_idx, e) * S + lf;
                    const int64_t ie = (int64_t)e * S + lf;
                    const float q = Lam[iv] - R[ie];
                    const float aq = __builtin_fminf(__builtin_fabsf(q), p.lmax);
                    const float rn = with_sign(p.alpha * ((aq == m1) ? m2 : m1), par ^ (q < 0.0f));
                    R[ie] = rn;
                    if (kFlood) Acc[iv] += rn;
                    else Lam[iv] = q + rn;  // eq. equ_s2e12
                }
            }
            if (kFlood)
                for (int v = 0; v < g.N; ++v) {
                    const int64_t iv = (int64_t)v * S + lf;
                    Lam[iv] = llr[f * g.N + v] + Acc[iv];  // eq. equ_s2e6
                }
            for (int v = 0; v < g.N; ++v) xb[(int64_t)v * S + lf] = Lam[(int64_t)v * S + lf] < 0.0f;
            if (t == d.sweep && f < d.frames) {
                if (d.lam)
                    for (int v = 0; v < g.N; ++v) d.lam[f * g.N + v] = Lam[(int64_t)v * S + lf];
                if (d.r)
                    for (int e = 0; e < g.E; ++e) d.r[f * g.E + e] = R[(int64_t)e * S + lf];
            }
            const bool stop = (p.stop_rule == 0 && lane_syndrome_ok(g, xb, S, lf)) || t == max_iter;
            if (stop) {
                write_out(g, xb, S, lf, bits, iters, f, t);
                active = false;
            }
        }
    }
    if (active) write_out(g, xb, S, lf, bits, iters, f, max_iter);
}

__global__ __launch_bounds__(kSyndromeBlock) void syndrome_kernel(SparseDev g, const uint8_t *__restrict__ bits,
                                                       uint8_t *__restrict__ ok, int64_t batch) {
    const int64_t f = (int64_t)gid_x() * kSyndromeBlock + tid_x();
    if (f >= batch) return;
    uint32_t bad = 0;
    for (int i = 0; i < g.M; ++i) {
        uint32_t par = 0;
        for (int e = ldc(g.row_ptr, i); e < ldc(g.row_ptr, i + 1); ++e) par ^= bits[f * g.N + ldc(g.col_idx, e)] & 1u;
        bad |= par;
    }
    ok[f] = bad == 0;
}

__global__ __launch_bounds__(kFillBlock) void fill_i32_kernel(int *p, int n, int value) {
    const int i = gid_x() * kFillBlock + tid_x();
    if (i < n) p[i] = value;
}

}  // namespace

static int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

size_t sparse_ws_bytes(int algo, const SparseDev &g, int64_t frames) {
    const int64_t S = round_up(frames, kWave);
    const bool belief = algo == kCBP || algo == kCBPNMS;
    int64_t floats = belief ? (2LL * g.N + g.E + 2LL * g.M) : (2LL * g.N + g.E);
    // each array starts on a 256-byte boundary
    return (size_t)(floats * S * 4 + (int64_t)g.N * S + 8 * 256);
}

SparseWs sparse_ws_carve(int algo, const SparseDev &g, int64_t frames, void *base) {
    SparseWs w{};
    w.stride = round_up(frames, kWave);
    const int64_t S = w.stride;
    char *p = (char *)base;
    auto take = [&](int64_t bytes) {
        char *r = p;
        p += round_up(bytes, 256);
        return r;
    };
    if (algo == kCBP || algo == kCBPNMS) {
        w.a0 = (float *)take(4LL * g.N * S);
        w.a1 = (float *)take(4LL * g.N * S);
        w.a2 = (float *)take(4LL * g.E * S);
        w.a3 = (float *)take(4LL * g.M * S);
        w.a4 = (float *)take(4LL * g.M * S);
    } else {
        w.a0 = (float *)take(4LL * g.N * S);
        w.a1 = (float *)take(4LL * g.E * S);
        w.a2 = (float *)take(4LL * g.N * S);
    }
    w.xb = (uint8_t *)take((int64_t)g.N * S);
    return w;
}

hipError_t launch_sparse(int algo, const SparseDev &g, const float *llr, uint8_t *bits,
                         int32_t *iters, int64_t f0, int64_t nf, int max_iter, const Params &p,
                         const SparseWs &ws, const Dump &d, hipStream_t s) {
    const dim3 grid((unsigned)((nf + kWave - 1) / kWave)), block(kWave);
    if (algo == kCBP)
        hipLaunchKernelGGL(cbp_sparse_kernel<false>, grid, block, 0, s, g, llr, bits, iters, f0, nf,
                           max_iter, p, ws, d);
    else if (algo == kCBPNMS)
        hipLaunchKernelGGL(cbp_sparse_kernel<true>, grid, block, 0, s, g, llr, bits, iters, f0, nf,
                           max_iter, p, ws, d);
    else if (algo == kLBPNMS)
        hipLaunchKernelGGL(nms_sparse_kernel<false>, grid, block, 0, s, g, llr, bits, iters, f0,
                           nf, max_iter, p, ws, d);
    else
        hipLaunchKernelGGL(nms_sparse_kernel<true>, grid, block, 0, s, g, llr, bits, iters, f0,
                           nf, max_iter, p, ws, d);
    return hipGetLastError();
}

hipError_t launch_syndrome(const SparseDev &g, const uint8_t *bits, uint8_t *ok, int64_t batch,
                           hipStream_t s) {
    const dim3 grid((unsigned)((batch + kSyndromeBlock - 1) / kSyndromeBlock)), block(kSyndromeBlock);
    hipLaunchKernelGGL(syndrome_kernel, grid, block, 0, s, g, bits, ok, batch);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int *ptr, int n, int value, hipStream_t s) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3((n + kFillBlock - 1) / kFillBlock), dim3(kFillBlock), 0, s, ptr,
                       n, value);
    return hipGetLastError();
}

}  // namespace cbp
