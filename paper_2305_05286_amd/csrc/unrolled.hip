// Unrolled, differentiable CBP: a fixed number of sweeps of CBP (Sec. IV-C)
// whose B2V outputs carry learnable weights, and its hand-written adjoint.
//
// In sweep t the B2V output R_new(c_j -> v) of eq. (equ_s4e18) becomes
//     sgn(R_new) * max(w[t][b] * |R_new| - beta[t][b], 0),   b = block-column of v,
// before it is committed (equ_s4e22) and added to Q_v (equ_s4e20); w = 1,
// beta = 0 is plain CBP.  The output is the soft value o_v = Q_v + (the same
// weighted B2V from v's latest check with the last sweep's weights).
//
// Layout and arithmetic follow the streamed QC decoder: a frame occupies Z
// lanes, lane l owns variable l of every block-column, block-rows are layers,
// the check-belief is kept as (max phi2 term | parity, rest of the sum), LLRs in
// log2 units (phi2 is its own inverse there).  With w = 1, beta = 0 the forward
// pass performs exactly the streamed kernel's operations.
//
// Memory: the forward pass stores the state (Q, R, Omega) at the start of every
// sweep after the first (checkpoints) and leaves the final state in the working
// area.  The backward pass walks the sweeps in reverse; for each it recomputes
// the sweep in place on the checkpoint it started from (which no later step
// needs), writing a per-edge tape (Q_v before the visit, the excluded phi-domain
// sum, R(c_i -> v) as read, the belief's parity), then applies the adjoint
// layer by layer in reverse order.  The backward pass therefore consumes the
// checkpoints: one backward per forward.  Adjoint state: lambda_Q [N],
// lambda_R [E], lambda_T [M] (adjoint of each check's phi-domain total).  The
// adjoint of a check total read by a B2V is scattered to the check's rows
// through LDS (row k gathers from lane (k + s) mod Z), so no atomics are used and
// the result is deterministic; weight gradients are summed per workgroup in LDS
// and over workgroups by a fixed-order reduction kernel.
//
// Derivatives: g(x) = phi(x ln2)/ln2 has g'(x) = -1/sinh(x ln2); the clamp of
// |Q| to [a, lmax] passes sign(Q) inside the interval and 0 outside; the
// exclusion S + (Mx - f) is the check total minus f; signs carry no gradient.
#include "internal.hpp"
#include "phi.hpp"
#include "stream_util.hpp"

namespace cbp {
namespace {

struct UnArgs {
    const float *llr;
    int64_t batch;
    int T;
    const StreamCode *code;
    const float *w, *beta;   // [T][NB]
    float *out;              // forward: soft output [B][N] (natural units)
    const float *gout;       // backward: dL/d out [B][N]
    float *gllr;             // backward: dL/d llr [B][N] or NULL
    float *gpart;            // backward: [groups][T][NB][2] per-workgroup weight gradients
    char *ws;                // workgroup workspaces, group_bytes apart
    int64_t group_bytes;
    int64_t frame_bytes;
    float a, lmax;           // natural units
    int lanes;
    int dcmax;
};

// g'(x) = -1 / sinh(x ln2), both forms evaluated and one selected
__device__ __forceinline__ float dphi2(float x) {
    const float y = x * kLn2;
    const float y2 = y * y;
    const float sh_small = y * (1.0f + y2 * (0.16666667f + y2 * (0.0083333333f + y2 * 0.00019841270f)));
    const float t = __builtin_amdgcn_exp2f(-x);
    const float sh_large = (1.0f - t * t) * __builtin_amdgcn_rcpf(2.0f * t);
    return -__builtin_amdgcn_rcpf(y < 0.35f ? sh_small : sh_large);  // 1 ulp reciprocal
}

// d clamp(|q|) / dq
__device__ __forceinline__ float dclamp(float q, float a2, float lmax2) {
    const float m = __builtin_fabsf(q);
    return (m > a2 && m < lmax2) ? (q < 0.0f ? -1.0f : 1.0f) : 0.0f;
}

__device__ __forceinline__ int wrapz(int x, int Z) {
    x += (x < 0) ? Z : 0;
    return x - ((x >= Z) ? Z : 0);
}

// Frame geometry inside its workgroup's buffer (byte offsets).
struct Frame {
    Ws W;
    int Z, NB, MB, E, l;
    uint32_t oQ, oR, oOM;            // working state
    uint32_t oCk;                    // checkpoint 1 (each is `ck` bytes)
    uint32_t ck;
    uint32_t oLQ, oLR, oLT, oTape;   // adjoints and tape (backward)
};

__device__ __forceinline__ Frame frame_of(const UnArgs &A, int slot, int l, int Z, int NB, int MB, int E) {
    Frame F;
    F.W = Ws{__builtin_amdgcn_make_buffer_rsrc(A.ws + (int64_t)gid_x() * A.group_bytes, 0, (int)A.group_bytes,
                                               kBufferWord3)};
    F.Z = Z;
    F.NB = NB;
    F.MB = MB;
    F.E = E;
    F.l = l;
    const uint32_t N = NB * Z, EZ = E * Z, M = MB * Z;
    const uint32_t base = (uint32_t)(slot * A.frame_bytes);
    F.ck = 4u * (N + EZ) + 8u * M;
    F.oQ = base;
    F.oR = base + 4u * N;
    F.oOM = base + 4u * (N + EZ);
    F.oCk = base + F.ck;
    const uint32_t after = F.oCk + F.ck * (uint32_t)(A.T - 1);  // checkpoints 1 .. T-1
    F.oLQ = after;
    F.oLR = after + 4u * N;
    F.oLT = after + 4u * (N + EZ);
    F.oTape = (after + 4u * (N + EZ + M) + 15u) & ~15u;
    return F;
}

// One sweep of weighted CBP, in place on the state at byte offset `st`
// (Q [N], R [E][Z], Omega [M] float2 back to back); kTape also writes the tape.
// kCk (sweeps t >= 1 of the forward pass) also writes the state as it was at
// the start of the sweep to the checkpoint at `ck`, each element when the sweep
// first reads it: Q_v at v's first visit; R(c_i -> v) at its own visit, except
// where the commit at the column's first visit has already replaced it (the
// column's last edge), whose old value is read just before that commit; a
// check's belief just before its row stores the new one.
template <bool kTape, bool kCk>
__device__ void sweep(const UnArgs &A, const Frame &F, uint32_t st, uint32_t ck, const int *rstart,
                      const int4 *erec, int t, float *sX, float a2, float lmax2) {
    const int Z = F.Z, l = F.l, NB = F.NB;
    const uint32_t oQ = st, oR = st + 4u * (NB * Z), oOM = st + 4u * (NB * Z + F.E * Z);
    const uint32_t cQ = ck, cR = ck + 4u * (NB * Z), cOM = ck + 4u * (NB * Z + F.E * Z);
    for (int r = 0; r < F.MB; ++r) {
        const int e0 = ldc(rstart, r), e1 = ldc(rstart, r + 1);
        // two edges at a time: all loads before any store (distinct block-columns;
        // R(c_i -> v) is read before R(c_j -> v) is stored, from rn in a degree-1 column)
        struct In {
            Edge ed;
            float q, rci, rep;  // rep: R(c_j -> v) before its commit (kCk, first visits)
            float2 om;
            bool has;
        };
        auto ld_edge = [&](int e, In &in) {
            in.ed = edge(erec, e);
            in.q = F.W.ld(oQ + 4u * (in.ed.b * Z + l));
            in.rci = F.W.ld(oR + 4u * (e * Z + l));
            in.has = !(t == 0 && in.ed.first);
            in.om = in.has ? F.W.ld2(oOM + 8u * (in.ed.epr * Z + wrapz(l - in.ed.epsh, Z))) : make_float2(0.0f, 0.0f);
            if constexpr (kCk)
                if (in.ed.first && in.ed.ep != e) in.rep = F.W.ld(oR + 4u * (in.ed.ep * Z + l));
        };
        auto fin_edge = [&](int e, const In &in) {
            const Edge &ed = in.ed;
            const float q = in.q;
            if constexpr (kCk) {
                if (ed.first) F.W.st(cQ + 4u * (ed.b * Z + l), q);
                if (!ed.last || ed.ep == e) F.W.st(cR + 4u * (e * Z + l), in.rci);
                if (ed.first && ed.ep != e) F.W.st(cR + 4u * (ed.ep * Z + l), in.rep);
            }
            float rn = 0.0f, d = -1.0f, par = 0.0f;
            bool own = false;
            if (in.has) {
                d = excl_sum(abs_bits(in.om.x), in.om.y, phi2_clamped(q, a2, lmax2));
                const int k = t * NB + ed.b;
                const float mag = __builtin_fmaxf(ldc(A.w, k) * phi2(d) - ldc(A.beta, k) * kLog2e, 0.0f);
                rn = with_sign(mag, sign_bit(in.om.x) ^ (q < 0.0f));
                F.W.st(oR + 4u * (ed.ep * Z + l), rn);  // commit R(c_j -> v)
                own = ed.ep == e;
                par = sign_bit(in.om.x) ? 1.0f : 0.0f;
            }
            const float rold = own ? rn : in.rci;
            const float qn = q + rn - rold;
            F.W.st(oQ + 4u * (ed.b * Z + l), qn);
            sX[(e - e0) * Z + wrapz(l - ed.sh, Z)] = with_sign(phi2_clamped(qn, a2, lmax2), qn < 0.0f);
            if constexpr (kTape) F.W.st4(F.oTape + 16u * (e * Z + l), make_float4(q, d, rold, par));
        };
        int e = e0;
        for (; e + 1 < e1; e += 2) {
            In p0, p1;
            ld_edge(e, p0);
            ld_edge(e + 1, p1);
            fin_edge(e, p0);
            fin_edge(e + 1, p1);
        }
        if (e < e1) {
            In p0;
            ld_edge(e, p0);
            fin_edge(e, p0);
        }
        __syncthreads();
        {
            bool p = false;
            float Mx = 0.0f, Sr = 0.0f;
            for (int j = 0; j < e1 - e0; ++j) {
                const float x = sX[j * Z + l];
                p ^= sign_bit(x);
                fold(Mx, Sr, abs_bits(x));
            }
            if constexpr (kCk) F.W.st2(cOM + 8u * (r * Z + l), F.W.ld2(oOM + 8u * (r * Z + l)));
            F.W.st2(oOM + 8u * (r * Z + l), make_float2(with_sign(Mx, p), Sr));
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void unrolled_fwd_kernel(UnArgs A) {
    extern __shared__ float smem[];
    using CS = const __attribute__((address_space(4))) StreamCode;
    CS *cs = (CS *)A.code;
    const int Z = cs->Z, NB = cs->nb, MB = cs->mb, E = cs->E;
    const int64_t N = cs->N;
    const int *rstart = cs->rstart;
    const int4 *erec = cs->erec;
    const int SL = A.lanes / Z;
    const int slot = tid_x() / Z, l = tid_x() - slot * Z;
    const int64_t f = (int64_t)gid_x() * SL + slot;
    const bool have = f < A.batch;
    const float a2 = A.a * kLog2e, lmax2 = A.lmax * kLog2e;
    float *sX = smem + (size_t)slot * A.dcmax * Z;
    const Frame F = frame_of(A, slot, l, Z, NB, MB, E);

    for (int b = 0; b < NB; ++b)
        F.W.st(F.oQ + 4u * (b * Z + l), have ? A.llr[f * N + b * Z + l] * kLog2e : 0.0f);
    for (int e = 0; e < E; ++e) F.W.st(F.oR + 4u * (e * Z + l), 0.0f);
    __syncthreads();
    for (int t = 0; t < A.T; ++t) {
        if (t > 0)  // the state at the start of sweep t goes to checkpoint t as the sweep reads it
            sweep<false, true>(A, F, F.oQ, F.oCk + F.ck * (uint32_t)(t - 1), rstart, erec, t, sX, a2, lmax2);
        else
            sweep<false, false>(A, F, F.oQ, 0, rstart, erec, t, sX, a2, lmax2);
    }
    for (int b = 0; b < NB; ++b) {
        const int el = ldc(cs->elast, b);
        const float2 om = F.W.ld2(F.oOM + 8u * (ldc(cs->er, el) * Z + wrapz(l - ldc(cs->esh, el), Z)));
        const float q = F.W.ld(F.oQ + 4u * (b * Z + l));
        const float d = excl_sum(abs_bits(om.x), om.y, phi2_clamped(q, a2, lmax2));
        const int k = (A.T - 1) * NB + b;
        const float mag = __builtin_fmaxf(ldc(A.w, k) * phi2(d) - ldc(A.beta, k) * kLog2e, 0.0f);
        const float o = q + with_sign(mag, sign_bit(om.x) ^ (q < 0.0f));
        if (have) A.out[f * N + b * Z + l] = o * kLn2;
    }
}

// Edges of a layer whose adjoint accesses are issued together.
#ifndef CBP_UNROLLED_ADJ_GROUP
#define CBP_UNROLLED_ADJ_GROUP 2
#endif
constexpr int kAdjGroup = CBP_UNROLLED_ADJ_GROUP;

// Sum over the 64 lanes of a wave (xor butterfly; every lane gets the total,
// lane 0's in a fixed order).  Only for workgroups of whole waves.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// kWaveSum: weight-gradient contributions are summed over each wave per edge
// and accumulated per (block-column, wave) in LDS (workgroups of whole waves);
// otherwise per (block-column, lane).
template <bool kWaveSum>
__global__ __launch_bounds__(1024) void unrolled_bwd_kernel(UnArgs A) {
    extern __shared__ float smem[];
    using CS = const __attribute__((address_space(4))) StreamCode;
    CS *cs = (CS *)A.code;
    const int Z = cs->Z, NB = cs->nb, MB = cs->mb, E = cs->E;
    const int64_t N = cs->N;
    const int *rstart = cs->rstart;
    const int4 *erec = cs->erec;
    const int SL = A.lanes / Z;
    const int tid = tid_x();
    const int slot = tid / Z, l = tid - slot * Z;
    const int64_t f = (int64_t)gid_x() * SL + slot;
    const bool have = f < A.batch;
    const float a2 = A.a * kLog2e, lmax2 = A.lmax * kLog2e;
    const int DM = A.dcmax;
    // LDS: exchange [SL][dcmax][Z], row adjoints [SL][Z], scatter [SL][dcmax][Z],
    // weight-gradient accumulators [NB][ACC] x 2, ACC = waves (kWaveSum) or lanes
    float *sX = smem + (size_t)slot * A.dcmax * Z;
    float *sLall = smem + (size_t)A.lanes * A.dcmax;
    float *sL = sLall + (size_t)slot * Z;
    float *sD = sLall + A.lanes + (size_t)slot * DM * Z;
    const int ACC = kWaveSum ? A.lanes / 64 : A.lanes;
    const int acc_i = kWaveSum ? tid / 64 : tid;  // this lane's accumulator column
    float *sAw = sLall + A.lanes + (size_t)A.lanes * DM;
    float *sAb = sAw + (size_t)NB * ACC;
    // add this edge's contributions (cw to w[b], cb to beta[b]); every lane of
    // the workgroup calls it for the same b
    auto accumulate = [&](int b, float cw, float cb) {
        if constexpr (kWaveSum) {
            cw = wave_sum(cw);
            cb = wave_sum(cb);
            if ((tid & 63) == 0) {
                sAw[b * ACC + acc_i] += cw;
                sAb[b * ACC + acc_i] += cb;
            }
        } else {
            sAw[b * ACC + acc_i] += cw;
            sAb[b * ACC + acc_i] += cb;
        }
    };
    const Frame F = frame_of(A, slot, l, Z, NB, MB, E);
    const uint32_t oFinal = F.oQ;  // the forward pass leaves the final state here

    for (int i = tid; i < NB * ACC; i += A.lanes) {
        sAw[i] = 0.0f;
        sAb[i] = 0.0f;
    }
    for (int e = 0; e < E; ++e) F.W.st(F.oLR + 4u * (e * Z + l), 0.0f);
    for (int r = 0; r < MB; ++r) F.W.st(F.oLT + 4u * (r * Z + l), 0.0f);

    // ---- adjoint of the soft output o_v = Q_v + weighted B2V (last weights),
    // block-columns in chunks of DM (the scatter buffer's depth)
    for (int b0 = 0; b0 < NB; b0 += DM) {
        const int b1 = b0 + DM < NB ? b0 + DM : NB;
        for (int b = b0; b < b1; ++b) {
            const int el = ldc(cs->elast, b);
            const float2 om = F.W.ld2(oFinal + 4u * (uint32_t)(N + E * Z) +
                                      8u * (ldc(cs->er, el) * Z + wrapz(l - ldc(cs->esh, el), Z)));
            const float q = F.W.ld(oFinal + 4u * (b * Z + l));
            const float go = have ? A.gout[f * N + b * Z + l] * kLn2 : 0.0f;
            const float d = excl_sum(abs_bits(om.x), om.y, phi2_clamped(q, a2, lmax2));
            const int k = (A.T - 1) * NB + b;
            const float wk = ldc(A.w, k), m = phi2(d);
            const bool act = wk * m - ldc(A.beta, k) * kLog2e > 0.0f;
            const bool neg = sign_bit(om.x) ^ (q < 0.0f);
            const float lmag = neg ? -go : go;            // d o / d mag = sgn
            const float lm = act ? lmag * wk : 0.0f;
            accumulate(b, act ? lmag * m : 0.0f, act ? -lmag : 0.0f);
            const float ld = lm * dphi2(d);
            const float lq = go - ld * dphi2(__builtin_fminf(__builtin_fmaxf(__builtin_fabsf(q), a2), lmax2)) *
                                      dclamp(q, a2, lmax2);
            F.W.st(F.oLQ + 4u * (b * Z + l), lq);
            sD[(b - b0) * Z + l] = ld;
        }
        __syncthreads();
        for (int b = b0; b < b1; ++b) {  // lane = row l of each check layer
            const int el = ldc(cs->elast, b);
            const uint32_t o = F.oLT + 4u * (ldc(cs->er, el) * Z + l);
            F.W.st(o, F.W.ld(o) + sD[(b - b0) * Z + wrapz(l + ldc(cs->esh, el), Z)]);
        }
        __syncthreads();
    }

    for (int t = A.T - 1; t >= 0; --t) {
        // recompute sweep t with the tape, in place on the state it started
        // from: checkpoint t (no longer needed once this sweep is differentiated),
        // or for t = 0 the initial state rebuilt in the working area
        uint32_t st = F.oQ;
        if (t > 0) {
            st = F.oCk + F.ck * (uint32_t)(t - 1);
        } else {
            for (int b = 0; b < NB; ++b)
                F.W.st(F.oQ + 4u * (b * Z + l), have ? A.llr[f * N + b * Z + l] * kLog2e : 0.0f);
            for (int e = 0; e < E; ++e) F.W.st(F.oR + 4u * (e * Z + l), 0.0f);
        }
        __syncthreads();
        sweep<true, false>(A, F, st, 0, rstart, erec, t, sX, a2, lmax2);

        for (int r = MB - 1; r >= 0; --r) {
            const int e0 = ldc(rstart, r), e1 = ldc(rstart, r + 1);
            {  // lane = row l: adjoint of the new total of check row l of layer r
                const uint32_t o = F.oLT + 4u * (r * Z + l);
                sL[l] = F.W.ld(o);
                F.W.st(o, 0.0f);
            }
            __syncthreads();
            // lane = variable.  Two edges at a time, all loads before any store:
            // the edges of a layer are distinct block-columns, so no load of
            // one reads what the other stores (its own R(c_j -> v) and
            // R(c_i -> v) coincide only in a degree-1 column, handled below).
            struct AIn {
                Edge ed;
                float4 tp;        // tape: Q before the visit, excluded sum d, R(c_i -> v) read, parity
                float lq, lrep, lre, lf;
            };
            auto ld_adj = [&](int e, AIn &in) {
                in.ed = edge(erec, e);
                in.tp = F.W.ld4(F.oTape + 16u * (e * Z + l));
                in.lq = F.W.ld(F.oLQ + 4u * (in.ed.b * Z + l));
                in.lrep = F.W.ld(F.oLR + 4u * (in.ed.ep * Z + l));
                in.lre = F.W.ld(F.oLR + 4u * (e * Z + l));
                in.lf = sL[wrapz(l - in.ed.sh, Z)];
            };
            auto fin_adj = [&](int e, const AIn &in) {
                float cw = 0.0f, cb = 0.0f;  // this edge's weight-gradient contributions
                const Edge &ed = in.ed;
                const int iv = ed.b * Z + l;
                const float q = in.tp.x, d = in.tp.y, rold = in.tp.z;
                const bool has = d >= 0.0f;
                float rn = 0.0f, m = 0.0f, wk = 0.0f;
                bool act = false, neg = false;
                const int k = t * NB + ed.b;
                if (has) {
                    wk = ldc(A.w, k);
                    m = phi2(d);
                    act = wk * m - ldc(A.beta, k) * kLog2e > 0.0f;
                    neg = (in.tp.w != 0.0f) ^ (q < 0.0f);
                    rn = with_sign(__builtin_fmaxf(wk * m - ldc(A.beta, k) * kLog2e, 0.0f), neg);
                }
                const bool own = has && ed.ep == e;
                const float qn = q + rn - rold;
                const float cn = __builtin_fminf(__builtin_fmaxf(__builtin_fabsf(qn), a2), lmax2);
                const float lqn = in.lq + in.lf * dphi2(cn) * dclamp(qn, a2, lmax2);
                float lq = lqn;  // through lam = q + rn
                float ld = 0.0f;
                if (has) {
                    const float lrn = lqn + (own ? -lqn : 0.0f) + in.lrep;
                    F.W.st(F.oLR + 4u * (ed.ep * Z + l), 0.0f);  // R(c_j -> v) before the commit is dead
                    const float lmag = neg ? -lrn : lrn;
                    const float lm = act ? lmag * wk : 0.0f;
                    cw = act ? lmag * m : 0.0f;
                    cb = act ? -lmag : 0.0f;
                    ld = lm * dphi2(d);
                    const float cq = __builtin_fminf(__builtin_fmaxf(__builtin_fabsf(q), a2), lmax2);
                    lq -= ld * dphi2(cq) * dclamp(q, a2, lmax2);
                }
                if (!own)  // R(c_i -> v) as read by this visit (a different slot from R(c_j -> v) above)
                    F.W.st(F.oLR + 4u * (e * Z + l), in.lre - lqn);
                F.W.st(F.oLQ + 4u * iv, lq);
                sD[(e - e0) * Z + l] = ld;
                accumulate(ed.b, cw, cb);
            };
            {
                int e = e0;
                for (; e + kAdjGroup <= e1; e += kAdjGroup) {
                    AIn in[kAdjGroup];
#pragma unroll
                    for (int k = 0; k < kAdjGroup; ++k) ld_adj(e + k, in[k]);
#pragma unroll
                    for (int k = 0; k < kAdjGroup; ++k) fin_adj(e + k, in[k]);
                }
                for (; e < e1; ++e) {
                    AIn in;
                    ld_adj(e, in);
                    fin_adj(e, in);
                }
            }
            __syncthreads();
            for (int e = e0; e < e1; ++e) {  // lane = row l of the B2V's latest check
                const Edge ed = edge(erec, e);
                if (t == 0 && ed.first) continue;
                const uint32_t o = F.oLT + 4u * (ed.epr * Z + l);
                F.W.st(o, F.W.ld(o) + sD[(e - e0) * Z + wrapz(l + ed.epsh, Z)]);
            }
            __syncthreads();
        }
        // this sweep's weight gradients: sum over the workgroup's accumulators
        for (int b = tid; b < NB; b += A.lanes) {
            float sw = 0.0f, sb = 0.0f;
            for (int i = 0; i < ACC; ++i) {
                sw += sAw[b * ACC + i];
                sb += sAb[b * ACC + i];
            }
            float *gp = A.gpart + (((int64_t)gid_x() * A.T + t) * NB + b) * 2;
            gp[0] = sw;
            gp[1] = sb;
        }
        __syncthreads();
        for (int i = tid; i < NB * ACC; i += A.lanes) {
            sAw[i] = 0.0f;
            sAb[i] = 0.0f;
        }
        __syncthreads();
    }
    if (have && A.gllr)
        for (int b = 0; b < NB; ++b)
            A.gllr[f * N + b * Z + l] = F.W.ld(F.oLQ + 4u * (b * Z + l)) * kLog2e;
}

// grad_w[t][b] = sum over workgroups (deterministic: thread k sums workgroups
// k, k + 256, ... in order, then a fixed-shape tree over the 256 partial sums);
// one workgroup per (t, b).  beta enters in log2 units, hence the log2 e factor.
constexpr int kReduceBlock = 256;
__global__ __launch_bounds__(kReduceBlock) void unrolled_reduce_kernel(const float *gpart, int groups, int TNB,
                                                                       float *gw, float *gb) {
    __shared__ float sw[kReduceBlock], sb[kReduceBlock];
    const int i = gid_x(), k = tid_x();
    float w = 0.0f, b = 0.0f;
    for (int g = k; g < groups; g += kReduceBlock) {
        w += gpart[((int64_t)g * TNB + i) * 2];
        b += gpart[((int64_t)g * TNB + i) * 2 + 1];
    }
    sw[k] = w;
    sb[k] = b;
    __syncthreads();
    for (int h = kReduceBlock / 2; h > 0; h /= 2) {
        if (k < h) {
            sw[k] += sw[k + h];
            sb[k] += sb[k + h];
        }
        __syncthreads();
    }
    if (k == 0) {
        gw[i] = sw[0];
        gb[i] = sb[0] * kLog2e;
    }
}

}  // namespace

int64_t unrolled_frame_bytes(const StreamCode &c, int T) {
    const int64_t N = c.N, EZ = (int64_t)c.E * c.Z, M = (int64_t)c.mb * c.Z;
    const int64_t state = 4 * (N + EZ) + 8 * M;
    int64_t b = state * T + 4 * (N + EZ + M);  // working state + T-1 checkpoints, adjoints
    b = (b + 15) & ~(int64_t)15;
    b += 16 * EZ;  // tape
    return (b + 255) & ~(int64_t)255;
}

size_t unrolled_lds_bytes(const StreamCode &c, int lanes, bool backward) {
    const size_t x = (size_t)lanes * c.dcmax;
    if (!backward) return 4 * x;
    const size_t acc = lanes % 64 == 0 ? lanes / 64 : lanes;
    return 4 * (2 * x + lanes + 2 * (size_t)c.nb * acc);
}

bool unrolled_fits(const StreamCode &c, int lanes) {
    int fw = 0, bw = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&fw, reinterpret_cast<const void *>(unrolled_fwd_kernel), lanes,
                                                     unrolled_lds_bytes(c, lanes, false)) != hipSuccess)
        return false;
    const void *bwd = lanes % 64 == 0 ? reinterpret_cast<const void *>(unrolled_bwd_kernel<true>)
                                      : reinterpret_cast<const void *>(unrolled_bwd_kernel<false>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bw, bwd, lanes, unrolled_lds_bytes(c, lanes, true)) != hipSuccess)
        return false;
    return fw > 0 && bw > 0;
}

hipError_t launch_unrolled(bool backward, const StreamCode &host_code, const StreamCode *dev_code, int lanes,
                           int groups, const float *llr, int64_t batch, int T, const float *w,
                           const float *beta, float *out, const float *gout, float *gllr, float *gpart,
                           float *gw, float *gb, const Params &p, void *ws, hipStream_t s) {
    UnArgs A{};
    A.llr = llr;
    A.batch = batch;
    A.T = T;
    A.code = dev_code;
    A.w = w;
    A.beta = beta;
    A.out = out;
    A.gout = gout;
    A.gllr = gllr;
    A.gpart = gpart;
    A.ws = (char *)ws;
    A.frame_bytes = unrolled_frame_bytes(host_code, T);
    A.group_bytes = (int64_t)(lanes / host_code.Z) * A.frame_bytes;
    A.a = p.a;
    A.lmax = p.lmax;
    A.lanes = lanes;
    A.dcmax = host_code.dcmax;
    const size_t lds = unrolled_lds_bytes(host_code, lanes, backward);
    if (!backward) {
        hipLaunchKernelGGL(unrolled_fwd_kernel, dim3(groups), dim3(lanes), lds, s, A);
        return hipGetLastError();
    }
    if (lanes % 64 == 0)
        hipLaunchKernelGGL(unrolled_bwd_kernel<true>, dim3(groups), dim3(lanes), lds, s, A);
    else
        hipLaunchKernelGGL(unrolled_bwd_kernel<false>, dim3(groups), dim3(lanes), lds, s, A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int TNB = T * host_code.nb;
    hipLaunchKernelGGL(unrolled_reduce_kernel, dim3(TNB), dim3(kReduceBlock), 0, s, gpart, groups, TNB, gw, gb);
    return hipGetLastError();
}

}  // namespace cbp
