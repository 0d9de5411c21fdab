// Any parity-check matrix (CSR) with each frame's whole state in LDS.
//
// A workgroup holds kF frames in LDS (CBP: Q [N], R [E], the rows' beliefs
// [M] by level position, decisions [N]; the BP layout is given with its
// kernel below) and runs their sweeps together, level by level: the rows of
// one level share no variable, so they commute in the paper's sequential row
// order (Sec. IV-C) and are updated at once with exactly the sequential
// result.  Within a level the work is split by edge, not by row, which gives
// the threads five to six times more independent items than rows alone:
//   phase A (thread = one edge of one frame): B2V from the latest check's
//            belief and its commit, V2C, the decision at the variable's last
//            visit, and the edge's check-rule term, parked in the edge's own
//            R slot (its old C2V message has just been read, and the next
//            visit of the variable overwrites it by its commit first);
//   phase B (thread = one row of one frame): the row's terms folded in
//            ascending column order into its new belief.
// Per edge these are the very instructions of the one-frame-per-lane kernel
// (the same check-rule functions, the same fold order), so the two layouts
// agree bit for bit.  Within a phase nothing one item writes is read by
// another: a level's rows share no variable, a commit goes to the R slot of a
// row in another level, and a belief read is of another level's row (in a
// weight-one column, of the row itself, whose new belief phase B stores after
// the barrier).  A CU holds several workgroups (one or a few frames each)
// rather than one large one: their barriers are independent, so one
// workgroup's wait is covered by another's work (measured on the PEG codes:
// three one-frame workgroups per CU decode 1.6x faster than one workgroup of
// three frames).  The grid is persistent: a slot whose frame stops writes the
// outputs and loads the next frame of the batch from a global counter; a
// fresh frame is syndrome-tested before its first sweep.  Every branch that
// contains a barrier is taken by the whole workgroup (its condition comes
// from LDS after a barrier).
#include <cstdlib>
#include <type_traits>

#include "internal.hpp"
#include "phi.hpp"
#include "sparse_rules.hpp"

namespace cbp {
namespace {

constexpr int kLdsFillBlock = 256;
constexpr int kLdsChunk = 8;  // loads of a row issued together
constexpr int kLdsCuThreads = 2048;

__global__ __launch_bounds__(kLdsFillBlock) void lds_zero_kernel(unsigned int *p) {
    if (tid_x() == 0) *p = 0u;
}

// Where a launch takes its frames: entries [qs, qs + qn) of a queue filled
// by a counter (frame = perm[qs + k], or k without perm), the frame's LLRs and
// decisions at element offset[frame] (frame * N without offset).
struct LdsQueue {
    const int32_t *perm;
    const int64_t *offset;
    int64_t qs, qn;
    unsigned int *counter;
};

// The persistent slot loop shared by the decoders: kF frame slots in dynamic
// LDS; `load(f, off)` runs Step 1 on a fresh slot whose frame starts at
// element off (all threads, no barrier), `sweep(live, s1)` one sweep of the
// live slots (bit f of s1: slot f's first sweep; it ends with a barrier),
// `dec(f, v)` is slot f's decision on variable v (0 or 1).  Returns once the
// queue is exhausted and every slot has stopped.
template <int kF, int kT, class Load, class Sweep, class Dec>
__device__ __forceinline__ void run_slots(const SparseDev &g, uint8_t *bits, int32_t *iters, const LdsQueue &q,
                                          int max_iter, const Params &p, Load &&load, Sweep &&sweep, Dec &&dec) {
    __shared__ int64_t sFrame[kF], sOff[kF];  // frame (-1: none) and its element offset
    __shared__ int sT[kF], sBad[kF], sFresh[kF];
    const int tid = tid_x();
    auto claim = [&](int f) {  // one thread
        const int64_t k = (int64_t)atomicAdd(q.counter, 1u);
        int64_t fr = -1, off = 0;
        if (k < q.qn) {
            fr = q.perm ? (int64_t)q.perm[q.qs + k] : k;
            off = q.offset ? q.offset[fr] : fr * (int64_t)g.N;
        }
        sFrame[f] = fr;
        sOff[f] = off;
        sT[f] = 0;
    };
    auto load_fresh = [&]() {
        for (int f = 0; f < kF; ++f)
            if (sFresh[f] && sFrame[f] >= 0) load(f, sOff[f]);
    };
    __syncthreads();  // a previous loop's last reads of the slot table are done
    if (tid < kF) {
        claim(tid);
        sFresh[tid] = 1;
    }
    __syncthreads();
    load_fresh();
    __syncthreads();
    for (;;) {
        // ---------------- syndrome of every live slot's decisions ------------
        if (tid < kF) sBad[tid] = 0;
        __syncthreads();
        uint32_t live = 0;
        for (int f = 0; f < kF; ++f) live |= (uint32_t)(sFrame[f] >= 0) << f;
        // a row per thread, its column and decision loads issued together (the
        // column table is padded past E; entries past the row name other
        // columns and are masked)
        for (int i = tid; i < kF * g.M; i += kT) {
            const int j = i / kF, f = i - j * kF;
            if (!((live >> f) & 1u)) continue;
            const int e0 = g.row_ptr[j], e1 = g.row_ptr[j + 1];
            uint32_t par = 0;
            for (int c0 = e0; c0 < e1; c0 += kLdsChunk) {
                int col[kLdsChunk];
                uint32_t x[kLdsChunk];
#pragma unroll
                for (int c = 0; c < kLdsChunk; ++c) col[c] = g.col_idx[c0 + c];
#pragma unroll
                for (int c = 0; c < kLdsChunk; ++c) x[c] = dec(f, col[c]);
#pragma unroll
                for (int c = 0; c < kLdsChunk; ++c) par ^= c0 + c < e1 ? x[c] : 0u;
            }
            if (par) sBad[f] = 1;
        }
        __syncthreads();
        // ---------------- stopped frames out, next frames in -----------------
        uint32_t done = 0;
        for (int f = 0; f < kF; ++f)
            if (((live >> f) & 1u) && ((p.stop_rule == 0 && sBad[f] == 0) || sT[f] >= max_iter))
                done |= 1u << f;
        for (int f = 0; f < kF; ++f) {
            if (!((done >> f) & 1u)) continue;
            const int64_t off = sOff[f];
            for (int v = tid; v < g.N; v += kT) bits[off + v] = (uint8_t)dec(f, v);
            if (tid == 0) iters[sFrame[f]] = sT[f];
        }
        __syncthreads();  // every thread has read sFrame / sOff / sT before they change
        if (tid < kF) {
            const bool d = (done >> tid) & 1u;
            if (d) claim(tid);
            sFresh[tid] = d;
        }
        __syncthreads();
        load_fresh();
        __syncthreads();
        live = 0;
        uint32_t fresh = 0, s1 = 0;
        for (int f = 0; f < kF; ++f) {
            const bool on = sFrame[f] >= 0;
            live |= (uint32_t)on << f;
            fresh |= (uint32_t)(on && sFresh[f] != 0) << f;
            s1 |= (uint32_t)(sT[f] == 0) << f;
        }
        if (!live) break;
        if (fresh) continue;  // test the new frames before they sweep
        sweep(live, s1);
        if (tid < kF && ((live >> tid) & 1u)) ++sT[tid];
    }
}

// CBP.  kMin: the normalized min-sum check rule (beliefs = (min1 | parity,
// min2)).  kT threads per workgroup.
template <bool kMin, int kF, int kT>
__device__ __forceinline__ void cbp_lds_body(const SparseDev &g, const float *__restrict__ llr,
                                             uint8_t *__restrict__ bits, int32_t *__restrict__ iters,
                                             const LdsQueue &q, int max_iter, Params p, const LdsItem &it) {
    extern __shared__ uint4 s_dyn[];
    const int tid = tid_x();
    const float us = kMin ? 1.0f : kLog2e;  // log2 units for the log-tanh rule
    p.a *= us;
    p.lmax *= us;
    char *const base = reinterpret_cast<char *>(s_dyn);
    auto Qp = [&](int f) { return reinterpret_cast<float *>(base + f * it.bytes); };
    auto Rp = [&](int f) { return reinterpret_cast<float *>(base + f * it.bytes + it.r); };
    auto Op = [&](int f) { return reinterpret_cast<float2 *>(base + f * it.bytes + it.om); };
    auto Xp = [&](int f) { return reinterpret_cast<uint8_t *>(base + f * it.bytes + it.xb); };

    // Step 2(1) a-e on the edge of record rec of frame slot f (s1 bit f: the
    // slot's first sweep)
    auto edge = [&](int f, uint32_t s1, const int4 &rec) {
        const int col = rec.x, pe = rec.y, pr = rec.z, e = rec.w & 0x3fffffff;
        const uint32_t fl = (uint32_t)rec.w >> 30;
        float *Q = Qp(f), *R = Rp(f);
        const float q = Q[col];
        float rc = R[e];
        const float2 om = Op(f)[pr];
        // the term of q that the latest check folded, still parked in that
        // edge's slot (only this visit's commit replaces it, and q has not
        // changed since): B2V needs no second evaluation of the check rule
        const float tp = R[pe];
        float rn = 0.0f;
        // no latest check yet on a variable's first visit of the first sweep
        if (!(((s1 >> f) & 1u) && (fl & kFirstVisit))) {
            rn = b2v_term<kMin>(om.x, om.y, tp, p);  // B2V, eq. equ_s4e18
            R[pe] = rn;                               // commit R(c_j -> v) first
            if (pe == e) rc = rn;
        }
        const float lam = q + rn;  // eq. equ_s4e20
        if (fl & kLastVisit) Xp(f)[col] = lam < 0.0f;
        const float qn = lam - rc;  // V2C, eq. equ_s4e19
        Q[col] = qn;
        const float term = kMin ? __builtin_fminf(__builtin_fabsf(qn), p.lmax) : phi2_clamped(qn, p.a, p.lmax);
        R[e] = with_sign(term, qn < 0.0f);
    };
    // Step 2(1)d / 2(2) for row rr = (row, first edge, end edge) of slot f, at
    // level position pos: the terms folded in ascending column order into the
    // new belief (C2B, eqs. equ_s4e21 / equ_s4e23), kLdsChunk loads at a time
    // (indices past the row clamped to its last edge)
    auto row_fold = [&](int f, const int4 &rr, int pos) {
        const float *R = Rp(f);
        float Mx = kMin ? __builtin_inff() : 0.0f, Sr = kMin ? __builtin_inff() : 0.0f;
        bool par = false;
        for (int c0 = rr.y; c0 < rr.z; c0 += kLdsChunk) {
            float x[kLdsChunk];
#pragma unroll
            for (int c = 0; c < kLdsChunk; ++c) x[c] = R[c0 + c < rr.z ? c0 + c : rr.z - 1];
#pragma unroll
            for (int c = 0; c < kLdsChunk; ++c) {
                if (c0 + c < rr.z) {
                    par ^= sign_bit(x[c]);
                    const float ax = abs_bits(x[c]);
                    if constexpr (!kMin) {
                        fold(Mx, Sr, ax);
                    } else {
                        Sr = __builtin_fminf(Sr, __builtin_fmaxf(Mx, ax));
                        Mx = __builtin_fminf(Mx, ax);
                    }
                }
            }
        }
        Op(f)[pos] = make_float2(with_sign(Mx, par), Sr);
    };
    // Step 1: latest V2C = channel LLR, R = 0, x = [L < 0]
    auto load = [&](int f, int64_t off) {
        float *Q = Qp(f), *R = Rp(f);
        uint8_t *xb = Xp(f);
        for (int v = tid; v < g.N; v += kT) {
            const float l = llr[off + v] * us;
            Q[v] = l;
            xb[v] = l < 0.0f;
        }
        for (int e = tid; e < g.E; e += kT) R[e] = 0.0f;
    };
    auto sweep = [&](uint32_t live, uint32_t s1) {
        // Each phase reads its thread's first table record one phase ahead, so
        // that the table latency overlaps the work before the barrier.
        int4 recA = make_int4(0, 0, 0, 0), recB = make_int4(0, 0, 0, 0);
        {
            const int ea = ldc(g.lvl_eptr, 0);
            if (tid < kF * (ldc(g.lvl_eptr, 1) - ea)) recA = g.lvl_edges[ea + tid / kF];
        }
        for (int l = 0; l < g.nlev; ++l) {
            // phase A: thread = (edge of the level, frame)
            const int ea = ldc(g.lvl_eptr, l), en = ldc(g.lvl_eptr, l + 1) - ea;
            const int ra = ldc(g.lvl_ptr, l), rows = ldc(g.lvl_ptr, l + 1) - ra;
            if (tid < kF * rows) recB = g.lvl_rows[ra + tid / kF];
            for (int i = tid; i < kF * en; i += kT) {
                const int j = i / kF, f = i - j * kF;
                if (!((live >> f) & 1u)) continue;
                edge(f, s1, i == tid ? recA : g.lvl_edges[ea + j]);
            }
            __syncthreads();
            // phase B: thread = (row of the level, frame)
            if (l + 1 < g.nlev) {
                const int eb = ldc(g.lvl_eptr, l + 1);
                if (tid < kF * (ldc(g.lvl_eptr, l + 2) - eb)) recA = g.lvl_edges[eb + tid / kF];
            }
            for (int i = tid; i < kF * rows; i += kT) {
                const int j = i / kF, f = i - j * kF;
                if (!((live >> f) & 1u)) continue;
                row_fold(f, i == tid ? recB : g.lvl_rows[ra + j], ra + j);
            }
            __syncthreads();
        }
    };
    run_slots<kF, kT>(g, bits, iters, q, max_iter, p, load, sweep,
                      [&](int f, int v) { return (uint32_t)Xp(f)[v]; });
}

template <bool kMin, int kF, int kT>
__global__ __launch_bounds__(kT) void cbp_lds_kernel(SparseDev g, const float *__restrict__ llr,
                                                     uint8_t *__restrict__ bits, int32_t *__restrict__ iters,
                                                     int64_t nf, int max_iter, Params p, unsigned int *counter,
                                                     LdsItem it) {
    cbp_lds_body<kMin, kF, kT>(g, llr, bits, iters, LdsQueue{nullptr, nullptr, 0, nf, counter}, max_iter, p, it);
}

// Layered (kFlood false) and flooding BP, Sec. II-A / II-B, with the
// normalized min-sum (kMin) or the log-tanh check rule, in the same layout:
// the posterior Lambda [N] at 0, R [E], the fold states of one level's rows
// (the two smallest |Q| or the (max, rest) of g(|Q|), the parity in the
// first's sign bit; a row's state is used only within its level, so the
// array holds the largest level, indexed by a row's position in its level),
// the flooding C2V sums [N].  The decisions are Lambda's signs (whenever the
// syndrome is taken, Lambda holds the value the decision is defined on: the
// channel LLR, the value after a variable's last visit, or the flooding
// posterior), so no decision array is kept.  The same operations as the
// one-frame-per-lane kernel's row update (a fold pass, then a C2V pass), so
// the results agree bit for bit.  Layered BP runs three phases per level
// (see the sweep below).  Flooding BP keeps Lambda for the whole sweep, so
// per level:
//   phase B (thread = row of a frame): the row's V2C messages Q = Lambda - R
//            of the previous sweep folded in ascending column order into its
//            state, each one's check-rule term (with its sign) left in its
//            edge's R slot in place of the old C2V message;
//   phase C (thread = edge of a frame): the C2V message from the row's state
//            and that term (Lambda is fixed for the sweep, so this is the
//            term the lane kernel recomputes), then R and the variable's C2V
//            sum (rows containing a variable meet it in index order, level by
//            level, as row by row);
// and the sweep ends with the posterior L + sum and the decisions of every
// variable.
template <bool kFlood, bool kMin, int kF, int kT>
__device__ __forceinline__ void bp_lds_body(const SparseDev &g, const float *__restrict__ llr,
                                            uint8_t *__restrict__ bits, int32_t *__restrict__ iters,
                                            const LdsQueue &q, int max_iter, Params p, const LdsItem &it) {
    extern __shared__ uint4 s_dyn[];
    const int tid = tid_x();
    const float us = kMin ? 1.0f : kLog2e;  // log2 units for the log-tanh rule
    p.a *= us;
    p.lmax *= us;
    char *const base = reinterpret_cast<char *>(s_dyn);
    auto Lp = [&](int f) { return reinterpret_cast<float *>(base + f * it.bytes); };
    auto Rp = [&](int f) { return reinterpret_cast<float *>(base + f * it.bytes + it.r); };
    auto Sp = [&](int f) { return reinterpret_cast<float2 *>(base + f * it.bytes + it.om); };
    auto Ap = [&](int f) { return reinterpret_cast<float *>(base + f * it.bytes + it.acc); };

    // fold of row rr (position j in its level) of slot f (V2C, eq. equ_s2e3 /
    // equ_s2e10)
    auto row_fold = [&](int f, const int4 &rr, int j) {
        const float *Lam = Lp(f);
        float *R = Rp(f);
        float m1 = kMin ? __builtin_inff() : 0.0f, m2 = kMin ? __builtin_inff() : 0.0f;
        bool par = false;
        for (int c0 = rr.y; c0 < rr.z; c0 += kLdsChunk) {
            int col[kLdsChunk];
            float lv[kLdsChunk], rv[kLdsChunk];
#pragma unroll
            for (int c = 0; c < kLdsChunk; ++c) col[c] = g.col_idx[c0 + c];  // padded table
#pragma unroll
            for (int c = 0; c < kLdsChunk; ++c) {
                const int e = c0 + c < rr.z ? c0 + c : rr.z - 1;
                lv[c] = Lam[c0 + c < rr.z ? col[c] : 0];
                rv[c] = R[e];
            }
#pragma unroll
            for (int c = 0; c < kLdsChunk; ++c) {
                if (c0 + c < rr.z) {
                    const float q = lv[c] - rv[c];
                    float t;
                    if constexpr (kMin) {
                        t = __builtin_fminf(__builtin_fabsf(q), p.lmax);
                        m2 = __builtin_fminf(m2, __builtin_fmaxf(m1, t));
                        m1 = __builtin_fminf(m1, t);
                    } else {
                        t = phi2_clamped(q, p.a, p.lmax);
                        fold(m1, m2, t);
                    }
                    par ^= (q < 0.0f);
                    // the term, with q's sign, replaces the old C2V message (read
                    // just now; Lambda stays fixed for the sweep, so phase C needs
                    // only this term of q)
                    R[c0 + c] = with_sign(t, q < 0.0f);
                }
            }
        }
        Sp(f)[j] = make_float2(with_sign(m1, par), m2);
    };
    // flooding: C2V of the edge of record rec of slot f, its row at position
    // row of the level (eq. equ_s2e4 or the min-sum rule) from the term of its
    // V2C message that the row fold left in R, then R and the C2V sum
    auto edge = [&](int f, const int4 &rec, int row) {
        const int col = rec.x, e = rec.w & 0x3fffffff;
        float *R = Rp(f), *A = Ap(f);
        const float2 st = Sp(f)[row];
        const float m1 = abs_bits(st.x), m2 = st.y;
        const bool par = sign_bit(st.x);
        const float t = R[e];
        const float rn = kMin ? with_sign(p.alpha * ((abs_bits(t) == m1) ? m2 : m1), par ^ sign_bit(t))
                              : with_sign(phi2(excl_sum(m1, m2, abs_bits(t))), par ^ sign_bit(t));
        R[e] = rn;
        A[col] = A[col] + rn;
    };
    __shared__ int64_t sCur[kF];  // the slot's frame offset, for the flooding posterior
    auto load = [&](int f, int64_t fr) {
        float *Lam = Lp(f), *R = Rp(f);
        for (int v = tid; v < g.N; v += kT) {
            Lam[v] = llr[fr + v] * us;
            if constexpr (kFlood) Ap(f)[v] = 0.0f;
        }
        for (int e = tid; e < g.E; e += kT) R[e] = 0.0f;
        if (tid == 0) sCur[f] = fr;
    };
    // layered: three phases per level, all but the fold edge-parallel.
    //   A (edge): Q = Lambda - R kept in Lambda (no other row of the level
    //     reads it), its check-rule term in R (the old C2V is no longer needed);
    //   B (row):  the terms folded in column order into the row's state;
    //   C (edge): the C2V message from the state and the edge's own term (the
    //     same bits the one-frame-per-lane kernel recomputes), R, Lambda = Q + C2V.
    auto term_edge = [&](int f, const int4 &rec) {
        const int col = rec.x, e = rec.w & 0x3fffffff;
        float *Lam = Lp(f), *R = Rp(f);
        const float q = Lam[col] - R[e];  // V2C, eq. equ_s2e10
        Lam[col] = q;
        R[e] = with_sign(kMin ? __builtin_fminf(__builtin_fabsf(q), p.lmax) : phi2_clamped(q, p.a, p.lmax), q < 0.0f);
    };
    auto term_fold = [&](int f, const int4 &rr, int j) {
        const float *R = Rp(f);
        float m1 = kMin ? __builtin_inff() : 0.0f, m2 = kMin ? __builtin_inff() : 0.0f;
        bool par = false;
        for (int c0 = rr.y; c0 < rr.z; c0 += kLdsChunk) {
            float x[kLdsChunk];
#pragma unroll
            for (int c = 0; c < kLdsChunk; ++c) x[c] = R[c0 + c < rr.z ? c0 + c : rr.z - 1];
#pragma unroll
            for (int c = 0; c < kLdsChunk; ++c) {
                if (c0 + c < rr.z) {
                    par ^= sign_bit(x[c]);
                    const float ax = abs_bits(x[c]);
                    if constexpr (kMin) {
                        m2 = __builtin_fminf(m2, __builtin_fmaxf(m1, ax));
                        m1 = __builtin_fminf(m1, ax);
                    } else {
                        fold(m1, m2, ax);
                    }
                }
            }
        }
        Sp(f)[j] = make_float2(with_sign(m1, par), m2);
    };
    auto c2v_edge = [&](int f, const int4 &rec, int row) {
        const int col = rec.x, e = rec.w & 0x3fffffff;
        float *Lam = Lp(f), *R = Rp(f);
        const float2 st = Sp(f)[row];
        const float m1 = abs_bits(st.x), m2 = st.y;
        const bool par = sign_bit(st.x);
        const float q = Lam[col], t = abs_bits(R[e]);
        const float rn = kMin ? with_sign(p.alpha * ((t == m1) ? m2 : m1), par ^ (q < 0.0f))
                              : with_sign(phi2(excl_sum(m1, m2, t)), par ^ (q < 0.0f));  // eq. equ_s2e4
        R[e] = rn;
        Lam[col] = q + rn;  // eq. equ_s2e12; its sign after the last visit is the decision (eq. equ_s2e7)
    };
    auto sweep = [&](uint32_t live, uint32_t) {
        // A thread's first edge record of a level (and the edge's row) is read
        // at the start of the level before, its first row record at the start
        // of the level; layered BP keeps the edge record from phase A to C.
        int4 recE = make_int4(0, 0, 0, 0);
        int rowE = 0;
        {
            const int ea = ldc(g.lvl_eptr, 0);
            if (tid < kF * (ldc(g.lvl_eptr, 1) - ea)) {
                recE = g.lvl_edges[ea + tid / kF];
                rowE = g.lvl_erow[ea + tid / kF];
            }
        }
        for (int l = 0; l < g.nlev; ++l) {
            const int ea = ldc(g.lvl_eptr, l), en = ldc(g.lvl_eptr, l + 1) - ea;
            const int ra = ldc(g.lvl_ptr, l), rows = ldc(g.lvl_ptr, l + 1) - ra;
            int4 recR = make_int4(0, 0, 0, 0), nextE = make_int4(0, 0, 0, 0);
            int nextRow = 0;
            if (tid < kF * rows) recR = g.lvl_rows[ra + tid / kF];
            if (l + 1 < g.nlev && tid < kF * (ldc(g.lvl_eptr, l + 2) - (ea + en))) {
                nextE = g.lvl_edges[ea + en + tid / kF];
                nextRow = g.lvl_erow[ea + en + tid / kF];
            }
            if constexpr (!kFlood) {
                for (int i = tid; i < kF * en; i += kT) {
                    const int j = i / kF, f = i - j * kF;
                    if ((live >> f) & 1u) term_edge(f, i == tid ? recE : g.lvl_edges[ea + j]);
                }
                __syncthreads();
                for (int i = tid; i < kF * rows; i += kT) {
                    const int j = i / kF, f = i - j * kF;
                    if ((live >> f) & 1u) term_fold(f, i == tid ? recR : g.lvl_rows[ra + j], j);
                }
                __syncthreads();
                for (int i = tid; i < kF * en; i += kT) {
                    const int j = i / kF, f = i - j * kF;
                    if ((live >> f) & 1u)
                        c2v_edge(f, i == tid ? recE : g.lvl_edges[ea + j], i == tid ? rowE : g.lvl_erow[ea + j]);
                }
                __syncthreads();
            } else {
                for (int i = tid; i < kF * rows; i += kT) {
                    const int j = i / kF, f = i - j * kF;
                    if ((live >> f) & 1u) row_fold(f, i == tid ? recR : g.lvl_rows[ra + j], j);
                }
                __syncthreads();
                for (int i = tid; i < kF * en; i += kT) {
                    const int j = i / kF, f = i - j * kF;
                    if ((live >> f) & 1u)
                        edge(f, i == tid ? recE : g.lvl_edges[ea + j], i == tid ? rowE : g.lvl_erow[ea + j]);
                }
                __syncthreads();
            }
            recE = nextE;
            rowE = nextRow;
        }
        if constexpr (kFlood) {  // eq. equ_s2e6 (its sign is the decision, eq. equ_s2e7)
            for (int f = 0; f < kF; ++f) {
                if (!((live >> f) & 1u)) continue;
                const int64_t fr = sCur[f];
                float *Lam = Lp(f), *A = Ap(f);
                for (int v = tid; v < g.N; v += kT) {
                    Lam[v] = flood_posterior(llr[fr + v], us, A[v]);
                    A[v] = 0.0f;
                }
            }
        }
    };
    run_slots<kF, kT>(g, bits, iters, q, max_iter, p, load, sweep,
                      [&](int f, int v) { return (uint32_t)(Lp(f)[v] < 0.0f); });
}

template <bool kFlood, bool kMin, int kF, int kT>
__global__ __launch_bounds__(kT) void bp_lds_kernel(SparseDev g, const float *__restrict__ llr,
                                                    uint8_t *__restrict__ bits, int32_t *__restrict__ iters,
                                                    int64_t nf, int max_iter, Params p, unsigned int *counter,
                                                    LdsItem it) {
    bp_lds_body<kFlood, kMin, kF, kT>(g, llr, bits, iters, LdsQueue{nullptr, nullptr, 0, nf, counter}, max_iter, p,
                                      it);
}

// Element i of a device array of structs that no launch writes, read with
// scalar loads (the index is workgroup-uniform).
template <class T>
__device__ __forceinline__ T ldc_struct(const T *p, int64_t i) {
    static_assert(sizeof(T) % 4 == 0, "read as words");
    T out;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(p + i);
    uint32_t *dst = reinterpret_cast<uint32_t *>(&out);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = ldc(src, k);
    return out;
}

// Mixed batches: every code c with frames[c] > 0 frames per workgroup (the
// codes whose frame fits the launch's LDS) is decoded from its queue (frames
// perm[qstart[c] .. qstart[c + 1]), claimed through counter[c]); a workgroup
// starts at code (its index mod ncodes) and moves on once that code's queue
// is exhausted and its slots have stopped.  Codes with frames[c] = 0 are
// left to the streamed kernel, which runs beside this one and finds the
// others' queues exhausted.
template <int kAlgo, int kT>
__global__ __launch_bounds__(kT) void mix_lds_kernel(const SparseDev *codes, const LdsItem *items,
                                                     const int *frames, int ncodes, const float *__restrict__ llr,
                                                     uint8_t *__restrict__ bits, int32_t *__restrict__ iters,
                                                     const int64_t *qstart, const int32_t *perm,
                                                     const int64_t *offset, unsigned int *counter, int max_iter,
                                                     Params p) {
    for (int ci = 0; ci < ncodes; ++ci) {
        const int c = (gid_x() + ci) % ncodes;
        const int F = ldc(frames, c);
        if (F == 0) continue;
        const SparseDev g = ldc_struct(codes, c);
        const LdsItem it = ldc_struct(items, c);
        const LdsQueue q{perm, offset, ldc(qstart, c), ldc(qstart, c + 1) - ldc(qstart, c), counter + c};
        auto go = [&](auto fc) {
            constexpr int kF = decltype(fc)::value;
            if constexpr (kAlgo == kCBP || kAlgo == kCBPNMS)
                cbp_lds_body<kAlgo == kCBPNMS, kF, kT>(g, llr, bits, iters, q, max_iter, p, it);
            else
                bp_lds_body<kAlgo == kFBPNMS || kAlgo == kFBP, kAlgo == kLBPNMS || kAlgo == kFBPNMS, kF, kT>(
                    g, llr, bits, iters, q, max_iter, p, it);
        };
        if (F >= 8) go(std::integral_constant<int, 8>{});
        else if (F >= 4) go(std::integral_constant<int, 4>{});
        else if (F >= 2) go(std::integral_constant<int, 2>{});
        else go(std::integral_constant<int, 1>{});
    }
}

template <class K>
hipError_t launch_k(K *k, int groups, int threads, size_t lds, hipStream_t s, const SparseDev &g, const float *llr,
                    uint8_t *bits, int32_t *iters, int64_t nf, int max_iter, const Params &p, unsigned int *counter,
                    const LdsItem &it) {
    if (lds > (64u << 10)) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, dim3((unsigned)groups), dim3(threads), lds, s, g, llr, bits, iters, nf, max_iter, p,
                       counter, it);
    return hipGetLastError();
}

// The kernel of algo for kF frames of kT threads.
template <int kF, int kT>
hipError_t launch_algo(int algo, int groups, size_t lds, hipStream_t s, const SparseDev &g, const float *llr,
                       uint8_t *bits, int32_t *iters, int64_t nf, int max_iter, const Params &p,
                       unsigned int *counter, const LdsItem &it) {
#define CBP_LDS_GO(KERNEL) return launch_k(KERNEL, groups, kT, lds, s, g, llr, bits, iters, nf, max_iter, p, counter, it)
    switch (algo) {
    case kCBP: CBP_LDS_GO((cbp_lds_kernel<false, kF, kT>));
    case kCBPNMS: CBP_LDS_GO((cbp_lds_kernel<true, kF, kT>));
    case kLBP: CBP_LDS_GO((bp_lds_kernel<false, false, kF, kT>));
    case kLBPNMS: CBP_LDS_GO((bp_lds_kernel<false, true, kF, kT>));
    case kFBP: CBP_LDS_GO((bp_lds_kernel<true, false, kF, kT>));
    case kFBPNMS: CBP_LDS_GO((bp_lds_kernel<true, true, kF, kT>));
    default: return hipErrorInvalidValue;
    }
#undef CBP_LDS_GO
}

int64_t align16(int64_t x) { return (x + 15) / 16 * 16; }

}  // namespace

LdsItem lds_item(int algo, const SparseDev &g) {
    LdsItem it{};
    if (algo < kCBP || algo > kFBP) return it;  // bytes = 0: not available
    const bool flood = algo == kFBP || algo == kFBPNMS, bp = algo != kCBP && algo != kCBPNMS;
    if (bp && g.M > 0 && g.lvl_maxrows < 1) return it;
    const int64_t q = align16(4 * (int64_t)g.N), r = align16(4 * (int64_t)g.E),
                  om = align16(8 * (int64_t)(bp ? g.lvl_maxrows : g.M)), acc = flood ? q : 0,
                  xb = bp ? 0 : align16(g.N);
    const int64_t total = q + r + om + acc + xb;
    if (total >= ((int64_t)1 << 31)) return it;
    it.r = (int)q;
    it.om = (int)(q + r);
    it.acc = flood ? (int)(q + r + om) : 0;
    it.xb = (int)(q + r + om + acc);
    it.bytes = (int)total;
    return it;
}

int lds_frames(const LdsItem &it, int64_t lds_limit) {
    if (it.bytes <= 0) return 0;
    const int64_t f = (lds_limit - kLdsStaticBytes) / it.bytes;
    return (int)(f < kLdsMaxFrames ? f : kLdsMaxFrames);
}

// Geometry: frames per CU that fit (LDS per CU = the per-workgroup maximum on
// gfx950).  Four or more: workgroups of 512 threads, four per CU, each with
// its share of the frames (1, 2, 4 or 8); two or three: one frame per
// workgroup of 512 threads; one: one workgroup of 1024 threads.
// CBP_SPARSE_LDS_FRAMES in the environment caps the frames per workgroup.
hipError_t launch_sparse_lds(int algo, const SparseDev &g, const float *llr, uint8_t *bits, int32_t *iters,
                             int64_t nf, int max_iter, const Params &p, unsigned int *counter, int device,
                             hipStream_t s) {
    const LdsItem it = lds_item(algo, g);
    int lim = 0, cus = 0;
    hipError_t e = hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    if (it.bytes <= 0 || cus < 1) return hipErrorInvalidValue;
    const int64_t per_cu_frames = ((int64_t)lim - 4 * kLdsStaticBytes) / it.bytes;
    if (per_cu_frames < 1 || lds_frames(it, lim) < 1) return hipErrorInvalidValue;
    int F = per_cu_frames >= 4 ? (int)(per_cu_frames / 4) : 1;
    if (F > kLdsMaxFrames) F = kLdsMaxFrames;
    if (const char *v = std::getenv("CBP_SPARSE_LDS_FRAMES")) {
        const int cap = std::atoi(v);
        if (cap >= 1 && cap < F) F = cap;
    }
    // small batches: fewer frames per workgroup, more workgroups
    const int64_t spread = (nf + cus - 1) / cus;
    if (spread < F) F = (int)(spread < 1 ? 1 : spread);
    F = F >= 8 ? 8 : F >= 4 ? 4 : F >= 2 ? 2 : 1;  // the compiled widths
    const int T = per_cu_frames == 1 ? 1024 : 512;
    const int64_t by_lds = (int64_t)lim / ((int64_t)F * it.bytes + kLdsStaticBytes);
    const int64_t by_threads = kLdsCuThreads / T;
    const int64_t per_cu = by_lds < 1 ? 1 : (by_lds < by_threads ? by_lds : by_threads);
    const int64_t need = (nf + F - 1) / F;
    const int groups = (int)(need < per_cu * cus ? need : per_cu * cus);
    const size_t lds = (size_t)F * (size_t)it.bytes;
    hipLaunchKernelGGL(lds_zero_kernel, dim3(1), dim3(kLdsFillBlock), 0, s, counter);
    if (T == 1024) return launch_algo<1, 1024>(algo, groups, lds, s, g, llr, bits, iters, nf, max_iter, p, counter, it);
    switch (F) {
    case 8: return launch_algo<8, 512>(algo, groups, lds, s, g, llr, bits, iters, nf, max_iter, p, counter, it);
    case 4: return launch_algo<4, 512>(algo, groups, lds, s, g, llr, bits, iters, nf, max_iter, p, counter, it);
    case 2: return launch_algo<2, 512>(algo, groups, lds, s, g, llr, bits, iters, nf, max_iter, p, counter, it);
    default: return launch_algo<1, 512>(algo, groups, lds, s, g, llr, bits, iters, nf, max_iter, p, counter, it);
    }
}

namespace {
__global__ __launch_bounds__(kLdsFillBlock) void mix_exhaust_kernel(const int *frames, const int64_t *qstart,
                                                                    int ncodes, unsigned int *counter) {
    for (int c = tid_x(); c < ncodes; c += kLdsFillBlock)
        counter[c] = frames[c] > 0 ? (unsigned int)(qstart[c + 1] - qstart[c]) : 0u;
}
}  // namespace

hipError_t launch_mix_exhaust(const int *frames, const int64_t *qstart, int ncodes, unsigned int *counter,
                              hipStream_t s) {
    hipLaunchKernelGGL(mix_exhaust_kernel, dim3(1), dim3(kLdsFillBlock), 0, s, frames, qstart, ncodes, counter);
    return hipGetLastError();
}

hipError_t prepare_mix_lds(int algo, size_t lds) {
    auto go = [&](auto *k) {
        if (lds <= (64u << 10)) return hipSuccess;
        return hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds);
    };
    switch (algo) {
    case kCBP: return go(mix_lds_kernel<kCBP, kLdsMixThreads>);
    case kCBPNMS: return go(mix_lds_kernel<kCBPNMS, kLdsMixThreads>);
    case kLBPNMS: return go(mix_lds_kernel<kLBPNMS, kLdsMixThreads>);
    case kFBPNMS: return go(mix_lds_kernel<kFBPNMS, kLdsMixThreads>);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_mix_lds(int algo, const SparseDev *codes, const LdsItem *items, const int *frames, int ncodes,
                          int groups, size_t lds, const float *llr, uint8_t *bits, int32_t *iters,
                          const int64_t *qstart, const int32_t *perm, const int64_t *offset, unsigned int *counter,
                          int max_iter, const Params &p, hipStream_t s) {
    auto go = [&](auto *k) {
        hipLaunchKernelGGL(k, dim3((unsigned)groups), dim3(kLdsMixThreads), lds, s, codes, items, frames, ncodes, llr,
                           bits, iters, qstart, perm, offset, counter, max_iter, p);
        return hipGetLastError();
    };
    switch (algo) {
    case kCBP: return go(mix_lds_kernel<kCBP, kLdsMixThreads>);
    case kCBPNMS: return go(mix_lds_kernel<kCBPNMS, kLdsMixThreads>);
    case kLBPNMS: return go(mix_lds_kernel<kLBPNMS, kLdsMixThreads>);
    case kFBPNMS: return go(mix_lds_kernel<kFBPNMS, kLdsMixThreads>);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace cbp
