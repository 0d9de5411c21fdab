// One frame per lane, any parity-check matrix (CSR).
//
// Every lane of a wave runs the whole sweep of its own frame in the paper's
// row order; since all lanes share the code, the row/edge loops and the table
// reads are wave-uniform (scalar loads through the constant address space)
// and the per-frame state is stored
// frame-interleaved (index-major, frame-minor) so that each access of a wave
// is one contiguous 256-byte line.  The grid is persistent: a lane owns one
// state slot and takes the next frame of the batch from a global counter as
// soon as its frame stops, so a slow frame holds up only its own lane; the
// wave leaves its loop once the batch is exhausted and every lane is done.
#include "internal.hpp"
#include "phi.hpp"
#include "sparse_rules.hpp"

namespace cbp {
namespace {

constexpr int kWave = 64;
constexpr int kChunk = 8;  // edges of a row whose loads are issued together
constexpr int kLevelThreads = 256;  // threads per frame in the level-parallel kernels
constexpr int kSyndromeBlock = 256;
constexpr int kFillBlock = 256;

// Element (index, lane) of an array of a wave's state block: 32-bit index
// arithmetic (a block stays below 2 GiB, checked at launch).
__device__ __forceinline__ uint32_t at(int idx, uint32_t lane) { return (uint32_t)idx * (uint32_t)kWave + lane; }

// Edges in chunks of kChunk: the chunk's column indices are read
// unconditionally (the table is padded) so the scalar loads go out together,
// then its decision bytes.
__device__ bool lane_syndrome_ok(const SparseDev &g, const uint8_t *xb, uint32_t lf) {
    uint32_t bad = 0;
    for (int i = 0; i < g.M; ++i) {
        uint32_t p = 0;
        const int e1 = ldc(g.row_ptr, i + 1);
        for (int c0 = ldc(g.row_ptr, i); c0 < e1; c0 += kChunk) {
            int col[kChunk];
#pragma unroll
            for (int k = 0; k < kChunk; ++k) col[k] = ldc(g.col_idx, c0 + k);
#pragma unroll
            for (int k = 0; k < kChunk; ++k)
                if (c0 + k < e1) p ^= xb[at(col[k], lf)];
        }
        bad |= p;
    }
    return bad == 0;
}

__device__ void write_out(const SparseDev &g, const uint8_t *xb, uint32_t lf,
                          uint8_t *bits, int32_t *iters, int64_t f, int t) {
    for (int v = 0; v < g.N; ++v) bits[f * g.N + v] = xb[at(v, lf)];
    iters[f] = t;
}

// This wave's block of the workspace.
__device__ __forceinline__ SparseWs wave_block(SparseWs w) {
    const int64_t off = (int64_t)gid_x() * w.block_bytes;
    auto at = [off](auto *p) { return p ? (decltype(p))((char *)p + off) : p; };
    w.a0 = at(w.a0);
    w.a1 = at(w.a1);
    w.a2 = at(w.a2);
    w.a3 = at(w.a3);
    w.a4 = at(w.a4);
    w.xb = at(w.xb);
    return w;
}

// The next frame index for every lane in `want` (a wave-uniform ballot): the
// leader adds the number of wanting lanes to the batch's frame counter, then
// each wanting lane takes base + (wanting lanes below it).  Values of other
// lanes are undefined.
__device__ __forceinline__ int64_t claim_frames(unsigned long long *counter, uint64_t want) {
    const int leader = __builtin_ctzll(want);
    // every active lane executes the atomic (the leader adds the count, the
    // others 0), so the leader's result is not behind a branch
    const unsigned long long base =
        atomicAdd(counter, tid_x() == leader ? (unsigned long long)__builtin_popcountll(want) : 0ull);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)base, leader);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(base >> 32), leader);
    const uint64_t below = want & ((1ull << tid_x()) - 1ull);
    return (int64_t)((((uint64_t)hi << 32) | lo) + (uint64_t)__builtin_popcountll(below));
}

// --------------------------------------------------------------------------
// CBP.  ws: a0 = Q[N] (latest V2C), a2 = R[E], a3 = Om[M] as float2 (max phi2
// term with the parity in its sign bit, rest of the phi2 sum), xb = hard
// decisions [N].  The phi2 term of Q_v that v's latest check folded is not
// stored: Q_v is still that V2C value, and phi2 of it is recomputed bit for
// bit (8 bytes per edge-update less state traffic).  The log-tanh rule keeps
// LLRs in log2 units (L / ln2), where phi2 serves both directions of the
// check rule; Params a and lmax arrive already scaled.
// --------------------------------------------------------------------------

template <bool kMin>
__device__ float cbp_flushed(const SparseDev &g, const SparseWs &w, uint32_t lf, int v, const Params &p) {
    const int e = ldc(g.last_edge, v);
    const int j = ldc(g.edge_row, e);
    const float q = w.a0[at(v, lf)];
    const float2 om = reinterpret_cast<const float2 *>(w.a3)[at(j, lf)];
    return q + b2v<kMin>(om.x, om.y, q, p);
}

// Flushed posterior after a stop in the middle of sweep t, right after row
// istop: v's latest check is its last row <= istop in this sweep, else (t > 1)
// its last row of the previous sweep, else none (B2V 0).  The column's edges
// are walked backwards from its last edge through pred_edge.
template <bool kMin>
__device__ float cbp_flushed_at(const SparseDev &g, const SparseWs &w, uint32_t lf, int v, const Params &p,
                                int istop, int t) {
    const float q = w.a0[at(v, lf)];
    int e = ldc(g.last_edge, v);
    while (ldc(g.edge_row, e) > istop) {
        if (ldc_u8(g.first, e) & kFirstVisit) {  // no visit of v yet in this sweep
            if (t == 1) return q;
            e = ldc(g.last_edge, v);
            break;
        }
        e = ldc(g.pred_edge, e);
    }
    const int j = ldc(g.edge_row, e);
    const float2 om = reinterpret_cast<const float2 *>(w.a3)[at(j, lf)];
    return q + b2v<kMin>(om.x, om.y, q, p);
}

// Entry r of the level-ordered row table: (row, first edge, end edge, 0).
__device__ __forceinline__ int4 level_row(const SparseDev &g, int r) {
    const int *q = reinterpret_cast<const int *>(g.lvl_rows) + 4 * (int64_t)r;
    return make_int4(ldc(q, 0), ldc(q, 1), ldc(q, 2), 0);
}

// Element idx of a state array whose frames are kStride apart: kStride = 64
// for lane lf of a wave's frame-interleaved block, 1 (lf = 0) for one frame's
// contiguous copy.
template <int kStride>
__device__ __forceinline__ uint32_t ix(int idx, uint32_t lf) {
    return (uint32_t)idx * (uint32_t)kStride + lf;
}

struct CbpState {
    float *Q, *R;
    float2 *Om;
    uint8_t *xb;
};

// One check-node update of CBP on one frame: Step 2(1) a-e for each edge of
// row i (edges e0 .. e1-1) in ascending column order, then Step 2(2).  Returns the sign parity of
// the new belief; with stop_rule 1 ors into flip whether a decision changed.
// sweep1: first sweep, where a first-visit edge has no latest check yet.
template <bool kMin, int kStride>
__device__ __forceinline__ bool cbp_row(const SparseDev &g, int i, int e0, int e1, bool sweep1, const CbpState &st,
                                        uint32_t lf, const Params &p, bool &flip) {
    float *Q = st.Q, *R = st.R;
    uint8_t *xb = st.xb;
    // decisions are stored at a variable's last visit of the sweep (the one
    // Step 3 reads), or at every visit for the paper's stopping rule
    const bool every = p.stop_rule == 1;
    float Mx = kMin ? __builtin_inff() : 0.0f, Sr = kMin ? __builtin_inff() : 0.0f;
    bool par = false;
    // The row's edges in chunks of kChunk: every load of a chunk is issued
    // before its first store, so a chunk costs one memory round trip instead
    // of one per edge.  Within a row the columns differ, so no load of a chunk
    // reads what an earlier edge of the same chunk stores, except R(c_i -> v)
    // when v's latest check is c_i itself (a column of weight one): that
    // commit is forwarded in registers.
    for (int c0 = e0; c0 < e1; c0 += kChunk) {
        const int n = e1 - c0 < kChunk ? e1 - c0 : kChunk;
        // the chunk's table entries, unconditionally (padded tables)
        int col[kChunk], pe[kChunk], pr[kChunk];
        uint32_t fi[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
            col[k] = ldc(g.col_idx, c0 + k);
            pe[k] = ldc(g.pred_edge, c0 + k);
            pr[k] = ldc(g.pred_row, c0 + k);
            fi[k] = ldc_u8(g.first, c0 + k);
        }
        float q[kChunk], r[kChunk];
        float2 om[kChunk];
        uint8_t x0[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
            if (k < n) {
                const uint32_t iv = ix<kStride>(col[k], lf);
                q[k] = Q[iv];
                if (!(sweep1 && (fi[k] & kFirstVisit))) om[k] = st.Om[ix<kStride>(pr[k], lf)];
                r[k] = R[ix<kStride>(c0 + k, lf)];
                if (p.stop_rule == 1) x0[k] = xb[iv];
            }
        }
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
            if (k < n) {
                const int e = c0 + k;
                const uint32_t iv = ix<kStride>(col[k], lf);
                float rn = 0.0f, rc = r[k];
                if (!(sweep1 && (fi[k] & kFirstVisit))) {
                    // B2V (eq. equ_s4e18): C2V of the latest check c_j recovered
                    // from its belief, then committed to R(c_j -> v) first.
                    rn = b2v<kMin>(om[k].x, om[k].y, q[k], p);
                    R[ix<kStride>(pe[k], lf)] = rn;
                    if (pe[k] == e) rc = rn;
                }
                const float lam = q[k] + rn;              // eq. equ_s4e20
                const uint8_t nx = lam < 0.0f;            // eq. equ_s2e7
                if (p.stop_rule == 1) flip |= nx != x0[k];
                if (every || (fi[k] & kLastVisit)) xb[iv] = nx;
                const float qn = lam - rc;                // V2C, eq. equ_s4e19
                Q[iv] = qn;
                if constexpr (!kMin) {
                    fold(Mx, Sr, phi2_clamped(qn, p.a, p.lmax));  // C2B, eq. equ_s4e21
                } else {                                  // eq. equ_s4e21xx
                    const float aq = __builtin_fminf(__builtin_fabsf(qn), p.lmax);
                    Sr = __builtin_fminf(Sr, __builtin_fmaxf(Mx, aq));
                    Mx = __builtin_fminf(Mx, aq);
                }
                par ^= (qn < 0.0f);
            }
        }
    }
    st.Om[ix<kStride>(i, lf)] = make_float2(with_sign(Mx, par), Sr);  // eq. equ_s4e23
    return par;
}

// Rows of one level handled together by the one-frame-per-lane kernel.
#ifndef CBP_SPARSE_ROWS
#define CBP_SPARSE_ROWS 4
#endif
constexpr int kRows = CBP_SPARSE_ROWS;
// Rows of a level updated together by the layered / flooding lane kernels
// (1: row by row in index order).  Measured on the PEG codes, n = 8192:
// flooding BP 951 ms row by row, 818 with 2, 738 with 4; layered BP 357 ms
// row by row, 452 with 2, 423 with 4 (level order scatters its R accesses,
// which index order walks contiguously, and it moves fewer bytes per edge to
// save on).
#ifndef CBP_SPARSE_ROWS_LAYERED
#define CBP_SPARSE_ROWS_LAYERED 1
#endif
#ifndef CBP_SPARSE_ROWS_FLOOD
#define CBP_SPARSE_ROWS_FLOOD 4
#endif
template <bool kFlood>
constexpr int kRowsBp() {
    return kFlood ? CBP_SPARSE_ROWS_FLOOD : CBP_SPARSE_ROWS_LAYERED;
}

// nr (<= kRows) rows of one level, each of at most kChunk edges, on the lane's
// frame: the same Step 2(1)-(2) updates as cbp_row, with every load of all
// the rows issued before any store.  Rows of a level share no variable, so no
// row reads what another stores (its Q, decisions and R slots are its own
// columns', and the beliefs it reads are of rows holding its variables, which
// are in other levels): nr rows cost one memory round trip instead of nr.
// Syndrome stopping only (decisions at last visits).
template <bool kMin>
__device__ __forceinline__ void cbp_level_rows(const SparseDev &g, const int4 (&rr)[kRows], int nr, bool sweep1,
                                               const CbpState &st, uint32_t lf, const Params &p) {
    float *Q = st.Q, *R = st.R;
    uint8_t *xb = st.xb;
    int col[kRows][kChunk], pe[kRows][kChunk], pr[kRows][kChunk];
    uint32_t fi[kRows][kChunk];
    float q[kRows][kChunk], r[kRows][kChunk];
    float2 om[kRows][kChunk];
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
        if (j < nr) {
#pragma unroll
            for (int k = 0; k < kChunk; ++k) {  // unconditionally (padded tables)
                col[j][k] = ldc(g.col_idx, rr[j].y + k);
                pe[j][k] = ldc(g.pred_edge, rr[j].y + k);
                pr[j][k] = ldc(g.pred_row, rr[j].y + k);
                fi[j][k] = ldc_u8(g.first, rr[j].y + k);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
        if (j < nr) {
            const int n = rr[j].z - rr[j].y;
#pragma unroll
            for (int k = 0; k < kChunk; ++k) {
                if (k < n) {
                    const uint32_t iv = at(col[j][k], lf);
                    q[j][k] = Q[iv];
                    if (!(sweep1 && (fi[j][k] & kFirstVisit))) om[j][k] = st.Om[at(pr[j][k], lf)];
                    r[j][k] = R[at(rr[j].y + k, lf)];
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
        if (j < nr) {
            const int n = rr[j].z - rr[j].y;
            float Mx = kMin ? __builtin_inff() : 0.0f, Sr = kMin ? __builtin_inff() : 0.0f;
            bool par = false;
#pragma unroll
            for (int k = 0; k < kChunk; ++k) {
                if (k < n) {
                    const int e = rr[j].y + k;
                    const uint32_t iv = at(col[j][k], lf);
                    float rn = 0.0f, rc = r[j][k];
                    if (!(sweep1 && (fi[j][k] & kFirstVisit))) {
                        rn = b2v<kMin>(om[j][k].x, om[j][k].y, q[j][k], p);  // eq. equ_s4e18
                        R[at(pe[j][k], lf)] = rn;
                        if (pe[j][k] == e) rc = rn;
                    }
                    const float lam = q[j][k] + rn;   // eq. equ_s4e20
                    if (fi[j][k] & kLastVisit) xb[iv] = lam < 0.0f;
                    const float qn = lam - rc;        // eq. equ_s4e19
                    Q[iv] = qn;
                    if constexpr (!kMin) {
                        fold(Mx, Sr, phi2_clamped(qn, p.a, p.lmax));  // eq. equ_s4e21
                    } else {
                        const float aq = __builtin_fminf(__builtin_fabsf(qn), p.lmax);
                        Sr = __builtin_fminf(Sr, __builtin_fmaxf(Mx, aq));
                        Mx = __builtin_fminf(Mx, aq);
                    }
                    par ^= (qn < 0.0f);
                }
            }
            st.Om[at(rr[j].x, lf)] = make_float2(with_sign(Mx, par), Sr);  // eq. equ_s4e23
        }
    }
}

// Hand-off of slow frames.  Once the batch is exhausted and a wave has only a
// few busy lanes left, their frames are copied, by the wave's active lanes, to
// contiguous items of h (while items are free) and finished by the
// level-parallel kernel.  An item: (frame, sweeps done) in h.items and the
// frame's state in h.state.
__device__ __forceinline__ char *item_base(const Handoff &h, uint32_t k) {
    return h.state + (int64_t)k * h.item_bytes;
}

__device__ __forceinline__ CbpState cbp_state(const SparseWs &w) {
    return CbpState{w.a0, w.a2, reinterpret_cast<float2 *>(w.a3), w.xb};
}

__device__ __forceinline__ CbpState cbp_layout(const SparseDev &g, char *b) {
    CbpState st;
    const int64_t n4 = round256(4 * (int64_t)g.N), e4 = round256(4 * (int64_t)g.E), m8 = round256(8 * (int64_t)g.M);
    st.Q = (float *)b;
    st.R = (float *)(b + n4);
    st.Om = (float2 *)(b + n4 + e4);
    st.xb = (uint8_t *)(b + n4 + e4 + m8);
    return st;
}

__device__ __forceinline__ CbpState cbp_item(const SparseDev &g, const Handoff &h, uint32_t k) {
    return cbp_layout(g, item_base(h, k));
}

// Copy of item k's state in LDS (the whole item, 16 bytes per thread and
// step), for the level-parallel kernels when a frame's state fits: their row
// accesses are scattered and each level pass waits on them, so LDS latency
// instead of cache latency shortens every pass.  The barrier in front keeps
// the previous item's readers ahead of the copy.
__device__ __forceinline__ char *stage_item(const Handoff &h, uint32_t k, uint4 *lds) {
    __syncthreads();
    const uint4 *src = reinterpret_cast<const uint4 *>(item_base(h, k));
    for (int64_t i = tid_x(); i < h.item_bytes / 16; i += kLevelThreads) lds[i] = src[i];
    __syncthreads();
    return reinterpret_cast<char *>(lds);
}

// The active lanes of the wave (rank r of na) copy lane d's slot
// (frame-interleaved) into item k (contiguous).
template <class T>
__device__ __forceinline__ void copy_slot(T *dst, const T *src, int n, uint32_t d, int r, int na) {
#pragma unroll 4
    for (int idx = r; idx < n; idx += na) dst[idx] = src[at(idx, d)];
}

// Rank of this lane among the active lanes, and their number.
__device__ __forceinline__ void active_rank(int &r, int &na) {
    const uint64_t act = __ballot(1);
    r = __builtin_popcountll(act & ((1ull << tid_x()) - 1ull));
    na = __builtin_popcountll(act);
}

// Unfinished frames of the lanes in `hand` (wave-uniform ballot) go to their
// items hk; each such lane then asks for a new frame.
__device__ __forceinline__ void hand_over_cbp(const SparseDev &g, const Handoff &h, const CbpState &w,
                                              uint64_t hand, uint32_t hk, int64_t f, int t) {
    for (uint64_t m = hand; m != 0; m &= m - 1) {
        const int d = __builtin_ctzll(m);
        const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)hk, d);
        const int fd = __builtin_amdgcn_readlane((int)f, d);
        const int td = __builtin_amdgcn_readlane(t, d);
        const CbpState it = cbp_item(g, h, k);
        int r, na;
        active_rank(r, na);
        copy_slot(it.Q, w.Q, g.N, d, r, na);
        copy_slot(it.xb, w.xb, g.N, d, r, na);
        copy_slot(it.R, w.R, g.E, d, r, na);
        copy_slot(it.Om, w.Om, g.M, d, r, na);
        if (r == 0) h.items[k] = make_int2(fd, td);
    }
}

// Whether this wave hands its frames over now: every frame of the batch has
// been taken and at most h.lanes of its lanes are still busy (each such lane
// then works alone for a whole sweep at a time).  Each busy lane claims an
// item; hand = a free item was left for it (hk), else its frame stays.
__device__ __forceinline__ bool handing_off(const Handoff &h, unsigned long long *counter, int64_t nf, bool busy,
                                            bool &hand, uint32_t &hk) {
    const uint64_t bm = __ballot(busy);
    if (bm == 0 || __builtin_popcountll(bm) > h.lanes) return false;
    const unsigned long long taken = __hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__builtin_amdgcn_readfirstlane((int)(taken < (unsigned long long)nf))) return false;
    // every active lane executes the atomic (lanes that are not busy add 0)
    hk = atomicAdd(h.count, busy ? 1u : 0u);
    hand = busy && hk < h.cap;
    return __ballot(hand) != 0;
}

// kMin: the normalized min-sum check rule (Om = (min1 | parity, min2)).
template <bool kMin>
__global__ __launch_bounds__(kWave) void cbp_sparse_kernel(
    SparseDev g, const float *__restrict__ llr, uint8_t *__restrict__ bits,
    int32_t *__restrict__ iters, int64_t nf, int max_iter, Params p, SparseWs w, Dump d,
    unsigned long long *counter, Handoff h) {
    w = wave_block(w);
    const uint32_t lf = tid_x();  // this lane's slot in its wave's block
    const CbpState st = cbp_state(w);
    float *Q = w.a0, *R = w.a2;
    const float2 *Om = st.Om;
    const float us = kMin ? 1.0f : kLog2e;  // log2 units for the log-tanh rule
    const float un = kMin ? 1.0f : kLn2;    // dumps in natural units
    p.a *= us;
    p.lmax *= us;
    uint8_t *xb = w.xb;
    int64_t f = 0;  // the lane's frame
    int t = 0;      // sweeps done on it
    bool need = true, done = false;
    // paper's stopping rule (stop_rule 1): check updates in a row, across
    // sweeps, whose belief is positive and that flipped no decision
    int64_t run = 0;
    for (;;) {
        for (uint64_t want = __ballot(need); want != 0; want = __ballot(need)) {
            const int64_t fn = claim_frames(counter, want);
            if (need) {
                need = false;
                f = fn;
                if (f >= nf) {
                    done = true;
                } else {
                    // Step 1: latest V2C = channel LLR, R = 0, x = [L < 0]
                    for (int v = 0; v < g.N; ++v) {
                        const float l = llr[f * g.N + v] * us;
                        Q[at(v, lf)] = l;
                        xb[at(v, lf)] = l < 0.0f;
                    }
                    for (int e = 0; e < g.E; ++e) R[at(e, lf)] = 0.0f;
                    t = 0;
                    run = 0;
                    if (max_iter == 0 || (p.stop_rule == 0 && lane_syndrome_ok(g, xb, lf))) {
                        write_out(g, xb, lf, bits, iters, f, 0);
                        need = true;
                    }
                }
            }
        }
        if (__ballot(!done) == 0) break;
        bool hand = false;
        uint32_t hk = 0;
        if (!done) {
            ++t;
            // Step 2: check-nodes in index order; with the syndrome stop, level by
            // level (the same result bit for bit), kRows rows of a level at a time
            bool paper_stop = false;
            int istop = 0;
            if (p.stop_rule == 1) {
                for (int i = 0; i < g.M; ++i) {
                    bool flip = false;
                    const bool par = cbp_row<kMin, kWave>(g, i, ldc(g.row_ptr, i), ldc(g.row_ptr, i + 1), t == 1, st,
                                                          lf, p, flip);
                    // Step 2(3): M updates in a row with Omega > 0, no flip
                    run = (!par && !flip) ? run + 1 : 0;
                    if (run >= g.M) {
                        paper_stop = true;
                        istop = i;
                        break;
                    }
                }
            } else {
                for (int l = 0; l < g.nlev; ++l) {
                    const int r1 = ldc(g.lvl_ptr, l + 1);
                    for (int r = ldc(g.lvl_ptr, l); r < r1; r += kRows) {
                        const int nr = r1 - r < kRows ? r1 - r : kRows;
                        int4 rr[kRows];
                        bool narrow = true;
#pragma unroll
                        for (int j = 0; j < kRows; ++j) {
                            rr[j] = level_row(g, j < nr ? r + j : r);
                            narrow &= rr[j].z - rr[j].y <= kChunk;
                        }
                        if (narrow) {
                            cbp_level_rows<kMin>(g, rr, nr, t == 1, st, lf, p);
                        } else {
                            for (int j = 0; j < nr; ++j) {
                                bool flip = false;
                                (void)cbp_row<kMin, kWave>(g, rr[j].x, rr[j].y, rr[j].z, t == 1, st, lf, p, flip);
                            }
                        }
                    }
                }
            }
            if (paper_stop) {
                if (p.hd_mode == 1)
                    for (int v = 0; v < g.N; ++v)
                        xb[at(v, lf)] = cbp_flushed_at<kMin>(g, w, lf, v, p, istop, t) < 0.0f;
                write_out(g, xb, lf, bits, iters, f, t);
                need = true;
                continue;
            }
            if (p.hd_mode == 1)
                for (int v = 0; v < g.N; ++v) xb[at(v, lf)] = cbp_flushed<kMin>(g, w, lf, v, p) < 0.0f;
            if (t == d.sweep && f < d.frames) {
                for (int v = 0; v < g.N; ++v) {
                    if (d.q) d.q[f * g.N + v] = Q[at(v, lf)] * un;
                    if (d.lam) d.lam[f * g.N + v] = cbp_flushed<kMin>(g, w, lf, v, p) * un;
                }
                if (d.r)
                    for (int e = 0; e < g.E; ++e) d.r[f * g.E + e] = R[at(e, lf)] * un;
                if (d.om)
                    for (int i = 0; i < g.M; ++i) {
                        const float2 om = Om[at(i, lf)];
                        d.om[f * g.M + i] =
                            kMin ? with_sign(p.alpha * abs_bits(om.x), sign_bit(om.x))
                                 : with_sign(phi2(abs_bits(om.x) + om.y) * un, sign_bit(om.x));
                    }
            }
            const bool stop = (p.stop_rule == 0 && lane_syndrome_ok(g, xb, lf)) || t == max_iter;
            if (stop) {
                write_out(g, xb, lf, bits, iters, f, t);
                need = true;
            }
        }
        if (h.lanes > 0 && handing_off(h, counter, nf, !done && !need, hand, hk))
            hand_over_cbp(g, h, st, __ballot(hand), hk, f, t);
        if (hand) need = true;
    }
}

// Syndrome of one contiguous frame, rows spread over the workgroup's threads.
// A row's column entries in chunks of kChunk, read unconditionally (padded
// table) so that the loads of a chunk go out together.  The result is
// workgroup-uniform.  Every thread clears and sets the LDS flag (no branch):
// a branch taken by some threads inside the sweep loop lets the compiler split
// that loop by lanes, and a split wave would meet the barriers out of step.
__device__ bool block_syndrome_ok(const SparseDev &g, const uint8_t *xb, int *s_flag) {
    uint32_t bad = 0;
    for (int i = tid_x(); i < g.M; i += kLevelThreads) {
        uint32_t par = 0;
        const int e1 = ldc(g.row_ptr, i + 1);
        for (int c0 = ldc(g.row_ptr, i); c0 < e1; c0 += kChunk) {
            int col[kChunk];
#pragma unroll
            for (int k = 0; k < kChunk; ++k) col[k] = ldc(g.col_idx, c0 + k);
#pragma unroll
            for (int k = 0; k < kChunk; ++k)
                if (c0 + k < e1) par ^= xb[col[k]];
        }
        bad |= par;
    }
    *s_flag = 0;
    __syncthreads();
    atomicOr(s_flag, (int)(bad != 0));
    __syncthreads();
    const int any = __builtin_amdgcn_readfirstlane(*s_flag);
    __syncthreads();  // every thread has read the flag before it is cleared again
    return any == 0;
}

// Items handed over, wave-uniform.  Workgroup g takes items g, g + G, ... (no
// claim: a counter read back by one thread would need a branch in the item
// loop, see block_syndrome_ok).
__device__ __forceinline__ uint32_t item_count(const Handoff &h) {
    const uint32_t n = *h.count;
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)(n < h.cap ? n : h.cap));
}

// Item k's (frame, sweeps done), wave-uniform.
__device__ __forceinline__ int2 item_head(const Handoff &h, uint32_t k) {
    const int2 it = h.items[k];
    return make_int2(__builtin_amdgcn_readfirstlane(it.x), __builtin_amdgcn_readfirstlane(it.y));
}

// Level-parallel CBP on handed-over frames, one frame per workgroup: each
// sweep runs the row levels in order, the rows of a level on separate threads
// (rows of a level share no variable, so every row sees exactly the state the
// sequential schedule gives it and the result is the same bit for bit).
// kLds: the frame's state is staged in LDS (dynamic, h.item_bytes).
template <bool kMin, bool kLds>
__global__ __launch_bounds__(kLevelThreads) void cbp_level_kernel(SparseDev g, uint8_t *__restrict__ bits,
                                                                  int32_t *__restrict__ iters, int max_iter,
                                                                  Params p, Handoff h) {
    __shared__ int s_flag;
    extern __shared__ uint4 s_item[];
    const float us = kMin ? 1.0f : kLog2e;
    p.a *= us;
    p.lmax *= us;
    const uint32_t n = item_count(h);
    for (uint32_t j = 0;; ++j) {
        const uint32_t k = (uint32_t)__builtin_amdgcn_readfirstlane((int)(gid_x() + j * gridDim.x));
        if (k >= n) break;
        CbpState st;
        if constexpr (kLds) st = cbp_layout(g, stage_item(h, k, s_item));
        else st = cbp_item(g, h, k);
        const int2 it = item_head(h, k);
        const int64_t f = it.x;
        int t = it.y;
        for (;;) {
            ++t;
            for (int l = 0; l < g.nlev; ++l) {
                const int r1 = ldc(g.lvl_ptr, l + 1);
                for (int r = ldc(g.lvl_ptr, l) + tid_x(); r < r1; r += kLevelThreads) {
                    bool flip = false;
                    const int4 rr = level_row(g, r);
                    (void)cbp_row<kMin, 1>(g, rr.x, rr.y, rr.z, false, st, 0, p, flip);
                }
                __syncthreads();
            }
            const bool stop = t >= max_iter || (p.stop_rule == 0 && block_syndrome_ok(g, st.xb, &s_flag));
            if (stop) {
                for (int v = tid_x(); v < g.N; v += kLevelThreads) bits[f * g.N + v] = st.xb[v];
                iters[f] = t;  // every thread, the same value
                break;
            }
        }
    }
}

// --------------------------------------------------------------------------
// Layered and flooding BP baselines (Sec. II-A, II-B).  ws: a0 = Lambda[N],
// a1 = R[E], a2 = Lambda accumulator of the flooding schedule [N].
// kMin: the normalized min-sum check rule (alpha * sign * min of the other
// clamped |Q|).  Otherwise the log-tanh rule of eq. equ_s2e4 in log2 units
// (as in the CBP kernel): each row folds g(|Q|) of its edges into a
// (max, rest) pair and excludes an edge's own term from it exactly.
// --------------------------------------------------------------------------
struct BpState {
    float *Lam, *R, *Acc;
    uint8_t *xb;
};

// One row (edges e0 .. e1-1) of the layered (kFlood false) or flooding schedule on one frame.
template <bool kFlood, bool kMin, int kStride>
__device__ __forceinline__ void bp_row(int e0, int e1, const SparseDev &g, const BpState &st, uint32_t lf,
                                       const Params &p) {
    float *Lam = st.Lam, *R = st.R, *Acc = st.Acc;
    // min-sum: (m1, m2) = two smallest |Q|; log-tanh: (m1, m2) = (max, rest) of g(|Q|)
    float m1 = kMin ? __builtin_inff() : 0.0f, m2 = kMin ? __builtin_inff() : 0.0f;
    bool par = false;
    // Edges in chunks of kChunk with all loads of a chunk issued together (the
    // columns of a row differ, so they never read what the chunk stores).  A
    // row of at most kChunk edges keeps its V2C messages in registers between
    // the two passes.
    float qs[kChunk];
    for (int c0 = e0; c0 < e1; c0 += kChunk) {
        const int n = e1 - c0 < kChunk ? e1 - c0 : kChunk;
        int col[kChunk];  // read unconditionally (padded table)
#pragma unroll
        for (int k = 0; k < kChunk; ++k) col[k] = ldc(g.col_idx, c0 + k);
        float lv[kChunk], rv[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k)
            if (k < n) {
                lv[k] = Lam[ix<kStride>(col[k], lf)];
                rv[k] = R[ix<kStride>(c0 + k, lf)];
            }
#pragma unroll
        for (int k = 0; k < kChunk; ++k)
            if (k < n) {
                // V2C, eq. equ_s2e3 (flooding: Lambda of the previous sweep) / equ_s2e10
                const float q = lv[k] - rv[k];
                qs[k] = q;
                if constexpr (kMin) {
                    const float aq = __builtin_fminf(__builtin_fabsf(q), p.lmax);
                    m2 = __builtin_fminf(m2, __builtin_fmaxf(m1, aq));
                    m1 = __builtin_fminf(m1, aq);
                } else {
                    fold(m1, m2, phi2_clamped(q, p.a, p.lmax));
                }
                par ^= (q < 0.0f);
            }
    }
    const bool kept = e1 - e0 <= kChunk;
    for (int c0 = e0; c0 < e1; c0 += kChunk) {
        const int n = e1 - c0 < kChunk ? e1 - c0 : kChunk;
        int col[kChunk];  // read unconditionally (padded table)
#pragma unroll
        for (int k = 0; k < kChunk; ++k) col[k] = ldc(g.col_idx, c0 + k);
        float qv[kChunk], av[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k)
            if (k < n) {
                const uint32_t iv = ix<kStride>(col[k], lf);
                qv[k] = kept ? qs[k] : Lam[iv] - R[ix<kStride>(c0 + k, lf)];
                if (kFlood) av[k] = Acc[iv];
            }
#pragma unroll
        for (int k = 0; k < kChunk; ++k)
            if (k < n) {
                const uint32_t iv = ix<kStride>(col[k], lf);
                const float q = qv[k];
                float rn;
                if constexpr (kMin) {
                    const float aq = __builtin_fminf(__builtin_fabsf(q), p.lmax);
                    rn = with_sign(p.alpha * ((aq == m1) ? m2 : m1), par ^ (q < 0.0f));
                } else {  // C2V, eq. equ_s2e4
                    rn = with_sign(phi2(excl_sum(m1, m2, phi2_clamped(q, p.a, p.lmax))), par ^ (q < 0.0f));
                }
                R[ix<kStride>(c0 + k, lf)] = rn;
                if (kFlood) Acc[iv] = av[k] + rn;
                else Lam[iv] = q + rn;  // eq. equ_s2e12
            }
    }
}

// nr (<= K) rows of one level, each of at most kChunk edges, of the
// layered or flooding schedule on the lane's frame: the updates of bp_row,
// with every load of all the rows issued before any store.  Rows of a level
// share no variable, so none reads what another writes (layered: its Lambda
// and R slots are its own columns'; flooding: it reads the previous sweep's
// Lambda and adds to its own columns' sums, in the same per-variable order as
// row by row).
template <bool kFlood, bool kMin, int K>
__device__ __forceinline__ void bp_level_rows(const int4 (&rr)[K], int nr, const SparseDev &g,
                                              const BpState &st, uint32_t lf, const Params &p) {
    float *Lam = st.Lam, *R = st.R, *Acc = st.Acc;
    int col[K][kChunk];
    float lv[K][kChunk], rv[K][kChunk], av[K][kChunk];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j < nr) {
#pragma unroll
            for (int k = 0; k < kChunk; ++k) col[j][k] = ldc(g.col_idx, rr[j].y + k);  // padded table
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j < nr) {
            const int n = rr[j].z - rr[j].y;
#pragma unroll
            for (int k = 0; k < kChunk; ++k) {
                if (k < n) {
                    const uint32_t iv = at(col[j][k], lf);
                    lv[j][k] = Lam[iv];
                    rv[j][k] = R[at(rr[j].y + k, lf)];
                    if (kFlood) av[j][k] = Acc[iv];
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j < nr) {
            const int n = rr[j].z - rr[j].y;
            float m1 = kMin ? __builtin_inff() : 0.0f, m2 = kMin ? __builtin_inff() : 0.0f;
            bool par = false;
            float qs[kChunk];
#pragma unroll
            for (int k = 0; k < kChunk; ++k) {
                if (k < n) {
                    const float q = lv[j][k] - rv[j][k];  // eq. equ_s2e3 / equ_s2e10
                    qs[k] = q;
                    if constexpr (kMin) {
                        const float aq = __builtin_fminf(__builtin_fabsf(q), p.lmax);
                        m2 = __builtin_fminf(m2, __builtin_fmaxf(m1, aq));
                        m1 = __builtin_fminf(m1, aq);
                    } else {
                        fold(m1, m2, phi2_clamped(q, p.a, p.lmax));
                    }
                    par ^= (q < 0.0f);
                }
            }
#pragma unroll
            for (int k = 0; k < kChunk; ++k) {
                if (k < n) {
                    const uint32_t iv = at(col[j][k], lf);
                    const float q = qs[k];
                    float rn;
                    if constexpr (kMin) {
                        const float aq = __builtin_fminf(__builtin_fabsf(q), p.lmax);
                        rn = with_sign(p.alpha * ((aq == m1) ? m2 : m1), par ^ (q < 0.0f));
                    } else {  // eq. equ_s2e4
                        rn = with_sign(phi2(excl_sum(m1, m2, phi2_clamped(q, p.a, p.lmax))), par ^ (q < 0.0f));
                    }
                    R[at(rr[j].y + k, lf)] = rn;
                    if (kFlood) Acc[iv] = av[j][k] + rn;
                    else Lam[iv] = q + rn;  // eq. equ_s2e12
                }
            }
        }
    }
}

// Posterior of the flooding schedule (eq. equ_s2e6) from the channel LLR in
// log2 units and the sum of the C2V messages.

__device__ __forceinline__ BpState bp_layout(const SparseDev &g, char *b) {
    const int64_t n4 = round256(4 * (int64_t)g.N), e4 = round256(4 * (int64_t)g.E);
    return BpState{(float *)b, (float *)(b + n4), (float *)(b + n4 + e4), (uint8_t *)(b + 2 * n4 + e4)};
}

__device__ __forceinline__ BpState bp_item(const SparseDev &g, const Handoff &h, uint32_t k) {
    return bp_layout(g, item_base(h, k));
}

__device__ __forceinline__ void hand_over_bp(const SparseDev &g, const Handoff &h, const BpState &w,
                                             uint64_t hand, uint32_t hk, int64_t f, int t) {
    for (uint64_t m = hand; m != 0; m &= m - 1) {
        const int d = __builtin_ctzll(m);
        const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)hk, d);
        const int fd = __builtin_amdgcn_readlane((int)f, d);
        const int td = __builtin_amdgcn_readlane(t, d);
        const BpState it = bp_item(g, h, k);
        int r, na;
        active_rank(r, na);
        copy_slot(it.Lam, w.Lam, g.N, d, r, na);
        copy_slot(it.xb, w.xb, g.N, d, r, na);
        copy_slot(it.R, w.R, g.E, d, r, na);
        if (r == 0) h.items[k] = make_int2(fd, td);
    }
}

template <bool kFlood, bool kMin>
__global__ __launch_bounds__(kWave) void bp_sparse_kernel(
    SparseDev g, const float *__restrict__ llr, uint8_t *__restrict__ bits,
    int32_t *__restrict__ iters, int64_t nf, int max_iter, Params p, SparseWs w, Dump d,
    unsigned long long *counter, Handoff h) {
    w = wave_block(w);
    const uint32_t lf = tid_x();  // this lane's slot in its wave's block
    float *Lam = w.a0, *R = w.a1, *Acc = w.a2;
    const BpState st{Lam, R, Acc, w.xb};
    const float us = kMin ? 1.0f : kLog2e;  // log2 units for the log-tanh rule
    const float un = kMin ? 1.0f : kLn2;    // dumps in natural units
    p.a *= us;
    p.lmax *= us;
    uint8_t *xb = w.xb;
    int64_t f = 0;  // the lane's frame
    int t = 0;      // sweeps done on it
    bool need = true, done = false;
    for (;;) {
        for (uint64_t want = __ballot(need); want != 0; want = __ballot(need)) {
            const int64_t fn = claim_frames(counter, want);
            if (need) {
                need = false;
                f = fn;
                if (f >= nf) {
                    done = true;
                } else {
                    for (int v = 0; v < g.N; ++v) {
                        const float l = llr[f * g.N + v] * us;
                        Lam[at(v, lf)] = l;
                        xb[at(v, lf)] = l < 0.0f;
                        if (kFlood) Acc[at(v, lf)] = 0.0f;
                    }
                    for (int e = 0; e < g.E; ++e) R[at(e, lf)] = 0.0f;
                    t = 0;
                    if (max_iter == 0 || (p.stop_rule == 0 && lane_syndrome_ok(g, xb, lf))) {
                        write_out(g, xb, lf, bits, iters, f, 0);
                        need = true;
                    }
                }
            }
        }
        if (__ballot(!done) == 0) break;
        bool hand = false;
        uint32_t hk = 0;
        if (!done) {
            ++t;
            if constexpr (kRowsBp<kFlood>() == 1) {
                for (int i = 0; i < g.M; ++i)
                    bp_row<kFlood, kMin, kWave>(ldc(g.row_ptr, i), ldc(g.row_ptr, i + 1), g, st, lf, p);
            } else {
                // rows level by level (the same result bit for bit as index
                // order), kRowsBp rows of a level at a time
                constexpr int K = kRowsBp<kFlood>();
                for (int l = 0; l < g.nlev; ++l) {
                    const int r1 = ldc(g.lvl_ptr, l + 1);
                    for (int r = ldc(g.lvl_ptr, l); r < r1; r += K) {
                        const int nr = r1 - r < K ? r1 - r : K;
                        int4 rr[K];
                        bool narrow = true;
#pragma unroll
                        for (int j = 0; j < K; ++j) {
                            rr[j] = level_row(g, j < nr ? r + j : r);
                            narrow &= rr[j].z - rr[j].y <= kChunk;
                        }
                        if (narrow)
                            bp_level_rows<kFlood, kMin, K>(rr, nr, g, st, lf, p);
                        else
                            for (int j = 0; j < nr; ++j) bp_row<kFlood, kMin, kWave>(rr[j].y, rr[j].z, g, st, lf, p);
                    }
                }
            }
            // flooding: posterior and decision of every variable, and its C2V sum
            // cleared for the next sweep, in one pass
            if (kFlood) {
                for (int v = 0; v < g.N; ++v) {
                    const uint32_t iv = at(v, lf);
                    const float lm = flood_posterior(llr[f * g.N + v], us, Acc[iv]);
                    Lam[iv] = lm;
                    xb[iv] = lm < 0.0f;
                    Acc[iv] = 0.0f;
                }
            } else {
                for (int v = 0; v < g.N; ++v) xb[at(v, lf)] = Lam[at(v, lf)] < 0.0f;  // eq. equ_s2e7
            }
            if (t == d.sweep && f < d.frames) {
                if (d.lam)
                    for (int v = 0; v < g.N; ++v) d.lam[f * g.N + v] = Lam[at(v, lf)] * un;
                if (d.r)
                    for (int e = 0; e < g.E; ++e) d.r[f * g.E + e] = R[at(e, lf)] * un;
            }
            const bool stop = (p.stop_rule == 0 && lane_syndrome_ok(g, xb, lf)) || t == max_iter;
            if (stop) {
                write_out(g, xb, lf, bits, iters, f, t);
                need = true;
            }
        }
        if (h.lanes > 0 && handing_off(h, counter, nf, !done && !need, hand, hk))
            hand_over_bp(g, h, st, __ballot(hand), hk, f, t);
        if (hand) need = true;
    }
}

// Level-parallel layered / flooding BP on handed-over frames (see
// cbp_level_kernel).  Flooding rows only read the previous sweep's posterior
// and add to per-variable sums in row order, which the levels keep.
template <bool kFlood, bool kMin, bool kLds>
__global__ __launch_bounds__(kLevelThreads) void bp_level_kernel(SparseDev g, const float *__restrict__ llr,
                                                                 uint8_t *__restrict__ bits,
                                                                 int32_t *__restrict__ iters, int max_iter,
                                                                 Params p, Handoff h) {
    __shared__ int s_flag;
    extern __shared__ uint4 s_item[];
    const float us = kMin ? 1.0f : kLog2e;
    p.a *= us;
    p.lmax *= us;
    const uint32_t n = item_count(h);
    for (uint32_t j = 0;; ++j) {
        const uint32_t k = (uint32_t)__builtin_amdgcn_readfirstlane((int)(gid_x() + j * gridDim.x));
        if (k >= n) break;
        BpState st;
        if constexpr (kLds) st = bp_layout(g, stage_item(h, k, s_item));
        else st = bp_item(g, h, k);
        const int2 it = item_head(h, k);
        const int64_t f = it.x;
        int t = it.y;
        for (;;) {
            ++t;
            if (kFlood) {
                for (int v = tid_x(); v < g.N; v += kLevelThreads) st.Acc[v] = 0.0f;
                __syncthreads();
            }
            for (int l = 0; l < g.nlev; ++l) {
                const int r1 = ldc(g.lvl_ptr, l + 1);
                for (int r = ldc(g.lvl_ptr, l) + tid_x(); r < r1; r += kLevelThreads) {
                    const int4 rr = level_row(g, r);
                    bp_row<kFlood, kMin, 1>(rr.y, rr.z, g, st, 0, p);
                }
                __syncthreads();
            }
            for (int v = tid_x(); v < g.N; v += kLevelThreads) {
                if (kFlood) st.Lam[v] = flood_posterior(llr[f * g.N + v], us, st.Acc[v]);
                st.xb[v] = st.Lam[v] < 0.0f;
            }
            __syncthreads();
            const bool stop = t >= max_iter || (p.stop_rule == 0 && block_syndrome_ok(g, st.xb, &s_flag));
            if (stop) {
                for (int v = tid_x(); v < g.N; v += kLevelThreads) bits[f * g.N + v] = st.xb[v];
                iters[f] = t;  // every thread, the same value
                break;
            }
        }
    }
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

constexpr int kScanBlock = 256;
constexpr int64_t kScanMaxBlocks = 16384;

// Flat index of the first NaN or +-Inf among n floats (exponent bits all
// ones): the atomic minimum over the offending indices is left in *pos, which
// starts at all ones.
__global__ __launch_bounds__(kScanBlock) void nonfinite_scan_kernel(const uint32_t *x, int64_t n,
                                                                    unsigned long long *pos) {
    const int64_t stride = (int64_t)gridDim.x * kScanBlock;
    for (int64_t i = (int64_t)gid_x() * kScanBlock + tid_x(); i < n; i += stride)
        if ((x[i] & 0x7f800000u) == 0x7f800000u) atomicMin(pos, (unsigned long long)i);
}

}  // namespace

static int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Bytes of one wave's block: each array padded to 256 bytes.
static int64_t sparse_block_bytes(int algo, const SparseDev &g) {
    auto arr = [](int64_t n, int64_t bytes) { return round_up(n * kWave * bytes, 256); };
    if (algo == kCBP || algo == kCBPNMS) return arr(g.N, 4) + arr(g.E, 4) + arr(g.M, 8) + arr(g.N, 1);
    return 2 * arr(g.N, 4) + arr(g.E, 4) + arr(g.N, 1);
}

int64_t sparse_item_bytes(int algo, const SparseDev &g) {
    const int64_t n4 = round256(4 * (int64_t)g.N), e4 = round256(4 * (int64_t)g.E), m8 = round256(8 * (int64_t)g.M);
    if (algo == kCBP || algo == kCBPNMS) return n4 + e4 + m8 + round256(g.N);
    return 2 * n4 + e4 + round256(g.N);
}

size_t sparse_ws_bytes(int algo, const SparseDev &g, int64_t frames) {
    return (size_t)(round_up(frames, kWave) / kWave * sparse_block_bytes(algo, g));
}

SparseWs sparse_ws_carve(int algo, const SparseDev &g, int64_t frames, void *base) {
    SparseWs w{};
    w.stride = kWave;
    w.block_bytes = sparse_block_bytes(algo, g);
    w.waves = round_up(frames, kWave) / kWave;
    char *p = (char *)base;
    auto take = [&](int64_t n, int64_t bytes) {
        char *r = p;
        p += round_up(n * kWave * bytes, 256);
        return r;
    };
    if (algo == kCBP || algo == kCBPNMS) {
        w.a0 = (float *)take(g.N, 4);
        w.a2 = (float *)take(g.E, 4);
        w.a3 = (float *)take(g.M, 8);  // float2
    } else {
        w.a0 = (float *)take(g.N, 4);
        w.a1 = (float *)take(g.E, 4);
        w.a2 = (float *)take(g.N, 4);
    }
    w.xb = (uint8_t *)take(g.N, 1);
    return w;
}

// Frames whose state fits a workgroup's LDS (160 KB on gfx950; above 64 KB
// the kernel's dynamic-LDS limit is raised first) are finished by the
// level-parallel kernels with the state in LDS.
static int64_t level_lds_limit() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 64 << 10;
    return (int64_t)v - 64;  // room for the kernels' static LDS
}

template <class K>
static bool allow_lds(K kernel, size_t bytes) {
    return bytes <= (64u << 10) ||
           hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes) == hipSuccess;
}

// Launches the level-parallel kernel of algo; with kLds the frame state is
// staged in `lds` bytes of dynamic LDS.  False if that LDS cannot be granted.
template <bool kLds>
static bool launch_level(int algo, dim3 grid, dim3 block, size_t lds, hipStream_t s, const SparseDev &g,
                         const float *llr, uint8_t *bits, int32_t *iters, int max_iter, const Params &p,
                         const Handoff &h) {
#define CBP_LEVEL_LAUNCH(KERNEL, ...)                                          \
    do {                                                                       \
        if (kLds && !allow_lds(KERNEL, lds)) return false;                     \
        hipLaunchKernelGGL(KERNEL, grid, block, lds, s, __VA_ARGS__);          \
    } while (0)
    if (algo == kCBP)
        CBP_LEVEL_LAUNCH((cbp_level_kernel<false, kLds>), g, bits, iters, max_iter, p, h);
    else if (algo == kCBPNMS)
        CBP_LEVEL_LAUNCH((cbp_level_kernel<true, kLds>), g, bits, iters, max_iter, p, h);
    else if (algo == kLBPNMS)
        CBP_LEVEL_LAUNCH((bp_level_kernel<false, true, kLds>), g, llr, bits, iters, max_iter, p, h);
    else if (algo == kFBPNMS)
        CBP_LEVEL_LAUNCH((bp_level_kernel<true, true, kLds>), g, llr, bits, iters, max_iter, p, h);
    else if (algo == kLBP)
        CBP_LEVEL_LAUNCH((bp_level_kernel<false, false, kLds>), g, llr, bits, iters, max_iter, p, h);
    else
        CBP_LEVEL_LAUNCH((bp_level_kernel<true, false, kLds>), g, llr, bits, iters, max_iter, p, h);
#undef CBP_LEVEL_LAUNCH
    return true;
}

hipError_t launch_sparse(int algo, const SparseDev &g, const float *llr, uint8_t *bits,
                         int32_t *iters, int64_t nf, int max_iter, const Params &p,
                         const SparseWs &ws, const Dump &d, unsigned long long *counter,
                         const Handoff &h, hipStream_t s) {
    // one lane per state slot; the frame counter and the hand-off count start at zero
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(kFillBlock), 0, s, (int *)counter, 4, 0);
    const dim3 grid((unsigned)ws.waves), block(kWave);
    if (algo == kCBP)
        hipLaunchKernelGGL(cbp_sparse_kernel<false>, grid, block, 0, s, g, llr, bits, iters, nf,
                           max_iter, p, ws, d, counter, h);
    else if (algo == kCBPNMS)
        hipLaunchKernelGGL(cbp_sparse_kernel<true>, grid, block, 0, s, g, llr, bits, iters, nf,
                           max_iter, p, ws, d, counter, h);
    else if (algo == kLBPNMS)
        hipLaunchKernelGGL((bp_sparse_kernel<false, true>), grid, block, 0, s, g, llr, bits, iters,
                           nf, max_iter, p, ws, d, counter, h);
    else if (algo == kFBPNMS)
        hipLaunchKernelGGL((bp_sparse_kernel<true, true>), grid, block, 0, s, g, llr, bits, iters,
                           nf, max_iter, p, ws, d, counter, h);
    else if (algo == kLBP)
        hipLaunchKernelGGL((bp_sparse_kernel<false, false>), grid, block, 0, s, g, llr, bits, iters,
                           nf, max_iter, p, ws, d, counter, h);
    else if (algo == kFBP)
        hipLaunchKernelGGL((bp_sparse_kernel<true, false>), grid, block, 0, s, g, llr, bits, iters,
                           nf, max_iter, p, ws, d, counter, h);
    else
        return hipErrorInvalidValue;
    if (h.lanes <= 0) return hipGetLastError();
    const dim3 lgrid((unsigned)h.groups), lblock(kLevelThreads);
    if (h.item_bytes > level_lds_limit() ||
        !launch_level<true>(algo, lgrid, lblock, (size_t)h.item_bytes, s, g, llr, bits, iters, max_iter, p, h))
        launch_level<false>(algo, lgrid, lblock, 0, s, g, llr, bits, iters, max_iter, p, h);
    return hipGetLastError();
}

hipError_t launch_syndrome(const SparseDev &g, const uint8_t *bits, uint8_t *ok, int64_t batch,
                           hipStream_t s) {
    const dim3 grid((unsigned)((batch + kSyndromeBlock - 1) / kSyndromeBlock)), block(kSyndromeBlock);
    hipLaunchKernelGGL(syndrome_kernel, grid, block, 0, s, g, bits, ok, batch);
    return hipGetLastError();
}

hipError_t launch_nonfinite_scan(const float *x, int64_t n, unsigned long long *pos, hipStream_t s) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(kFillBlock), 0, s, (int *)pos, 2, -1);
    if (n > 0) {
        const int64_t need = (n + kScanBlock - 1) / kScanBlock;
        const dim3 grid((unsigned)(need < kScanMaxBlocks ? need : kScanMaxBlocks)), block(kScanBlock);
        hipLaunchKernelGGL(nonfinite_scan_kernel, grid, block, 0, s, (const uint32_t *)x, n, pos);
    }
    return hipGetLastError();
}

hipError_t launch_fill_i32(int *ptr, int n, int value, hipStream_t s) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3((n + kFillBlock - 1) / kFillBlock), dim3(kFillBlock), 0, s, ptr,
                       n, value);
    return hipGetLastError();
}

}  // namespace cbp
