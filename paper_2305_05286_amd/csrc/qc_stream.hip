// Quasi-cyclic decoders for any base matrix and any mix of codes, with the
// per-frame state in a device workspace instead of registers (frames too
// large for the register file, base patterns that are not compiled in, and
// batches that mix codes, lengths and rates in one launch).
//
// Same mapping as the register-resident kernels: a frame occupies Z lanes,
// lane l owns variable l of every block-column, block-rows are the layers of
// the sweep and the only cross-lane traffic of a layer is one rotated LDS
// exchange of the new V2C terms plus the rotated reads of the latest checks'
// beliefs.  The base structure is a runtime edge table (sweep order: layer
// major, block-column ascending), read through the constant address space so
// that its wave-uniform reads are scalar loads: a vector load there would put
// a full memory round trip in front of every state access of the edge.
//
// Scheduling.  The launch is persistent: every workgroup has the same number
// of lanes, a multiple of each code's Z, and decodes lanes / Z frames of one
// code at a time ("slots").  Frames wait in one queue per code; a slot whose
// frame stops (at a sweep boundary, per-frame early termination) writes its
// outputs and claims the next frame of the queue, and when a code's queue is
// empty and its last frames are done the workgroup moves on to the next
// code.  A single-code launch is the case of one queue.
//
// The kernel is bound by memory latency (a layer's accesses depend on the
// edge table and end in a barrier), so what matters is the number of frames
// in flight: the state per edge is kept to what the method needs and the
// kernel is compiled for 8 waves per SIMD.
//
// Workspace of one slot (element [i][l] of a Z-vector array at i*Z + l, so a
// lane's accesses are coalesced across the slot):
//   Q  [NB][Z]  CBP: latest V2C; NMS: posterior Lambda
//   PQ [NB][Z]  FBP only: accumulator of the new C2V messages
//   R  [E][Z]   C2V message of every edge
//   OM [MB][Z]  CBP: check-beliefs (max phi2 term | parity, rest of the sum)
//   XB [NB][Z]  hard decisions (bytes)
// CBP keeps LLRs in log2 units and needs no cached phi2(|Q_v|): Q_v is still
// the V2C value the latest check folded, and phi2 of it is recomputed
// bit-identically.
#include "internal.hpp"
#include "phi.hpp"
#include "stream_util.hpp"

#ifndef STREAM_WPE_N
#define STREAM_WPE_N 8
#endif
#ifndef STREAM_GROUP_N
#define STREAM_GROUP_N 2
#endif

namespace cbp {
namespace {

// Edges of a layer whose memory accesses are issued together (measured on
// MI355X, n = 26112: 2 beats 1 by 29% for CBP and 15-18% for the min-sum
// layers; 3 runs out of registers at 8 waves per SIMD).
constexpr int kGroup = STREAM_GROUP_N;

struct StreamArgs {
    const float *llr;
    uint8_t *bits;
    int32_t *iters;
    const StreamCode *codes;
    int ncodes;
    int lanes;
    int dcmax;
    int xfloats;              // LDS floats of one exchange array (lanes * dcmax, even)
    int max_slots;
    const int64_t *qstart;    // [ncodes+1] or NULL (one code, frames [0, batch))
    const int32_t *perm;      // frame ids grouped by code, or NULL (identity)
    const int64_t *offset;    // element offset of each frame, or NULL (f * N)
    unsigned int *counter;    // [ncodes] claims per queue
    int64_t batch;
    int max_iter;
    Params p;
    Dump d;
    char *ws;                 // workgroup workspaces, group_bytes apart
    int64_t group_bytes;
};

// kDbg: the instantiation that also serves hd_mode = 1 and the state dumps
// (cold code still costs registers in a kernel held to 64 VGPRs).
template <int kAlgo, bool kDbg>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(STREAM_WPE_N)))
void qc_stream_kernel(StreamArgs A) {
    extern __shared__ float smem[];
    using CS = const __attribute__((address_space(4))) StreamCode;
    CS *codes = (CS *)A.codes;
    constexpr bool kBelief = kAlgo == kCBP || kAlgo == kCBPNMS;
    // The log-tanh rule keeps every LLR in log2 units (L / ln2), where one
    // function (phi2) serves both directions of the check rule.
    constexpr bool kLog2 = kAlgo == kCBP;
    const float us = kLog2 ? kLog2e : 1.0f;
    const float a = A.p.a * us, lmax = A.p.lmax * us, alpha = A.p.alpha;

    // LDS, sized for the largest code of the launch: exchange [lanes*dcmax],
    // NMS V2C stash [lanes*dcmax], row state [lanes] float2, 5 flag arrays
    float *sXall = smem;
    float *sQall = smem + A.xfloats;
    float2 *sRowAll = reinterpret_cast<float2 *>(smem + (kBelief ? 1 : 2) * (size_t)A.xfloats);
    int *sFlags = reinterpret_cast<int *>(sRowAll + A.lanes);
    const int MS = A.max_slots;
    int64_t *sF = reinterpret_cast<int64_t *>(sFlags);  // [MS] claimed queue position
    int *sBad = sFlags + 2 * MS;                         // [2][MS]
    int *sAct = sFlags + 4 * MS;                         // [MS]
    int *sFresh = sFlags + 5 * MS;                       // [MS]
    // paper's stopping rule (debug instantiation only; its launches allocate
    // these): per-row outcomes [lanes], per-edge flips and previous decisions
    // [dcmax][lanes] bytes, stop row and run per slot
    constexpr bool kStop = kDbg && kBelief;
    long long *sRunAll = reinterpret_cast<long long *>(sFlags + 6 * MS);  // [MS]
    int *sStopAll = reinterpret_cast<int *>(sRunAll + MS);                 // [MS]
    uint8_t *sGoodAll = reinterpret_cast<uint8_t *>(sStopAll + MS);        // [lanes]
    uint8_t *sFlAll = sGoodAll + A.lanes;                                  // [lanes * dcmax]
    uint8_t *sOldAll = sFlAll + (size_t)A.lanes * A.dcmax;                 // [lanes * dcmax]

    for (int visit = 0; visit < A.ncodes; ++visit) {
        const int c = (int)(((unsigned)gid_x() + (unsigned)visit) % (unsigned)A.ncodes);
        const int Z = codes[c].Z, NB = codes[c].nb, MB = codes[c].mb, E = codes[c].E;
        const int dcm = codes[c].dcmax;
        const int64_t N = codes[c].N;
        const int *rstart = codes[c].rstart;
        const int4 *erec = codes[c].erec;
        const int64_t q0 = A.qstart ? ldc(A.qstart, c) : 0;
        const int64_t qn = (A.qstart ? ldc(A.qstart, c + 1) : A.batch) - q0;
        const int SL = A.lanes / Z;
        const int slot = tid_x() / Z;
        const int l = tid_x() - slot * Z;
        float *sX = sXall + (size_t)slot * dcm * Z;
        float *sQ = sQall + (size_t)slot * dcm * Z;
        float2 *sRow = sRowAll + (size_t)slot * Z;
        [[maybe_unused]] uint8_t *sGood = sGoodAll + (size_t)slot * Z;
        [[maybe_unused]] uint8_t *sFl = sFlAll + (size_t)slot * dcm * Z;
        [[maybe_unused]] uint8_t *sOld = sOldAll + (size_t)slot * dcm * Z;
        // paper's stopping rule: rows in a row (across sweeps) with Omega > 0 and
        // no flipped decision; on reaching M mid-layer the decisions of the
        // layer's later rows are reverted and the frame's decisions frozen
        const bool paper = kStop && A.p.stop_rule == 1;
        long long run = 0;
        bool pstop = false;

        // State: byte offsets of this slot's arrays in the workgroup's buffer.
        const Ws W{__builtin_amdgcn_make_buffer_rsrc(A.ws + (int64_t)gid_x() * A.group_bytes, 0,
                                                     (int)A.group_bytes, kBufferWord3)};
        const uint32_t oQ = (uint32_t)(slot * stream_slot_bytes(kAlgo, N, E, MB, Z));
        const uint32_t oPQ = oQ + 4u * (uint32_t)N;
        const uint32_t oR = oQ + 4u * (uint32_t)((kAlgo == kFBPNMS ? 2 : 1) * N);
        const uint32_t oOM = (oR + 4u * (uint32_t)(E * Z) + 7u) & ~7u;
        const uint32_t oXB = oOM + (kBelief ? 8u * (uint32_t)(MB * Z) : 0u);

        // frame id and element offset of queue position k
        auto frame_of = [&](int64_t k) -> int { return A.perm ? A.perm[q0 + k] : (int)(q0 + k); };
        auto offset_of = [&](int fr) -> int64_t { return A.offset ? A.offset[fr] : (int64_t)fr * N; };

        auto load = [&](int64_t fo) {
            for (int b = 0; b < NB; ++b) {
                const float v = A.llr[fo + (int64_t)b * Z + l] * us;
                W.st(oQ + 4u * (b * Z + l), v);
                if constexpr (kAlgo == kFBPNMS) W.st(oPQ + 4u * (b * Z + l), 0.0f);
                W.stb(oXB + b * Z + l, v < 0.0f);
            }
            for (int e = 0; e < E; ++e) W.st(oR + 4u * (e * Z + l), 0.0f);
        };

        if (l == 0) sF[slot] = (int64_t)atomicAdd(A.counter + c, 1u);
        __syncthreads();
        int64_t k = sF[slot];
        bool have = k < qn;
        int f = have ? frame_of(k) : 0;
        int64_t fo = have ? offset_of(f) : 0;
        int t = 0, it = 0;
        if (have) load(fo);

        for (;;) {
            // ---------------- syndrome of the current decisions ----------
            const int pb = it & 1;
            ++it;
            if (l == 0) sBad[pb * MS + slot] = 0;
            __syncthreads();  // decisions of all lanes written
            uint32_t bad = 0;
            for (int r = 0; r < MB; ++r) {
                uint32_t par = 0;
                for (int e = ldc(rstart, r); e < ldc(rstart, r + 1); ++e) {
                    const Edge ed = edge(erec, e);
                    int idx = l + ed.sh;
                    idx -= (idx >= Z) ? Z : 0;
                    par ^= W.ldb(oXB + ed.b * Z + idx);
                }
                bad |= par;
            }
            if (bad) sBad[pb * MS + slot] = 1;
            __syncthreads();
            const bool ok = sBad[pb * MS + slot] == 0;
            const bool done = !have || t >= A.max_iter || (A.p.stop_rule == 0 && ok) || (paper && pstop);
            const bool claim = done && have;
            if (claim) {
                for (int b = 0; b < NB; ++b) A.bits[fo + (int64_t)b * Z + l] = (uint8_t)W.ldb(oXB + b * Z + l);
                if (l == 0) {
                    A.iters[f] = t;
                    sF[slot] = (int64_t)atomicAdd(A.counter + c, 1u);
                }
            }
            __syncthreads();
            if (claim) {
                k = sF[slot];
                have = k < qn;
                t = 0;
                run = 0;
                pstop = false;
                if (have) {
                    f = frame_of(k);
                    fo = offset_of(f);
                    load(fo);
                }
            }
            if (l == 0) {
                sAct[slot] = have;
                sFresh[slot] = claim && have;
            }
            __syncthreads();
            bool anyAct = false, anyFresh = false;
            for (int s2 = 0; s2 < SL; ++s2) {
                anyAct |= sAct[s2] != 0;
                anyFresh |= sFresh[s2] != 0;
            }
            if (!anyAct) break;
            if (anyFresh) continue;

            // ---------------- one sweep -----------------------------------
            const bool first = (t == 0);
            for (int r = 0; r < MB; ++r) {
                const int e0 = ldc(rstart, r), e1 = ldc(rstart, r + 1);
                // phase 1: lane = variable
                if constexpr (kBelief) {
                    // kGroup edges at a time: all their loads are issued before any of
                    // their stores (the edges of a layer are distinct block-columns, so
                    // no store of one aliases a load of another; R(c_i -> v) differs from
                    // R(c_j -> v) except in a degree-1 column, where rn is used).  The
                    // stores count in the same in-order memory counter as the loads, so
                    // one edge at a time costs a full round trip per edge.
                    struct In {
                        Edge ed;
                        int iv, kc;
                        float q, rci;
                        float2 om;
                        bool has;
                        uint32_t xold;
                    };
                    auto ld_edge = [&](int e, In &in) {
                        in.ed = edge(erec, e);
                        in.iv = in.ed.b * Z + l;
                        in.kc = l - in.ed.sh;
                        in.kc += (in.kc < 0) ? Z : 0;
                        in.q = W.ld(oQ + 4u * in.iv);
                        in.rci = W.ld(oR + 4u * (e * Z + l));
                        in.has = !(first && in.ed.first);
                        if constexpr (kStop) in.xold = paper ? W.ldb(oXB + in.iv) : 0u;
                        in.om = make_float2(0.0f, 0.0f);
                        if (in.has) {
                            int kp = l - in.ed.epsh;
                            kp += (kp < 0) ? Z : 0;
                            in.om = W.ld2(oOM + 8u * (in.ed.epr * Z + kp));
                        }
                    };
                    auto fin_edge = [&](int e, const In &in) {
                        const float q = in.q;
                        float rn = 0.0f;
                        bool own = false;
                        if (in.has) {
                            const float2 om = in.om;
                            if constexpr (kAlgo == kCBP) {
                                const float dd = excl_sum(abs_bits(om.x), om.y, phi2_clamped(q, a, lmax));
                                rn = with_sign(phi2(dd), sign_bit(om.x) ^ (q < 0.0f));
                            } else {
                                const float aq = __builtin_fminf(__builtin_fabsf(q), lmax);
                                const float m1 = abs_bits(om.x);
                                rn = with_sign(alpha * ((aq == m1) ? om.y : m1), sign_bit(om.x) ^ (q < 0.0f));
                            }
                            W.st(oR + 4u * (in.ed.ep * Z + l), rn);
                            own = in.ed.ep == e;
                        }
                        const float lam = q + rn;
                        if (kStop && paper) {  // every visit decides; frozen once stopped
                            const uint32_t nx = lam < 0.0f;
                            sFl[(e - e0) * Z + in.kc] = (uint8_t)(nx != in.xold);
                            sOld[(e - e0) * Z + l] = (uint8_t)in.xold;
                            if (!pstop) W.stb(oXB + in.iv, nx != 0);
                        } else if (in.ed.last) {
                            W.stb(oXB + in.iv, lam < 0.0f);
                        }
                        const float qn2 = lam - (own ? rn : in.rci);
                        const float fq = kAlgo == kCBP ? phi2_clamped(qn2, a, lmax)
                                                       : __builtin_fminf(__builtin_fabsf(qn2), lmax);
                        W.st(oQ + 4u * in.iv, qn2);
                        sX[(e - e0) * Z + in.kc] = with_sign(fq, qn2 < 0.0f);
                    };
                    int e = e0;
                    for (; e + kGroup - 1 < e1; e += kGroup) {
                        In p[kGroup];
#pragma unroll
                        for (int j = 0; j < kGroup; ++j) ld_edge(e + j, p[j]);
#pragma unroll
                        for (int j = 0; j < kGroup; ++j) fin_edge(e + j, p[j]);
                    }
                    for (; e < e1; ++e) {
                        In p0;
                        ld_edge(e, p0);
                        fin_edge(e, p0);
                    }
                } else {
                    // min-sum layers: the V2C loads of kGroup edges are issued together
                    int e = e0;
                    auto nms1 = [&](int e, float q) {
                        const Edge ed = edge(erec, e);
                        int kc = l - ed.sh;
                        kc += (kc < 0) ? Z : 0;
                        sQ[(e - e0) * Z + l] = q;  // kept for phase 3
                        sX[(e - e0) * Z + kc] = with_sign(__builtin_fminf(__builtin_fabsf(q), lmax), q < 0.0f);
                    };
                    auto nmsq = [&](int e) {
                        const Edge ed = edge(erec, e);
                        return W.ld(oQ + 4u * (ed.b * Z + l)) - W.ld(oR + 4u * (e * Z + l));
                    };
                    for (; e + kGroup - 1 < e1; e += kGroup) {
                        float qq[kGroup];
#pragma unroll
                        for (int j = 0; j < kGroup; ++j) qq[j] = nmsq(e + j);
#pragma unroll
                        for (int j = 0; j < kGroup; ++j) nms1(e + j, qq[j]);
                    }
                    for (; e < e1; ++e) nms1(e, nmsq(e));
                }
                __syncthreads();
                // phase 2: lane = row l of layer r
                {
                    bool par = false;
                    if constexpr (kAlgo == kCBP) {
                        float Mx = 0.0f, Sr = 0.0f;
                        for (int j = 0; j < e1 - e0; ++j) {
                            const float x = sX[j * Z + l];
                            par ^= sign_bit(x);
                            fold(Mx, Sr, abs_bits(x));
                        }
                        W.st2(oOM + 8u * (r * Z + l), make_float2(with_sign(Mx, par), Sr));
                    } else {
                        float m1 = __builtin_inff(), m2 = __builtin_inff();
                        for (int j = 0; j < e1 - e0; ++j) {
                            const float x = sX[j * Z + l];
                            par ^= sign_bit(x);
                            const float ax = abs_bits(x);
                            m2 = __builtin_fminf(m2, __builtin_fmaxf(m1, ax));
                            m1 = __builtin_fminf(m1, ax);
                        }
                        if constexpr (kBelief) W.st2(oOM + 8u * (r * Z + l), make_float2(with_sign(m1, par), m2));
                        else sRow[l] = make_float2(with_sign(m1, par), m2);
                    }
                    if constexpr (kStop) {
                        if (paper) {  // Step 2(3): this row keeps Omega > 0 and flips nothing
                            uint8_t fl = 0;
                            for (int j = 0; j < e1 - e0; ++j) fl |= sFl[j * Z + l];
                            sGood[l] = (uint8_t)(!par && fl == 0);
                        }
                    }
                }
                __syncthreads();
                if constexpr (kStop) {
                    if (paper) {
                        if (l == 0) {  // rows of this layer in index order, continuing the run
                            const long long Mrows = (long long)MB * Z;
                            int lead = 0, trail = 0;
                            bool all = true;
                            for (int kk = 0; kk < Z; ++kk) {
                                if (sGood[kk]) {
                                    ++trail;
                                    if (all) ++lead;
                                } else {
                                    all = false;
                                    trail = 0;
                                }
                            }
                            sStopAll[slot] = (!pstop && run + lead >= Mrows) ? (int)(Mrows - run - 1) : -1;
                            sRunAll[slot] = all ? run + Z : trail;
                        }
                        __syncthreads();
                        const int kstop = sStopAll[slot];
                        run = sRunAll[slot];
                        if (!pstop && kstop >= 0) {
                            // stop after row kstop: the layer's later rows are undone
                            for (int e = e0; e < e1; ++e) {
                                const Edge ed = edge(erec, e);
                                int kc = l - ed.sh;
                                kc += (kc < 0) ? Z : 0;
                                if (kc > kstop) W.stb(oXB + ed.b * Z + l, sOld[(e - e0) * Z + l] != 0);
                            }
                            pstop = true;
                        }
                        __syncthreads();
                    }
                }
                if constexpr (!kBelief) {
                    // phase 3: lane = variable
                    auto c2v = [&](int e, const Edge &ed) {
                        int kc = l - ed.sh;
                        kc += (kc < 0) ? Z : 0;
                        const float2 rw = sRow[kc];
                        const float q = sQ[(e - e0) * Z + l];
                        const float aq = __builtin_fminf(__builtin_fabsf(q), lmax);
                        const float m1 = abs_bits(rw.x);
                        return with_sign(alpha * ((aq == m1) ? rw.y : m1), sign_bit(rw.x) ^ (q < 0.0f));
                    };
                    if constexpr (kAlgo == kLBPNMS) {
                        for (int e = e0; e < e1; ++e) {
                            const Edge ed = edge(erec, e);
                            const float rn = c2v(e, ed);
                            W.st(oR + 4u * (e * Z + l), rn);
                            W.st(oQ + 4u * (ed.b * Z + l), sQ[(e - e0) * Z + l] + rn);
                        }
                    } else {
                        // flooding accumulator: the reads of kGroup edges go first
                        int e = e0;
                        auto acc = [&](int e, float pq) {
                            const Edge ed = edge(erec, e);
                            const float rn = c2v(e, ed);
                            W.st(oR + 4u * (e * Z + l), rn);
                            W.st(oPQ + 4u * (ed.b * Z + l), pq + rn);
                        };
                        for (; e + kGroup - 1 < e1; e += kGroup) {
                            float pq[kGroup];
#pragma unroll
                            for (int j = 0; j < kGroup; ++j)
                                pq[j] = W.ld(oPQ + 4u * (edge(erec, e + j).b * Z + l));
#pragma unroll
                            for (int j = 0; j < kGroup; ++j) acc(e + j, pq[j]);
                        }
                        for (; e < e1; ++e) acc(e, W.ld(oPQ + 4u * (edge(erec, e).b * Z + l)));
                    }
                }
            }
            ++t;

            // ---------------- end of sweep --------------------------------
            if constexpr (!kBelief) {
                for (int b = 0; b < NB; ++b) {
                    const int iv = b * Z + l;
                    float lam = W.ld(oQ + 4u * iv);
                    if constexpr (kAlgo == kFBPNMS) {
                        if (have) lam = A.llr[fo + iv] + W.ld(oPQ + 4u * iv);
                        W.st(oQ + 4u * iv, lam);
                        W.st(oPQ + 4u * iv, 0.0f);
                    }
                    W.stb(oXB + iv, lam < 0.0f);
                }
            }
            auto flushed = [&](int b) {
                const int el = ldc(codes[c].elast, b);
                int kk = l - ldc(codes[c].esh, el);
                kk += (kk < 0) ? Z : 0;
                const float2 om = W.ld2(oOM + 8u * (ldc(codes[c].er, el) * Z + kk));
                const float q = W.ld(oQ + 4u * (b * Z + l));
                if constexpr (kAlgo == kCBP) {
                    const float dd = excl_sum(abs_bits(om.x), om.y, phi2_clamped(q, a, lmax));
                    return q + with_sign(phi2(dd), sign_bit(om.x) ^ (q < 0.0f));
                } else {
                    const float aq = __builtin_fminf(__builtin_fabsf(q), lmax);
                    const float m1 = abs_bits(om.x);
                    return q + with_sign(alpha * ((aq == m1) ? om.y : m1), sign_bit(om.x) ^ (q < 0.0f));
                }
            };
            if constexpr (kBelief && kDbg) {
                if (A.p.hd_mode == 1)
                    for (int b = 0; b < NB; ++b) W.stb(oXB + b * Z + l, flushed(b) < 0.0f);
            }
            if (kDbg && have && t == A.d.sweep && f < A.d.frames) {  // one-code launches only
                const int64_t Etot = (int64_t)E * Z, M = (int64_t)MB * Z;
                const float un = kLog2 ? kLn2 : 1.0f;  // dumps in natural units
                for (int b = 0; b < NB; ++b) {
                    if constexpr (kBelief) {
                        if (A.d.q) A.d.q[f * N + b * Z + l] = W.ld(oQ + 4u * (b * Z + l)) * un;
                        if (A.d.lam) A.d.lam[f * N + b * Z + l] = flushed(b) * un;
                    } else {
                        if (A.d.lam) A.d.lam[f * N + b * Z + l] = W.ld(oQ + 4u * (b * Z + l));
                    }
                }
                if (A.d.r)
                    for (int e = 0; e < E; ++e) {
                        const int r = ldc(codes[c].er, e);
                        int kk = l - ldc(codes[c].esh, e);
                        kk += (kk < 0) ? Z : 0;
                        const int r0 = ldc(rstart, r), dc = ldc(rstart, r + 1) - r0;
                        A.d.r[f * Etot + (int64_t)r0 * Z + (int64_t)kk * dc + (e - r0)] = W.ld(oR + 4u * (e * Z + l)) * un;
                    }
                if constexpr (kBelief) {
                    if (A.d.om)
                        for (int r = 0; r < MB; ++r) {
                            const float2 om = W.ld2(oOM + 8u * (r * Z + l));
                            A.d.om[f * M + (int64_t)r * Z + l] =
                                kAlgo == kCBP ? with_sign(phi2(abs_bits(om.x) + om.y) * un, sign_bit(om.x))
                                              : with_sign(alpha * abs_bits(om.x), sign_bit(om.x));
                        }
                }
            }
        }
        __syncthreads();  // the flags are reused by the next code
    }
}

// Groups a mixed batch by code (one workgroup): per-code histogram in LDS,
// exclusive scan, scatter of the frame ids.  The order of the frames within
// a code's queue is whatever the atomics give; it does not affect results.
__global__ __launch_bounds__(1024) void mix_prepare_kernel(const int32_t *frame_code,
                                                           const int64_t *offset, int64_t batch,
                                                           int64_t llr_elems, const StreamCode *codes,
                                                           int ncodes, int64_t *qstart, int32_t *perm,
                                                           unsigned int *counter, int32_t *iters) {
    __shared__ unsigned int hist[kMaxMixCodes];
    __shared__ int64_t cur[kMaxMixCodes];
    using CS = const __attribute__((address_space(4))) StreamCode;
    CS *cs = (CS *)codes;
    for (int i = tid_x(); i < ncodes; i += 1024) {
        hist[i] = 0;
        counter[i] = 0;
    }
    __syncthreads();
    auto valid = [&](int64_t f, int cc) {
        if (cc < 0 || cc >= ncodes) return false;
        const int64_t o = offset[f];
        return o >= 0 && o <= llr_elems - cs[cc].N;
    };
    for (int64_t f = tid_x(); f < batch; f += 1024) {
        const int cc = frame_code[f];
        if (valid(f, cc)) atomicAdd(&hist[cc], 1u);
        else iters[f] = -1;
    }
    __syncthreads();
    if (tid_x() == 0) {
        int64_t acc = 0;
        for (int i = 0; i < ncodes; ++i) {
            qstart[i] = acc;
            cur[i] = acc;
            acc += hist[i];
        }
        qstart[ncodes] = acc;
    }
    __syncthreads();
    for (int64_t f = tid_x(); f < batch; f += 1024) {
        const int cc = frame_code[f];
        if (valid(f, cc)) perm[atomicAdd((unsigned long long *)&cur[cc], 1ull)] = (int32_t)f;
    }
}

template <bool kDbg>
const void *stream_kernel(int algo) {
    return algo == kCBP      ? reinterpret_cast<const void *>(qc_stream_kernel<kCBP, kDbg>)
           : algo == kLBPNMS ? reinterpret_cast<const void *>(qc_stream_kernel<kLBPNMS, kDbg>)
           : algo == kFBPNMS ? reinterpret_cast<const void *>(qc_stream_kernel<kFBPNMS, kDbg>)
                             : reinterpret_cast<const void *>(qc_stream_kernel<kCBPNMS, kDbg>);
}

template <bool kDbg>
void launch_algo(int algo, dim3 grid, dim3 block, size_t lds, hipStream_t s, const StreamArgs &A) {
    if (algo == kCBP)
        hipLaunchKernelGGL((qc_stream_kernel<kCBP, kDbg>), grid, block, lds, s, A);
    else if (algo == kLBPNMS)
        hipLaunchKernelGGL((qc_stream_kernel<kLBPNMS, kDbg>), grid, block, lds, s, A);
    else if (algo == kFBPNMS)
        hipLaunchKernelGGL((qc_stream_kernel<kFBPNMS, kDbg>), grid, block, lds, s, A);
    else
        hipLaunchKernelGGL((qc_stream_kernel<kCBPNMS, kDbg>), grid, block, lds, s, A);
}

}  // namespace

size_t stream_lds_bytes(int algo, int lanes, int dcmax, int max_slots, bool dbg) {
    const bool belief = algo == kCBP || algo == kCBPNMS;
    const size_t xfloats = ((size_t)lanes * dcmax + 1) & ~(size_t)1;
    size_t b = 4 * xfloats * (belief ? 1 : 2) + 8 * (size_t)lanes + 4 * 6 * (size_t)max_slots;
    if (dbg && belief) b += 12 * (size_t)max_slots + (size_t)lanes * (1 + 2 * (size_t)dcmax);
    return b;
}

int stream_groups_per_cu(int algo, int lanes, size_t lds) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stream_kernel<false>(algo), lanes, lds) != hipSuccess)
        return 0;
    return per_cu;
}

hipError_t launch_qc_stream(int algo, const StreamLaunch &L, const float *llr, uint8_t *bits,
                            int32_t *iters, int64_t batch, const int64_t *qstart,
                            const int32_t *perm, const int64_t *offset, unsigned int *counter,
                            int max_iter, const Params &p, const Dump &d, void *ws, hipStream_t s) {
    StreamArgs A{};
    A.llr = llr;
    A.bits = bits;
    A.iters = iters;
    A.codes = L.codes;
    A.ncodes = L.ncodes;
    A.lanes = L.lanes;
    A.dcmax = L.dcmax;
    A.xfloats = (int)(((size_t)L.lanes * L.dcmax + 1) & ~(size_t)1);
    A.max_slots = L.max_slots;
    A.qstart = qstart;
    A.perm = perm;
    A.offset = offset;
    A.counter = counter;
    A.batch = batch;
    A.max_iter = max_iter;
    A.p = p;
    A.d = d;
    A.ws = (char *)ws;
    A.group_bytes = L.group_bytes;
    const bool dbg = (d.sweep > 0 && d.frames > 0) || p.hd_mode == 1 || p.stop_rule == 1;
    const size_t lds = stream_lds_bytes(algo, L.lanes, L.dcmax, L.max_slots, dbg);
    const dim3 grid(L.groups), block(L.lanes);
    if (dbg) launch_algo<true>(algo, grid, block, lds, s, A);
    else launch_algo<false>(algo, grid, block, lds, s, A);
    return hipGetLastError();
}

hipError_t launch_mix_prepare(const int32_t *frame_code, const int64_t *offset, int64_t batch,
                              int64_t llr_elems, const StreamCode *codes, int ncodes,
                              int64_t *qstart, int32_t *perm, unsigned int *counter,
                              int32_t *iters, hipStream_t s) {
    hipLaunchKernelGGL(mix_prepare_kernel, dim3(1), dim3(1024), 0, s, frame_code, offset, batch,
                       llr_elems, codes, ncodes, qstart, perm, counter, iters);
    return hipGetLastError();
}

}  // namespace cbp
