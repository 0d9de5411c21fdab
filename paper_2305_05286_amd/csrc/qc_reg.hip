// Register-resident decoders for quasi-cyclic codes whose base pattern is
// compiled in (qc_graphs.inc); circulant shifts are runtime arguments.
//
// Layout.  A frame occupies Z lanes ("a slot"); lane l owns variable l of
// every block-column b (v = b*Z + l): its latest V2C message Q[b], the phi2
// term of that message as folded into its latest check PQ[b], the C2V message
// of each of its edges R[e] and its hard decisions (bit b of xb) all live in
// VGPRs (log-tanh CBP in log2 units, see phi.hpp).
// Block-row r is one layer of the sweep: its Z rows share no variable, so the
// Z lanes update them at once with exactly the result of the paper's
// row-by-row order.  Row k of block-row r meets variable (k + s) mod Z of
// block-column b, i.e. lane l talks to row (l - s) mod Z: the only cross-lane
// traffic is through LDS, one rotated (bank-conflict-free) access per edge:
//   phase 1 (lane = variable): B2V from the latest check's belief (LDS read),
//            V2C, hard decision, phi2 of the new V2C -> exchange slot of its row;
//   phase 2 (lane = row k):    fold the row's exchange entries into the
//            check-belief (max term, rest-of-sum, sign parity) -> LDS.
// Two barriers per layer.  Workgroups hold lcm(Z, 64)/Z slots (Z = 96: two
// frames in three waves) and are persistent: a slot whose frame stops (at a
// sweep boundary) writes its outputs and claims the next frame from a global
// counter, so long-running frames do not hold the rest of the chip.
#include <type_traits>
#include <utility>

#include "internal.hpp"
#include "phi.hpp"


namespace cbp {
namespace {

#include "qc_graphs.inc"

template <int B, int E, class F>
__host__ __device__ __forceinline__ constexpr void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <class G>
constexpr int count_edges() {
    int n = 0;
    for (int i = 0; i < G::MB * G::NB; ++i) n += G::P[i] ? 1 : 0;
    return n;
}

template <class G>
constexpr int slots_for() {
    int s = 1;
    while ((s * G::Z) % 64 != 0) ++s;
    return s;
}

// Compile-time description of a base pattern: edges in sweep order
// (block-row major, block-column ascending).
template <class G>
struct Tab {
    static constexpr int MB = G::MB, NB = G::NB, E = count_edges<G>();
    int er[E], eb[E], epred[E], ejpos[E];
    bool efirst[E];
    int rstart[MB + 1], dc[MB], csr_off[MB];
    int elast[NB];
    int dcmax;
};

template <class G>
constexpr Tab<G> make_tab() {
    Tab<G> T{};
    int e = 0;
    for (int r = 0; r < G::MB; ++r) {
        T.rstart[r] = e;
        for (int b = 0; b < G::NB; ++b)
            if (G::P[r * G::NB + b]) {
                T.er[e] = r;
                T.eb[e] = b;
                T.ejpos[e] = e - T.rstart[r];
                ++e;
            }
        T.dc[r] = e - T.rstart[r];
    }
    T.rstart[G::MB] = e;
    for (int b = 0; b < G::NB; ++b) {
        int first = -1, last = -1;
        for (int k = 0; k < e; ++k)
            if (T.eb[k] == b) {
                if (first < 0) first = k;
                last = k;
            }
        T.elast[b] = last;
        int prev = last;  // the latest check of a column's first row is its last row
        for (int k = 0; k < e; ++k)
            if (T.eb[k] == b) {
                T.epred[k] = prev;
                T.efirst[k] = (k == first);
                prev = k;
            }
    }
    int off = 0, mx = 0;
    for (int r = 0; r < G::MB; ++r) {
        T.csr_off[r] = off;
        off += T.dc[r] * G::Z;
        mx = T.dc[r] > mx ? T.dc[r] : mx;
    }
    T.dcmax = mx;
    return T;
}

template <class G>
struct TabOf {
    static constexpr Tab<G> T = make_tab<G>();
};

template <class G>
struct QcArgs {
    static constexpr int E = count_edges<G>();
    const float *llr;
    uint8_t *bits;
    int32_t *iters;
    unsigned int *counter;
    int64_t batch;
    int max_iter;
    Params p;
    Dump d;
    // device table [2E]: [e] = shift of the block of edge e, [E + e] = shift
    // of the block of the latest-check edge of e
    const int *sht;
};

// Opaque copies: recomputing a lane's rotated LDS indices per layer is cheaper
// than letting the compiler hoist all of them (two per edge) into VGPRs.
__device__ __forceinline__ int opaque_v(int x) {
    asm volatile("" : "+v"(x));
    return x;
}
// The shift table is never written during a launch: read through the
// constant address space it is loaded with scalar loads into SGPRs (as a
// generic pointer it would take flat vector loads and a VGPR per shift).
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *opaque_s(const T *p) {
    asm volatile("" : "+s"(p));
    return (const __attribute__((address_space(4))) T *)p;
}

// Occupancy target (waves per SIMD) handed to the register allocator.  The
// per-lane state is ~2 NB + E registers; measured on MI355X with the n=2304
// code, CBP is fastest at 3 (160 VGPRs; 2 leaves the SIMDs idle at the
// barriers, 4 spills in the loop), layered min-sum and min-sum CBP at 4
// (128 VGPRs; min-sum CBP 7% faster than at 3), flooding min-sum at 3.  The
// instantiations that also serve the dumps and the paper's stopping rule
// stay at 3 (at 4 the allocator gives up on them).
template <int kAlgo, bool kDbg>
constexpr int waves_per_simd() {
    return (kAlgo == kLBPNMS || (kAlgo == kCBPNMS && !kDbg)) ? 4 : 3;
}

// (x mod Z) for x in (-Z, 2Z)
template <int Z>
__device__ __forceinline__ int wrap(int x) {
    x += (x < 0) ? Z : 0;
    return x - ((x >= Z) ? Z : 0);
}

// (x mod Z) for x in (-Z, Z): as unsigned, a negative x exceeds x + Z.
template <int Z>
__device__ __forceinline__ int wrap_lo(int x) {
    const unsigned u = (unsigned)x, v = (unsigned)(x + Z);
    return (int)(u < v ? u : v);
}

// kDbg: the instantiation that also serves hd_mode = 1 and the state dumps;
// the production instantiation carries neither (cold code still costs
// registers in a kernel this close to its register budget).
template <class G, int kAlgo, bool kDbg>
__global__ __launch_bounds__(slots_for<G>() * G::Z, (waves_per_simd<kAlgo, kDbg>())) void qc_reg_kernel(QcArgs<G> A) {
    using TT = TabOf<G>;
    constexpr int MB = G::MB, NB = G::NB, Z = G::Z, E = count_edges<G>();
    constexpr int SL = slots_for<G>(), DCM = TT::T.dcmax;
    constexpr int64_t N = (int64_t)NB * Z;
    using Mask = std::conditional_t<(NB > 32), uint64_t, uint32_t>;
    // CBP in either check rule keeps check-beliefs; every rule but log-tanh
    // CBP folds a row into (min1, min2, parity)
    constexpr bool kBelief = kAlgo == kCBP || kAlgo == kCBPNMS;
    constexpr bool kMinRow = kAlgo != kCBP;

    // The exchange buffer, the min-sum row states and the decision words are
    // stored twice ([i] and [i + Z]) so that every rotated read (index i + s,
    // 0 <= i, s < Z) needs no wrap-around.
    __shared__ float2 sOm[kBelief ? SL : 1][kBelief ? MB * Z : 1];
    // Row of the latest check's block-row that lane l meets at edge e,
    // (l - s) mod Z for that check's shift s: the same for every frame and
    // sweep, so it is worked out once per launch and each B2V read costs one
    // byte load instead of a wrap-around in VALU.
    // (Log-tanh CBP only: min-sum CBP runs at four waves per SIMD, where
    // these E*Z bytes would cost a workgroup per CU.)
    constexpr bool kKp = kAlgo == kCBP;
    static_assert(!kKp || Z <= 256, "row indices are stored as bytes");
    __shared__ uint8_t sKp[kKp ? E : 1][kKp ? Z : 1];
    __shared__ float2 sRow[kBelief ? 1 : SL][kBelief ? 1 : 2 * Z];
    __shared__ float sX[SL][DCM][2 * Z];
    __shared__ Mask sXB[SL][2 * Z];
    // paper's stopping rule (kDbg): per-edge decision flips, per-row verdicts
    constexpr bool kStop = kDbg && kBelief;
    __shared__ uint8_t sFl[kStop ? SL : 1][kStop ? DCM : 1][kStop ? 2 * Z : 1];
    __shared__ uint8_t sGood[kStop ? SL : 1][kStop ? Z : 1];
    __shared__ int sStop[SL];
    __shared__ long long sRun[SL];
    __shared__ unsigned int sF[SL];
    __shared__ int sBad[2][SL];
    __shared__ int sAct[SL], sFresh[SL];

    const int slot = tid_x() / Z;
    const int l = tid_x() - slot * Z;
    // The log-tanh rule keeps every LLR in log2 units (L / ln2), where one
    // function (phi2) serves both directions of the check rule; the min-sum
    // rules are linear and keep natural units.
    constexpr bool kLog2 = kAlgo == kCBP;
    const float us = kLog2 ? kLog2e : 1.0f;
    const float a = A.p.a * us, lmax = A.p.lmax * us, alpha = A.p.alpha;

    // CBP: Q = latest V2C, PQ = phi2(clamped Q) as folded.  NMS: Q = posterior
    // Lambda, PQ = flooding accumulator of the new C2V messages.
    float Q[NB], PQ[NB], R[E];
    Mask xb = 0;
    int64_t f;
    int t = 0, it = 0;
    // paper's stopping rule: rows in a row (across sweeps) with Omega > 0 and no
    // flipped decision; when the run reaches M mid-layer, the decisions of the
    // layer's later rows are reverted and frozen in xb_stop
    const bool paper = kStop && A.p.stop_rule == 1;
    long long run = 0;
    bool pstop = false;
    Mask xb_stop = 0;

    auto load = [&](int64_t fr) {
        xb = 0;
        static_for<0, NB>([&](auto bc) {
            constexpr int b = bc;
            const float v = A.llr[fr * N + b * Z + l] * us + 0.0f;  // -0.0 -> +0.0
            Q[b] = v;
            PQ[b] = 0.0f;
            if (v < 0.0f) xb |= Mask(1) << b;
        });
        static_for<0, E>([&](auto ec) { R[decltype(ec)::value] = 0.0f; });
        if constexpr (kBelief) {
            // A variable's first visit in a frame has no latest check and its
            // B2V message is 0 (Step 1's infinite belief only seeds the C2B
            // fold).  A stored belief whose exclusion is +inf (log-tanh: g(inf)
            // = 0) or whose two smallest terms are 0 (min-sum) yields exactly
            // that 0, so the first sweep needs no test of its own; its first
            // visits also commit that 0 to R, which already holds 0.
            const float z = kAlgo == kCBP ? __builtin_inff() : 0.0f;
            static_for<0, MB>([&](auto rc) { sOm[slot][decltype(rc)::value * Z + l] = make_float2(z, z); });
        }
    };

    if constexpr (kKp)
        for (int i = tid_x(); i < E * Z; i += SL * Z) {
            const int e = i / Z, k = i - e * Z;
            sKp[e][k] = (uint8_t)wrap_lo<Z>(k - A.sht[E + e]);
        }
    if (l == 0) sF[slot] = atomicAdd(A.counter, 1u);
    __syncthreads();
    f = sF[slot];
    if (f < A.batch) load(f);

    for (;;) {
        // ---------------- syndrome of the current decisions --------------
        const int pb = it & 1;
        ++it;
        if (l == 0) sBad[pb][slot] = 0;
        sXB[slot][l] = xb;
        sXB[slot][l + Z] = xb;
        __syncthreads();
        uint32_t bad = 0;
        static_for<0, MB>([&](auto rc) {
            constexpr int r = rc;
            constexpr int e0 = TT::T.rstart[r], D = TT::T.rstart[r + 1] - e0;
            const int lv = opaque_v(l);
            const auto sh = opaque_s(A.sht);
            // row l meets lane l + s; bit 0 of the XOR of the words shifted
            // down by their block-columns is the row's parity, two at a time
            auto word = [&](auto ec) {
                constexpr int e = ec;
                return (uint32_t)(sXB[slot][lv + sh[e]] >> TT::T.eb[e]);
            };
            uint32_t par = 0;
            static_for<0, D / 2>([&](auto pc) {
                constexpr int e = e0 + 2 * pc;
                par = xor3(par, word(std::integral_constant<int, e>{}), word(std::integral_constant<int, e + 1>{}));
            });
            if constexpr (D % 2) par ^= word(std::integral_constant<int, e0 + D - 1>{});
            bad |= par & 1u;
        });
        if (bad) sBad[pb][slot] = 1;
        __syncthreads();
        const bool ok = sBad[pb][slot] == 0;
        const bool have = f < A.batch;
        const bool done = !have || t >= A.max_iter || (A.p.stop_rule == 0 && ok) || (paper && pstop);
        const bool claim = done && have;
        if (claim) {
            const Mask xo = (paper && pstop) ? xb_stop : xb;
            static_for<0, NB>([&](auto bc) {
                constexpr int b = bc;
                A.bits[f * N + b * Z + l] = (uint8_t)((xo >> b) & 1u);
            });
            if (l == 0) {
                A.iters[f] = t;
                sF[slot] = atomicAdd(A.counter, 1u);
            }
        }
        __syncthreads();
        if (claim) {
            f = sF[slot];
            t = 0;
            run = 0;
            pstop = false;
            if (f < A.batch) load(f);
        }
        if (l == 0) {
            sAct[slot] = f < A.batch;
            sFresh[slot] = claim && f < A.batch;
        }
        __syncthreads();
        bool anyAct = false, anyFresh = false;
        static_for<0, SL>([&](auto sc) {
            anyAct |= sAct[decltype(sc)::value] != 0;
            anyFresh |= sFresh[decltype(sc)::value] != 0;
        });
        if (!anyAct) break;
        if (anyFresh) continue;  // pre-check the new frames first

        // ---------------- one sweep over the layers -------------------------
        static_for<0, MB>([&](auto rc) {
            constexpr int r = rc;
            constexpr int e0 = TT::T.rstart[r], e1 = TT::T.rstart[r + 1];
            float qk[e1 - e0];
            const int lv = opaque_v(l);
            const auto sh = opaque_s(A.sht);
            [[maybe_unused]] const Mask xb_prev = xb;  // decisions before this layer
            // phase 1: lane = variable
            static_for<e0, e1>([&](auto ec) {
                constexpr int e = ec;
                constexpr int b = TT::T.eb[e], j = e - e0;
                if constexpr (kBelief) {
                    constexpr int ep = TT::T.epred[e], rp = TT::T.er[ep];
                    // B2V (eq. equ_s4e18) from the latest check's belief
                    int kp;
                    if constexpr (kKp) kp = sKp[e][lv];
                    else kp = wrap_lo<Z>(lv - sh[E + e]);
                    const float2 om = sOm[slot][rp * Z + kp];
                    float rn;
                    if constexpr (kAlgo == kCBP) {
                        const float dd = excl_sum(abs_bits(om.x), om.y, PQ[b]);
                        rn = or_sign(phi2(dd), fbits(om.x) ^ fbits(Q[b]));
                    } else {  // min-sum rule (eq. equ_s4e18xx)
                        const float aq = __builtin_fminf(__builtin_fabsf(Q[b]), lmax);
                        const float m1 = abs_bits(om.x);
                        rn = or_sign(alpha * ((aq == m1) ? om.y : m1), fbits(om.x) ^ fbits(Q[b]));
                    }
                    R[ep] = rn;                       // commit R(c_j -> v) first
                    const float lam = Q[b] + rn;      // eq. equ_s4e20
                    xb = (xb & ~(Mask(1) << b)) | (Mask(fbits(lam) >> 31) << b);  // [lam < 0]
                    if constexpr (kStop) {
                        if (paper) {
                            const uint8_t fl = (uint8_t)(((xb ^ xb_prev) >> b) & 1u);
                            sFl[slot][j][lv] = fl;
                            sFl[slot][j][lv + Z] = fl;
                        }
                    }
                    const float qn = lam - R[e];      // V2C, eq. equ_s4e19
                    float fq;
                    if constexpr (kAlgo == kCBP) {
                        fq = phi2_clamped(qn, a, lmax);
                        PQ[b] = fq;
                    } else {
                        fq = __builtin_fminf(__builtin_fabsf(qn), lmax);
                    }
                    Q[b] = qn;
                    const float xv = or_sign(fq, fbits(qn));
                    sX[slot][j][lv] = xv;
                    sX[slot][j][lv + Z] = xv;
                } else {
                    const float q = Q[b] - R[e];      // eq. equ_s2e10 / equ_s2e3
                    qk[j] = q;
                    const float xv = or_sign(__builtin_fminf(__builtin_fabsf(q), lmax), fbits(q));
                    sX[slot][j][lv] = xv;
                    sX[slot][j][lv + Z] = xv;
                }
            });
            __syncthreads();
            // phase 2: lane = row l of this layer; its entry from block-column
            // b_j was written by lane (l + s_j) mod Z
            {
                uint32_t par = 0;
                const int lr = opaque_v(l);
                const auto shr = opaque_s(A.sht);
                // the row's entries two at a time (a lone last one for odd degree)
                constexpr int D = e1 - e0;
                auto entry = [&](auto jc) { return sX[slot][decltype(jc)::value][lr + shr[e0 + decltype(jc)::value]]; };
                if constexpr (!kMinRow) {
                    float Mx = 0.0f, Sr = 0.0f;
                    static_for<0, D / 2>([&](auto pc) {
                        constexpr int j = 2 * pc;
                        const float x = entry(std::integral_constant<int, j>{});
                        const float y = entry(std::integral_constant<int, j + 1>{});
                        par = xor3(par, fbits(x), fbits(y));
                        fold2(Mx, Sr, abs_bits(x), abs_bits(y));  // C2B, eq. equ_s4e21
                    });
                    if constexpr (D % 2) {
                        const float x = entry(std::integral_constant<int, D - 1>{});
                        par ^= fbits(x);
                        fold(Mx, Sr, abs_bits(x));
                    }
                    sOm[slot][r * Z + l] = make_float2(or_sign(Mx, par), Sr);  // eq. equ_s4e23
                } else {
                    float m1 = __builtin_inff(), m2 = __builtin_inff();
                    static_for<0, D / 2>([&](auto pc) {
                        constexpr int j = 2 * pc;
                        const float x = entry(std::integral_constant<int, j>{});
                        const float y = entry(std::integral_constant<int, j + 1>{});
                        par = xor3(par, fbits(x), fbits(y));
                        fold_min2(m1, m2, abs_bits(x), abs_bits(y));
                    });
                    if constexpr (D % 2) {
                        const float x = entry(std::integral_constant<int, D - 1>{});
                        par ^= fbits(x);
                        fold_min(m1, m2, abs_bits(x));
                    }
                    const float2 rs = make_float2(or_sign(m1, par), m2);
                    if constexpr (kBelief) {
                        sOm[slot][r * Z + l] = rs;  // C2B, eq. equ_s4e21xx
                    } else {
                        sRow[slot][l] = rs;
                        sRow[slot][l + Z] = rs;
                    }
                }
                if constexpr (kStop) {
                    if (paper) {  // Step 2(3): this row's update keeps Omega > 0 and flips nothing
                        uint8_t fl = 0;
                        static_for<0, e1 - e0>([&](auto jc) {
                            constexpr int j = jc;
                            fl |= sFl[slot][j][lr + shr[e0 + j]];
                        });
                        sGood[slot][l] = (uint8_t)(((par >> 31) == 0) && fl == 0);
                    }
                }
            }
            __syncthreads();
            if constexpr (kStop) {
                if (paper) {
                    // rows of this layer in index order, continuing the run
                    if (l == 0) {
                        constexpr long long Mrows = (long long)MB * Z;
                        int lead = 0, trail = 0;
                        bool all = true;
                        for (int k = 0; k < Z; ++k) {
                            if (sGood[slot][k]) {
                                ++trail;
                                if (all) ++lead;
                            } else {
                                all = false;
                                trail = 0;
                            }
                        }
                        int kstop = -1;
                        if (!pstop && run + lead >= Mrows) kstop = (int)(Mrows - run - 1);
                        sStop[slot] = kstop;
                        sRun[slot] = all ? run + Z : trail;
                    }
                    __syncthreads();
                    const int kstop = sStop[slot];
                    run = sRun[slot];
                    if (!pstop && kstop >= 0) {
                        // stop after row kstop: rows beyond it in this layer are undone
                        Mask xs = xb;
                        static_for<e0, e1>([&](auto ec) {
                            constexpr int e = ec;
                            constexpr int b = TT::T.eb[e];
                            if (wrap_lo<Z>(lv - sh[e]) > kstop)
                                xs = (xs & ~(Mask(1) << b)) | (xb_prev & (Mask(1) << b));
                        });
                        xb_stop = xs;
                        pstop = true;
                    }
                    __syncthreads();
                }
            }
            if constexpr (!kBelief) {
                // phase 3: lane = variable, normalized min-sum C2V
                static_for<e0, e1>([&](auto ec) {
                    constexpr int e = ec;
                    constexpr int b = TT::T.eb[e], j = e - e0;
                    const float2 rw = sRow[slot][lv + Z - sh[e]];
                    const float aq = __builtin_fminf(__builtin_fabsf(qk[j]), lmax);
                    const float m1 = abs_bits(rw.x);
                    const float rn = or_sign(alpha * ((aq == m1) ? rw.y : m1), fbits(rw.x) ^ fbits(qk[j]));
                    R[e] = rn;
                    if constexpr (kAlgo == kLBPNMS) Q[b] = qk[j] + rn;  // eq. equ_s2e12
                    else PQ[b] += rn;
                });
            }
        });
        ++t;

        // ---------------- end of sweep ------------------------------------
        if constexpr (kAlgo == kFBPNMS) {
            if (f < A.batch)
                static_for<0, NB>([&](auto bc) {
                    constexpr int b = bc;
                    Q[b] = (A.llr[f * N + b * Z + l] + 0.0f) + PQ[b];  // eq. equ_s2e6
                    PQ[b] = 0.0f;
                });
        }
        if constexpr (!kBelief) {
            xb = 0;
            static_for<0, NB>([&](auto bc) {
                constexpr int b = bc;
                if (Q[b] < 0.0f) xb |= Mask(1) << b;
            });
        }
        auto flushed = [&](auto bc) {
            constexpr int b = bc;
            constexpr int el = TT::T.elast[b], rl = TT::T.er[el];
            const float2 om = sOm[slot][rl * Z + wrap_lo<Z>(opaque_v(l) - opaque_s(A.sht)[el])];
            if constexpr (kAlgo == kCBP) {
                const float dd = excl_sum(abs_bits(om.x), om.y, PQ[b]);
                return Q[b] + with_sign(phi2(dd), sign_bit(om.x) ^ (Q[b] < 0.0f));
            } else {
                const float aq = __builtin_fminf(__builtin_fabsf(Q[b]), lmax);
                const float m1 = abs_bits(om.x);
                return Q[b] + with_sign(alpha * ((aq == m1) ? om.y : m1), sign_bit(om.x) ^ (Q[b] < 0.0f));
            }
        };
        if constexpr (kBelief && kDbg) {
            if (A.p.hd_mode == 1) {
                xb = 0;
                static_for<0, NB>([&](auto bc) {
                    if (flushed(bc) < 0.0f) xb |= Mask(1) << decltype(bc)::value;
                });
            }
        }
        if (kDbg && t == A.d.sweep && f < A.d.frames) {
            const int64_t Etot = (int64_t)E * Z, M = (int64_t)MB * Z;
            const float un = kLog2 ? kLn2 : 1.0f;  // dumps in natural units
            static_for<0, NB>([&](auto bc) {
                constexpr int b = bc;
                if constexpr (kBelief) {
                    if (A.d.q) A.d.q[f * N + b * Z + l] = Q[b] * un;
                    if (A.d.lam) A.d.lam[f * N + b * Z + l] = flushed(bc) * un;
                } else {
                    if (A.d.lam) A.d.lam[f * N + b * Z + l] = Q[b];
                }
            });
            if (A.d.r)
                static_for<0, E>([&](auto ec) {
                    constexpr int e = ec;
                    constexpr int r = TT::T.er[e];
                    const int k = wrap<Z>(l - A.sht[e]);
                    A.d.r[f * Etot + TT::T.csr_off[r] + k * TT::T.dc[r] + TT::T.ejpos[e]] = R[e] * un;
                });
            if constexpr (kBelief) {
                if (A.d.om)
                    static_for<0, MB>([&](auto rc) {
                        constexpr int r = rc;
                        const float2 om = sOm[slot][r * Z + l];
                        A.d.om[f * M + r * Z + l] =
                            kAlgo == kCBP ? with_sign(phi2(abs_bits(om.x) + om.y) * un, sign_bit(om.x))
                                          : with_sign(alpha * abs_bits(om.x), sign_bit(om.x));
                    });
            }
        }
    }
}

template <class G>
void graph_entry(int *mb, int *nb, int *Z, const uint8_t **pat) {
    *mb = G::MB;
    *nb = G::NB;
    *Z = G::Z;
    *pat = G::P;
}

template <class G>
int graph_shift_table(const int *shifts, int *out) {
    using TT = TabOf<G>;
    constexpr int E = count_edges<G>();
    for (int e = 0; e < E; ++e) {
        out[e] = shifts[TT::T.er[e] * G::NB + TT::T.eb[e]];
        const int ep = TT::T.epred[e];
        out[E + e] = shifts[TT::T.er[ep] * G::NB + TT::T.eb[ep]];
    }
    return 2 * E;
}

template <class G, int kAlgo, bool kDbg>
hipError_t launch_graph(const int *sht, const float *llr, uint8_t *bits, int32_t *iters,
                        int64_t batch, int max_iter, const Params &p, const Dump &d,
                        int *counter, int device, hipStream_t s) {
    constexpr int SL = slots_for<G>(), threads = SL * G::Z;
    QcArgs<G> A{};
    A.llr = llr;
    A.bits = bits;
    A.iters = iters;
    A.counter = (unsigned int *)counter;
    A.batch = batch;
    A.max_iter = max_iter;
    A.p = p;
    A.d = d;
    A.sht = sht;
    // persistent grid: as many workgroups as fit on the device at once
    static int cached_blocks[64] = {0};
    const int dev = device < 64 ? device : 0;
    if (cached_blocks[dev] == 0) {
        int per_cu = 0, cus = 0;
        hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(qc_reg_kernel<G, kAlgo, kDbg>), threads, 0);
        if (err != hipSuccess) return err;
        err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
        if (err != hipSuccess) return err;
        cached_blocks[dev] = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
    }
    const int64_t need = (batch + SL - 1) / SL;
    const int blocks = (int)(need < cached_blocks[dev] ? need : cached_blocks[dev]);
    hipError_t err = launch_fill_i32(counter, 1, 0, s);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL((qc_reg_kernel<G, kAlgo, kDbg>), dim3(blocks), dim3(threads), 0, s, A);
    return hipGetLastError();
}

}  // namespace

int qc_reg_count() { return CBP_QC_GRAPH_COUNT; }

void qc_reg_entry(int k, int *mb, int *nb, int *Z, const uint8_t **pattern) {
#define CBP_ENTRY(K, G) \
    if (k == K) graph_entry<G>(mb, nb, Z, pattern);
    CBP_QC_GRAPHS(CBP_ENTRY)
#undef CBP_ENTRY
}

int qc_reg_shift_table(int k, const int *shifts, int *out) {
#define CBP_TABLE(K, G) \
    if (k == K) return graph_shift_table<G>(shifts, out);
    CBP_QC_GRAPHS(CBP_TABLE)
#undef CBP_TABLE
    return 0;
}

hipError_t launch_qc_reg(int k, int algo, const int *sht, const float *llr, uint8_t *bits,
                         int32_t *iters, int64_t batch, int max_iter, const Params &p,
                         const Dump &d, int *counter, int device, hipStream_t s) {
#define CBP_LAUNCH_ALGO(G, DBG)                                                               \
    switch (algo) {                                                                           \
    case kCBP:                                                                                \
        return launch_graph<G, kCBP, DBG>(sht, llr, bits, iters, batch, max_iter, p, d,       \
                                          counter, device, s);                                \
    case kLBPNMS:                                                                             \
        return launch_graph<G, kLBPNMS, DBG>(sht, llr, bits, iters, batch, max_iter, p, d,    \
                                             counter, device, s);                             \
    case kFBPNMS:                                                                             \
        return launch_graph<G, kFBPNMS, DBG>(sht, llr, bits, iters, batch, max_iter, p, d,    \
                                             counter, device, s);                             \
    default:                                                                                  \
        return launch_graph<G, kCBPNMS, DBG>(sht, llr, bits, iters, batch, max_iter, p, d,    \
                                             counter, device, s);                             \
    }
#define CBP_LAUNCH(K, G)                                                                      \
    if (k == K) {                                                                             \
        if (dbg) {                                                                            \
            CBP_LAUNCH_ALGO(G, true)                                                          \
        }                                                                                     \
        CBP_LAUNCH_ALGO(G, false)                                                             \
    }
    const bool dbg = (d.sweep > 0 && d.frames > 0) || p.hd_mode == 1 || p.stop_rule == 1;
    CBP_QC_GRAPHS(CBP_LAUNCH)
#undef CBP_LAUNCH
#undef CBP_LAUNCH_ALGO
    return hipErrorInvalidValue;
}

}  // namespace cbp
