// Quasi-cyclic decoders for any base matrix, with the per-frame state in a
// device workspace instead of registers (frames too large for the register
// file, or base patterns that are not compiled in).
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

#ifndef STREAM_WPE_N
#define STREAM_WPE_N 8
#endif

namespace cbp {
namespace {

struct StreamArgs {
    const float *llr;
    uint8_t *bits;
    int32_t *iters;
    unsigned int *counter;
    int64_t batch;
    int max_iter;
    Params p;
    Dump d;
    QcStreamDev g;
    char *ws;           // slot workspaces, ws_stride bytes apart
    int64_t ws_stride;
};

struct Edge {
    int b, sh, ep, epsh, epr;
    bool last, first;
};
__device__ __forceinline__ Edge edge(const QcStreamDev &g, int e) {
    const int *rec = reinterpret_cast<const int *>(g.erec) + 4 * (int64_t)e;
    const int x = ldc(rec, 0), w = ldc(rec, 3);
    return Edge{x & 0xffff, ldc(rec, 1), ldc(rec, 2), w & 0xffff, w >> 16, ((x >> 29) & 1) != 0,
                ((x >> 30) & 1) != 0};
}

template <int kAlgo>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(STREAM_WPE_N)))
void qc_stream_kernel(StreamArgs A) {
    extern __shared__ float smem[];
    const QcStreamDev &g = A.g;
    const int Z = g.Z, NB = g.nb, MB = g.mb, E = g.E;
    const int64_t N = (int64_t)NB * Z;
    const int SL = g.slots;
    const int slot = threadIdx.x / Z;
    const int l = threadIdx.x - slot * Z;
    // LDS: exchange [SL][dcmax][Z] floats, NMS V2C stash [SL][dcmax][Z] floats,
    // row state [SL][Z] float2, flags
    const size_t xfloats = ((size_t)2 * SL * g.dcmax * Z + 1) & ~(size_t)1;  // keep sRow 8-byte aligned
    float *sX = smem + (size_t)slot * g.dcmax * Z;
    float *sQ = smem + (size_t)(SL + slot) * g.dcmax * Z;
    float2 *sRow = reinterpret_cast<float2 *>(smem + xfloats) + (size_t)slot * Z;
    int *sFlags = reinterpret_cast<int *>(smem + xfloats + 2 * (size_t)SL * Z);
    unsigned int *sF = reinterpret_cast<unsigned int *>(sFlags);  // [SL]
    int *sBad = sFlags + SL;                                        // [2][SL]
    int *sAct = sFlags + 3 * SL;                                    // [SL]
    int *sFresh = sFlags + 4 * SL;                                  // [SL]

    constexpr bool kBelief = kAlgo == kCBP || kAlgo == kCBPNMS;
    const int64_t gslot = (int64_t)blockIdx.x * SL + slot;
    char *base = A.ws + gslot * A.ws_stride;
    float *Q = reinterpret_cast<float *>(base);
    float *PQ = Q + N;                                     // FBP only
    float *R = Q + (kAlgo == kFBPNMS ? 2 * N : N);
    float2 *OM = reinterpret_cast<float2 *>(base + ((4 * ((kAlgo == kFBPNMS ? 2 : 1) * N + (int64_t)E * Z) + 7) & ~(int64_t)7));
    uint8_t *XB = reinterpret_cast<uint8_t *>(OM + (kBelief ? (int64_t)MB * Z : 0));  // slot end = qc_stream_slot_bytes

    // The log-tanh rule keeps every LLR in log2 units (L / ln2), where one
    // function (phi2) serves both directions of the check rule.
    constexpr bool kLog2 = kAlgo == kCBP;
    const float us = kLog2 ? kLog2e : 1.0f;
    const float a = A.p.a * us, lmax = A.p.lmax * us, alpha = A.p.alpha;

    auto load = [&](int64_t fr) {
        for (int b = 0; b < NB; ++b) {
            const float v = A.llr[fr * N + (int64_t)b * Z + l] * us;
            Q[b * Z + l] = v;
            if constexpr (kAlgo == kFBPNMS) PQ[b * Z + l] = 0.0f;
            XB[b * Z + l] = v < 0.0f;
        }
        for (int e = 0; e < E; ++e) R[(int64_t)e * Z + l] = 0.0f;
    };

    if (l == 0) sF[slot] = atomicAdd(A.counter, 1u);
    __syncthreads();
    int64_t f = sF[slot];
    int t = 0, it = 0;
    if (f < A.batch) load(f);

    for (;;) {
        // ---------------- syndrome of the current decisions --------------
        const int pb = it & 1;
        ++it;
        if (l == 0) sBad[pb * SL + slot] = 0;
        __syncthreads();  // decisions of all lanes written
        uint32_t bad = 0;
        for (int r = 0; r < MB; ++r) {
            uint32_t par = 0;
            for (int e = ldc(g.rstart, r); e < ldc(g.rstart, r + 1); ++e) {
                const Edge ed = edge(g, e);
                int idx = l + ed.sh;
                idx -= (idx >= Z) ? Z : 0;
                par ^= XB[ed.b * Z + idx];
            }
            bad |= par;
        }
        if (bad) sBad[pb * SL + slot] = 1;
        __syncthreads();
        const bool ok = sBad[pb * SL + slot] == 0;
        const bool have = f < A.batch;
        const bool done = !have || t >= A.max_iter || (A.p.stop_rule == 0 && ok);
        const bool claim = done && have;
        if (claim) {
            for (int b = 0; b < NB; ++b) A.bits[f * N + (int64_t)b * Z + l] = XB[b * Z + l];
            if (l == 0) {
                A.iters[f] = t;
                sF[slot] = atomicAdd(A.counter, 1u);
            }
        }
        __syncthreads();
        if (claim) {
            f = sF[slot];
            t = 0;
            if (f < A.batch) load(f);
        }
        if (l == 0) {
            sAct[slot] = f < A.batch;
            sFresh[slot] = claim && f < A.batch;
        }
        __syncthreads();
        bool anyAct = false, anyFresh = false;
        for (int s = 0; s < SL; ++s) {
            anyAct |= sAct[s] != 0;
            anyFresh |= sFresh[s] != 0;
        }
        if (!anyAct) break;
        if (anyFresh) continue;

        // ---------------- one sweep ---------------------------------------
        const bool first = (t == 0);
        for (int r = 0; r < MB; ++r) {
            const int e0 = ldc(g.rstart, r), e1 = ldc(g.rstart, r + 1);
            // phase 1: lane = variable
            for (int e = e0; e < e1; ++e) {
                const Edge ed = edge(g, e);
                const int iv = ed.b * Z + l;
                int kc = l - ed.sh;
                kc += (kc < 0) ? Z : 0;
                if constexpr (kBelief) {
                    const float q = Q[iv];
                    float rn = 0.0f;
                    bool own = false;  // R(c_j -> v) is R(c_i -> v): a degree-1 column
                    if (!(first && ed.first)) {
                        int kp = l - ed.epsh;
                        kp += (kp < 0) ? Z : 0;
                        const float2 om = OM[ed.epr * Z + kp];
                        if constexpr (kAlgo == kCBP) {
                            // Q_v is still the V2C value whose phi2 c_j folded
                            const float dd = excl_sum(abs_bits(om.x), om.y, phi2_clamped(q, a, lmax));
                            rn = with_sign(phi2(dd), sign_bit(om.x) ^ (q < 0.0f));
                        } else {
                            const float aq = __builtin_fminf(__builtin_fabsf(q), lmax);
                            const float m1 = abs_bits(om.x);
                            rn = with_sign(alpha * ((aq == m1) ? om.y : m1), sign_bit(om.x) ^ (q < 0.0f));
                        }
                        R[(int64_t)ed.ep * Z + l] = rn;  // commit R(c_j -> v) first
                        own = ed.ep == e;
                    }
                    const float lam = q + rn;
                    if (ed.last) XB[iv] = lam < 0.0f;  // v's last visit of the sweep decides
                    const float qn = lam - (own ? rn : R[(int64_t)e * Z + l]);
                    const float fq = kAlgo == kCBP ? phi2_clamped(qn, a, lmax)
                                                   : __builtin_fminf(__builtin_fabsf(qn), lmax);
                    Q[iv] = qn;
                    sX[(e - e0) * Z + kc] = with_sign(fq, qn < 0.0f);
                } else {
                    const float q = Q[iv] - R[(int64_t)e * Z + l];
                    sQ[(e - e0) * Z + l] = q;  // kept for phase 3
                    sX[(e - e0) * Z + kc] = with_sign(__builtin_fminf(__builtin_fabsf(q), lmax), q < 0.0f);
                }
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
                    OM[r * Z + l] = make_float2(with_sign(Mx, par), Sr);
                } else {
                    float m1 = __builtin_inff(), m2 = __builtin_inff();
                    for (int j = 0; j < e1 - e0; ++j) {
                        const float x = sX[j * Z + l];
                        par ^= sign_bit(x);
                        const float ax = abs_bits(x);
                        m2 = __builtin_fminf(m2, __builtin_fmaxf(m1, ax));
                        m1 = __builtin_fminf(m1, ax);
                    }
                    if constexpr (kBelief) OM[r * Z + l] = make_float2(with_sign(m1, par), m2);
                    else sRow[l] = make_float2(with_sign(m1, par), m2);
                }
            }
            __syncthreads();
            if constexpr (!kBelief) {
                // phase 3: lane = variable
                for (int e = e0; e < e1; ++e) {
                    const Edge ed = edge(g, e);
                    const int iv = ed.b * Z + l;
                    int kc = l - ed.sh;
                    kc += (kc < 0) ? Z : 0;
                    const float2 rw = sRow[kc];
                    const float q = sQ[(e - e0) * Z + l];
                    const float aq = __builtin_fminf(__builtin_fabsf(q), lmax);
                    const float m1 = abs_bits(rw.x);
                    const float rn = with_sign(alpha * ((aq == m1) ? rw.y : m1), sign_bit(rw.x) ^ (q < 0.0f));
                    R[(int64_t)e * Z + l] = rn;
                    if constexpr (kAlgo == kLBPNMS) Q[iv] = q + rn;
                    else PQ[iv] += rn;
                }
            }
        }
        ++t;

        // ---------------- end of sweep ------------------------------------
        if constexpr (!kBelief) {
            for (int b = 0; b < NB; ++b) {
                const int iv = b * Z + l;
                float lam = Q[iv];
                if constexpr (kAlgo == kFBPNMS) {
                    if (f < A.batch) lam = A.llr[f * N + iv] + PQ[iv];
                    Q[iv] = lam;
                    PQ[iv] = 0.0f;
                }
                XB[iv] = lam < 0.0f;
            }
        }
        auto flushed = [&](int b) {
            const int el = ldc(g.elast, b);
            int k = l - ldc(g.esh, el);
            k += (k < 0) ? Z : 0;
            const float2 om = OM[ldc(g.er, el) * Z + k];
            const float q = Q[b * Z + l];
            if constexpr (kAlgo == kCBP) {
                const float dd = excl_sum(abs_bits(om.x), om.y, phi2_clamped(q, a, lmax));
                return q + with_sign(phi2(dd), sign_bit(om.x) ^ (q < 0.0f));
            } else {
                const float aq = __builtin_fminf(__builtin_fabsf(q), lmax);
                const float m1 = abs_bits(om.x);
                return q + with_sign(alpha * ((aq == m1) ? om.y : m1), sign_bit(om.x) ^ (q < 0.0f));
            }
        };
        if constexpr (kBelief) {
            if (A.p.hd_mode == 1)
                for (int b = 0; b < NB; ++b) XB[b * Z + l] = flushed(b) < 0.0f;
        }
        if (t == A.d.sweep && f < A.d.frames) {
            const int64_t Etot = (int64_t)E * Z, M = (int64_t)MB * Z;
            const float un = kLog2 ? kLn2 : 1.0f;  // dumps in natural units
            for (int b = 0; b < NB; ++b) {
                if constexpr (kBelief) {
                    if (A.d.q) A.d.q[f * N + b * Z + l] = Q[b * Z + l] * un;
                    if (A.d.lam) A.d.lam[f * N + b * Z + l] = flushed(b) * un;
                } else {
                    if (A.d.lam) A.d.lam[f * N + b * Z + l] = Q[b * Z + l];
                }
            }
            if (A.d.r)
                for (int e = 0; e < E; ++e) {
                    const int r = ldc(g.er, e);
                    int k = l - ldc(g.esh, e);
                    k += (k < 0) ? Z : 0;
                    const int r0 = ldc(g.rstart, r), dc = ldc(g.rstart, r + 1) - r0;
                    A.d.r[f * Etot + (int64_t)r0 * Z + (int64_t)k * dc + (e - r0)] = R[(int64_t)e * Z + l] * un;
                }
            if constexpr (kBelief) {
                if (A.d.om)
                    for (int r = 0; r < MB; ++r) {
                        const float2 om = OM[r * Z + l];
                        A.d.om[f * M + (int64_t)r * Z + l] =
                            kAlgo == kCBP ? with_sign(phi2(abs_bits(om.x) + om.y) * un, sign_bit(om.x))
                                          : with_sign(alpha * abs_bits(om.x), sign_bit(om.x));
                    }
            }
        }
    }
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

int slots_per_group(int Z) {
    if (Z >= 64) return (Z % 64 == 0) ? 1 : (Z % 32 == 0 ? 2 : 1);
    int s = 1;
    while ((s * Z) % 64 != 0 && s * Z < 1024) ++s;
    return s;
}

}  // namespace

int64_t qc_stream_slot_bytes(int algo, const QcStreamDev &g) {
    const int64_t N = (int64_t)g.nb * g.Z;
    int64_t b = round_up(4 * ((algo == kFBPNMS ? 2 : 1) * N + (int64_t)g.E * g.Z), 8);
    if (algo == kCBP || algo == kCBPNMS) b += 8LL * g.mb * g.Z;
    b += N;
    return round_up(b, 256);
}

void qc_stream_shape(const QcStreamDev &g, int *slots, int *threads, size_t *lds) {
    const int SL = slots_per_group(g.Z);
    *slots = SL;
    *threads = SL * g.Z;
    const size_t xfloats = ((size_t)2 * SL * g.dcmax * g.Z + 1) & ~(size_t)1;
    *lds = xfloats * 4 + (size_t)SL * g.Z * 8 + 8 * 4 * (size_t)SL;
}

int qc_stream_groups(int algo, const QcStreamDev &g, int device) {
    int slots, threads;
    size_t lds;
    qc_stream_shape(g, &slots, &threads, &lds);
    int per_cu = 0, cus = 0;
    const void *fn = algo == kCBP      ? reinterpret_cast<const void *>(qc_stream_kernel<kCBP>)
                     : algo == kLBPNMS ? reinterpret_cast<const void *>(qc_stream_kernel<kLBPNMS>)
                     : algo == kFBPNMS ? reinterpret_cast<const void *>(qc_stream_kernel<kFBPNMS>)
                                       : reinterpret_cast<const void *>(qc_stream_kernel<kCBPNMS>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess) per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) cus = 1;
    return (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
}

hipError_t launch_qc_stream(int algo, const QcStreamDev &g, const float *llr, uint8_t *bits,
                            int32_t *iters, int64_t batch, int max_iter, const Params &p,
                            const Dump &d, int groups, void *ws, int *counter, hipStream_t s) {
    int slots, threads;
    size_t lds;
    qc_stream_shape(g, &slots, &threads, &lds);
    StreamArgs A{};
    A.llr = llr;
    A.bits = bits;
    A.iters = iters;
    A.counter = (unsigned int *)counter;
    A.batch = batch;
    A.max_iter = max_iter;
    A.p = p;
    A.d = d;
    A.g = g;
    A.g.slots = slots;
    A.ws = (char *)ws;
    A.ws_stride = qc_stream_slot_bytes(algo, g);
    hipError_t err = launch_fill_i32(counter, 1, 0, s);
    if (err != hipSuccess) return err;
    if (algo == kCBP)
        hipLaunchKernelGGL(qc_stream_kernel<kCBP>, dim3(groups), dim3(threads), lds, s, A);
    else if (algo == kLBPNMS)
        hipLaunchKernelGGL(qc_stream_kernel<kLBPNMS>, dim3(groups), dim3(threads), lds, s, A);
    else if (algo == kFBPNMS)
        hipLaunchKernelGGL(qc_stream_kernel<kFBPNMS>, dim3(groups), dim3(threads), lds, s, A);
    else
        hipLaunchKernelGGL(qc_stream_kernel<kCBPNMS>, dim3(groups), dim3(threads), lds, s, A);
    return hipGetLastError();
}

}  // namespace cbp
