// C ABI of the decoder library: argument checking, code handles, per-device
// tables, workspace and kernel selection.  Declarations and contracts are in
// include/cbp.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "cbp.h"
#include "internal.hpp"

using namespace cbp;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(CBP_EHIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr int kMaxDevices = 64;

struct DevTables {
    bool ready = false;
    void *buf = nullptr;
    SparseDev g{};
    const int *qc_sht = nullptr;  // shift table of the register-resident kernel
    StreamCode sc{};              // streamed kernel: base structure (device pointers)
    const StreamCode *sc_dev = nullptr;  // the same descriptor in device memory
};

}  // namespace

// Workspace of cbp_decode_static: one copy per GPU, held until the process
// ends.  Host code never passes `scratch` itself to a kernel or a copy (on the
// host it names a stand-in, not device memory): it uses the device address
// that hipGetSymbolAddress returns for the current device, kept per device.
static constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

struct cbp_code {
    int M = 0, N = 0;
    int64_t E = 0;
    std::vector<int> row_ptr, col_idx, edge_row, pred_edge, pred_row, last_edge;
    std::vector<uint8_t> first;
    // Row levels: rows that share no variable commute in the sequential
    // schedule, so a sweep may run level by level, each level's rows at once.
    // Rows sorted by (level, index): lvl_rows[lvl_ptr[l] .. lvl_ptr[l + 1]).
    int nlev = 0, lvl_maxrows = 0;
    std::vector<int> lvl_ptr, lvl_rows;
    bool qc = false;
    int mb = 0, nb = 0, Z = 0;
    std::vector<int> shifts;
    int qc_reg_id = -1;
    int qE = 0, qdcmax = 0;  // base edges and max block-row degree (QC codes)
    std::mutex mu;
    DevTables dev[kMaxDevices];
};

struct cbp_mix {
    std::vector<const cbp_code *> codes;
    int lcm = 1, zmin = 0, zmax = 0, dcmax = 0, default_lanes = 0;
    cbp_mix_schedule_t sched{};
    std::mutex mu;
    StreamCode *dev_codes[kMaxDevices] = {};  // the codes' descriptors per device
    // LDS-staged part of a mixed launch, per device: the codes' CSR tables
    // [n], then per algorithm a (kCBP, kLBPNMS, kFBPNMS, kCBPNMS) the layouts
    // [n] and frames per workgroup [n] (0: the code goes to the streamed
    // kernel), and the dynamic LDS each algorithm's launch needs (0: none)
    void *lds_tab[kMaxDevices] = {};
    size_t lds_bytes[kMaxDevices][4] = {};
    // the LDS-staged launch runs beside the streamed one: a second stream and
    // the fork / join events, per device
    hipStream_t side[kMaxDevices] = {};
    hipEvent_t fork[kMaxDevices] = {}, join[kMaxDevices] = {};
};

struct cbp_graph {
    hipGraphExec_t exec = nullptr;
};

namespace {

// Column lists in row order give each edge its latest check in steady state
// (the cyclically previous row of the same column) and the first- and
// last-visit flags.
int finish_code(cbp_code *c) {
    const int M = c->M, N = c->N;
    const int64_t E = c->E;
    c->edge_row.resize(E);
    c->pred_edge.resize(E);
    c->pred_row.resize(E);
    c->first.assign(E, 0);
    c->last_edge.assign(N, -1);
    std::vector<int> first_edge(N, -1);
    for (int i = 0; i < M; ++i)
        for (int e = c->row_ptr[i]; e < c->row_ptr[i + 1]; ++e) {
            c->edge_row[e] = i;
            const int v = c->col_idx[e];
            if (first_edge[v] < 0) {
                first_edge[v] = e;
                c->first[e] = (uint8_t)kFirstVisit;
            } else {
                c->pred_edge[e] = c->last_edge[v];
            }
            c->last_edge[v] = e;
        }
    for (int v = 0; v < N; ++v)
        if (c->last_edge[v] >= 0) c->first[c->last_edge[v]] |= (uint8_t)kLastVisit;
    for (int v = 0; v < N; ++v) {
        if (first_edge[v] < 0) return fail(CBP_EINVAL, "column %d has no edge", v);
        c->pred_edge[first_edge[v]] = c->last_edge[v];
    }
    for (int64_t e = 0; e < E; ++e) c->pred_row[e] = c->edge_row[c->pred_edge[e]];
    // level of a row = 1 + the highest level among the earlier rows sharing a
    // variable with it (rows in index order), so every pair of rows with a
    // common variable keeps its order and rows of one level are disjoint
    std::vector<int> lev(M), col_lev(N, 0);
    int nlev = 0;
    for (int i = 0; i < M; ++i) {
        int l = 0;
        for (int e = c->row_ptr[i]; e < c->row_ptr[i + 1]; ++e) l = std::max(l, col_lev[c->col_idx[e]]);
        lev[i] = l;
        for (int e = c->row_ptr[i]; e < c->row_ptr[i + 1]; ++e) col_lev[c->col_idx[e]] = l + 1;
        nlev = std::max(nlev, l + 1);
    }
    c->nlev = nlev;
    c->lvl_ptr.assign(nlev + 1, 0);
    for (int i = 0; i < M; ++i) ++c->lvl_ptr[lev[i] + 1];
    for (int l = 0; l < nlev; ++l) c->lvl_maxrows = std::max(c->lvl_maxrows, c->lvl_ptr[l + 1]);
    for (int l = 0; l < nlev; ++l) c->lvl_ptr[l + 1] += c->lvl_ptr[l];
    c->lvl_rows.resize(M);
    std::vector<int> fill(c->lvl_ptr.begin(), c->lvl_ptr.end() - 1);
    for (int i = 0; i < M; ++i) c->lvl_rows[fill[lev[i]]++] = i;
    return CBP_OK;
}

int check_csr(int32_t M, int32_t N, const int32_t *row_ptr, const int32_t *col_idx) {
    if (M <= 0 || N <= 0) return fail(CBP_EINVAL, "M and N must be positive (M=%d N=%d)", M, N);
    if (!row_ptr || !col_idx) return fail(CBP_EINVAL, "row_ptr/col_idx is NULL");
    if (row_ptr[0] != 0) return fail(CBP_EINVAL, "row_ptr[0] must be 0");
    for (int i = 0; i < M; ++i) {
        const int d = row_ptr[i + 1] - row_ptr[i];
        if (d < 2) return fail(CBP_EINVAL, "row %d has degree %d (< 2)", i, d);
        for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            if (col_idx[e] < 0 || col_idx[e] >= N) return fail(CBP_EINVAL, "col_idx[%d] out of range", e);
            if (e > row_ptr[i] && col_idx[e] <= col_idx[e - 1])
                return fail(CBP_EINVAL, "row %d is not strictly ascending", i);
        }
    }
    if ((int64_t)row_ptr[M] >= (int64_t)1 << 31) return fail(CBP_EINVAL, "too many edges");
    return CBP_OK;
}

double phi64(double x) { return std::log1p(2.0 / std::expm1(x)); }

// The code's device tables on the current device, built on first use unless
// `build` is false (then a missing table set is an error: nothing allocated).
int ensure_device(const cbp_code *cc, int *device_out, const SparseDev **g,
                  const int **qc_sht = nullptr, const DevTables **tab = nullptr, bool build = true) {
    cbp_code *c = const_cast<cbp_code *>(cc);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(CBP_EUNSUPPORTED, "device %d", dev);
    *device_out = dev;
    std::lock_guard<std::mutex> lock(c->mu);
    DevTables &t = c->dev[dev];
    if (!t.ready && !build)
        return fail(CBP_EUNSUPPORTED,
                    "the code's device tables are not built on device %d (any allocating call with this "
                    "code on this device, e.g. cbp_syndrome, builds them)", dev);
    if (!t.ready) {
        const int64_t E = c->E;
        const int M = c->M, N = c->N;
        std::vector<int> sht;
        if (c->qc_reg_id >= 0) {
            sht.resize(2 * (size_t)c->mb * c->nb);
            sht.resize(qc_reg_shift_table(c->qc_reg_id, c->shifts.data(), sht.data()));
        }
        // streamed-kernel edge table (QC codes)
        std::vector<int> qt;
        int qE = 0, dcmax = 0;
        size_t q_rstart = 0, q_er = 0, q_esh = 0, q_elast = 0, q_erec = 0, q_sc = 0;
        if (c->qc) {
            const int mb = c->mb, nb = c->nb;
            std::vector<int> rstart(mb + 1), eb, esh, er, ep, epr, epsh, efirst, elast(nb, -1);
            for (int r = 0; r < mb; ++r) {
                rstart[r] = (int)eb.size();
                for (int b = 0; b < nb; ++b)
                    if (c->shifts[r * nb + b] >= 0) {
                        eb.push_back(b);
                        esh.push_back(c->shifts[r * nb + b]);
                        er.push_back(r);
                    }
                dcmax = std::max(dcmax, (int)eb.size() - rstart[r]);
            }
            qE = (int)eb.size();
            rstart[mb] = qE;
            ep.assign(qE, 0);
            efirst.assign(qE, 0);
            std::vector<int> firstq(nb, -1);
            for (int e = 0; e < qE; ++e) {
                const int b = eb[e];
                if (firstq[b] < 0) {
                    firstq[b] = e;
                    efirst[e] = 1;
                } else {
                    ep[e] = elast[b];
                }
                elast[b] = e;
            }
            for (int b = 0; b < nb; ++b)
                if (firstq[b] >= 0) ep[firstq[b]] = elast[b];
            epr.resize(qE);
            epsh.resize(qE);
            for (int e = 0; e < qE; ++e) {
                epr[e] = er[ep[e]];
                epsh[e] = esh[ep[e]];
            }
            // layout (offsets in ints from the start of qt): rstart, er, esh,
            // elast, then 16-byte aligned the edge records and the descriptor
            q_rstart = 0;
            for (auto *v : {&rstart, &er, &esh, &elast}) qt.insert(qt.end(), v->begin(), v->end());
            q_er = mb + 1;
            q_esh = q_er + qE;
            q_elast = q_esh + qE;
            const size_t off0 = (size_t)(M + 1) + 4 * (size_t)E + 3 * (size_t)kSparseTablePad + (size_t)N + sht.size();
            while ((off0 + qt.size()) % 4) qt.push_back(0);
            q_erec = qt.size();
            for (int e = 0; e < qE; ++e) {
                const int last = elast[eb[e]] == e;
                qt.push_back(eb[e] | last << 29 | efirst[e] << 30);
                qt.push_back(esh[e]);
                qt.push_back(ep[e]);
                qt.push_back(epsh[e] | epr[e] << 16);
            }
            q_sc = qt.size();
            qt.resize(q_sc + (sizeof(StreamCode) + 3) / 4, 0);  // filled once the device address is known
        }
        const size_t P = kSparseTablePad;  // padding of col_idx, pred_edge, pred_row, first
        // level pointers, then (16-byte aligned) one int4 per row in level order
        const size_t lvl_pad = (4 - ((size_t)(M + 1) + 4 * (size_t)E + 3 * P + (size_t)N + sht.size() + qt.size() +
                                     (size_t)c->nlev + 1) % 4) % 4;
        // then one int4 per edge in the same order, the level edge pointers and
        // the row of each of those edges
        const size_t lvl_ints =
            (size_t)c->nlev + 1 + lvl_pad + 4 * (size_t)M + 4 * (size_t)E + (size_t)c->nlev + 1 + (size_t)E;
        const size_t ints =
            (size_t)(M + 1) + 4 * (size_t)E + 3 * P + (size_t)N + sht.size() + qt.size() + lvl_ints;
        const size_t bytes = ints * 4 + (size_t)E + P + 64;
        void *buf = nullptr;
        e = hipMalloc(&buf, bytes);
        if (e != hipSuccess) return fail(CBP_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
        std::vector<int> host(ints, 0);
        int *p = host.data();
        std::memcpy(p, c->row_ptr.data(), 4 * (size_t)(M + 1));
        p += M + 1;
        std::memcpy(p, c->col_idx.data(), 4 * (size_t)E);
        p += E + P;
        std::memcpy(p, c->edge_row.data(), 4 * (size_t)E);
        p += E;
        std::memcpy(p, c->pred_edge.data(), 4 * (size_t)E);
        p += E + P;
        std::memcpy(p, c->pred_row.data(), 4 * (size_t)E);
        p += E + P;
        std::memcpy(p, c->last_edge.data(), 4 * (size_t)N);
        p += N;
        if (!sht.empty()) std::memcpy(p, sht.data(), 4 * sht.size());
        p += sht.size();
        if (c->qc) {
            int *dq = (int *)buf + (p - host.data());  // device address of qt
            StreamCode &sc = t.sc;
            sc = StreamCode{};
            sc.Z = c->Z;
            sc.mb = c->mb;
            sc.nb = c->nb;
            sc.E = qE;
            sc.dcmax = dcmax;
            sc.N = (int64_t)c->nb * c->Z;
            sc.rstart = dq + q_rstart;
            sc.erec = reinterpret_cast<const int4 *>(dq + q_erec);
            sc.elast = dq + q_elast;
            sc.er = dq + q_er;
            sc.esh = dq + q_esh;
            std::memcpy(qt.data() + q_sc, &sc, sizeof sc);
            t.sc_dev = reinterpret_cast<const StreamCode *>(dq + q_sc);
        }
        if (!qt.empty()) std::memcpy(p, qt.data(), 4 * qt.size());
        p += qt.size();
        std::memcpy(p, c->lvl_ptr.data(), 4 * ((size_t)c->nlev + 1));
        p += c->nlev + 1 + lvl_pad;
        for (int k = 0; k < M; ++k) {
            const int i = c->lvl_rows[k];
            p[4 * k] = i;
            p[4 * k + 1] = c->row_ptr[i];
            p[4 * k + 2] = c->row_ptr[i + 1];
            p[4 * k + 3] = 0;
        }
        p += 4 * (size_t)M;
        {
            // position of every row in level order (the LDS-staged CBP kernel
            // keeps the beliefs in that order)
            std::vector<int> rpos(M);
            for (int r = 0; r < M; ++r) rpos[c->lvl_rows[r]] = r;
            int *eptr = p + 4 * (size_t)E, *erow = eptr + c->nlev + 1;
            int64_t k = 0;
            for (int l = 0; l < c->nlev; ++l) {
                eptr[l] = (int)k;
                for (int r = c->lvl_ptr[l]; r < c->lvl_ptr[l + 1]; ++r) {
                    const int i = c->lvl_rows[r];
                    for (int e = c->row_ptr[i]; e < c->row_ptr[i + 1]; ++e, ++k) {
                        p[4 * k] = c->col_idx[e];
                        p[4 * k + 1] = c->pred_edge[e];
                        p[4 * k + 2] = rpos[c->pred_row[e]];
                        p[4 * k + 3] = e | (int)((uint32_t)c->first[e] << 30);
                        erow[k] = r - c->lvl_ptr[l];
                    }
                }
            }
            eptr[c->nlev] = (int)k;
        }
        e = hipMemcpy(buf, host.data(), ints * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            std::vector<uint8_t> fp(c->first);
            fp.resize((size_t)E + P, 0);
            e = hipMemcpy((char *)buf + ints * 4, fp.data(), (size_t)E + P, hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) {
            (void)hipFree(buf);
            return hip_fail(e, "hipMemcpy of code tables");
        }
        int *d = (int *)buf;
        t.g.M = M;
        t.g.N = N;
        t.g.E = (int)E;
        t.g.row_ptr = d;
        d += M + 1;
        t.g.col_idx = d;
        d += E + P;
        t.g.edge_row = d;
        d += E;
        t.g.pred_edge = d;
        d += E + P;
        t.g.pred_row = d;
        d += E + P;
        t.g.last_edge = d;
        d += N;
        t.qc_sht = sht.empty() ? nullptr : d;
        d += sht.size();
        d += qt.size();
        t.g.nlev = c->nlev;
        t.g.lvl_ptr = d;
        d += c->nlev + 1 + lvl_pad;
        t.g.lvl_rows = reinterpret_cast<const int4 *>(d);
        d += 4 * (size_t)M;
        t.g.lvl_edges = reinterpret_cast<const int4 *>(d);
        d += 4 * (size_t)E;
        t.g.lvl_eptr = d;
        t.g.lvl_erow = d + c->nlev + 1;
        t.g.lvl_maxrows = c->lvl_maxrows;
        t.g.first = (const uint8_t *)((char *)buf + ints * 4);
        t.buf = buf;
        t.ready = true;
    }
    *g = &t.g;
    if (qc_sht) *qc_sht = t.qc_sht;
    if (tab) *tab = &t;
    return CBP_OK;
}

struct Resolved {
    Params p;
    Dump d;
    int kernel;
    bool handoff;  // the sparse kernel may hand slow frames to the level-parallel kernel
    void *ws;
    size_t ws_bytes;
};

// True if the LDS-staged CSR kernel serves algo on this code: at least one
// frame's state fits the LDS of a gfx950 workgroup.
bool lds_kernel_fits(int algo, const cbp_code_t *code) {
    SparseDev g{};
    g.M = code->M;
    g.N = code->N;
    g.E = code->E < ((int64_t)1 << 30) ? (int)code->E : (1 << 30);
    g.lvl_maxrows = code->lvl_maxrows;
    return lds_frames(lds_item(algo, g), kLdsPlanBytes) >= 1;
}

int resolve_opts(const cbp_code_t *code, int algo, int64_t batch, const cbp_opts_t *o, Resolved *r) {
    cbp_opts_t def;
    cbp_opts_default(&def);
    if (!o) o = &def;
    if (o->stop_rule < 0 || o->stop_rule > 2) return fail(CBP_EINVAL, "stop_rule must be 0, 1 or 2");
    if (o->stop_rule == 1 && algo != kCBP && algo != kCBPNMS)
        return fail(CBP_EINVAL, "stop_rule 1 (the paper's rule) applies to cbp_decode only");
    if (o->hd_mode != 0 && o->hd_mode != 1) return fail(CBP_EINVAL, "hd_mode must be 0 or 1");
    if (o->hd_mode == 1 && algo != kCBP && algo != kCBPNMS)
        return fail(CBP_EINVAL, "hd_mode 1 applies to cbp_decode only");
    if (!(o->lmax > 0.0f) || !std::isfinite(o->lmax) || o->lmax > 80.0f)
        return fail(CBP_EINVAL, "lmax must be in (0, 80]");
    if (!std::isfinite(o->alpha) || !(o->alpha > 0.0f)) return fail(CBP_EINVAL, "alpha must be positive");
    if (o->check_rule != CBP_RULE_LOG_TANH && o->check_rule != CBP_RULE_MIN_SUM)
        return fail(CBP_EINVAL, "check_rule must be CBP_RULE_LOG_TANH or CBP_RULE_MIN_SUM");
    if (o->dump_sweep < 0 || o->dump_frames < 0) return fail(CBP_EINVAL, "negative dump option");
    int k = o->kernel;
    const bool stream_ok = code->qc && code->Z <= 1024 && code->mb < 32768 && code->nb < 65536;
    // the LDS-staged CSR kernel: the one-frame-per-lane kernel's results, for
    // the syndrome stop or fixed sweeps, decisions of Step 3, no dumps
    const bool lds_opts = o->stop_rule != 1 && o->hd_mode == 0 && (o->dump_sweep == 0 || o->dump_frames == 0);
    const bool lds_fits = lds_kernel_fits(algo, code);
    if ((algo == kLBP || algo == kFBP) && k != CBP_KERNEL_AUTO && k != CBP_KERNEL_SPARSE &&
        k != CBP_KERNEL_SPARSE_LDS)
        return fail(CBP_EUNSUPPORTED, "lbp_decode and fbp_decode run on the CSR kernels only");
    if ((algo == kLBP || algo == kFBP) && k == CBP_KERNEL_AUTO)
        k = (lds_fits && lds_opts) ? CBP_KERNEL_SPARSE_LDS : CBP_KERNEL_SPARSE;
    // AUTO: a compiled base pattern keeps the register-resident kernel; else
    // frames staged in LDS where they fit (for QC codes as fast as the
    // streamed kernel at Z = 128 and up to 2.9x faster for smaller Z, with the
    // same results), else the streamed kernel for QC codes, else one frame per
    // lane
    if (k == CBP_KERNEL_AUTO)
        k = code->qc_reg_id >= 0     ? CBP_KERNEL_QC_REG
            : (lds_fits && lds_opts) ? CBP_KERNEL_SPARSE_LDS
            : stream_ok              ? CBP_KERNEL_QC_STREAM
                                     : CBP_KERNEL_SPARSE;
    if (k == CBP_KERNEL_QC_REG && code->qc_reg_id < 0)
        return fail(CBP_EUNSUPPORTED, "no register-resident kernel is compiled for this base pattern");
    if (k == CBP_KERNEL_QC_STREAM && !stream_ok)
        return fail(CBP_EUNSUPPORTED, "the streamed kernel needs a QC code with Z <= 1024, mb < 32768, nb < 65536");
    if (k == CBP_KERNEL_SPARSE_LDS && !lds_fits)
        return fail(CBP_EUNSUPPORTED, "the LDS-staged kernel serves codes whose frame state fits a CU's LDS");
    if (k == CBP_KERNEL_SPARSE_LDS && !lds_opts)
        return fail(CBP_EUNSUPPORTED, "the LDS-staged kernel runs with stop_rule 0 or 2, hd_mode 0 and no dumps");
    if (k != CBP_KERNEL_QC_REG && k != CBP_KERNEL_QC_STREAM && k != CBP_KERNEL_SPARSE && k != CBP_KERNEL_SPARSE_LDS)
        return fail(CBP_EINVAL, "unknown kernel %d", o->kernel);
    if (o->stop_rule == 1 && o->hd_mode == 1 && k != CBP_KERNEL_SPARSE)
        return fail(CBP_EUNSUPPORTED, "stop_rule 1 with hd_mode 1 needs the sparse kernel (a mid-layer stop would "
                                      "have to undo the layer's messages)");
    r->kernel = k;
    r->p.lmax = o->lmax;
    // lower clamp of a magnitude entering a check: phi(lmax), but never above
    // lmax (for lmax below phi's fixed point 0.88 both clamps give lmax), so a
    // kernel may clamp with one median-of-three
    r->p.a = std::fmin((float)phi64((double)o->lmax), o->lmax);
    r->p.alpha = o->alpha;
    r->p.stop_rule = o->stop_rule;
    r->p.hd_mode = o->hd_mode;
    r->d.sweep = o->dump_sweep;
    r->d.frames = o->dump_frames < batch ? o->dump_frames : batch;
    r->d.q = o->dump_q;
    r->d.r = o->dump_r;
    r->d.om = o->dump_om;
    r->d.lam = o->dump_lam;
    if (r->d.sweep == 0) r->d.frames = 0;
    // the level-parallel kernel runs whole sweeps with the syndrome test on the
    // V2C-phase decisions (or fixed sweeps), and writes no dumps
    r->handoff = k == CBP_KERNEL_SPARSE && o->stop_rule != 1 && o->hd_mode == 0 &&
                 (o->dump_sweep == 0 || o->dump_frames == 0);
    if (o->workspace && ((uintptr_t)o->workspace & 255))
        return fail(CBP_EINVAL, "workspace must be 256-byte aligned");
    r->ws = o->workspace;
    r->ws_bytes = o->workspace_bytes;
    return CBP_OK;
}

// State slots (lanes) of the persistent sparse launch: one per frame, up to
// 2048 waves and at most 32 GiB of frame state (e.g. 131k slots, 25 GB, for an
// n = 8192 code).  Measured on n = 2048 and 8192 codes, throughput stops
// growing at about 1000 waves; once the batch is drained a launch waits only
// for its slowest frames.
#ifndef CBP_SPARSE_MAX_WAVES
#define CBP_SPARSE_MAX_WAVES 2048
#endif
constexpr int64_t kSparseMaxLanes = (int64_t)CBP_SPARSE_MAX_WAVES * 64;
constexpr int64_t kSparseMaxBytes = (int64_t)32 << 30;
constexpr size_t kSparseCounterBytes = 256;  // frame counter, hand-off counters ahead of the slots

// Hand-off of slow frames (sparse kernel): once the batch is exhausted, a wave
// with at most this many busy lanes hands their frames to the level-parallel
// kernel.  CBP_SPARSE_HANDOFF in the environment overrides it (0 = never,
// 64 = as soon as the batch is exhausted).  Items take at most
// kHandoffMaxBytes (CBP_SPARSE_HANDOFF_ITEMS can lower their number; frames
// beyond it finish on their lanes).
constexpr int kHandoffLanes = 16;
constexpr int64_t kHandoffMaxBytes = (int64_t)8 << 30;
// Workgroups of the level-parallel launch: at most kHandoffGroups, and few
// enough that the frames in flight fit in kLevelResident bytes (their rows
// touch scattered words of the frame state, which then stay in cache).
constexpr int64_t kHandoffGroups = 2048;
constexpr int64_t kLevelResident = (int64_t)192 << 20;

// A non-negative integer from the environment, else `def`.
int64_t env_count(const char *name, int64_t def) {
    const char *v = std::getenv(name);
    if (!v || !*v) return def;
    char *end = nullptr;
    const long long n = std::strtoll(v, &end, 10);
    if (*end || n < 0) return def;
    return n > ((int64_t)1 << 40) ? ((int64_t)1 << 40) : (int64_t)n;
}

int handoff_lanes() { return (int)std::min<int64_t>(env_count("CBP_SPARSE_HANDOFF", kHandoffLanes), 64); }

// Workspace of a sparse decode: header (kSparseCounterBytes), hand-off items
// (cap x 8 bytes, then cap frame states), then the lanes' blocks.
struct SparsePlan {
    int64_t lanes = 0;
    uint32_t cap = 0;
    int64_t item_bytes = 0;
    size_t items_off = 0, state_off = 0, blocks_off = 0, total = 0;
};

int64_t sparse_lanes(int algo, const SparseDev &g, int64_t batch) {
    const int64_t per = (int64_t)(sparse_ws_bytes(algo, g, 64) / 64) + 1;
    int64_t n = std::min<int64_t>(kSparseMaxLanes, kSparseMaxBytes / per) / 64 * 64;
    if (n < 64) n = 64;
    const int64_t b = (batch + 63) / 64 * 64;
    return b < n ? b : n;
}

// Streamed QC kernel: at most this many frames (slots) in flight per call,
// which bounds its workspace (e.g. 2048 x 0.68 MB for the n = 26112 code).
constexpr int64_t kStreamMaxSlots = 2048;

// Frames per workgroup of a one-code streamed launch: whole waves where Z
// allows it (Z = 96: two frames in three waves).
int stream_slots(int Z) {
    if (Z >= 64) return (Z % 64 == 0) ? 1 : (Z % 32 == 0 ? 2 : 1);
    int s = 1;
    while ((s * Z) % 64 != 0 && s * Z < 1024) ++s;
    return s;
}

// Geometry of a one-code streamed launch (groups capped by the batch and by
// kStreamMaxSlots frames in flight; device occupancy is applied at launch).
StreamLaunch single_stream(int algo, const cbp_code_t *c, int64_t batch) {
    StreamLaunch L{};
    const int SL = stream_slots(c->Z);
    L.ncodes = 1;
    L.lanes = SL * c->Z;
    L.dcmax = c->qdcmax;
    L.max_slots = SL;
    const int64_t need = (batch + SL - 1) / SL;
    const int64_t cap = std::max<int64_t>(1, kStreamMaxSlots / SL);
    L.groups = (int)std::min(need, cap);
    L.group_bytes = SL * stream_slot_bytes(algo, (int64_t)c->nb * c->Z, c->qE, c->mb, c->Z);
    return L;
}

int device_cus(int dev) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 1;
    return cus;
}

SparsePlan sparse_plan(int algo, const SparseDev &g, int64_t batch, bool handoff, int64_t max_lanes = 0) {
    SparsePlan sp;
    sp.lanes = sparse_lanes(algo, g, batch);
    if (max_lanes > 0) sp.lanes = std::min(sp.lanes, max_lanes);
    sp.item_bytes = sparse_item_bytes(algo, g);
    if (handoff && handoff_lanes() > 0) {
        // CBP_SPARSE_HANDOFF_ITEMS (> 0) lowers the number of items
        const int64_t lim = env_count("CBP_SPARSE_HANDOFF_ITEMS", 0);
        int64_t cap = std::min<int64_t>(sp.lanes, kHandoffMaxBytes / sp.item_bytes);
        if (lim > 0) cap = std::min(cap, lim);
        sp.cap = (uint32_t)cap;
    }
    sp.items_off = kSparseCounterBytes;
    sp.state_off = sp.items_off + (size_t)round256(8 * (int64_t)sp.cap);
    sp.blocks_off = sp.state_off + (size_t)sp.cap * (size_t)sp.item_bytes;
    sp.total = sp.blocks_off + sparse_ws_bytes(algo, g, sp.lanes);
    return sp;
}

// The widest sparse plan (lanes a multiple of 64, at most the default) whose
// workspace fits in `budget` bytes; lanes = 0 if not even one wave fits.
SparsePlan sparse_plan_fit(int algo, const SparseDev &g, int64_t batch, bool handoff, size_t budget) {
    SparsePlan sp = sparse_plan(algo, g, batch, handoff);
    if (sp.total <= budget) return sp;
    int64_t lo = 0, hi = sp.lanes / 64;  // in waves; plan(lo) fits, plan(hi) does not
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (sparse_plan(algo, g, batch, handoff, mid * 64).total <= budget) lo = mid;
        else hi = mid;
    }
    if (lo == 0) return SparsePlan{};
    return sparse_plan(algo, g, batch, handoff, lo * 64);
}

size_t needed_ws(int algo, const cbp_code_t *code, const SparseDev &g, int kernel, int64_t batch,
                 bool handoff) {
    if (kernel == CBP_KERNEL_QC_REG || kernel == CBP_KERNEL_SPARSE_LDS) return 256;
    if (kernel == CBP_KERNEL_QC_STREAM) {
        const StreamLaunch L = single_stream(algo, code, batch);
        return 256 + (size_t)L.groups * L.group_bytes;
    }
    return sparse_plan(algo, g, batch, handoff).total;
}

// opts.validate: scan n LLRs for NaN / +-Inf (frames of `row` values, 0 = no frame
// structure); blocks on s.
// `fixed`: a device word to use for the result (nothing is then allocated).
int validate_llr(const float *llr, int64_t n, int64_t row, hipStream_t s,
                 unsigned long long *fixed = nullptr) {
    unsigned long long *pos = fixed;
    hipError_t e = hipSuccess;
    if (!fixed) {
        e = hipMallocAsync((void **)&pos, sizeof(*pos), s);
        if (e != hipSuccess) return fail(CBP_ENOMEM, "hipMallocAsync(8): %s", hipGetErrorString(e));
    }
    unsigned long long h = ~0ull;
    e = launch_nonfinite_scan(llr, n, pos, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, pos, sizeof(h), hipMemcpyDeviceToHost, s);
    hipError_t e2 = fixed ? hipSuccess : hipFreeAsync(pos, s);
    if (e == hipSuccess) e = e2;
    e2 = hipStreamSynchronize(s);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return hip_fail(e, "llr_in scan");
    if (h != ~0ull && row <= 0) return fail(CBP_EINVAL, "llr_in element %llu is NaN or infinite", h);
    if (h != ~0ull)
        return fail(CBP_EINVAL, "llr_in element %llu (frame %lld, position %lld) is NaN or infinite", h,
                    (long long)(h / (unsigned long long)row), (long long)(h % (unsigned long long)row));
    return CBP_OK;
}

// A workspace the caller of decode() fixes in advance (the static scratch of
// cbp_decode_static): decode() then allocates nothing, builds no tables, and
// fits the persistent kernels' frames in flight to its size.
struct FixedWs {
    void *base = nullptr;  // 256-byte aligned; the first 256 bytes hold the input-scan word
    size_t bytes = 0;
};

int decode(int algo, const cbp_code_t *code, const float *llr, uint8_t *bits, int32_t *iters,
           int32_t max_iter, int64_t batch, const cbp_opts_t *opts, void *stream,
           const FixedWs *fixed = nullptr) {
    if (!code) return fail(CBP_EINVAL, "code is NULL");
    if (batch < 0) return fail(CBP_EINVAL, "batch < 0");
    if (max_iter < 0) return fail(CBP_EINVAL, "max_iter < 0");
    if (batch == 0) return CBP_OK;
    if (!llr || !bits || !iters) return fail(CBP_EINVAL, "llr_in/bits_out/iters_out is NULL");
    if (batch > ((int64_t)1 << 30)) return fail(CBP_EINVAL, "batch above 2^30 frames per call");
    Resolved r;
    int rc = resolve_opts(code, algo, batch, opts, &r);
    if (rc) return rc;
    int dev = 0;
    const SparseDev *g = nullptr;
    const int *qc_sht = nullptr;
    const DevTables *tab = nullptr;
    rc = ensure_device(code, &dev, &g, &qc_sht, &tab, fixed == nullptr);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (opts && opts->validate) {
        rc = validate_llr(llr, batch * (int64_t)code->N, code->N, s,
                          fixed ? (unsigned long long *)fixed->base : nullptr);
        if (rc) return rc;
    }
    // with a fixed workspace: the part after its first 256 bytes, and no
    // more frames in flight than fit in it
    size_t budget = 0;
    if (fixed) {
        r.ws = (char *)fixed->base + 256;
        r.ws_bytes = budget = fixed->bytes - 256;
    }
    const size_t need = fixed ? 0 : needed_ws(algo, code, *g, r.kernel, batch, r.handoff);
    void *ws = r.ws;
    bool own = false;
    if (!fixed && (!ws || r.ws_bytes < need)) {
        hipError_t e = hipMallocAsync(&ws, need, s);
        if (e != hipSuccess) return fail(CBP_ENOMEM, "hipMallocAsync(%zu): %s", need, hipGetErrorString(e));
        own = true;
    }
    hipError_t e = hipSuccess;
    if (r.kernel == CBP_KERNEL_QC_REG) {
        e = launch_qc_reg(code->qc_reg_id, algo, qc_sht, llr, bits, iters, batch,
                          max_iter, r.p, r.d, (int *)ws, dev, s);
    } else if (r.kernel == CBP_KERNEL_SPARSE_LDS) {
        e = launch_sparse_lds(algo, *g, llr, bits, iters, batch, max_iter, r.p, (unsigned int *)ws, dev, s);
    } else if (r.kernel == CBP_KERNEL_QC_STREAM) {
        StreamLaunch L = single_stream(algo, code, batch);
        L.codes = tab->sc_dev;
        if (L.group_bytes >= ((int64_t)1 << 31)) {
            if (own) (void)hipFreeAsync(ws, s);
            return fail(CBP_EUNSUPPORTED, "frame state above 2 GiB per workgroup");
        }
        const int per_cu = stream_groups_per_cu(algo, L.lanes, stream_lds_bytes(algo, L.lanes, L.dcmax, L.max_slots));
        if (per_cu <= 0) {
            if (own) (void)hipFreeAsync(ws, s);
            return fail(CBP_EUNSUPPORTED, "the streamed kernel's LDS for this code (Z=%d, row degree %d) exceeds a CU",
                        code->Z, code->qdcmax);
        }
        L.groups = (int)std::min<int64_t>(L.groups, (int64_t)per_cu * device_cus(dev));
        if (fixed) {
            const int64_t fit = (int64_t)(budget - 256) / L.group_bytes;
            if (fit < 1)
                return fail(CBP_EUNSUPPORTED, "one workgroup's frame state (%lld bytes) exceeds the %zu-byte "
                            "static scratch", (long long)L.group_bytes, budget);
            L.groups = (int)std::min<int64_t>(L.groups, fit);
        }
        e = launch_fill_i32((int *)ws, 1, 0, s);
        if (e == hipSuccess)
            e = launch_qc_stream(algo, L, llr, bits, iters, batch, nullptr, nullptr, nullptr,
                                 (unsigned int *)ws, max_iter, r.p, r.d, (char *)ws + 256, s);
    } else {
        if ((int64_t)std::max({g->N, g->M, g->E}) * 64 >= ((int64_t)1 << 32)) {
            if (own) (void)hipFreeAsync(ws, s);
            return fail(CBP_EUNSUPPORTED, "the sparse kernel indexes its state with 32 bits: at most 2^26 edges");
        }
        const SparsePlan sp = fixed ? sparse_plan_fit(algo, *g, batch, r.handoff, budget)
                                    : sparse_plan(algo, *g, batch, r.handoff);
        if (sp.lanes == 0)
            return fail(CBP_EUNSUPPORTED, "the state of 64 frames on the sparse kernel (%lld bytes) exceeds the "
                        "%zu-byte static scratch",
                        (long long)sparse_plan(algo, *g, 64, r.handoff).total, budget);
        const SparseWs w = sparse_ws_carve(algo, *g, sp.lanes, (char *)ws + sp.blocks_off);
        Handoff h{};
        const int hl = handoff_lanes();
        if (sp.cap > 0 && hl > 0 && max_iter > 1) {
            h.lanes = hl;
            h.cap = sp.cap;
            h.groups = (int)std::min<int64_t>(
                {(int64_t)sp.cap, kHandoffGroups, std::max<int64_t>(64, kLevelResident / sp.item_bytes)});
            h.count = (unsigned int *)((char *)ws + 8);
            h.items = (int2 *)((char *)ws + sp.items_off);
            h.state = (char *)ws + sp.state_off;
            h.item_bytes = sp.item_bytes;
        }
        e = launch_sparse(algo, *g, llr, bits, iters, batch, max_iter, r.p, w, r.d,
                          (unsigned long long *)ws, h, s);
    }
    if (own) {
        hipError_t e2 = hipFreeAsync(ws, s);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return CBP_OK;
}

// ---- the static scratch of cbp_decode_static -----------------------------

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (the current device), looked up
// once per device.
int static_scratch(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(CBP_EUNSUPPORTED, "device %d", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the static scratch");
        if (!p || ((uintptr_t)p & 255)) return fail(CBP_EHIP, "static scratch at %p is not 256-byte aligned", p);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CBP_OK;
}

// ---- mixed-code batches ---------------------------------------------------

// Byte offsets in cbp_mix::lds_tab of n codes: tables, then per algorithm
// the layouts and the frames per workgroup.
size_t mix_lds_items_off(size_t n, int a) {
    const size_t t = (sizeof(SparseDev) * n + 15) / 16 * 16, per = (sizeof(LdsItem) * n + 4 * n + 15) / 16 * 16;
    return t + per * (size_t)a;
}

int mix_ensure_device(cbp_mix *m, int *dev_out, const StreamCode **codes) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(CBP_EUNSUPPORTED, "device %d", dev);
    *dev_out = dev;
    std::lock_guard<std::mutex> lock(m->mu);
    if (!m->lds_tab[dev]) {
        // the LDS-staged part: a code takes frames_per_workgroup (1, 2, 4 or 8)
        // slots if its frame fits a workgroup's share of the CU's LDS
        const size_t n = m->codes.size();
        int lim = 0;
        e = hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
        const int64_t budget = (int64_t)lim / kLdsMixGroupsPerCu - kLdsStaticBytes;
        std::vector<char> host(mix_lds_items_off(n, 4), 0);
        for (size_t i = 0; i < n; ++i) {
            int d2 = 0;
            const SparseDev *g = nullptr;
            int rc = ensure_device(m->codes[i], &d2, &g);
            if (rc) return rc;
            std::memcpy(host.data() + sizeof(SparseDev) * i, g, sizeof(SparseDev));
        }
        for (int a = 0; a < 4; ++a) {
            LdsItem *items = (LdsItem *)(host.data() + mix_lds_items_off(n, a));
            int *frames = (int *)(host.data() + mix_lds_items_off(n, a) + sizeof(LdsItem) * n);
            size_t need = 0;
            for (size_t i = 0; i < n; ++i) {
                SparseDev g{};
                g.M = m->codes[i]->M;
                g.N = m->codes[i]->N;
                g.E = (int)m->codes[i]->E;
                g.lvl_maxrows = m->codes[i]->lvl_maxrows;
                items[i] = lds_item(a, g);
                int f = items[i].bytes > 0 ? (int)std::min<int64_t>(8, budget / items[i].bytes) : 0;
                f = f >= 8 ? 8 : f >= 4 ? 4 : f >= 2 ? 2 : f;
                frames[i] = f;
                need = std::max(need, (size_t)f * (size_t)items[i].bytes);
            }
            m->lds_bytes[dev][a] = need;
            e = prepare_mix_lds(a, need);
            if (e != hipSuccess) return hip_fail(e, "dynamic LDS of the mixed LDS-staged kernel");
        }
        void *buf = nullptr;
        e = hipMalloc(&buf, host.size());
        if (e != hipSuccess) return fail(CBP_ENOMEM, "hipMalloc: %s", hipGetErrorString(e));
        e = hipMemcpy(buf, host.data(), host.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(buf);
            return hip_fail(e, "hipMemcpy of the plan's LDS tables");
        }
        m->lds_tab[dev] = buf;
        e = hipStreamCreateWithFlags(&m->side[dev], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&m->fork[dev], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&m->join[dev], hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "stream / event for the LDS-staged launch");
    }
    if (!m->dev_codes[dev]) {
        std::vector<StreamCode> host;
        for (const cbp_code *c : m->codes) {
            int d2 = 0;
            const SparseDev *g = nullptr;
            const DevTables *tab = nullptr;
            int rc = ensure_device(c, &d2, &g, nullptr, &tab);
            if (rc) return rc;
            host.push_back(tab->sc);
        }
        void *buf = nullptr;
        e = hipMalloc(&buf, sizeof(StreamCode) * host.size());
        if (e != hipSuccess) return fail(CBP_ENOMEM, "hipMalloc: %s", hipGetErrorString(e));
        e = hipMemcpy(buf, host.data(), sizeof(StreamCode) * host.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(buf);
            return hip_fail(e, "hipMemcpy of the plan's code descriptors");
        }
        m->dev_codes[dev] = (StreamCode *)buf;
    }
    *codes = m->dev_codes[dev];
    return CBP_OK;
}

int mix_algo(int32_t decoder, const cbp_opts_t *opts, int *algo) {
    if (decoder < 0 || decoder > 2) return fail(CBP_EINVAL, "decoder must be 0, 1 or 2");
    *algo = decoder == 0 ? ((opts && opts->check_rule == CBP_RULE_MIN_SUM) ? kCBPNMS : kCBP) : decoder;
    return CBP_OK;
}

// counter[256] (1 KB), qstart[257] (int64) at 1024, the streamed kernel's
// counters [256] at 4096
constexpr size_t kMixHeader = 8192;



int mix_geometry(const cbp_mix *m, int algo, const cbp_mix_schedule_t &sc, int dev, int64_t batch,
                 StreamLaunch *L) {
    *L = StreamLaunch{};
    L->ncodes = (int)m->codes.size();
    L->lanes = sc.lanes;
    L->dcmax = m->dcmax;
    L->max_slots = sc.lanes / m->zmin;
    const size_t lds = stream_lds_bytes(algo, L->lanes, L->dcmax, L->max_slots);
    int per_cu = stream_groups_per_cu(algo, L->lanes, lds);
    if (per_cu <= 0)
        return fail(CBP_EUNSUPPORTED, "%d lanes with row degree %d need %zu B of LDS: no workgroup fits a CU",
                    L->lanes, L->dcmax, lds);
    if (sc.groups_per_cu > 0) per_cu = std::min(per_cu, sc.groups_per_cu);
    int64_t groups = (int64_t)per_cu * device_cus(dev);
    groups = std::min<int64_t>(groups, std::max<int64_t>(1, batch));
    L->groups = (int)groups;
    int64_t gb = 0;
    for (const cbp_code *c : m->codes)
        gb = std::max(gb, (int64_t)(sc.lanes / c->Z) *
                              stream_slot_bytes(algo, (int64_t)c->nb * c->Z, c->qE, c->mb, c->Z));
    L->group_bytes = gb;
    if (gb >= ((int64_t)1 << 31)) return fail(CBP_EUNSUPPORTED, "workgroup workspace above 2 GiB");
    return CBP_OK;
}

size_t mix_ws_bytes(const StreamLaunch &L, int64_t batch) {
    const size_t perm = ((size_t)4 * batch + 255) & ~(size_t)255;
    return kMixHeader + perm + (size_t)L.groups * L.group_bytes;
}

int mix_decode_impl(const cbp_mix *mc, int32_t decoder, const float *llr, int64_t llr_elems,
                    const int32_t *fcode, const int64_t *foff, uint8_t *bits, int32_t *iters,
                    int32_t max_iter, int64_t batch, const cbp_opts_t *opts, void *ws,
                    size_t ws_bytes, void *stream, const cbp_mix_schedule_t &sched) {
    cbp_mix *m = const_cast<cbp_mix *>(mc);
    if (!m) return fail(CBP_EINVAL, "mix is NULL");
    if (batch < 0 || max_iter < 0 || llr_elems < 0) return fail(CBP_EINVAL, "negative batch/max_iter/llr_elems");
    if (batch > INT32_MAX) return fail(CBP_EINVAL, "batch above 2^31 - 1 frames");
    int algo = 0;
    int rc = mix_algo(decoder, opts, &algo);
    if (rc) return rc;
    if (batch == 0) return CBP_OK;
    if (!llr || !fcode || !foff || !bits || !iters) return fail(CBP_EINVAL, "NULL buffer");
    cbp_opts_t o;
    if (opts) o = *opts;
    else cbp_opts_default(&o);
    o.kernel = CBP_KERNEL_QC_STREAM;  // every code of a plan has it
    Resolved r;
    rc = resolve_opts(m->codes[0], algo, batch, &o, &r);
    if (rc) return rc;
    if (r.d.sweep > 0 && r.d.frames > 0) return fail(CBP_EUNSUPPORTED, "state dumps are not available for mixed batches");
    int dev = 0;
    const StreamCode *dc = nullptr;
    rc = mix_ensure_device(m, &dev, &dc);
    if (rc) return rc;
    StreamLaunch L;
    rc = mix_geometry(m, algo, sched, dev, batch, &L);
    if (rc) return rc;
    L.codes = dc;
    const size_t need = mix_ws_bytes(L, batch);
    if (!ws || ws_bytes < need) return fail(CBP_EINVAL, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((uintptr_t)ws & 255) return fail(CBP_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    if (o.validate) {
        rc = validate_llr(llr, llr_elems, 0, s);
        if (rc) return rc;
    }
    char *w = (char *)ws;
    unsigned int *counter = (unsigned int *)w;
    int64_t *qstart = (int64_t *)(w + 1024);
    int32_t *perm = (int32_t *)(w + kMixHeader);
    char *groups = w + kMixHeader + (((size_t)4 * batch + 255) & ~(size_t)255);
    hipError_t e = launch_mix_prepare(fcode, foff, batch, llr_elems, dc, L.ncodes, qstart, perm, counter, iters, s);
    // The codes whose frame fits a workgroup's share of the LDS are decoded
    // staged in LDS, on a second stream beside the streamed launch; the
    // streamed kernel's own counters mark those codes' queues as exhausted.
    // The two persistent launches share the CUs as their resources allow and
    // do not wait on each other (disjoint queues).  The streamed kernel is
    // issued first, eagerly and as the first of the two graph nodes when
    // captured: its workgroups then take their place on every CU before the
    // LDS-staged ones fill the LDS that is left (the other order starves the
    // streamed kernel, the longer of the two, for the LDS kernel's run).
    const size_t lds = m->lds_bytes[dev][algo];
    const int lds_groups_cu = sched.lds_groups_per_cu;
    const bool side = e == hipSuccess && lds > 0 && lds_groups_cu > 0;
    unsigned int *scounter = counter;
    std::unique_lock<std::mutex> side_lock(m->mu, std::defer_lock);  // one fork / join at a time
    const size_t n = m->codes.size();
    const char *tab = (const char *)m->lds_tab[dev];
    const int *frames = side ? (const int *)(tab + mix_lds_items_off(n, algo) + sizeof(LdsItem) * n) : nullptr;
    if (side) {
        side_lock.lock();
        scounter = (unsigned int *)(w + 4096);
        e = launch_mix_exhaust(frames, qstart, (int)n, scounter, s);
        if (e == hipSuccess) e = hipEventRecord(m->fork[dev], s);
    }
    if (e == hipSuccess)
        e = launch_qc_stream(algo, L, llr, bits, iters, batch, qstart, perm, foff, scounter, max_iter, r.p,
                             r.d, groups, s);
    if (side && e == hipSuccess) {
        e = hipStreamWaitEvent(m->side[dev], m->fork[dev], 0);
        const int groups_lds = (int)std::min<int64_t>((int64_t)lds_groups_cu * device_cus(dev), batch);
        if (e == hipSuccess)
            e = launch_mix_lds(algo, (const SparseDev *)tab, (const LdsItem *)(tab + mix_lds_items_off(n, algo)),
                               frames, (int)n, groups_lds, lds, llr, bits, iters, qstart, perm, foff, counter, max_iter,
                               r.p, m->side[dev]);
        if (e == hipSuccess) e = hipEventRecord(m->join[dev], m->side[dev]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, m->join[dev], 0);
    }
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return CBP_OK;
}

}  // namespace

extern "C" {

// ---- unrolled differentiable CBP ------------------------------------------

namespace {

struct UnrolledGeom {
    int lanes, groups;
    int64_t gpart_bytes, group_bytes;
};

int unrolled_geom(const cbp_code_t *code, int32_t sweeps, int64_t batch, UnrolledGeom *g) {
    if (!code) return fail(CBP_EINVAL, "code is NULL");
    if (!(code->qc && code->Z <= 1024 && code->mb < 32768 && code->nb < 65536))
        return fail(CBP_EUNSUPPORTED, "the unrolled decoder needs a QC code with the streamed layout");
    if (sweeps < 1 || sweeps > 64) return fail(CBP_EINVAL, "sweeps must be in [1, 64]");
    if (batch < 0 || batch > INT32_MAX) return fail(CBP_EINVAL, "batch out of range");
    StreamCode sc{};
    sc.Z = code->Z;
    sc.mb = code->mb;
    sc.nb = code->nb;
    sc.E = code->qE;
    sc.dcmax = code->qdcmax;
    sc.N = (int64_t)code->nb * code->Z;
    const int SL = stream_slots(code->Z);
    g->lanes = SL * code->Z;
    g->groups = (int)((batch + SL - 1) / SL);
    g->group_bytes = SL * unrolled_frame_bytes(sc, sweeps);
    if (g->group_bytes >= ((int64_t)1 << 31)) return fail(CBP_EUNSUPPORTED, "frame state above 2 GiB per workgroup");
    g->gpart_bytes = ((int64_t)g->groups * sweeps * code->nb * 8 + 255) & ~(int64_t)255;
    return CBP_OK;
}

int unrolled_run(bool backward, const cbp_code_t *code, const float *llr, int64_t batch, int32_t sweeps,
                 const float *w, const float *beta, float *out, const float *gout, float *gllr, float *gw,
                 float *gb, const cbp_opts_t *opts, void *ws, size_t ws_bytes, void *stream) {
    UnrolledGeom G;
    int rc = unrolled_geom(code, sweeps, batch, &G);
    if (rc) return rc;
    cbp_opts_t o;
    if (opts) o = *opts;
    else cbp_opts_default(&o);
    o.kernel = CBP_KERNEL_QC_STREAM;
    Resolved r;
    rc = resolve_opts(code, kCBP, batch, &o, &r);
    if (rc) return rc;
    if (!w || !beta) return fail(CBP_EINVAL, "w/beta is NULL");
    if (batch == 0) {
        if (backward && gw && gb) {  // no frames: zero gradients
            hipStream_t s = (hipStream_t)stream;
            hipError_t e = launch_fill_i32((int *)gw, sweeps * code->nb, 0, s);
            if (e == hipSuccess) e = launch_fill_i32((int *)gb, sweeps * code->nb, 0, s);
            if (e != hipSuccess) return hip_fail(e, "kernel launch");
        }
        return CBP_OK;
    }
    if (!llr || (!backward && !out) || (backward && (!gout || !gw || !gb)))
        return fail(CBP_EINVAL, "NULL buffer");
    const size_t need = (size_t)G.gpart_bytes + (size_t)G.groups * G.group_bytes;
    if (!ws || ws_bytes < need) return fail(CBP_EINVAL, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((uintptr_t)ws & 255) return fail(CBP_EINVAL, "workspace must be 256-byte aligned");
    int dev = 0;
    const SparseDev *sg = nullptr;
    const DevTables *tab = nullptr;
    rc = ensure_device(code, &dev, &sg, nullptr, &tab);
    if (rc) return rc;
    if (!unrolled_fits(tab->sc, G.lanes))
        return fail(CBP_EUNSUPPORTED, "the unrolled decoder's LDS for this code exceeds a CU");
    hipError_t e = launch_unrolled(backward, tab->sc, tab->sc_dev, G.lanes, G.groups, llr, batch, sweeps, w, beta,
                                   out, gout, gllr, (float *)ws, gw, gb, r.p, (char *)ws + G.gpart_bytes,
                                   (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return CBP_OK;
}

}  // namespace

int cbp_unrolled_workspace_size(const cbp_code_t *code, int32_t sweeps, int64_t batch, size_t *bytes) {
    if (!bytes) return fail(CBP_EINVAL, "bytes is NULL");
    UnrolledGeom G;
    int rc = unrolled_geom(code, sweeps, batch, &G);
    if (rc) return rc;
    *bytes = batch == 0 ? 0 : (size_t)G.gpart_bytes + (size_t)G.groups * G.group_bytes;
    return CBP_OK;
}

int cbp_unrolled_forward(const cbp_code_t *code, const float *llr_in, int64_t batch, int32_t sweeps,
                         const float *w, const float *beta, float *soft_out, const cbp_opts_t *opts,
                         void *workspace, size_t workspace_bytes, void *stream) {
    return unrolled_run(false, code, llr_in, batch, sweeps, w, beta, soft_out, nullptr, nullptr, nullptr,
                        nullptr, opts, workspace, workspace_bytes, stream);
}

int cbp_unrolled_backward(const cbp_code_t *code, const float *llr_in, int64_t batch, int32_t sweeps,
                          const float *w, const float *beta, const float *grad_out, float *grad_llr,
                          float *grad_w, float *grad_beta, const cbp_opts_t *opts, void *workspace,
                          size_t workspace_bytes, void *stream) {
    return unrolled_run(true, code, llr_in, batch, sweeps, w, beta, nullptr, grad_out, grad_llr, grad_w,
                        grad_beta, opts, workspace, workspace_bytes, stream);
}

int cbp_mix_create(const cbp_code_t *const *codes, int32_t ncodes, cbp_mix_t **out) {
    if (!out) return fail(CBP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!codes || ncodes <= 0 || ncodes > kMaxMixCodes) return fail(CBP_EINVAL, "need 1..%d codes", kMaxMixCodes);
    cbp_mix *m = new (std::nothrow) cbp_mix;
    if (!m) return fail(CBP_ENOMEM, "out of host memory");
    int64_t lcm = 1;
    for (int i = 0; i < ncodes; ++i) {
        const cbp_code *c = codes[i];
        if (!c) {
            delete m;
            return fail(CBP_EINVAL, "code %d is NULL", i);
        }
        if (!(c->qc && c->Z <= 1024 && c->mb < 32768 && c->nb < 65536)) {
            delete m;
            return fail(CBP_EUNSUPPORTED, "code %d has no streamed layout", i);
        }
        int64_t a = lcm, b = c->Z;
        while (b) {
            const int64_t t = a % b;
            a = b;
            b = t;
        }
        lcm = lcm / a * c->Z;
        if (lcm > 1024) {
            delete m;
            return fail(CBP_EUNSUPPORTED, "the Z values need workgroups of %lld lanes (> 1024)", (long long)lcm);
        }
        m->codes.push_back(c);
        m->zmin = m->zmin ? std::min(m->zmin, c->Z) : c->Z;
        m->zmax = std::max(m->zmax, c->Z);
        m->dcmax = std::max(m->dcmax, c->qdcmax);
    }
    m->lcm = (int)lcm;
    int lanes = m->lcm;
    while (lanes % 64 != 0 && lanes * 2 <= 1024) lanes *= 2;
    m->default_lanes = lanes;
    m->sched.lanes = lanes;
    m->sched.groups_per_cu = 0;
    *out = m;
    return CBP_OK;
}

void cbp_mix_free(cbp_mix_t *m) {
    if (!m) return;
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    for (int d = 0; d < kMaxDevices; ++d) {
        if (m->dev_codes[d] && hipSetDevice(d) == hipSuccess) (void)hipFree(m->dev_codes[d]);
        if (m->lds_tab[d] && hipSetDevice(d) == hipSuccess) (void)hipFree(m->lds_tab[d]);
        if (m->side[d] && hipSetDevice(d) == hipSuccess) {
            (void)hipStreamDestroy(m->side[d]);
            (void)hipEventDestroy(m->fork[d]);
            (void)hipEventDestroy(m->join[d]);
        }
    }
    if (have_cur) (void)hipSetDevice(cur);
    delete m;
}

int cbp_mix_get_schedule(const cbp_mix_t *m, cbp_mix_schedule_t *sched) {
    if (!m || !sched) return fail(CBP_EINVAL, "mix/sched is NULL");
    *sched = m->sched;
    return CBP_OK;
}

int cbp_mix_set_schedule(cbp_mix_t *m, const cbp_mix_schedule_t *sched) {
    if (!m || !sched) return fail(CBP_EINVAL, "mix/sched is NULL");
    if (sched->lanes <= 0 || sched->lanes > 1024 || sched->lanes % m->lcm != 0)
        return fail(CBP_EINVAL, "lanes must be a multiple of %d in (0, 1024]", m->lcm);
    if (sched->groups_per_cu < 0) return fail(CBP_EINVAL, "groups_per_cu < 0");
    if (sched->lds_groups_per_cu < 0 || sched->lds_groups_per_cu > 2)
        return fail(CBP_EINVAL, "lds_groups_per_cu must be 0, 1 or 2");
    m->sched = *sched;
    return CBP_OK;
}

int cbp_mix_workspace_size(const cbp_mix_t *m, int32_t decoder, int64_t batch, const cbp_opts_t *opts,
                           size_t *bytes) {
    if (!m || !bytes) return fail(CBP_EINVAL, "mix/bytes is NULL");
    if (batch < 0) return fail(CBP_EINVAL, "batch < 0");
    int algo = 0;
    int rc = mix_algo(decoder, opts, &algo);
    if (rc) return rc;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    StreamLaunch L;
    rc = mix_geometry(m, algo, m->sched, dev, batch, &L);
    if (rc) return rc;
    *bytes = mix_ws_bytes(L, batch);
    return CBP_OK;
}

int cbp_mix_decode(const cbp_mix_t *m, int32_t decoder, const float *llr_in, int64_t llr_elems,
                   const int32_t *frame_code, const int64_t *frame_offset, uint8_t *bits_out,
                   int32_t *iters_out, int32_t max_iter, int64_t batch, const cbp_opts_t *opts,
                   void *workspace, size_t workspace_bytes, void *stream) {
    if (!m) return fail(CBP_EINVAL, "mix is NULL");
    return mix_decode_impl(m, decoder, llr_in, llr_elems, frame_code, frame_offset, bits_out, iters_out,
                           max_iter, batch, opts, workspace, workspace_bytes, stream, m->sched);
}

int cbp_mix_tune(cbp_mix_t *m, int32_t decoder, const float *llr_in, int64_t llr_elems,
                 const int32_t *frame_code, const int64_t *frame_offset, uint8_t *bits_out,
                 int32_t *iters_out, int32_t max_iter, int64_t batch, const cbp_opts_t *opts,
                 void *stream, cbp_mix_schedule_t *best, float *best_ms) {
    if (!m) return fail(CBP_EINVAL, "mix is NULL");
    if (batch <= 0) return fail(CBP_EINVAL, "tuning needs frames");
    int algo = 0;
    int rc = mix_algo(decoder, opts, &algo);
    if (rc) return rc;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::vector<cbp_mix_schedule_t> cand;
    size_t need = 0;
    for (int lanes = m->default_lanes; lanes <= 1024 && lanes <= 4 * m->default_lanes; lanes *= 2) {
        cbp_mix_schedule_t sc{lanes, 0};
        StreamLaunch L;
        if (mix_geometry(m, algo, sc, dev, batch, &L) != CBP_OK) continue;
        const int per_cu = stream_groups_per_cu(algo, lanes, stream_lds_bytes(algo, lanes, L.dcmax, L.max_slots));
        for (int g = 1; g <= per_cu; ++g) {
            sc.groups_per_cu = g;
            StreamLaunch Lg;
            if (mix_geometry(m, algo, sc, dev, batch, &Lg) != CBP_OK) continue;
            need = std::max(need, mix_ws_bytes(Lg, batch));
            // without and with the LDS-staged part (1 or 2 of its workgroups per CU)
            for (int lg = 0; lg <= 2; ++lg) {
                sc.lds_groups_per_cu = lg;
                cand.push_back(sc);
            }
            sc.lds_groups_per_cu = 0;
        }
    }
    if (cand.empty()) return fail(CBP_EUNSUPPORTED, "no schedule fits the device");
    hipStream_t s = (hipStream_t)stream;
    void *ws = nullptr;
    e = hipMalloc(&ws, need);
    if (e != hipSuccess) return fail(CBP_ENOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e));
    hipEvent_t t0 = nullptr, t1 = nullptr;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    float best_t = -1.0f;
    cbp_mix_schedule_t best_s = m->sched;
    for (size_t i = 0; i < cand.size() && rc == CBP_OK; ++i) {
        // an untimed launch before each timed one (the first launch of a kernel
        // or a stream pays for loading and caches)
        for (int rep = 0; rep < 2 && rc == CBP_OK; ++rep) {
            if (rep == 1 && (e = hipEventRecord(t0, s)) != hipSuccess) break;
            rc = mix_decode_impl(m, decoder, llr_in, llr_elems, frame_code, frame_offset, bits_out, iters_out,
                                 max_iter, batch, opts, ws, need, stream, cand[i]);
            if (rep == 1 && rc == CBP_OK) e = hipEventRecord(t1, s);
        }
        if (rc != CBP_OK || e != hipSuccess) break;
        if ((e = hipEventSynchronize(t1)) != hipSuccess) break;
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, t0, t1);
        if (best_t < 0.0f || ms < best_t) {
            best_t = ms;
            best_s = cand[i];
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    (void)hipFree(ws);
    if (rc != CBP_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, "timing");
    m->sched = best_s;
    if (best) *best = best_s;
    if (best_ms) *best_ms = best_t;
    return CBP_OK;
}

int cbp_mix_graph_create(const cbp_mix_t *mc, int32_t decoder, const float *llr_in, int64_t llr_elems,
                         const int32_t *frame_code, const int64_t *frame_offset, uint8_t *bits_out,
                         int32_t *iters_out, int32_t max_iter, int64_t batch, const cbp_opts_t *opts,
                         void *workspace, size_t workspace_bytes, cbp_graph_t **out) {
    if (!out) return fail(CBP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!mc) return fail(CBP_EINVAL, "mix is NULL");
    if (opts && opts->validate)
        return fail(CBP_EUNSUPPORTED, "opts.validate reads a flag back to the host and cannot be captured");
    cbp_mix *m = const_cast<cbp_mix *>(mc);
    // device tables first: their upload is not capturable
    int dev = 0;
    const StreamCode *dc = nullptr;
    int rc = mix_ensure_device(m, &dev, &dc);
    if (rc) return rc;
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    rc = mix_decode_impl(m, decoder, llr_in, llr_elems, frame_code, frame_offset, bits_out, iters_out, max_iter,
                         batch, opts, workspace, workspace_bytes, cs, m->sched);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    hipGraphExec_t exec = nullptr;
    if (rc == CBP_OK && e2 == hipSuccess) e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cs);
    if (rc != CBP_OK) return rc;
    if (e2 != hipSuccess) return hip_fail(e2, "graph capture");
    cbp_graph *g = new (std::nothrow) cbp_graph;
    if (!g) {
        (void)hipGraphExecDestroy(exec);
        return fail(CBP_ENOMEM, "out of host memory");
    }
    g->exec = exec;
    *out = g;
    return CBP_OK;
}

int cbp_graph_launch(cbp_graph_t *g, void *stream) {
    if (!g || !g->exec) return fail(CBP_EINVAL, "graph is NULL");
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return CBP_OK;
}

void cbp_graph_free(cbp_graph_t *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    delete g;
}

void cbp_opts_default(cbp_opts_t *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->stop_rule = 0;
    o->hd_mode = 0;
    o->lmax = 20.0f;
    o->alpha = 0.75f;
    o->kernel = CBP_KERNEL_AUTO;
}

int cbp_code_from_csr(int32_t M, int32_t N, const int32_t *row_ptr, const int32_t *col_idx,
                      cbp_code_t **out) {
    if (!out) return fail(CBP_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_csr(M, N, row_ptr, col_idx);
    if (rc) return rc;
    cbp_code *c = new (std::nothrow) cbp_code;
    if (!c) return fail(CBP_ENOMEM, "out of host memory");
    c->M = M;
    c->N = N;
    c->E = row_ptr[M];
    c->row_ptr.assign(row_ptr, row_ptr + M + 1);
    c->col_idx.assign(col_idx, col_idx + c->E);
    rc = finish_code(c);
    if (rc) {
        delete c;
        return rc;
    }
    *out = c;
    return CBP_OK;
}

int cbp_code_from_qc(int32_t mb, int32_t nb, int32_t Z, const int32_t *shifts, cbp_code_t **out) {
    if (!out) return fail(CBP_EINVAL, "out is NULL");
    *out = nullptr;
    if (mb <= 0 || nb <= 0 || Z <= 0 || !shifts) return fail(CBP_EINVAL, "bad QC shape or NULL shifts");
    if ((int64_t)nb * Z >= ((int64_t)1 << 31) || (int64_t)mb * Z >= ((int64_t)1 << 31))
        return fail(CBP_EINVAL, "QC code too large");
    for (int i = 0; i < mb * nb; ++i)
        if (shifts[i] < -1 || shifts[i] >= Z) return fail(CBP_EINVAL, "shift[%d] = %d out of range", i, shifts[i]);
    std::vector<int> row_ptr((size_t)mb * Z + 1, 0), col_idx;
    for (int r = 0; r < mb; ++r)
        for (int k = 0; k < Z; ++k) {
            for (int b = 0; b < nb; ++b) {
                const int s = shifts[r * nb + b];
                if (s >= 0) col_idx.push_back(b * Z + (k + s) % Z);
            }
            row_ptr[(size_t)r * Z + k + 1] = (int)col_idx.size();
        }
    cbp_code_t *c = nullptr;
    int rc = cbp_code_from_csr(mb * Z, nb * Z, row_ptr.data(), col_idx.data(), &c);
    if (rc) return rc;
    c->qc = true;
    c->mb = mb;
    c->nb = nb;
    c->Z = Z;
    c->shifts.assign(shifts, shifts + mb * nb);
    for (int r = 0; r < mb; ++r) {
        int d = 0;
        for (int b = 0; b < nb; ++b) d += shifts[r * nb + b] >= 0;
        c->qE += d;
        c->qdcmax = std::max(c->qdcmax, d);
    }
    for (int k = 0; k < qc_reg_count(); ++k) {
        int kmb, knb, kz;
        const uint8_t *pat;
        qc_reg_entry(k, &kmb, &knb, &kz, &pat);
        if (kmb != mb || knb != nb || kz != Z) continue;
        bool same = true;
        for (int i = 0; i < mb * nb && same; ++i) same = (pat[i] != 0) == (shifts[i] >= 0);
        if (same) {
            c->qc_reg_id = k;
            break;
        }
    }
    *out = c;
    return CBP_OK;
}

void cbp_code_free(cbp_code_t *c) {
    if (!c) return;
    int cur = 0;
    bool have_cur = hipGetDevice(&cur) == hipSuccess;
    for (int d = 0; d < kMaxDevices; ++d)
        if (c->dev[d].ready && c->dev[d].buf) {
            if (hipSetDevice(d) == hipSuccess) (void)hipFree(c->dev[d].buf);
        }
    if (have_cur) (void)hipSetDevice(cur);
    delete c;
}

int cbp_code_levels(const cbp_code_t *c, int32_t *nlev, int32_t *lvl_ptr, int32_t *rows) {
    if (!c) return fail(CBP_EINVAL, "code is NULL");
    if (nlev) *nlev = c->nlev;
    if (lvl_ptr) std::memcpy(lvl_ptr, c->lvl_ptr.data(), 4 * ((size_t)c->nlev + 1));
    if (rows) std::memcpy(rows, c->lvl_rows.data(), 4 * (size_t)c->M);
    return CBP_OK;
}

int cbp_code_info(const cbp_code_t *c, int32_t *M, int32_t *N, int64_t *E, int32_t *Z,
                  int32_t *kernels) {
    if (!c) return fail(CBP_EINVAL, "code is NULL");
    if (M) *M = c->M;
    if (N) *N = c->N;
    if (E) *E = c->E;
    if (Z) *Z = c->qc ? c->Z : 0;
    if (kernels)
        *kernels = CBP_KERNEL_SPARSE | (c->qc_reg_id >= 0 ? CBP_KERNEL_QC_REG : 0) |
                   (c->qc && c->Z <= 1024 && c->mb < 32768 && c->nb < 65536 ? CBP_KERNEL_QC_STREAM : 0) |
                   (lds_kernel_fits(kCBP, c) ? CBP_KERNEL_SPARSE_LDS : 0);
    return CBP_OK;
}

int cbp_decode(const cbp_code_t *code, const float *llr_in, uint8_t *bits_out, int32_t *iters_out,
               int32_t max_iter, int64_t batch, const cbp_opts_t *opts, void *stream) {
    const int algo = (opts && opts->check_rule == CBP_RULE_MIN_SUM) ? kCBPNMS : kCBP;
    return decode(algo, code, llr_in, bits_out, iters_out, max_iter, batch, opts, stream);
}

int lbp_nms_decode(const cbp_code_t *code, const float *llr_in, uint8_t *bits_out,
                   int32_t *iters_out, int32_t max_iter, int64_t batch, const cbp_opts_t *opts,
                   void *stream) {
    return decode(kLBPNMS, code, llr_in, bits_out, iters_out, max_iter, batch, opts, stream);
}

int fbp_nms_decode(const cbp_code_t *code, const float *llr_in, uint8_t *bits_out,
                   int32_t *iters_out, int32_t max_iter, int64_t batch, const cbp_opts_t *opts,
                   void *stream) {
    return decode(kFBPNMS, code, llr_in, bits_out, iters_out, max_iter, batch, opts, stream);
}

int lbp_decode(const cbp_code_t *code, const float *llr_in, uint8_t *bits_out, int32_t *iters_out,
               int32_t max_iter, int64_t batch, const cbp_opts_t *opts, void *stream) {
    return decode(kLBP, code, llr_in, bits_out, iters_out, max_iter, batch, opts, stream);
}

int fbp_decode(const cbp_code_t *code, const float *llr_in, uint8_t *bits_out, int32_t *iters_out,
               int32_t max_iter, int64_t batch, const cbp_opts_t *opts, void *stream) {
    return decode(kFBP, code, llr_in, bits_out, iters_out, max_iter, batch, opts, stream);
}

int cbp_decode_static(const cbp_code_t *code, int32_t decoder, const float *llr_in, uint8_t *bits_out,
                      int32_t *iters_out, int32_t max_iter, int64_t batch, const cbp_opts_t *opts,
                      void *stream) {
    if (decoder < 0 || decoder > 4) return fail(CBP_EINVAL, "decoder must be 0 .. 4");
    static const int kDecoderAlgo[5] = {kCBP, kLBPNMS, kFBPNMS, kLBP, kFBP};
    int algo = kDecoderAlgo[decoder];
    if (algo == kCBP && opts && opts->check_rule == CBP_RULE_MIN_SUM) algo = kCBPNMS;
    // the checks decode() makes before any device work, so that an empty batch
    // is a no-op here too
    if (!code) return fail(CBP_EINVAL, "code is NULL");
    if (batch < 0) return fail(CBP_EINVAL, "batch < 0");
    if (max_iter < 0) return fail(CBP_EINVAL, "max_iter < 0");
    if (batch == 0) return CBP_OK;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    FixedWs fx;
    int rc = static_scratch(dev, &fx.base);
    if (rc) return rc;
    fx.bytes = kStaticScratchBytes;
    return decode(algo, code, llr_in, bits_out, iters_out, max_iter, batch, opts, stream, &fx);
}

int cbp_workspace_size(const cbp_code_t *code, int32_t decoder, int64_t batch, const cbp_opts_t *opts,
                       size_t *bytes) {
    if (!code || !bytes) return fail(CBP_EINVAL, "code/bytes is NULL");
    if (decoder < 0 || decoder > 4) return fail(CBP_EINVAL, "decoder must be 0 .. 4");
    static const int kDecoderAlgo[5] = {kCBP, kLBPNMS, kFBPNMS, kLBP, kFBP};
    int algo = kDecoderAlgo[decoder];
    if (algo == kCBP && opts && opts->check_rule == CBP_RULE_MIN_SUM) algo = kCBPNMS;
    if (batch < 0) return fail(CBP_EINVAL, "batch < 0");
    Resolved r;
    int rc = resolve_opts(code, algo, batch, opts, &r);
    if (rc) return rc;
    SparseDev g{};
    g.M = code->M;
    g.N = code->N;
    g.E = (int)code->E;
    *bytes = batch == 0 ? 0 : needed_ws(algo, code, g, r.kernel, batch, r.handoff);
    return CBP_OK;
}

int cbp_syndrome(const cbp_code_t *code, const uint8_t *bits, uint8_t *ok_out, int64_t batch,
                 void *stream) {
    if (!code) return fail(CBP_EINVAL, "code is NULL");
    if (batch < 0) return fail(CBP_EINVAL, "batch < 0");
    if (batch == 0) return CBP_OK;
    if (!bits || !ok_out) return fail(CBP_EINVAL, "bits/ok_out is NULL");
    int dev = 0;
    const SparseDev *g = nullptr;
    int rc = ensure_device(code, &dev, &g);
    if (rc) return rc;
    hipError_t e = launch_syndrome(*g, bits, ok_out, batch, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "syndrome launch");
    return CBP_OK;
}

const char *cbp_strerror(int status) {
    switch (status) {
    case CBP_OK: return "ok";
    case CBP_EINVAL: return "invalid argument";
    case CBP_EUNSUPPORTED: return "unsupported";
    case CBP_EHIP: return "HIP error";
    case CBP_ENOMEM: return "out of memory";
    default: return "unknown status";
    }
}

const char *cbp_last_error(void) { return g_err.c_str(); }

int32_t cbp_version(void) { return 100; }

}  // extern "C"
