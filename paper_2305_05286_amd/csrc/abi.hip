// C ABI of the decoder library: argument checking, code handles, per-device
// tables, workspace and kernel selection.  Declarations and contracts are in
// include/cbp.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
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
    QcStreamDev qs{};             // base structure of the streamed kernel
    bool qs_ready = false;
};

}  // namespace

struct cbp_code {
    int M = 0, N = 0;
    int64_t E = 0;
    std::vector<int> row_ptr, col_idx, edge_row, pred_edge, pred_row, last_edge;
    std::vector<uint8_t> first;
    bool qc = false;
    int mb = 0, nb = 0, Z = 0;
    std::vector<int> shifts;
    int qc_reg_id = -1;
    int qE = 0, qdcmax = 0;  // base edges and max block-row degree (QC codes)
    std::mutex mu;
    DevTables dev[kMaxDevices];
};

namespace {

// Column lists in row order give each edge its latest check in steady state
// (the cyclically previous row of the same column) and the first-visit flag.
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
                c->first[e] = 1;
            } else {
                c->pred_edge[e] = c->last_edge[v];
            }
            c->last_edge[v] = e;
        }
    for (int v = 0; v < N; ++v) {
        if (first_edge[v] < 0) return fail(CBP_EINVAL, "column %d has no edge", v);
        c->pred_edge[first_edge[v]] = c->last_edge[v];
    }
    for (int64_t e = 0; e < E; ++e) c->pred_row[e] = c->edge_row[c->pred_edge[e]];
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

int ensure_device(const cbp_code *cc, int *device_out, const SparseDev **g,
                  const int **qc_sht = nullptr, const QcStreamDev **qs = nullptr) {
    cbp_code *c = const_cast<cbp_code *>(cc);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(CBP_EUNSUPPORTED, "device %d", dev);
    *device_out = dev;
    std::lock_guard<std::mutex> lock(c->mu);
    DevTables &t = c->dev[dev];
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
            for (auto *v : {&rstart, &eb, &esh, &er, &ep, &epr, &epsh, &efirst, &elast})
                qt.insert(qt.end(), v->begin(), v->end());
            // the records start 16-byte aligned in the device buffer
            const size_t off0 = (size_t)(M + 1) + 4 * (size_t)E + (size_t)N + sht.size();
            while ((off0 + qt.size()) % 4) qt.push_back(0);
            for (int e = 0; e < qE; ++e) {
                const int last = elast[eb[e]] == e;
                qt.push_back(eb[e] | last << 29 | efirst[e] << 30);
                qt.push_back(esh[e]);
                qt.push_back(ep[e]);
                qt.push_back(epsh[e] | epr[e] << 16);
            }
        }
        const size_t ints = (size_t)(M + 1) + 4 * (size_t)E + (size_t)N + sht.size() + qt.size();
        const size_t bytes = ints * 4 + (size_t)E + 64;
        void *buf = nullptr;
        e = hipMalloc(&buf, bytes);
        if (e != hipSuccess) return fail(CBP_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
        std::vector<int> host(ints);
        int *p = host.data();
        std::memcpy(p, c->row_ptr.data(), 4 * (size_t)(M + 1));
        p += M + 1;
        std::memcpy(p, c->col_idx.data(), 4 * (size_t)E);
        p += E;
        std::memcpy(p, c->edge_row.data(), 4 * (size_t)E);
        p += E;
        std::memcpy(p, c->pred_edge.data(), 4 * (size_t)E);
        p += E;
        std::memcpy(p, c->pred_row.data(), 4 * (size_t)E);
        p += E;
        std::memcpy(p, c->last_edge.data(), 4 * (size_t)N);
        p += N;
        if (!sht.empty()) std::memcpy(p, sht.data(), 4 * sht.size());
        p += sht.size();
        if (!qt.empty()) std::memcpy(p, qt.data(), 4 * qt.size());
        e = hipMemcpy(buf, host.data(), ints * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy((char *)buf + ints * 4, c->first.data(), (size_t)E, hipMemcpyHostToDevice);
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
        d += E;
        t.g.edge_row = d;
        d += E;
        t.g.pred_edge = d;
        d += E;
        t.g.pred_row = d;
        d += E;
        t.g.last_edge = d;
        d += N;
        t.qc_sht = sht.empty() ? nullptr : d;
        d += sht.size();
        if (c->qc) {
            QcStreamDev &q = t.qs;
            q.Z = c->Z;
            q.mb = c->mb;
            q.nb = c->nb;
            q.E = qE;
            q.dcmax = dcmax;
            q.rstart = d;
            d += c->mb + 1;
            q.eb = d;
            d += qE;
            q.esh = d;
            d += qE;
            q.er = d;
            d += qE;
            q.ep = d;
            d += qE;
            q.epr = d;
            d += qE;
            q.epsh = d;
            d += qE;
            q.efirst = d;
            d += qE;
            q.elast = d;
            d += c->nb;
            d = reinterpret_cast<int *>(((uintptr_t)d + 15) & ~(uintptr_t)15);
            q.erec = reinterpret_cast<const int4 *>(d);
            d += 4 * (size_t)qE;
            t.qs_ready = true;
        }
        t.g.first = (const uint8_t *)((char *)buf + ints * 4);
        t.buf = buf;
        t.ready = true;
    }
    *g = &t.g;
    if (qc_sht) *qc_sht = t.qc_sht;
    if (qs) *qs = t.qs_ready ? &t.qs : nullptr;
    return CBP_OK;
}

struct Resolved {
    Params p;
    Dump d;
    int kernel;
    void *ws;
    size_t ws_bytes;
};

int resolve_opts(const cbp_code_t *code, int algo, int64_t batch, const cbp_opts_t *o, Resolved *r) {
    cbp_opts_t def;
    cbp_opts_default(&def);
    if (!o) o = &def;
    if (o->stop_rule == 1)
        return fail(CBP_EUNSUPPORTED, "stop_rule 1 (consecutive positive check-beliefs) is not implemented on the GPU");
    if (o->stop_rule != 0 && o->stop_rule != 2) return fail(CBP_EINVAL, "stop_rule must be 0 or 2");
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
    if (k == CBP_KERNEL_AUTO)
        k = code->qc_reg_id >= 0 ? CBP_KERNEL_QC_REG : stream_ok ? CBP_KERNEL_QC_STREAM : CBP_KERNEL_SPARSE;
    if (k == CBP_KERNEL_QC_REG && code->qc_reg_id < 0)
        return fail(CBP_EUNSUPPORTED, "no register-resident kernel is compiled for this base pattern");
    if (k == CBP_KERNEL_QC_STREAM && !stream_ok)
        return fail(CBP_EUNSUPPORTED, "the streamed kernel needs a QC code with Z <= 1024, mb < 32768, nb < 65536");
    if (k != CBP_KERNEL_QC_REG && k != CBP_KERNEL_QC_STREAM && k != CBP_KERNEL_SPARSE)
        return fail(CBP_EINVAL, "unknown kernel %d", o->kernel);
    r->kernel = k;
    r->p.lmax = o->lmax;
    r->p.a = (float)phi64((double)o->lmax);
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
    r->ws = o->workspace;
    r->ws_bytes = o->workspace_bytes;
    return CBP_OK;
}

constexpr int64_t kSparseChunkBytes = (int64_t)1 << 30;

int64_t sparse_chunk_frames(int algo, const SparseDev &g, int64_t batch) {
    const size_t per = sparse_ws_bytes(algo, g, 64) / 64 + 1;
    int64_t n = kSparseChunkBytes / (int64_t)per;
    n = n / 64 * 64;
    if (n < 64) n = 64;
    return batch < n ? batch : n;
}

// Streamed QC kernel: at most this many frames (slots) in flight per call,
// which bounds its workspace (e.g. 2048 x 0.68 MB for the n = 26112 code).
constexpr int64_t kStreamMaxSlots = 2048;

QcStreamDev stream_shape_of(const cbp_code_t *c) {
    QcStreamDev q{};
    q.Z = c->Z;
    q.mb = c->mb;
    q.nb = c->nb;
    q.E = c->qE;
    q.dcmax = c->qdcmax;
    return q;
}

int64_t stream_groups_cap(const QcStreamDev &q, int64_t batch) {
    int slots, threads;
    size_t lds;
    qc_stream_shape(q, &slots, &threads, &lds);
    const int64_t need = (batch + slots - 1) / slots;
    const int64_t cap = std::max<int64_t>(1, kStreamMaxSlots / slots);
    return std::min(need, cap);
}

size_t needed_ws(int algo, const cbp_code_t *code, const SparseDev &g, int kernel, int64_t batch) {
    if (kernel == CBP_KERNEL_QC_REG) return 256;
    if (kernel == CBP_KERNEL_QC_STREAM) {
        const QcStreamDev q = stream_shape_of(code);
        int slots, threads;
        size_t lds;
        qc_stream_shape(q, &slots, &threads, &lds);
        return 256 + (size_t)stream_groups_cap(q, batch) * slots * qc_stream_slot_bytes(algo, q);
    }
    return sparse_ws_bytes(algo, g, sparse_chunk_frames(algo, g, batch));
}

int decode(int algo, const cbp_code_t *code, const float *llr, uint8_t *bits, int32_t *iters,
           int32_t max_iter, int64_t batch, const cbp_opts_t *opts, void *stream) {
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
    const QcStreamDev *qs = nullptr;
    rc = ensure_device(code, &dev, &g, &qc_sht, &qs);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const size_t need = needed_ws(algo, code, *g, r.kernel, batch);
    void *ws = r.ws;
    bool own = false;
    if (!ws || r.ws_bytes < need) {
        hipError_t e = hipMallocAsync(&ws, need, s);
        if (e != hipSuccess) return fail(CBP_ENOMEM, "hipMallocAsync(%zu): %s", need, hipGetErrorString(e));
        own = true;
    }
    hipError_t e = hipSuccess;
    if (r.kernel == CBP_KERNEL_QC_REG) {
        e = launch_qc_reg(code->qc_reg_id, algo, qc_sht, llr, bits, iters, batch,
                          max_iter, r.p, r.d, (int *)ws, dev, s);
    } else if (r.kernel == CBP_KERNEL_QC_STREAM) {
        const int64_t cap = stream_groups_cap(*qs, batch);
        const int64_t groups = std::min<int64_t>(cap, qc_stream_groups(algo, *qs, dev));
        e = launch_qc_stream(algo, *qs, llr, bits, iters, batch, max_iter, r.p, r.d, (int)groups,
                             (char *)ws + 256, (int *)ws, s);
    } else {
        const int64_t chunk = sparse_chunk_frames(algo, *g, batch);
        SparseWs w = sparse_ws_carve(algo, *g, chunk, ws);
        for (int64_t f0 = 0; f0 < batch && e == hipSuccess; f0 += chunk) {
            const int64_t nf = batch - f0 < chunk ? batch - f0 : chunk;
            e = launch_sparse(algo, *g, llr, bits, iters, f0, nf, max_iter, r.p, w, r.d, s);
        }
    }
    if (own) {
        hipError_t e2 = hipFreeAsync(ws, s);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return CBP_OK;
}

}  // namespace

extern "C" {

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

int cbp_code_info(const cbp_code_t *c, int32_t *M, int32_t *N, int64_t *E, int32_t *Z,
                  int32_t *kernels) {
    if (!c) return fail(CBP_EINVAL, "code is NULL");
    if (M) *M = c->M;
    if (N) *N = c->N;
    if (E) *E = c->E;
    if (Z) *Z = c->qc ? c->Z : 0;
    if (kernels)
        *kernels = CBP_KERNEL_SPARSE | (c->qc_reg_id >= 0 ? CBP_KERNEL_QC_REG : 0) |
                   (c->qc && c->Z <= 1024 && c->mb < 32768 && c->nb < 65536 ? CBP_KERNEL_QC_STREAM : 0);
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

int cbp_workspace_size(const cbp_code_t *code, int32_t decoder, int64_t batch, const cbp_opts_t *opts,
                       size_t *bytes) {
    if (!code || !bytes) return fail(CBP_EINVAL, "code/bytes is NULL");
    if (decoder < 0 || decoder > 2) return fail(CBP_EINVAL, "decoder must be 0, 1 or 2");
    if (decoder == 0 && opts && opts->check_rule == CBP_RULE_MIN_SUM) decoder = kCBPNMS;
    if (batch < 0) return fail(CBP_EINVAL, "batch < 0");
    Resolved r;
    int rc = resolve_opts(code, decoder, batch, opts, &r);
    if (rc) return rc;
    SparseDev g{};
    g.M = code->M;
    g.N = code->N;
    g.E = (int)code->E;
    *bytes = batch == 0 ? 0 : needed_ws(decoder, code, g, r.kernel, batch);
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
