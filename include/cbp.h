/*
 * cbp.h -- C ABI of the MI355X check-belief propagation (CBP) LDPC decoder.
 *
 * Method: W. Guan, L. Liang, "Check-Belief Propagation Decoding of LDPC
 * Codes", IEEE Trans. Commun. (arXiv 2305.05286).
 *
 * All entry points use C linkage, plain pointers and sizes, and return an int
 * status (CBP_OK or a negative CBP_E* code); none aborts or prints.  A
 * human-readable message for the last failure of the calling thread is
 * returned by cbp_last_error().
 *
 * Device buffers are owned by the caller; the decoders read and write them
 * asynchronously on the caller's HIP stream (passed as void*, NULL = the
 * default stream) and results are valid once that stream has synchronised.
 * A code handle owns copies of the parity-check tables (host and, created on
 * first use, per device); it is immutable and may be shared by any number of
 * threads and streams.
 */
#ifndef CBP_H
#define CBP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define CBP_OK 0
#define CBP_EINVAL (-1)       /* null pointer, bad shape/size/option, malformed H */
#define CBP_EUNSUPPORTED (-2) /* valid request the library does not implement     */
#define CBP_EHIP (-3)         /* HIP runtime or launch error                      */
#define CBP_ENOMEM (-4)       /* device or host allocation failed                 */

/* ---- code handles ------------------------------------------------------ */
typedef struct cbp_code cbp_code_t;

/*
 * Parity-check matrix H (M x N) in CSR form: row i is check-node c_i, column v
 * is variable-node v (paper Sec. II).  row_ptr has M+1 entries (row_ptr[0] = 0,
 * non-decreasing, row_ptr[M] = E); col_idx has E entries, strictly ascending
 * within each row (ascending order is the order in which the C2B recursion
 * folds a row's V2C messages).  Every row needs degree >= 2 and every column
 * degree >= 1, else CBP_EINVAL.  Host pointers; copied.
 */
int cbp_code_from_csr(int32_t M, int32_t N, const int32_t *row_ptr, const int32_t *col_idx,
                      cbp_code_t **out);

/*
 * Quasi-cyclic H from a base matrix of mb x nb circulant shifts (row-major,
 * host pointer, copied): -1 is a Z x Z zero block, s in [0, Z) is the identity
 * cyclically shifted so that row k of the block connects to column (k+s) mod Z
 * of the block-column.  Row r*Z+k of H is row k of block-row r; the lifted H
 * is also available to every decoder as CSR.  Block-rows are the layers of the
 * sweep: the Z rows of a block-row share no variable, so they are updated in
 * parallel with a result identical to the paper's row-by-row order.
 */
int cbp_code_from_qc(int32_t mb, int32_t nb, int32_t Z, const int32_t *shifts, cbp_code_t **out);

void cbp_code_free(cbp_code_t *code);

/* Shape of a handle.  Any output pointer may be NULL.  *kernels is a bit set of
 * the decoder layouts available for this code (CBP_KERNEL_* below). */
int cbp_code_info(const cbp_code_t *code, int32_t *M, int32_t *N, int64_t *E, int32_t *Z,
                  int32_t *kernels);

/* Row levels of a code (library-computed at creation): level(i) = 1 + the
 * highest level of the rows before i that share a variable with it (0 if none),
 * so rows of one level share no variable and every two rows with a common
 * variable keep their index order.  Such rows commute in the sequential row
 * schedule of Sec. IV-C (a row reads and writes only messages of its own
 * variables), which lets the sparse kernel run a frame's sweep level by level
 * with its rows in parallel.  Outputs (each may be NULL): *nlev; lvl_ptr
 * [nlev + 1]; rows [M] sorted by (level, index), level l holding
 * rows[lvl_ptr[l] .. lvl_ptr[l + 1]). */
int cbp_code_levels(const cbp_code_t *code, int32_t *nlev, int32_t *lvl_ptr, int32_t *rows);

/* ---- options ----------------------------------------------------------- */
#define CBP_KERNEL_AUTO 0
#define CBP_KERNEL_QC_REG 1    /* QC: frame state in VGPRs + LDS (compiled base patterns) */
#define CBP_KERNEL_QC_STREAM 2 /* QC: messages streamed from device memory, any base     */
#define CBP_KERNEL_SPARSE 4    /* any H: one frame per lane, persistent (lanes take new  */
                               /* frames as theirs stop), state per wave contiguous      */
#define CBP_KERNEL_SPARSE_LDS 8 /* any H whose frame state (CBP 4N + 4E + 8M + N bytes,   */
                               /* rounded; the BP decoders 4N + 4E + 8 x the rows of the */
                               /* largest level, flooding 4N more) fits a CU's LDS: frames */
                               /* staged in LDS, each sweep level by level (see          */
                               /* cbp_code_levels), the edges of a level on separate     */
                               /* threads; persistent.  Every decoder, with stop_rule 0  */
                               /* or 2, hd_mode 0 and no dumps (else CBP_EUNSUPPORTED).  */
                               /* Results are bit-identical to CBP_KERNEL_SPARSE.  AUTO  */
                               /* picks it, when the options and the state allow, for    */
                               /* every code whose base pattern is not compiled in.      */
                               /* CBP_SPARSE_LDS_FRAMES (>= 1) in the environment caps   */
                               /* the frames per workgroup (tuning).                     */
/* Sparse kernel, slow frames: once every frame of the batch has been taken, a
 * wave with at most 16 busy lanes (CBP_SPARSE_HANDOFF in the environment:
 * 0 = never, 1..64) copies their frames into the workspace and a second launch
 * finishes them one frame per workgroup, running each sweep level by level (see
 * cbp_code_levels) with the rows of a level on separate lanes.  Results are
 * bit-identical to finishing them on their lanes.  Not used with stop_rule 1,
 * hd_mode 1 or state dumps.  CBP_SPARSE_HANDOFF_ITEMS (> 0) caps the frames
 * handed over (the rest finish on their lanes); the items take at most 8 GiB. */

#define CBP_RULE_LOG_TANH 0
#define CBP_RULE_MIN_SUM 1

typedef struct {
    /* 0: stop when the syndrome H x^T = 0, tested on [L < 0] before the first
     *    sweep and after every sweep (default).  1: the paper's rule (Sec.
     *    IV-C Step 2(3)), cbp_decode only: stop as soon as M consecutive check
     *    updates (rows in index order, across sweeps) each leave Omega > 0 and
     *    flip no hard decision; the decisions are those after that row, and
     *    iters_out counts the sweep it falls in.  With hd_mode 1 it needs the
     *    sparse kernel (else CBP_EUNSUPPORTED).  2: run exactly max_iter sweeps. */
    int32_t stop_rule;
    /* CBP hard decision.  0: x_v = [Lambda_v < 0] from the V2C phase of v's
     * last visit in the sweep (paper Step 3; default).  1: from the flushed
     * posterior Q_v + psi-(Omega_latest(v), Q_v) at the end of each sweep. */
    int32_t hd_mode;
    /* Saturation of V2C magnitudes entering the check rule (default 20). */
    float lmax;
    /* Normalisation factor of the min-sum baselines (default 0.75). */
    float alpha;
    /* CBP_KERNEL_AUTO or one CBP_KERNEL_* value (CBP_EUNSUPPORTED if that
     * layout is unavailable for the code). */
    int32_t kernel;
    /* cbp_decode check rule.  CBP_RULE_LOG_TANH (default): B2V and C2B with
     * phi (eqs. equ_s4e18, equ_s4e21).  CBP_RULE_MIN_SUM: the normalized
     * min-sum form of Sec. IV-D: each check keeps the two smallest clamped
     * |Q| (unscaled) and the sign parity of its V2C messages; B2V = parity *
     * sgn(Q) * alpha * (|Q| == min1 ? min2 : min1). */
    int32_t check_rule;
    /* Debug dump of the decoder state after sweep dump_sweep (0 = off) for
     * frames [0, dump_frames): float32 device buffers, frame-major, each may
     * be NULL.  CBP: dump_q = latest V2C Q [N], dump_r = C2V R [E, CSR edge
     * order], dump_om = check-belief Omega in the LLR domain [M] (min-sum
     * rule: parity * alpha * min1), dump_lam = flushed posterior [N].
     * Min-sum baselines: dump_lam = posterior, dump_r = R.  Rows of frames
     * that stopped before dump_sweep are not written. */
    int32_t dump_sweep;
    /* Nonzero: scan llr_in for NaN and +-Inf before decoding and return
     * CBP_EINVAL, decoding nothing, if one is found (the message names the
     * first such frame and position).  The scan reads the flag back, so the
     * call synchronises `stream`; not available in cbp_mix_graph_create
     * (CBP_EUNSUPPORTED).  Zero (default): no scan; a non-finite LLR leaves
     * the decisions and iteration count of its own frame unspecified (every
     * memory access is still indexed from the code tables alone, never from a
     * value, and every loop is bounded by max_iter). */
    int32_t validate;
    int64_t dump_frames;
    float *dump_q;
    float *dump_r;
    float *dump_om;
    float *dump_lam;
    /* Optional caller-provided device workspace (see cbp_workspace_size),
     * 256-byte aligned; if NULL or too small the call allocates one
     * stream-ordered.  Its contents on entry are ignored (frame counters in it
     * are reset by the call); calls sharing one workspace must not overlap. */
    void *workspace;
    size_t workspace_bytes;
} cbp_opts_t;

/* Fill *opts with the defaults listed above. */
void cbp_opts_default(cbp_opts_t *opts);

/* ---- decoders ---------------------------------------------------------- */
/*
 * Decode `batch` frames.
 *   llr_in    device float32 [batch][N]: channel LLRs ln Pr(y|x=0)/Pr(y|x=1)
 *             (Sec. IV-C Step 1), L > 0 favours bit 0.
 *   bits_out  device uint8   [batch][N]: hard decisions, 0/1 (Lambda = 0 -> 0).
 *   iters_out device int32   [batch]: sweeps executed, 0..max_iter (0 when
 *             [L < 0] already has a zero syndrome).  A frame with
 *             iters_out == max_iter may have failed: test with cbp_syndrome.
 *   max_iter  >= 0; 0 outputs [L < 0].  batch == 0 is a no-op.
 *   opts      NULL for defaults.
 *   stream    hipStream_t as void* (NULL = default stream).
 *
 * cbp_decode: CBP, Sec. IV-C Steps 1-3 (B2V eq. equ_s4e18, V2C eq. equ_s4e19,
 *   posterior eq. equ_s4e20, C2B eq. equ_s4e21, commits eqs. equ_s4e22/23);
 *   rows in index order, a row's V2C messages folded in ascending column order;
 *   a check not yet updated in this decode contributes a zero B2V message; the
 *   commit of Step 2(1)e stores R(c_j -> v) before R(c_i -> v) is read.
 * lbp_nms_decode: layered BP (Sec. II-B, eqs. equ_s2e10/equ_s2e12) with the
 *   normalized min-sum check rule alpha * prod sgn * min |Q| (|Q| <= lmax).
 * fbp_nms_decode: flooding BP (Sec. II-A, eqs. equ_s2e3/equ_s2e6/equ_s2e7)
 *   with the same normalized min-sum check rule.
 * lbp_decode, fbp_decode: the same two schedules with the paper's own check
 *   rule, the log-tanh C2V of eq. equ_s2e4 (phi of the sum of phi(|Q|) over
 *   the row's other edges, |Q| clamped to [phi(lmax), lmax] as in
 *   cbp_decode): the LBP and FBP the paper compares CBP with (Sec. V).
 *   They run on the CSR kernels (opts->kernel AUTO, CBP_KERNEL_SPARSE or
 *   CBP_KERNEL_SPARSE_LDS, else CBP_EUNSUPPORTED) for any code.
 */
int cbp_decode(const cbp_code_t *code, const float *llr_in, uint8_t *bits_out,
               int32_t *iters_out, int32_t max_iter, int64_t batch,
               const cbp_opts_t *opts, void *stream);
int lbp_nms_decode(const cbp_code_t *code, const float *llr_in, uint8_t *bits_out,
                   int32_t *iters_out, int32_t max_iter, int64_t batch,
                   const cbp_opts_t *opts, void *stream);
int fbp_nms_decode(const cbp_code_t *code, const float *llr_in, uint8_t *bits_out,
                   int32_t *iters_out, int32_t max_iter, int64_t batch,
                   const cbp_opts_t *opts, void *stream);
int lbp_decode(const cbp_code_t *code, const float *llr_in, uint8_t *bits_out,
               int32_t *iters_out, int32_t max_iter, int64_t batch,
               const cbp_opts_t *opts, void *stream);
int fbp_decode(const cbp_code_t *code, const float *llr_in, uint8_t *bits_out,
               int32_t *iters_out, int32_t max_iter, int64_t batch,
               const cbp_opts_t *opts, void *stream);

/* Device workspace (bytes) the given decoder needs for `batch` frames with
 * these options; decoder: 0 = cbp_decode, 1 = lbp_nms_decode, 2 = fbp_nms_decode,
 * 3 = lbp_decode, 4 = fbp_decode.  The sparse kernel's workspace holds at most
 * 131072 frames' state (and at most 32 GiB): it does not grow with larger
 * batches. */
int cbp_workspace_size(const cbp_code_t *code, int32_t decoder, int64_t batch,
                       const cbp_opts_t *opts, size_t *bytes);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the decoder
 * selected by `decoder` (0 = cbp_decode, 1 = lbp_nms_decode, 2 = fbp_nms_decode,
 * 3 = lbp_decode, 4 = fbp_decode; opts->check_rule picks CBP's rule as in
 * cbp_decode) with the same arguments, options and results, allocating
 * nothing: no hipMalloc / hipFree, stream-ordered or not.
 *   Workspace: a static device array of 64 MiB per GPU inside the library,
 *   held until the process ends; opts->workspace is ignored.  The persistent
 *   kernels take no more frames in flight than fit in it (the decoded results
 *   do not depend on that number); a code whose smallest unit of work does not
 *   fit (one streamed workgroup's frame state, or 64 frames on the sparse
 *   kernel) is rejected with CBP_EUNSUPPORTED, and so is a code whose device
 *   tables have not been built on the current device: any allocating call
 *   with that code on that device (e.g. cbp_syndrome) builds them.
 *   Calls on one GPU share its array and keep the last call's contents (each
 *   call resets the counters it uses): calls that overlap on one GPU, on any
 *   streams, race and must not be issued.  opts->validate reads its result
 *   back through the same array and synchronises `stream`, as in cbp_decode.
 */
int cbp_decode_static(const cbp_code_t *code, int32_t decoder, const float *llr_in,
                     uint8_t *bits_out, int32_t *iters_out, int32_t max_iter, int64_t batch,
                     const cbp_opts_t *opts, void *stream);

/*
 * Syndrome test (the stopping test of FBP, Sec. II-A): ok_out[f] = 1 if
 * H bits[f]^T = 0 over GF(2), else 0.  bits: device uint8 [batch][N] (0/1);
 * ok_out: device uint8 [batch].
 */
int cbp_syndrome(const cbp_code_t *code, const uint8_t *bits, uint8_t *ok_out, int64_t batch,
                 void *stream);

/* ---- mixed-code batches ------------------------------------------------- */
/*
 * One persistent launch decodes frames of several QC codes (different rates,
 * lengths and lifting sizes Z) with per-frame early termination.  Frames wait
 * in one queue per code; every workgroup has the same number of lanes, a
 * multiple of each code's Z, and decodes lanes / Z frames of one code at a
 * time, refilling a slot from the queue as soon as its frame stops; when a
 * code's queue is empty the workgroup moves on to the next code.  Every code
 * must offer the streamed layout (CBP_KERNEL_QC_STREAM in cbp_code_info).
 */
typedef struct cbp_mix cbp_mix_t;

/* A plan over ncodes (1..256) QC code handles.  The handles are referenced,
 * not copied: they must outlive the plan.  CBP_EUNSUPPORTED if a code lacks
 * the streamed layout or the least common multiple of the Z values exceeds
 * 1024. */
int cbp_mix_create(const cbp_code_t *const *codes, int32_t ncodes, cbp_mix_t **out);
void cbp_mix_free(cbp_mix_t *mix);

/* Schedule of the persistent launch: lanes per workgroup (a multiple of every
 * Z of the plan, at most 1024; it sets the frames per workgroup, lanes / Z)
 * and workgroups per CU (0 = as many as fit).  The default is the smallest
 * multiple of the Z values that fills whole 64-lane waves, and 0. */
typedef struct {
    int32_t lanes;
    int32_t groups_per_cu;
    /* 0 (default): every code on the streamed kernel.  1 or 2: the codes whose
     * frame state fits half a CU's LDS are decoded staged in LDS (the layout of
     * CBP_KERNEL_SPARSE_LDS) by this many workgroups per CU, on a second
     * stream beside the streamed launch (the plan's own stream, joined back
     * before the call's work ends; calls with one plan on one device take
     * turns on it); results are identical either way.  cbp_mix_tune tries 0,
     * 1 and 2 with every streamed schedule. */
    int32_t lds_groups_per_cu;
} cbp_mix_schedule_t;
int cbp_mix_get_schedule(const cbp_mix_t *mix, cbp_mix_schedule_t *sched);
int cbp_mix_set_schedule(cbp_mix_t *mix, const cbp_mix_schedule_t *sched);

/* Device workspace (bytes) of cbp_mix_decode for `batch` frames on the
 * current device under the plan's schedule; decoder as for
 * cbp_workspace_size (0 = cbp_decode with opts->check_rule, 1 = layered
 * NMS, 2 = flooding NMS). */
int cbp_mix_workspace_size(const cbp_mix_t *mix, int32_t decoder, int64_t batch,
                           const cbp_opts_t *opts, size_t *bytes);

/*
 * Decode a mixed batch with one decoder (same rules and options as the
 * single-code entry points; state dumps are not supported here).
 *   llr_in       device float32 [llr_elems]: the frames' channel LLRs, packed.
 *   frame_code   device int32 [batch]: index in the plan of frame f's code.
 *   frame_offset device int64 [batch]: element offset of frame f in llr_in and
 *                bits_out; the frame occupies N of its code elements.
 *   bits_out     device uint8 [llr_elems]: hard decisions at the same offsets.
 *   iters_out    device int32 [batch]: sweeps executed; -1 for a frame whose
 *                code index is outside the plan or whose LLRs leave
 *                [0, llr_elems) (its decisions are not written).
 *   workspace    device buffer of at least cbp_mix_workspace_size bytes, 256-byte
 *                aligned (CBP_EINVAL otherwise).
 * The call only launches kernels on `stream` (with lds_groups_per_cu > 0 also
 * on the plan's own side stream, forked from `stream` by an event and joined
 * back to it before the call's work ends): no allocation, no host
 * synchronisation, no memset node, so it may be captured in a HIP graph once
 * the plan has been used on the device (the first call uploads the code
 * tables and creates the side stream) — see cbp_mix_graph_create.
 */
int cbp_mix_decode(const cbp_mix_t *mix, int32_t decoder, const float *llr_in, int64_t llr_elems,
                   const int32_t *frame_code, const int64_t *frame_offset, uint8_t *bits_out,
                   int32_t *iters_out, int32_t max_iter, int64_t batch, const cbp_opts_t *opts,
                   void *workspace, size_t workspace_bytes, void *stream);

/*
 * Autotuner: decodes the given batch (arguments as for cbp_mix_decode, minus
 * the workspace) twice per candidate schedule — lanes in {L, 2L, 4L} up to
 * 1024 (L = the default lanes) times workgroups per CU from 1 to what fits
 * times lds_groups_per_cu in {0, 1, 2} — timing the second launch with HIP
 * events on `stream` (the call synchronises it and allocates its own
 * workspace), and sets the fastest as the plan's schedule.
 * best and best_ms may be NULL.  The outputs hold the last candidate's
 * (identical) decode.
 */
int cbp_mix_tune(cbp_mix_t *mix, int32_t decoder, const float *llr_in, int64_t llr_elems,
                 const int32_t *frame_code, const int64_t *frame_offset, uint8_t *bits_out,
                 int32_t *iters_out, int32_t max_iter, int64_t batch, const cbp_opts_t *opts,
                 void *stream, cbp_mix_schedule_t *best, float *best_ms);

/* A HIP graph of one cbp_mix_decode call with these arguments (captured on a
 * private stream; every replay reads and writes the same buffers, so refill
 * llr_in / frame_code / frame_offset in place between replays).
 * cbp_graph_launch replays it on `stream`. */
typedef struct cbp_graph cbp_graph_t;
int cbp_mix_graph_create(const cbp_mix_t *mix, int32_t decoder, const float *llr_in,
                         int64_t llr_elems, const int32_t *frame_code,
                         const int64_t *frame_offset, uint8_t *bits_out, int32_t *iters_out,
                         int32_t max_iter, int64_t batch, const cbp_opts_t *opts, void *workspace,
                         size_t workspace_bytes, cbp_graph_t **out);
int cbp_graph_launch(cbp_graph_t *graph, void *stream);
void cbp_graph_free(cbp_graph_t *graph);

/* ---- unrolled differentiable CBP ---------------------------------------- */
/*
 * A fixed number of CBP sweeps (Sec. IV-C, no stopping test) whose B2V outputs
 * carry learnable weights: in sweep t, the B2V output R_new(c_j -> v) of eq.
 * equ_s4e18 is replaced by
 *     sgn(R_new) * max(w[t][b] * |R_new| - beta[t][b], 0)
 * (b = the base block-column of v) before it is committed and added to Q_v.
 * w = 1, beta = 0 is plain CBP.  The output is the soft value
 * o_v = Q_v + (the same weighted B2V from v's latest check with the weights of
 * the last sweep), in LLR units (o_v > 0 favours bit 0).  QC codes with the
 * streamed layout only.
 *
 * Memory: the forward pass keeps a checkpoint of the frame state (Q, R,
 * check-beliefs) at the start of every sweep after the first, and the final
 * state, in the workspace; the backward pass recomputes one sweep at a time in
 * place on its checkpoint and runs the adjoint backwards through it, so the
 * workspace grows with sweeps x frame state, not with the per-edge history of
 * all sweeps.  The backward pass consumes the checkpoints: call it at most
 * once per forward call (a second call on the same workspace gives wrong
 * gradients; run the forward again first).
 *
 *   w, beta      device float32 [sweeps][nb] (nb = base block-columns).
 *   llr_in       device float32 [batch][N].
 *   soft_out     device float32 [batch][N].
 *   grad_out     device float32 [batch][N]: dLoss/d soft_out.
 *   grad_llr     device float32 [batch][N]: dLoss/d llr_in, or NULL.
 *   grad_w, grad_beta  device float32 [sweeps][nb]: dLoss/dw, dLoss/dbeta
 *                (summed over the batch; written, not accumulated).
 *   workspace    device buffer of at least cbp_unrolled_workspace_size bytes,
 *                256-byte aligned (CBP_EINVAL otherwise);
 *                cbp_unrolled_backward must get the workspace of the
 *                cbp_unrolled_forward call with the same code, llr_in, batch,
 *                sweeps, w and beta, unmodified in between.
 *   opts         NULL or options (lmax is used).
 * Deterministic: repeated calls give identical results.
 */
int cbp_unrolled_workspace_size(const cbp_code_t *code, int32_t sweeps, int64_t batch, size_t *bytes);
int cbp_unrolled_forward(const cbp_code_t *code, const float *llr_in, int64_t batch, int32_t sweeps,
                         const float *w, const float *beta, float *soft_out, const cbp_opts_t *opts,
                         void *workspace, size_t workspace_bytes, void *stream);
int cbp_unrolled_backward(const cbp_code_t *code, const float *llr_in, int64_t batch, int32_t sweeps,
                          const float *w, const float *beta, const float *grad_out, float *grad_llr,
                          float *grad_w, float *grad_beta, const cbp_opts_t *opts, void *workspace,
                          size_t workspace_bytes, void *stream);

/* ---- diagnostics --------------------------------------------------------- */
const char *cbp_strerror(int status);
const char *cbp_last_error(void);
/* Library version, 100 * major + minor. */
int32_t cbp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CBP_H */
