// Internal interfaces between the C ABI (abi.cpp) and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cbp {

// kCBPNMS: CBP with the normalized min-sum check rule (cbp_decode with
// CBP_RULE_MIN_SUM).  kLBP / kFBP: layered / flooding BP with the log-tanh
// check rule (sparse kernel only).
enum Algo : int { kCBP = 0, kLBPNMS = 1, kFBPNMS = 2, kCBPNMS = 3, kLBP = 4, kFBP = 5 };

// Work-item and workgroup ids straight from the hardware registers.  (The
// device code is built with relaxed NaN handling, which keeps the compiler
// from inlining the device library's id functions: threadIdx / blockIdx would
// become calls, with a stack frame and clobbered registers.)
__device__ __forceinline__ int tid_x() { return (int)__builtin_amdgcn_workitem_id_x(); }
__device__ __forceinline__ int gid_x() { return (int)__builtin_amdgcn_workgroup_id_x(); }

// Read of a table that no launch writes, through the constant address space:
// where the index is wave-uniform the compiler emits a scalar load (through a
// generic pointer it could not rule out aliasing with the kernel's stores and
// would issue a vector load, a full memory round trip, instead).
template <class T>
__device__ __forceinline__ T ldc(const T *p, int64_t i) {
    return ((const __attribute__((address_space(4))) T *)p)[i];
}

// A byte of such a table.  Scalar loads are dword-sized, so a byte read through
// ldc would become a vector load; this reads the containing dword (the table
// must start 4-byte aligned and be readable up to the next multiple of 4 bytes)
// and extracts the byte.
__device__ __forceinline__ uint32_t ldc_u8(const uint8_t *p, int64_t i) {
    return (ldc((const uint32_t *)p, i >> 2) >> (8 * (uint32_t)(i & 3))) & 0xffu;
}

// Bits of SparseDev::first.
constexpr uint32_t kFirstVisit = 1u, kLastVisit = 2u;

struct Params {
    float a;       // phi(lmax): lower clamp of |Q| entering phi
    float lmax;    // upper clamp
    float alpha;   // min-sum normalisation
    int stop_rule; // 0 syndrome, 2 fixed sweeps
    int hd_mode;   // CBP: 0 V2C-phase decision, 1 flushed posterior
};

struct Dump {
    int sweep;       // 0 = off
    int64_t frames;  // frames [0, frames) are dumped
    float *q, *r, *om, *lam;
};

// Device tables of a CSR code for the one-frame-per-lane kernels.
struct SparseDev {
    int M, N, E;
    const int *row_ptr;   // [M+1]
    const int *col_idx;   // [E]
    const int *edge_row;  // [E]  row of each edge
    const int *pred_edge; // [E]  edge of the cyclically previous row of the same column
    const int *pred_row;  // [E]  row of pred_edge
    const uint8_t *first; // [E]  visit flags: kFirstVisit if this is the lowest row of its
                          //      column, kLastVisit if the highest (both for weight one)
    const int *last_edge; // [N]  edge of the highest row of each column
    int nlev;             // row levels (rows of one level share no variable)
    const int *lvl_ptr;   // [nlev+1] first entry of each level in lvl_rows
    const int4 *lvl_rows; // [M] (row, first edge, end edge, 0) by (level, index)
    const int *lvl_eptr;  // [nlev+1] first entry of each level in lvl_edges
    const int4 *lvl_edges;// [E] the edges of lvl_rows' rows in that order: (column,
                          //      pred_edge, level position of pred_row (its entry
                          //      in lvl_rows), edge | first << 30)
    const int *lvl_erow;  // [E] the position of each lvl_edges entry's row
                          //      within its level
    int lvl_maxrows;      // rows of the largest level
};

// col_idx, pred_edge, pred_row and first are readable (zeros) for this many
// entries past E: the sparse kernels read a chunk's entries unconditionally,
// so that the scalar loads of a chunk go out together.
constexpr int kSparseTablePad = 16;

// Workspace of the sparse kernels: one contiguous block per wave (its 64
// lanes' state), frame-interleaved inside it — element (index, lane) of wave
// w lives at array[w * block_bytes + index * stride + lane] with stride = 64,
// so a wave's accesses are 256-byte lines within a few MB of its own.
struct SparseWs {
    int64_t stride;       // lanes per block (64)
    int64_t block_bytes;  // bytes from one wave's block to the next
    int64_t waves;        // blocks (= state slots / 64)
    float *a0, *a1, *a2, *a3, *a4;  // wave 0's arrays; meaning depends on the algorithm
    uint8_t *xb;
};

__host__ __device__ inline int64_t round256(int64_t x) { return (x + 255) / 256 * 256; }

// Hand-off of slow frames from the one-frame-per-lane kernels to a
// level-parallel kernel (one frame per workgroup, the rows of each level on
// separate threads).  An item holds one frame's state contiguously: CBP Q [N],
// R [E], Om [M] (float2), decisions [N]; BP Lambda [N], R [E], sums [N],
// decisions [N]; each array 256-byte aligned.
struct Handoff {
    int lanes;            // a wave hands over once the batch is exhausted and at most
                          // this many of its lanes are busy (0 = never)
    uint32_t cap;         // items
    int groups;           // workgroups of the level-parallel launch (one frame each at a time)
    unsigned int *count;  // frames handed over (any beyond cap stay on their lanes)
    int2 *items;          // [cap] (frame, sweeps done)
    char *state;          // [cap] frame states, item_bytes apart
    int64_t item_bytes;
};
int64_t sparse_item_bytes(int algo, const SparseDev &g);

size_t sparse_ws_bytes(int algo, const SparseDev &g, int64_t frames);
SparseWs sparse_ws_carve(int algo, const SparseDev &g, int64_t frames, void *base);
// Persistent sparse launch: one wave per block of `ws`, lanes take frames
// 0 .. nf-1 from `counter` (16 bytes: the frame counter, then h.count;
// reset by the launch).  With h.lanes > 0 a level-parallel launch
// over the handed-over frames follows on the same stream.
hipError_t launch_sparse(int algo, const SparseDev &g, const float *llr, uint8_t *bits,
                         int32_t *iters, int64_t nf, int max_iter, const Params &p,
                         const SparseWs &ws, const Dump &d, unsigned long long *counter,
                         const Handoff &h, hipStream_t s);
hipError_t launch_syndrome(const SparseDev &g, const uint8_t *bits, uint8_t *ok, int64_t batch,
                           hipStream_t s);

// ---- CSR codes with each frame's state in LDS ------------------------------
// Byte offsets of one frame's arrays in LDS: Q (CBP) or the posterior (BP)
// [N] at 0, R [E] at r, the rows' beliefs (CBP, [M]) or the fold states of one
// level's rows (BP, [lvl_maxrows]) (float2) at om, decisions [N] at xb (CBP;
// BP decides from the posterior's sign); bytes = 0 if the algorithm has no
// such kernel.
struct LdsItem {
    int r, om, xb, bytes;
    int acc;  // flooding BP: the C2V sums [N] (0 otherwise)
};
constexpr int kLdsMaxFrames = 8;       // frames per workgroup
constexpr int64_t kLdsStaticBytes = 256;  // the kernel's own LDS (slot table)
// Planning limit of a workgroup's LDS (gfx950: 160 KiB per CU); the launch
// uses the device's own figure.
constexpr int64_t kLdsPlanBytes = (int64_t)160 << 10;
LdsItem lds_item(int algo, const SparseDev &g);
// Frames per workgroup that fit in lds_limit bytes (0: none).
int lds_frames(const LdsItem &it, int64_t lds_limit);
// Mixed batches: workgroups of kLdsMixThreads threads, kLdsMixGroupsPerCu per
// CU; code c runs frames[c] (1, 2, 4 or 8; 0: not in this launch) frames per
// workgroup with layout items[c] from its queue (qstart / perm / counter as
// filled by launch_mix_prepare), frame f's LLRs and decisions at offset[f].
constexpr int kLdsMixThreads = 512;
constexpr int kLdsMixGroupsPerCu = 2;  // the LDS budget of a workgroup: half a CU
// Raises the kernel's dynamic-LDS limit to lds (done when a plan is set up on
// a device, outside any graph capture).
hipError_t prepare_mix_lds(int algo, size_t lds);
hipError_t launch_mix_lds(int algo, const SparseDev *codes, const LdsItem *items, const int *frames, int ncodes,
                          int groups, size_t lds, const float *llr, uint8_t *bits, int32_t *iters,
                          const int64_t *qstart, const int32_t *perm, const int64_t *offset, unsigned int *counter,
                          int max_iter, const Params &p, hipStream_t s);
// counter[c] = the length of code c's queue where frames[c] > 0, else 0: the
// streamed kernel's counters when the LDS-staged kernel takes those codes.
hipError_t launch_mix_exhaust(const int *frames, const int64_t *qstart, int ncodes, unsigned int *counter,
                              hipStream_t s);
// Persistent launch over frames 0 .. nf-1 (counter: 4 bytes, reset by the call).
hipError_t launch_sparse_lds(int algo, const SparseDev &g, const float *llr, uint8_t *bits, int32_t *iters,
                             int64_t nf, int max_iter, const Params &p, unsigned int *counter, int device,
                             hipStream_t s);
hipError_t launch_fill_i32(int *p, int n, int value, hipStream_t s);
// *pos (8 bytes, reset by the call) = flat index of the first NaN / +-Inf
// among x[0 .. n), or all ones if there is none.
hipError_t launch_nonfinite_scan(const float *x, int64_t n, unsigned long long *pos, hipStream_t s);

// ---- QC streamed kernels (any base matrix, any mix of codes) --------------
// Base structure of one QC code in sweep order (block-row major, block-column
// ascending), device pointers.  A device array of these describes the codes
// of one launch; the kernels read it with scalar loads.
struct StreamCode {
    int Z, mb, nb, E, dcmax, pad0;
    int64_t N;            // nb * Z
    const int *rstart;    // [mb+1] first edge of each block-row
    // [E] one 16-byte record per edge: x = block-column | last << 29 |
    // first << 30 (last: the column's last visit of the sweep; first: the
    // column's first block-row), y = shift, z = latest-check edge (the
    // cyclically previous block-row of the column), w = its shift | its
    // block-row << 16
    const int4 *erec;
    const int *elast;     // [nb] last edge of each block-column
    const int *er;        // [E] block-row of the edge
    const int *esh;       // [E] shift of the edge
};

// Device workspace of one frame in flight (bytes, 256-aligned).
__host__ __device__ inline int64_t stream_slot_bytes(int algo, int64_t N, int E, int mb, int Z) {
    const bool belief = algo == kCBP || algo == kCBPNMS;
    int64_t b = 4 * ((algo == kFBPNMS ? 2 : 1) * N + (int64_t)E * Z);
    b = (b + 7) & ~(int64_t)7;
    if (belief) b += 8LL * mb * Z;
    b += N;
    return (b + 255) & ~(int64_t)255;
}

// Geometry of one streamed launch.  Every workgroup has `lanes` threads, a
// multiple of each code's Z, and holds lanes / Z frames of one code at a time.
struct StreamLaunch {
    const StreamCode *codes;  // device [ncodes]
    int ncodes;
    int lanes;
    int dcmax;                // largest block-row degree over the codes
    int max_slots;            // lanes / smallest Z
    int groups;
    int64_t group_bytes;      // workspace per workgroup
};
size_t stream_lds_bytes(int algo, int lanes, int dcmax, int max_slots, bool dbg = false);
// Workgroups of the streamed kernel that fit on one CU (0 if none).
int stream_groups_per_cu(int algo, int lanes, size_t lds);
// Frames: queue q of code c holds perm[qstart[c] + q] (perm == NULL: frame
// qstart[c] + q; qstart == NULL: one code, frames [0, batch)); frame f's LLRs
// and decisions start at offset[f] (NULL: f * N).  counter[ncodes] must be 0.
hipError_t launch_qc_stream(int algo, const StreamLaunch &L, const float *llr, uint8_t *bits,
                            int32_t *iters, int64_t batch, const int64_t *qstart,
                            const int32_t *perm, const int64_t *offset, unsigned int *counter,
                            int max_iter, const Params &p, const Dump &d, void *ws, hipStream_t s);
// Groups the frames of a mixed batch by code: writes qstart[ncodes+1],
// perm[batch], zeroes counter[ncodes]; frames with a code index outside
// [0, ncodes) or LLRs outside [0, llr_elems) get iters = -1 and no queue slot.
constexpr int kMaxMixCodes = 256;
hipError_t launch_mix_prepare(const int32_t *frame_code, const int64_t *offset, int64_t batch,
                              int64_t llr_elems, const StreamCode *codes, int ncodes,
                              int64_t *qstart, int32_t *perm, unsigned int *counter,
                              int32_t *iters, hipStream_t s);

// ---- unrolled differentiable CBP (one QC code, fixed sweeps) --------------
// Device workspace of one frame (state, T checkpoints, adjoints, tape).
int64_t unrolled_frame_bytes(const StreamCode &c, int T);
size_t unrolled_lds_bytes(const StreamCode &c, int lanes, bool backward);
// True if both kernels can run a workgroup of `lanes` threads on a CU.
bool unrolled_fits(const StreamCode &c, int lanes);
// Forward (soft output, checkpoints in ws) or backward (gradients; reads the
// checkpoints the forward pass left in the same ws).  gpart: [groups][T][NB][2].
hipError_t launch_unrolled(bool backward, const StreamCode &host_code, const StreamCode *dev_code, int lanes,
                           int groups, const float *llr, int64_t batch, int T, const float *w,
                           const float *beta, float *out, const float *gout, float *gllr, float *gpart,
                           float *gw, float *gb, const Params &p, void *ws, hipStream_t s);

// ---- QC register-resident kernels (compiled base patterns) ----------------
// Number of compiled base patterns and the pattern table for matching.
int qc_reg_count();
// Fills mb, nb, Z and a pointer to the mb*nb 0/1 pattern of entry k.
void qc_reg_entry(int k, int *mb, int *nb, int *Z, const uint8_t **pattern);
// Host shift table of entry k for a base matrix (mb*nb, -1 = zero block):
// writes 2*E ints to out (E = edges of the base pattern), returns their count.
int qc_reg_shift_table(int k, const int *shifts, int *out);
// Launch entry k.  sht: device copy of the entry's shift table.
hipError_t launch_qc_reg(int k, int algo, const int *sht, const float *llr, uint8_t *bits,
                         int32_t *iters, int64_t batch, int max_iter, const Params &p,
                         const Dump &d, int *counter, int device, hipStream_t s);

}  // namespace cbp
