// Internal interfaces between the C ABI (abi.cpp) and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cbp {

// kCBPNMS: CBP with the normalized min-sum check rule (cbp_decode with
// CBP_RULE_MIN_SUM).
enum Algo : int { kCBP = 0, kLBPNMS = 1, kFBPNMS = 2, kCBPNMS = 3 };

// Read of a table that no launch writes, through the constant address space:
// where the index is wave-uniform the compiler emits a scalar load (through a
// generic pointer it could not rule out aliasing with the kernel's stores and
// would issue a vector load, a full memory round trip, instead).
template <class T>
__device__ __forceinline__ T ldc(const T *p, int64_t i) {
    return ((const __attribute__((address_space(4))) T *)p)[i];
}

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
    const uint8_t *first; // [E]  1 if this is the lowest row of its column
    const int *last_edge; // [N]  edge of the highest row of each column
};

// Frame-interleaved workspace of the sparse kernels: element (index, frame)
// lives at array[index * stride + frame].
struct SparseWs {
    int64_t stride;
    float *a0, *a1, *a2, *a3, *a4;  // meaning depends on the algorithm
    uint8_t *xb;
};

size_t sparse_ws_bytes(int algo, const SparseDev &g, int64_t frames);
SparseWs sparse_ws_carve(int algo, const SparseDev &g, int64_t frames, void *base);
hipError_t launch_sparse(int algo, const SparseDev &g, const float *llr, uint8_t *bits,
                         int32_t *iters, int64_t f0, int64_t nf, int max_iter,
                         const Params &p, const SparseWs &ws, const Dump &d, hipStream_t s);
hipError_t launch_syndrome(const SparseDev &g, const uint8_t *bits, uint8_t *ok, int64_t batch,
                           hipStream_t s);
hipError_t launch_fill_i32(int *p, int n, int value, hipStream_t s);

// ---- QC streamed kernels (any base matrix) ---------------------------------
// Base structure in sweep order (block-row major, block-column ascending).
struct QcStreamDev {
    int Z, mb, nb, E, dcmax, slots;
    const int *rstart;  // [mb+1] first edge of each block-row
    const int *eb;      // [E] block-column of the edge
    const int *esh;     // [E] circulant shift of the edge
    const int *er;      // [E] block-row of the edge
    const int *ep;      // [E] latest-check edge (cyclically previous block-row of the column)
    const int *epr;     // [E] block-row of ep
    const int *epsh;    // [E] shift of ep
    const int *efirst;  // [E] 1 if the edge's block-row is the first of its column
    const int *elast;   // [nb] last edge of each block-column
    // [E] the fields the sweep reads, one 16-byte record per edge:
    //   x = eb | last << 29 | first << 30  (last: the edge is its column's
    //       last visit of the sweep; first: efirst), y = esh, z = ep,
    //   w = epsh | epr << 16
    const int4 *erec;
};
int64_t qc_stream_slot_bytes(int algo, const QcStreamDev &g);
void qc_stream_shape(const QcStreamDev &g, int *slots, int *threads, size_t *lds);
int qc_stream_groups(int algo, const QcStreamDev &g, int device);
hipError_t launch_qc_stream(int algo, const QcStreamDev &g, const float *llr, uint8_t *bits,
                            int32_t *iters, int64_t batch, int max_iter, const Params &p,
                            const Dump &d, int groups, void *ws, int *counter, hipStream_t s);

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
