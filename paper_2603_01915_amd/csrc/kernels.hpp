// Launch interface between the C ABI and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dtans {

// Rows split over lanes (nonzero-balanced layouts): row, first and last lane
// of each; `longs` lists the ones summed by a whole wavefront: those spanning
// more than kLongSplit lanes, or kLongSplitRuns when the middle lanes' pieces
// were already summed per wavefront (the dtANS kernels).
constexpr int kLongSplit = 4, kLongSplitRuns = 256;
struct SplitRows {
    const int32_t *row, *first, *last, *longs;
    int64_t n, n_long;
};

// Device view of one encoded matrix (all pointers are device pointers).
struct DevMat {
    const uint64_t *tab;     // K table entries (see dtans_core.hpp)
    const void *tabval;      // K values (float or double)
    const int32_t *row_ptr;  // m + 1
    const uint64_t *woff, *doff, *voff;  // per-wave word / escape offsets
    const uint32_t *words;
    const uint32_t *escd;
    const void *escv;        // raw escaped values (float or double)
    const int32_t *lane_row; // layout NNZ: index in nzr of the row of each lane's first nonzero
    SplitRows split;         // layout NNZ
    const int2 *nzr;         // layout NNZ: {row, end} of every nonempty row, then {m, nnz}
    const int32_t *empty_rows;  // layout NNZ: the rows without nonzeros
    int64_t m, n, nnz, num_lanes, num_waves;
    int64_t n_nzr, n_empty;    // layout NNZ: nonempty rows (nzr has n_nzr + 1 entries), empty rows
    int32_t lane_nnz, layout;  // layout: 1 row per lane, 2 nonzeros per lane
    int32_t base_direct;       // 1: table metadata holds bases, not bases - 1
    int32_t no_escape;         // 1: neither table holds the escape symbol
    uint32_t first_mode;       // first delta of a row: 0 its column, 1 relative to the row
    int32_t esc_in_stream;     // 1: escaped symbols sit in the word stream (else escd / escv)
    // layout ROW with rows sorted within windows (else null): the original
    // row of every encoded row, and the original matrix's row pointers
    const int32_t *row_perm;
    const int32_t *orig_row_ptr;
};

struct Launch {
    int waves_per_wg;   // 1..16
    int grid;           // number of workgroups (direct-read kernels)
    int ring = 0;       // 1: SpMV/SpMM read their streams through an LDS ring
    int ring_waves_per_wg = 16;  // ring kernels: wavefronts per workgroup
    int num_cus = 256;  // compute units of the device
    int wg_per_cu = 0;  // ring kernels: resident workgroups per CU (0: as many as fit)
    int fixed_shape = 0;  // 1: waves_per_wg / grid as given; 0: the direct-read kernels pick
                          // the workgroup size that keeps the most waves resident
};

// Columns of X/Y one SpMM launch takes at most (wider products run in
// column passes that reuse the same scratch, in stream order).
constexpr int kMaxPassCols = 32;
// Device scratch launch_spmm needs for k columns: layout NNZ keeps a head and
// a tail partial sum (double) per lane and column of a pass; 0 for layout ROW.
size_t spmm_scratch_bytes(const DevMat &a, int k);
// Size of the library-owned scratch array (one per device, kept until the
// process ends) that dtans_spmm_noalloc uses instead of the handle's scratch.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
// Device address of the current device's copy of that array (looked up once
// per device, then cached); never the array's host-side name.
hipError_t static_scratch(void **ptr);
// y = alpha*A*x + beta*y; k columns of X/Y (k = 1: SpMV); partial: device
// scratch of at least spmm_scratch_bytes(a, k) bytes.
hipError_t launch_spmm(const DevMat &a, bool f64, int k, const void *X, int64_t ldx, void *Y,
                       int64_t ldy, double alpha, double beta, double *partial, Launch L,
                       hipStream_t st);
// dX = alpha*A^T*dY + beta*dX via decode-and-scatter.  When an n x c block
// of dX fits in LDS (c >= 1) and `work` holds spmm_t_work_bytes, each CU
// scatters into its own block and the blocks are summed; otherwise global
// atomic adds.
size_t spmm_t_work_bytes(const DevMat &a, bool f64, int num_cus);
hipError_t launch_spmm_t(const DevMat &a, bool f64, int k, const void *dY, int64_t lddy, void *dX,
                         int64_t lddx, double alpha, double beta, Launch L, void *work,
                         size_t work_bytes, hipStream_t st);
// decode to CSR (col / raw value bits); row_ptr copied by the caller
hipError_t launch_decode(const DevMat &a, bool f64, int32_t *col, void *vals, Launch L,
                         hipStream_t st);

// read `bytes` (multiple of 16) of buf so that later launches find nothing of
// theirs in L2 or the last-level cache; sink: one writable 32-bit word
hipError_t launch_flush(const void *buf, int64_t bytes, uint32_t *sink, hipStream_t st);

// many matrices (same dtype, layout ROW) in one persistent launch
struct BatchTask {  // a contiguous run of waves of one matrix for one workgroup
    int32_t mat;
    int32_t first_wave;
    int32_t num_waves;
    int32_t pad;
};
constexpr int kMaxBatch = 128;
struct BatchDev {
    const DevMat *mats;      // device array of matrix views
    const BatchTask *tasks;  // device array, grouped per workgroup
    const int32_t *wg_task;  // device, grid + 1 offsets into tasks
    void *const *ptrs;       // device table: x, y pointer of each matrix
};
// x / y device pointers of one call, passed by value with a launch
struct BatchPtrs {
    const void *xs[kMaxBatch];
    void *ys[kMaxBatch];
};
// Rewrites the pointer table on `st` and launches; calls on one batch must
// stay on one stream (the table is shared by its launches).
hipError_t launch_batch(const BatchDev &b, const BatchPtrs &ptrs, int count, bool f64, double alpha,
                        double beta, Launch L, hipStream_t st);
// k right-hand sides per matrix (X_i n_i x k, Y_i m_i x k, leading dimension
// k); aligned: every X_i and Y_i starts 16-byte aligned and k * sizeof(value)
// is a multiple of 16 (lane groups read 16-byte pieces of the rows of X)
hipError_t launch_batch_spmm(const BatchDev &b, const BatchPtrs &ptrs, int count, bool f64, int k,
                             bool aligned, double alpha, double beta, Launch L, hipStream_t st);

// plain CSR baseline.  variant 1: G lanes per row; variant 2: lane_nnz
// nonzeros per lane with partials + fix-up (lane_row, split_* as for DevMat).
// variant 3: CSR-stream row blocks (blk: first row of each block, nblk + 1
// entries) for single-vector products; other k fall back to variant 1.
struct CsrDev {
    const int32_t *row_ptr, *col;
    const void *val;
    const int32_t *lane_row;
    SplitRows split;
    const int32_t *blk;
    int64_t m, n, nnz, num_lanes, nblk;
    int32_t variant, group, lane_nnz;
};
hipError_t launch_csr(const CsrDev &c, bool f64, int k, const void *X, int64_t ldx, void *Y,
                      int64_t ldy, double alpha, double beta, double *partial, int num_cus,
                      hipStream_t st);

}  // namespace dtans
