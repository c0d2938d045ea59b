/*
 * dtans.h - C ABI of libdtans: sparse matrix-vector multiplication fused with
 * dtANS entropy decoding on AMD Instinct MI355X (gfx950).
 *
 * The method is the one of "Fast Entropy Decoding for Sparse MVM on GPUs"
 * (Schaetzle, Pegolotti, Pueschel, 2026): a CSR matrix is entropy coded once
 * on the host (column deltas per row, Sec. IV-A; interleaved delta/value
 * symbols and wave-interleaved 32-bit word streams, Sec. IV-B; coding tables
 * of K = 4096 slots with multiplicity cap M = 256, Sec. IV-C; two-pass
 * encoder, Sec. IV-E), and every multiplication decodes the streams on the
 * fly while multiplying (Sec. II-B, Alg. 3), so the uncompressed matrix never
 * exists in device memory.
 *
 * Conventions for every entry point:
 *   - Return value: DTANS_OK (0) or a positive error code; a thread-local
 *     message for the last error is available from dtans_last_error().
 *   - "host" pointers point to CPU memory and are only read during the call
 *     (borrowed).  "device" pointers are HIP device allocations owned by the
 *     caller (e.g. torch tensor data_ptr()); the library never frees them.
 *   - Product calls (dtans_spmv, dtans_spmm, dtans_spmm_t, dtans_spmv_sym,
 *     dtans_decode_csr, dtans_batch_spmv, dtans_batch_spmm, dtans_csr_spmv,
 *     dtans_csr_spmm)
 *     are asynchronous on the caller's HIP stream (NULL = the null stream),
 *     allocate nothing and never synchronize.  They need the matrix on the
 *     current device with scratch for their number of right-hand sides:
 *     dtans_to_device uploads it and reserves for one right-hand side,
 *     dtans_reserve for more; otherwise a product call returns DTANS_EINVAL
 *     without launching.  Only dtans_to_device, dtans_reserve, the encoders,
 *     dtans_batch_create, dtans_csr_create and dtans_autotune allocate device
 *     memory or wait for the device.  Arguments are validated on the host
 *     before anything is launched; a launch failure returns DTANS_EHIP.
 *   - Vectors have the matrix's value type (float for DTANS_F32, double for
 *     DTANS_F64); alpha/beta are passed as double and rounded to that type.
 *     beta == 0 means the output is not read (it may hold NaN).
 *   - Indices are 32-bit (Sec. V: int32 CSR); nnz, rows and columns must be
 *     below 2^31.
 *   - A handle is used by one thread at a time; calls on different handles
 *     may run concurrently.  A handle's device scratch (partial sums of the
 *     nonzero layout, the transposed product's copies of dX) is shared by its
 *     calls, so calls on one handle that may use it are ordered on one stream.
 */
#ifndef DTANS_H
#define DTANS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dtans_status;
enum {
    DTANS_OK = 0,
    DTANS_EINVAL = 1,      /* bad argument (null pointer, size, dtype, option) */
    DTANS_EUNSORTED = 2,   /* columns not ascending within a row */
    DTANS_ERANGE = 3,      /* nnz, row or column count or index >= 2^31 */
    DTANS_ENOMEM = 4,      /* host or device allocation failed */
    DTANS_EHIP = 5,        /* HIP runtime error (message has the HIP error) */
    DTANS_ECORRUPT = 6,    /* container fails its checksum or consistency check */
    DTANS_EUNSUPPORTED = 7,/* valid request the library does not implement */
    DTANS_EIO = 8          /* file could not be read or written */
};

typedef enum { DTANS_F32 = 1, DTANS_F64 = 2 } dtans_dtype;

/* Stream layouts.  ROW: lane = one row, wave = 64 consecutive rows (the
 * paper's slice-to-warp mapping, Sec. II-B/IV-B, with 64-lane wavefronts).
 * NNZ: lane = lane_nnz consecutive nonzeros in row-major order, so every lane
 * does the same work whatever the row lengths; rows that cross lanes are
 * summed by a fix-up pass.  AUTO lets the encoder choose. */
typedef enum { DTANS_LAYOUT_AUTO = 0, DTANS_LAYOUT_ROW = 1, DTANS_LAYOUT_NNZ = 2 } dtans_layout;

/* How SpMV and SpMM read their word streams (dtans_encode_opts). */
enum { DTANS_STAGE_AUTO = 0, DTANS_STAGE_DIRECT = 1, DTANS_STAGE_RING = 2 };

typedef struct {
    int32_t layout;        /* dtans_layout */
    int32_t lane_nnz;      /* NNZ layout: nonzeros per lane, multiple of 4; 0 = auto */
    int32_t waves_per_wg;  /* kernel launch: wavefronts per workgroup (1..16); 0 = auto */
    int32_t wg_per_cu;     /* kernel launch: persistent workgroups per CU; 0 = auto */
    int32_t sort_rows;     /* 1: sort columns within rows first (values follow) */
    int32_t stream_stage;  /* SpMV/SpMM: 0 = auto (direct), 1 = read stream words
                              directly from device memory, 2 = stage them through an
                              LDS ring (SpMM then takes 2 FP64 / 4 FP32 columns per pass) */
    int32_t max_mult;      /* largest number of slots per symbol, 1..256 (Sec. IV-C's
                              cap M = 256); 0 = 255, which keeps every base within a
                              byte so that the kernels use it without a correction */
    int32_t first_delta_column; /* 1: the first delta of a row is its column (Sec. IV-A);
                              0: column - row + 2^29 (mod 2^32), which banded and
                              stencil matrices keep within the table */
    int32_t escape_in_stream; /* where escaped symbols' raw bits go (Sec. IV-F): 0 = a
                              separate region per wave; 1 = inside the word stream,
                              read right after the decoding step that meets them (every
                              step's word positions then depend on its escape count;
                              SpMV/SpMM read such streams directly, never through the
                              LDS ring; dtans_encode_csr only, the device encoders
                              return DTANS_EUNSUPPORTED) */
    int32_t sort_window;   /* ROW layout: 0 = rows in CSR order; a multiple of 64 = a
                              SELL-C-sigma base (Sec. VII's other starting formats;
                              Kreutzer et al. 2014): within each window of that many
                              rows, rows are encoded by descending length (ties in
                              order), so a wave's 64 lanes get rows of similar
                              length; the order is stored and every product and
                              dtans_decode_csr work in the original row order.
                              dtans_encode_csr and dtans_encode_csr_gpu (the rows
                              are permuted on the host first); dtans_encode_csr_device
                              and dtans_spmv_sym return DTANS_EUNSUPPORTED */
    int32_t reserved0;
    uint64_t perm_seed;    /* seed of the random slot permutation (Sec. IV-F) */
} dtans_encode_opts;

/* Sizes and statistics of an encoded matrix. */
typedef struct {
    int64_t m, n, nnz;
    int32_t dtype, layout, lane_nnz, waves_per_wg;
    int64_t num_lanes, num_waves;
    int64_t words, esc_delta, esc_value;   /* counts of 32-bit words / raw symbols */
    int64_t table_bytes;                   /* device coding tables (K slots x 16 or 12 B) */
    int64_t stream_bytes;                  /* words + escapes */
    int64_t index_bytes;                   /* row pointers, per-wave offsets, lane metadata */
    int64_t total_bytes;                   /* everything one multiplication reads besides x, y */
    int64_t csr_bytes, coo_bytes, sell_bytes; /* same matrix in CSR / COO / SELL-64 */
    int32_t delta_symbols, value_symbols;  /* table symbols per alphabet (escape excluded) */
    double delta_entropy, value_entropy;   /* H of the delta / value distribution, bits (Eq. 1) */
    double delta_cross_entropy, value_cross_entropy; /* H(P, P') of the fitted tables (Eq. 2) */
    double bits_per_nnz;                   /* 8 * stream_bytes / nnz */
    int32_t stream_stage;                  /* SpMV word reads: 1 direct, 2 LDS ring */
    int32_t direct_table;                  /* 1: every base <= 255, used without correction */
    int32_t first_delta_column;            /* 1: first deltas are columns (the paper's form) */
    int32_t escape_in_stream;              /* 1: escapes inside the word stream */
    int32_t sort_window;                   /* rows sorted within windows of this many (0: none) */
    int32_t reserved;
} dtans_info;

typedef struct dtans_matrix dtans_matrix; /* owns its host container and device copy */
typedef struct dtans_batch dtans_batch;   /* references matrices, does not own them */

/* Library version string. */
const char *dtans_version(void);

/* Message for the last non-OK status returned on this thread. */
const char *dtans_last_error(void);

/* Fill *opts with defaults (layout AUTO, everything else auto, seed 1). */
void dtans_default_opts(dtans_encode_opts *opts);

/*
 * Encode a CSR matrix (Sec. II-A, IV-A..F).  Host pointers: row_ptr (m+1),
 * col_idx (nnz), vals (nnz floats or doubles).  Columns ascending within each
 * row (duplicates allowed) unless opts->sort_rows.  opts may be NULL.
 * On success *out owns a new handle (release with dtans_destroy).
 */
dtans_status dtans_encode_csr(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr,
                              const int32_t *col_idx, const void *vals, dtans_dtype dtype,
                              const dtans_encode_opts *opts, dtans_matrix **out);

/*
 * Same arguments, result and errors as dtans_encode_csr, and a container
 * byte-identical to its: the per-stream base and digit passes (Sec. IV-E) and
 * the interleave of each wave's streams in the decoder's load order
 * (Sec. IV-B) run on the current GPU, on `stream` (a hipStream_t, NULL = the
 * null stream); the alphabet fit, tables and escape regions stay on the host.
 * All arrays are host pointers; the call allocates its own device buffers
 * (about 8 bytes per nonzero plus the words), frees them before returning and
 * blocks until the words are back on the host.  DTANS_EHIP / DTANS_ENOMEM for
 * runtime or allocation failures; DTANS_ECORRUPT if the device's word counts
 * disagree (never expected).
 */
dtans_status dtans_encode_csr_gpu(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr,
                                  const int32_t *col_idx, const void *vals, dtans_dtype dtype,
                                  const dtans_encode_opts *opts, void *stream, dtans_matrix **out);

/*
 * As dtans_encode_csr_gpu, for CSR arrays already in device memory (e.g. a
 * weight re-encoded after pruning): row_ptr, col_idx and vals are DEVICE
 * pointers, read on `stream` (they must stay valid and unchanged until the
 * call returns).  row_ptr is copied to the host (the container keeps it);
 * columns are checked on the device with the same error classes and rows as
 * dtans_encode_csr (DTANS_ERANGE / DTANS_EUNSORTED for the first failing row).
 * opts->sort_rows is not supported here (DTANS_EUNSUPPORTED).  The container
 * is byte-identical to dtans_encode_csr's on the same arrays.
 */
dtans_status dtans_encode_csr_device(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr,
                                     const int32_t *col_idx, const void *vals, dtans_dtype dtype,
                                     const dtans_encode_opts *opts, void *stream, dtans_matrix **out);

/* Write / read the container file (Sec. II-A: the encoded matrix can be kept
 * for repeated decoding).  dtans_load checks the checksum and structure and
 * verifies by a full host decode before returning a handle. */
dtans_status dtans_save(const dtans_matrix *mat, const char *path);
dtans_status dtans_load(const char *path, dtans_matrix **out);

/* Copy the encoded matrix to the current HIP device and reserve the scratch
 * of products with one right-hand side (idempotent).  The copies are
 * enqueued on `stream` and the call waits for them, so that products on any
 * stream of this device find the matrix in place.  DTANS_EINVAL when the
 * matrix already lives on another device. */
dtans_status dtans_to_device(dtans_matrix *mat, void *stream);

/* Upload the matrix if needed (as dtans_to_device) and grow its device
 * scratch so that dtans_spmm and dtans_spmm_t with up to k right-hand sides
 * need no allocation (the nonzero-balanced layout keeps two partial sums per
 * lane and column of a pass of at most 32 columns; the transposed product
 * keeps per-CU copies of a block of dX).  Growing waits for the device
 * before the smaller buffer is freed.  k >= 1; DTANS_ENOMEM / DTANS_EHIP on
 * allocation failure. */
dtans_status dtans_reserve(dtans_matrix *mat, int32_t k, void *stream);

/* Sizes, entropies and launch configuration. */
dtans_status dtans_matrix_info(const dtans_matrix *mat, dtans_info *out);

/* Change the launch configuration of an encoded matrix (0 keeps the value). */
dtans_status dtans_set_launch(dtans_matrix *mat, int32_t waves_per_wg, int32_t wg_per_cu,
                              int32_t stream_stage);

/*
 * y = alpha * A x + beta * y (Sec. III-A; the paper's y = Ax is alpha=1,
 * beta=0).  Device pointers: x (n values), y (m values).
 */
dtans_status dtans_spmv(dtans_matrix *mat, const void *x, void *y, double alpha, double beta,
                        void *stream);

/*
 * Multi-vector product Y = alpha * A X + beta * Y (Sec. IV-B: the decoded
 * nonzeros are used for all right-hand sides while decoding).  X is n x k
 * row-major with leading dimension ldx >= k; Y is m x k row-major with
 * ldy >= k (device pointers).  Every stream is decoded once per column chunk:
 * chunks of 32 / 16 / 8 FP32 or 16 / 8 / 4 FP64 columns, whose rows of X lane
 * groups read as 16-byte pieces, when X is 16-byte aligned, ldx * sizeof(value)
 * a multiple of 16 and n * ldx * sizeof(value) <= 2^32 (so k = 32 FP32 is one
 * decode); the remaining columns (or all of them otherwise) in chunks of at
 * most 16 FP32 / 8 FP64 columns read per lane.  dtans_reserve(k) sizes the
 * partial sums of rows split over lanes.
 */
dtans_status dtans_spmm(dtans_matrix *mat, int32_t k, const void *X, int64_t ldx, void *Y,
                        int64_t ldy, double alpha, double beta, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as dtans_spmm, on the same kernels, with the partial sums of rows
 * split across lanes (nonzero-balanced layout) kept in a scratch array that
 * the library itself holds, one per device (64 MiB, held from the first call
 * on a device until the process ends) instead of the handle's scratch.  The
 * call allocates nothing and never synchronizes; the matrix must be on the
 * current device (dtans_to_device), and dtans_reserve is not needed.
 * DTANS_ERANGE, before any launch, when the product needs more scratch than
 * the array holds (2 * lanes * min(k, 32) doubles; nothing for the row
 * layout).  Every call on one device shares that device's array and leaves
 * its contents behind (each call writes every partial sum it reads), so
 * calls that may overlap on one device (concurrent streams or threads)
 * race: order them on one stream.
 */
dtans_status dtans_spmm_noalloc(dtans_matrix *mat, int32_t k, const void *X, int64_t ldx, void *Y,
                                int64_t ldy, double alpha, double beta, void *stream);

/*
 * Transposed product dX = alpha * A^T dY + beta * dX by decode-and-scatter of
 * the same streams.  When n x c values of dX (c up to 8) fit in LDS beside
 * the tables, every CU scatters into its own copy with LDS atomic adds and a
 * second kernel sums the copies (the copies live in the handle's scratch);
 * otherwise the scatter uses global atomic adds.  Either way the summation
 * order is not deterministic.  dY is m x k (lddy >= k), dX is n x k
 * (lddx >= k), device pointers.
 */
dtans_status dtans_spmm_t(dtans_matrix *mat, int32_t k, const void *dY, int64_t lddy, void *dX,
                          int64_t lddx, double alpha, double beta, void *stream);

/*
 * Symmetric product from one triangle (Sec. V: symmetric matrices multiplied
 * through one half, off-diagonal entries not duplicated).  mat holds the
 * strictly upper (or strictly lower) triangle S of a symmetric n x n matrix
 * A = S + S^T + diag(d); diag holds d (n values of the matrix's dtype,
 * device pointer; NULL for a zero diagonal).  Computes
 * y = alpha * (S x + S^T x + d .* x) + beta * y on `stream`: the product on
 * S (beta applied there), the diagonal term, then the transposed product on S
 * adding into y, so the summation order of the S^T part is not deterministic.
 * x and y are n-vectors in device memory and must not overlap.  DTANS_EINVAL
 * for a non-square mat, null or aliased vectors; otherwise as dtans_spmv and
 * dtans_spmm_t.  mat must not contain diagonal entries (they would count twice).
 */
dtans_status dtans_spmv_sym(dtans_matrix *mat, const void *diag, const void *x, void *y, double alpha,
                            double beta, void *stream);

/*
 * Decode the whole matrix back to CSR on the device (verification; the
 * result is bit-identical to the encoded CSR).  Device pointers: row_ptr
 * (m+1 int32), col_idx (nnz int32), vals (nnz values).
 */
dtans_status dtans_decode_csr(dtans_matrix *mat, int32_t *row_ptr, int32_t *col_idx, void *vals,
                              void *stream);

/*
 * Many matrices (at most 128, same dtype, ROW layout, each x at most 4 GiB)
 * in one persistent launch: workgroups walk contiguous, cost-balanced runs of encoded waves and
 * restage their LDS tables only when the matrix changes.  xs[i] / ys[i] are
 * device pointers for matrix i (host array of pointers, read during the
 * call).  The batch keeps a device table of these pointers that each call
 * rewrites on its stream, so calls on one batch must not run concurrently on
 * different streams.  The batch references the matrices; they must outlive it.
 */
dtans_status dtans_batch_create(int32_t count, dtans_matrix *const *mats, dtans_batch **out);
dtans_status dtans_batch_spmv(dtans_batch *batch, const void *const *xs, void *const *ys,
                              double alpha, double beta, void *stream);
/* Y_i = alpha * A_i X_i + beta * Y_i for every matrix of the batch with k >= 1
 * right-hand sides: Xs[i] (device, n_i x k) and Ys[i] (device, m_i x k) are
 * row major with leading dimension k.  Each launch decodes every matrix once
 * for a chunk of columns: 32 / 16 / 8 FP32 or 16 / 8 / 4 FP64 columns by
 * lane groups sharing 16-byte pieces of the rows of X (when every X_i and
 * Y_i is 16-byte aligned and k * sizeof(value) is a multiple of 16), the
 * rest 4, 2 or 1 at a time (the multi-vector product of Sec. IV-B over the
 * multi-matrix launch).  Same stream rule as dtans_batch_spmv. */
dtans_status dtans_batch_spmm(dtans_batch *batch, int32_t k, const void *const *Xs, void *const *Ys,
                              double alpha, double beta, void *stream);
void dtans_batch_destroy(dtans_batch *batch);

/*
 * Plain CSR baseline on the same GPU (the uncompressed comparison format of
 * Sec. V).  dtans_csr_create copies host CSR arrays (row_ptr m+1, col_idx
 * nnz, vals nnz) to the current device and plans the launch; variant:
 * 0 = automatic (3), 1 = a group of lanes per row sized by the mean row
 * length, 2 = equal nonzeros per lane with a fix-up for rows that cross lanes,
 * 3 = CSR-stream: row blocks of at most 1024 nonzeros staged through LDS
 * (single-vector products; several right-hand sides use variant 1).
 * dtans_csr_spmv / dtans_csr_spmm compute y = alpha*A*x + beta*y and
 * Y = alpha*A*X + beta*Y with the same conventions as dtans_spmv / _spmm.
 */
typedef struct dtans_csr dtans_csr;
dtans_status dtans_csr_create(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr,
                              const int32_t *col_idx, const void *vals, dtans_dtype dtype,
                              int32_t variant, dtans_csr **out);
dtans_status dtans_csr_spmv(dtans_csr *csr, const void *x, void *y, double alpha, double beta,
                            void *stream);
dtans_status dtans_csr_spmm(dtans_csr *csr, int32_t k, const void *X, int64_t ldx, void *Y,
                            int64_t ldy, double alpha, double beta, void *stream);
/* bytes one multiplication reads besides x and y (row_ptr, col_idx, vals, plan) */
int64_t dtans_csr_bytes(const dtans_csr *csr);
void dtans_csr_destroy(dtans_csr *csr);

/*
 * The platform's own sparse library on the same CSR arrays, as context for
 * the baselines above (rocSPARSE generic API: SpMV with the adaptive CSR
 * algorithm, preprocessed once by dtans_rocsparse_create; SpMM with the
 * library's default CSR algorithm, X and Y row-major).  Same argument
 * conventions as dtans_csr_*.  dtans_rocsparse_create copies the host arrays
 * to the current device and waits for it; the first dtans_rocsparse_spmm with
 * a given k sizes the library's work buffer (it may allocate and wait), later
 * calls with that k allocate nothing.  Not part of the compressed format's
 * path; DTANS_EHIP carries rocSPARSE's status code.
 */
typedef struct dtans_rocsparse dtans_rocsparse;
dtans_status dtans_rocsparse_create(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr,
                                    const int32_t *col_idx, const void *vals, dtans_dtype dtype,
                                    dtans_rocsparse **out);
dtans_status dtans_rocsparse_spmv(dtans_rocsparse *rs, const void *x, void *y, double alpha, double beta,
                                  void *stream);
dtans_status dtans_rocsparse_spmm(dtans_rocsparse *rs, int32_t k, const void *X, int64_t ldx, void *Y,
                                  int64_t ldy, double alpha, double beta, void *stream);
void dtans_rocsparse_destroy(dtans_rocsparse *rs);

/*
 * Autotuner (encode-time parameters; no equivalent in the paper, which uses
 * one fixed launch per GPU).  Candidate options are the fields of *in left at
 * 0 / AUTO, searched over: layout {ROW, NNZ}; for NNZ, nonzeros per lane
 * around the automatic choice (multiples of 4 between 32 and 512); launch
 * shapes of the direct-read kernels (workgroups per CU up to the LDS limit,
 * waves per workgroup filling the CU's wave slots, then half and a quarter of
 * that); and the LDS-ring stream stage with 16, 8 or 4 waves per workgroup and
 * as many workgroups per CU as fit.
 * Fields set in *in are kept in every candidate.
 *
 * dtans_autotune_candidates is host-only: it writes at most `cap` candidates,
 * in the order the autotuner times them (the automatic choice first), to out
 * (host array, may be NULL when cap == 0) and returns how many there are, or
 * -1 on a bad argument (message in dtans_last_error).  Encoding candidates
 * are grouped: all launch shapes of one encoding follow each other.
 *
 * dtans_autotune encodes each candidate encoding, uploads it to the current
 * device and times y = A*x (k = 1) or Y = A*X (X n x k, ldx = k) with HIP
 * events, reading a 512 MiB buffer before every timed launch so that the
 * matrix is not served from the last-level cache.  It stops starting new
 * encodings once budget_s seconds of wall time are spent (the first is always
 * finished), writes the fastest options to *inout and the best time per
 * multiplication to *best_ms.  cache_path (may be NULL) names a text file of
 * earlier results, one line per (matrix fingerprint, dtype, k, fixed options,
 * device name): a hit returns the stored options without encoding; a new
 * result is appended (a file that cannot be written gives DTANS_EIO after
 * *inout is filled).  Needs a GPU; blocks until its work is done.
 */
int32_t dtans_autotune_candidates(int64_t m, int64_t nnz, const int32_t *row_ptr,
                                  dtans_dtype dtype, int32_t k, const dtans_encode_opts *in,
                                  dtans_encode_opts *out, int32_t cap);
dtans_status dtans_autotune(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr,
                            const int32_t *col_idx, const void *vals, dtans_dtype dtype, int32_t k,
                            double budget_s, const char *cache_path, dtans_encode_opts *inout,
                            double *best_ms);

/* Release a handle and its device memory (NULL is ignored). */
void dtans_destroy(dtans_matrix *mat);

#ifdef __cplusplus
}
#endif
#endif /* DTANS_H */
