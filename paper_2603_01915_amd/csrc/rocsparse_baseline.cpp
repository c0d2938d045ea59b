// The vendor library's CSR products (rocSPARSE generic SpMV / SpMM) on the
// same GPU, as context for the plain HIP CSR kernels and the dtANS kernels:
// the uncompressed comparison format of Sec. V run by the platform's own
// sparse library.  Not part of the method: only bench.py times it.
//
// SpMV uses the adaptive CSR algorithm (the library's fastest for general
// sparsity, with a preprocessing step done once at creation); SpMM uses the
// library's default CSR algorithm with row-major X and Y.  The library's
// work buffer for SpMM is sized on the first call with a given k (that call
// allocates and waits for the device); later calls allocate nothing.
#include <hip/hip_runtime.h>
#include <rocsparse/rocsparse.h>

#include <string>

#include "dtans.h"

// rocsparse_spmv is marked deprecated in favour of a descriptor-based v2 call
// with the same algorithms; the generic call is kept for its simplicity
#pragma clang diagnostic ignored "-Wdeprecated-declarations"

namespace dtans {
dtans_status set_error(dtans_status s, const std::string &msg);  // capi.cpp
}

struct dtans_rocsparse {
    rocsparse_handle h = nullptr;
    rocsparse_spmat_descr A = nullptr;
    void *rp = nullptr, *ci = nullptr, *val = nullptr;
    void *xbuf = nullptr, *ybuf = nullptr;  // preprocessing vectors
    void *spmv_buf = nullptr, *spmm_buf = nullptr;
    size_t spmm_bytes = 0;
    int32_t spmm_k = 0;
    int64_t m = 0, n = 0, nnz = 0;
    bool f64 = true;
};

namespace {

dtans_status set_err(dtans_status s, const std::string &msg) { return dtans::set_error(s, msg); }

dtans_status rs_err(rocsparse_status s, const char *what) {
    return set_err(DTANS_EHIP, std::string(what) + ": rocSPARSE status " + std::to_string((int)s));
}
dtans_status hip_fail(hipError_t e, const char *what) {
    return set_err(DTANS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

void release(dtans_rocsparse *r) {
    if (r->A) rocsparse_destroy_spmat_descr(r->A);
    if (r->h) rocsparse_destroy_handle(r->h);
    for (void *p : {r->rp, r->ci, r->val, r->xbuf, r->ybuf, r->spmv_buf, r->spmm_buf})
        if (p) (void)hipFree(p);
    delete r;
}

}  // namespace

extern "C" {

dtans_status dtans_rocsparse_create(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr,
                                    const int32_t *col_idx, const void *vals, dtans_dtype dtype,
                                    dtans_rocsparse **out) {
    if (!out || m < 0 || n < 0 || nnz < 0 || !row_ptr || (nnz > 0 && (!col_idx || !vals)))
        return set_err(DTANS_EINVAL, "dtans_rocsparse_create: bad arguments");
    if (dtype != DTANS_F32 && dtype != DTANS_F64) return set_err(DTANS_EINVAL, "dtype must be F32 or F64");
    *out = nullptr;
    dtans_rocsparse *r = new dtans_rocsparse;
    r->m = m;
    r->n = n;
    r->nnz = nnz;
    r->f64 = dtype == DTANS_F64;
    const size_t vb = r->f64 ? 8 : 4;
    const rocsparse_datatype dt = r->f64 ? rocsparse_datatype_f64_r : rocsparse_datatype_f32_r;
    hipError_t e;
    if ((e = hipMalloc(&r->rp, 4 * (size_t)(m + 1))) != hipSuccess ||
        (e = hipMalloc(&r->ci, 4 * (size_t)(nnz > 0 ? nnz : 1))) != hipSuccess ||
        (e = hipMalloc(&r->val, vb * (size_t)(nnz > 0 ? nnz : 1))) != hipSuccess ||
        (e = hipMalloc(&r->xbuf, vb * (size_t)(n > 0 ? n : 1))) != hipSuccess ||
        (e = hipMalloc(&r->ybuf, vb * (size_t)(m > 0 ? m : 1))) != hipSuccess ||
        (e = hipMemcpy(r->rp, row_ptr, 4 * (size_t)(m + 1), hipMemcpyHostToDevice)) != hipSuccess ||
        (nnz > 0 && (e = hipMemcpy(r->ci, col_idx, 4 * (size_t)nnz, hipMemcpyHostToDevice)) != hipSuccess) ||
        (nnz > 0 && (e = hipMemcpy(r->val, vals, vb * (size_t)nnz, hipMemcpyHostToDevice)) != hipSuccess) ||
        (e = hipMemset(r->xbuf, 0, vb * (size_t)(n > 0 ? n : 1))) != hipSuccess) {
        release(r);
        return hip_fail(e, "dtans_rocsparse_create");
    }
    rocsparse_status s;
    if ((s = rocsparse_create_handle(&r->h)) != rocsparse_status_success ||
        (s = rocsparse_create_csr_descr(&r->A, m, n, nnz, r->rp, r->ci, r->val, rocsparse_indextype_i32,
                                        rocsparse_indextype_i32, rocsparse_index_base_zero, dt)) !=
            rocsparse_status_success) {
        release(r);
        return rs_err(s, "dtans_rocsparse_create");
    }
    // SpMV: buffer and preprocessing of the adaptive algorithm, once
    rocsparse_dnvec_descr x = nullptr, y = nullptr;
    rocsparse_create_dnvec_descr(&x, n, r->xbuf, dt);
    rocsparse_create_dnvec_descr(&y, m, r->ybuf, dt);
    const double one = 1.0, zero = 0.0;
    const float onef = 1.0f, zerof = 0.0f;
    const void *al = r->f64 ? (const void *)&one : (const void *)&onef;
    const void *be = r->f64 ? (const void *)&zero : (const void *)&zerof;
    size_t bytes = 0;
    s = rocsparse_spmv(r->h, rocsparse_operation_none, al, r->A, x, be, y, dt, rocsparse_spmv_alg_csr_adaptive,
                       rocsparse_spmv_stage_buffer_size, &bytes, nullptr);
    if (s == rocsparse_status_success && (e = hipMalloc(&r->spmv_buf, bytes > 0 ? bytes : 1)) != hipSuccess) {
        rocsparse_destroy_dnvec_descr(x);
        rocsparse_destroy_dnvec_descr(y);
        release(r);
        return hip_fail(e, "dtans_rocsparse_create buffer");
    }
    if (s == rocsparse_status_success)
        s = rocsparse_spmv(r->h, rocsparse_operation_none, al, r->A, x, be, y, dt,
                           rocsparse_spmv_alg_csr_adaptive, rocsparse_spmv_stage_preprocess, &bytes, r->spmv_buf);
    rocsparse_destroy_dnvec_descr(x);
    rocsparse_destroy_dnvec_descr(y);
    if (s != rocsparse_status_success) {
        release(r);
        return rs_err(s, "dtans_rocsparse_create preprocess");
    }
    if ((e = hipDeviceSynchronize()) != hipSuccess) {
        release(r);
        return hip_fail(e, "dtans_rocsparse_create");
    }
    *out = r;
    return DTANS_OK;
}

dtans_status dtans_rocsparse_spmv(dtans_rocsparse *r, const void *x, void *y, double alpha, double beta,
                                  void *stream) {
    if (!r || (r->m > 0 && !y) || (r->n > 0 && !x)) return set_err(DTANS_EINVAL, "dtans_rocsparse_spmv: null argument");
    const rocsparse_datatype dt = r->f64 ? rocsparse_datatype_f64_r : rocsparse_datatype_f32_r;
    rocsparse_set_stream(r->h, (hipStream_t)stream);
    rocsparse_dnvec_descr xd = nullptr, yd = nullptr;
    rocsparse_create_dnvec_descr(&xd, r->n, const_cast<void *>(x), dt);
    rocsparse_create_dnvec_descr(&yd, r->m, y, dt);
    const float af = (float)alpha, bf = (float)beta;
    const void *al = r->f64 ? (const void *)&alpha : (const void *)&af;
    const void *be = r->f64 ? (const void *)&beta : (const void *)&bf;
    size_t bytes = 0;
    rocsparse_status s = rocsparse_spmv(r->h, rocsparse_operation_none, al, r->A, xd, be, yd, dt,
                                        rocsparse_spmv_alg_csr_adaptive, rocsparse_spmv_stage_compute, &bytes,
                                        r->spmv_buf);
    rocsparse_destroy_dnvec_descr(xd);
    rocsparse_destroy_dnvec_descr(yd);
    return s == rocsparse_status_success ? DTANS_OK : rs_err(s, "dtans_rocsparse_spmv");
}

dtans_status dtans_rocsparse_spmm(dtans_rocsparse *r, int32_t k, const void *X, int64_t ldx, void *Y,
                                  int64_t ldy, double alpha, double beta, void *stream) {
    if (!r || k < 1 || ldx < k || ldy < k || (r->m > 0 && !Y) || (r->n > 0 && !X))
        return set_err(DTANS_EINVAL, "dtans_rocsparse_spmm: bad arguments");
    const rocsparse_datatype dt = r->f64 ? rocsparse_datatype_f64_r : rocsparse_datatype_f32_r;
    rocsparse_set_stream(r->h, (hipStream_t)stream);
    rocsparse_dnmat_descr Xd = nullptr, Yd = nullptr;
    rocsparse_create_dnmat_descr(&Xd, r->n, k, ldx, const_cast<void *>(X), dt, rocsparse_order_row);
    rocsparse_create_dnmat_descr(&Yd, r->m, k, ldy, Y, dt, rocsparse_order_row);
    const float af = (float)alpha, bf = (float)beta;
    const void *al = r->f64 ? (const void *)&alpha : (const void *)&af;
    const void *be = r->f64 ? (const void *)&beta : (const void *)&bf;
    rocsparse_status s = rocsparse_status_success;
    if (k != r->spmm_k) {
        size_t bytes = 0;
        s = rocsparse_spmm(r->h, rocsparse_operation_none, rocsparse_operation_none, al, r->A, Xd, be, Yd, dt,
                           rocsparse_spmm_alg_default, rocsparse_spmm_stage_buffer_size, &bytes, nullptr);
        if (s == rocsparse_status_success && bytes > r->spmm_bytes) {
            hipError_t e = hipDeviceSynchronize();
            if (e == hipSuccess && r->spmm_buf) e = hipFree(r->spmm_buf);
            r->spmm_buf = nullptr;
            if (e == hipSuccess) e = hipMalloc(&r->spmm_buf, bytes);
            if (e != hipSuccess) {
                rocsparse_destroy_dnmat_descr(Xd);
                rocsparse_destroy_dnmat_descr(Yd);
                r->spmm_bytes = 0;
                return hip_fail(e, "dtans_rocsparse_spmm buffer");
            }
            r->spmm_bytes = bytes;
        }
        if (s == rocsparse_status_success)
            s = rocsparse_spmm(r->h, rocsparse_operation_none, rocsparse_operation_none, al, r->A, Xd, be, Yd, dt,
                               rocsparse_spmm_alg_default, rocsparse_spmm_stage_preprocess, &bytes, r->spmm_buf);
        if (s == rocsparse_status_success) r->spmm_k = k;
    }
    size_t bytes = r->spmm_bytes;
    if (s == rocsparse_status_success)
        s = rocsparse_spmm(r->h, rocsparse_operation_none, rocsparse_operation_none, al, r->A, Xd, be, Yd, dt,
                           rocsparse_spmm_alg_default, rocsparse_spmm_stage_compute, &bytes, r->spmm_buf);
    rocsparse_destroy_dnmat_descr(Xd);
    rocsparse_destroy_dnmat_descr(Yd);
    return s == rocsparse_status_success ? DTANS_OK : rs_err(s, "dtans_rocsparse_spmm");
}

void dtans_rocsparse_destroy(dtans_rocsparse *r) {
    if (r) release(r);
}

}  // extern "C"
