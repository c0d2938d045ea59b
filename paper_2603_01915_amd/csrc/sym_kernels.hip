// The diagonal term of the symmetric product from one triangle (Sec. V: a
// symmetric matrix multiplied through one of its halves, without duplicated
// off-diagonal entries): y[i] += alpha * d[i] * x[i].  The off-diagonal
// halves use the ordinary product and the transposed product kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dtans {
namespace {

template <typename VT>
__global__ __launch_bounds__(256) void diag_axpy_kernel(const VT *__restrict__ d, const VT *__restrict__ x,
                                                        VT *__restrict__ y, int64_t n, double alpha) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (VT)((double)y[i] + alpha * (double)d[i] * (double)x[i]);
}

}  // namespace

hipError_t launch_diag_axpy(bool f64, const void *d, const void *x, void *y, int64_t n, double alpha,
                            hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned grid = (unsigned)(n / 256 + 1 < 65536 ? n / 256 + 1 : 65536);
    if (f64)
        hipLaunchKernelGGL(diag_axpy_kernel<double>, dim3(grid), dim3(256), 0, st, (const double *)d,
                           (const double *)x, (double *)y, n, alpha);
    else
        hipLaunchKernelGGL(diag_axpy_kernel<float>, dim3(grid), dim3(256), 0, st, (const float *)d,
                           (const float *)x, (float *)y, n, alpha);
    return hipGetLastError();
}

}  // namespace dtans
