// Mixed-precision solve helpers: Jacobi scaling of A, conversion to the FP32
// factor storage, the FP64 residual R = B - A X and column norms for the
// iterative refinement.  The residual uses the FP64 matrix A (near entries
// exact in FP64, far entries as assembled), so refinement converges to the
// solution of the assembled FP64 system.
#include "gbem_internal.h"

namespace gbem {

__global__ void jacobi_scale_kernel(const double *__restrict__ A, int64_t lda, int npad,
                                    double *__restrict__ s)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npad) s[i] = 1.0 / sqrt(A[i + (int64_t)i * lda]);
}

hipError_t launch_jacobi_scale(const double *A, int64_t lda, int npad, double *s, hipStream_t st)
{
    hipLaunchKernelGGL(jacobi_scale_kernel, dim3((npad + 255) / 256), dim3(256), 0, st, A, lda, npad, s);
    return hipGetLastError();
}

// F = S A S in FP32, lower triangle (column j = blockIdx.x, rows i >= j).
__global__ void scale_convert_kernel(const double *__restrict__ A, int64_t lda,
                                     const double *__restrict__ s, int npad, float *__restrict__ F,
                                     int64_t ldf)
{
    const int j = blockIdx.x;
    const int i = blockIdx.y * blockDim.x + threadIdx.x;
    if (i >= npad || i < j) return;
    F[i + (int64_t)j * ldf] = (float)(s[i] * A[i + (int64_t)j * lda] * s[j]);
}

hipError_t launch_scale_convert(const double *A, int64_t lda, const double *s, int npad, float *F,
                                int64_t ldf, hipStream_t st)
{
    hipLaunchKernelGGL(scale_convert_kernel, dim3(npad, (npad + 255) / 256), dim3(256), 0, st, A, lda,
                       s, npad, F, ldf);
    return hipGetLastError();
}

// norms[c] = sum_i R[i, c]^2 (fixed-order reduction, one workgroup per column)
__global__ __launch_bounds__(256) void col_norms_kernel(const double *__restrict__ R, int64_t ldr,
                                                        int npad, double *__restrict__ norms)
{
    __shared__ double red[4];
    const int c = blockIdx.x, tid = threadIdx.x;
    double s = 0.0;
    for (int i = tid; i < npad; i += 256) {
        double v = R[i + (int64_t)c * ldr];
        s = __builtin_fma(v, v, s);
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) norms[c] = (red[0] + red[1]) + (red[2] + red[3]);
}

hipError_t launch_col_norms(const double *R, int64_t ldr, int npad, int m, double *norms,
                            hipStream_t st)
{
    hipLaunchKernelGGL(col_norms_kernel, dim3(m), dim3(256), 0, st, R, ldr, npad, norms);
    return hipGetLastError();
}

__global__ void scale_rows_kernel(double *__restrict__ X, int64_t ldx, const double *__restrict__ s,
                                  int npad)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int c = blockIdx.y;
    if (i < npad) X[i + (int64_t)c * ldx] *= s[i];
}

hipError_t launch_scale_rows(double *X, int64_t ldx, const double *s, int npad, int m, hipStream_t st)
{
    hipLaunchKernelGGL(scale_rows_kernel, dim3((npad + 255) / 256, m), dim3(256), 0, st, X, ldx, s,
                       npad);
    return hipGetLastError();
}

__global__ void axpy_cols_kernel(double *__restrict__ X, int64_t ldx, const double *__restrict__ D,
                                 int64_t ldd, int npad)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int c = blockIdx.y;
    if (i < npad) X[i + (int64_t)c * ldx] += D[i + (int64_t)c * ldd];
}

hipError_t launch_axpy_cols(double *X, int64_t ldx, const double *D, int64_t ldd, int npad, int m,
                            hipStream_t st)
{
    hipLaunchKernelGGL(axpy_cols_kernel, dim3((npad + 255) / 256, m), dim3(256), 0, st, X, ldx, D, ldd,
                       npad);
    return hipGetLastError();
}

}  // namespace gbem
