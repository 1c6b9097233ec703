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

__global__ void fill_i32_kernel(int32_t *__restrict__ p, int n, int32_t v)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

// A kernel in place of hipMemsetAsync for flags and counters: a fill of this
// kind is a kernel node when the stream is captured into a graph.
hipError_t launch_fill_i32(int32_t *p, int n, int32_t v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_jacobi_scale(const double *A, int64_t lda, int npad, double *s, hipStream_t st)
{
    hipLaunchKernelGGL(jacobi_scale_kernel, dim3((npad + 255) / 256), dim3(256), 0, st, A, lda, npad, s);
    return hipGetLastError();
}

// F = S A S (lower triangle) in FP32.  Workgroup: 1024 rows x 8 columns;
// thread: 4 consecutive rows (one 32-byte load and one 16-byte store per
// column).  npad is a multiple of 512 and lda, ldf multiples of 4, so every
// access is aligned; threads whose rows all lie above the diagonal return.
__global__ __launch_bounds__(256) void scale_convert_kernel(const double *__restrict__ A, int64_t lda,
                                                            const double *__restrict__ s, int npad,
                                                            float *__restrict__ F, int64_t ldf)
{
    typedef double d4_t __attribute__((ext_vector_type(4)));
    typedef float f4_t __attribute__((ext_vector_type(4)));
    const int j0 = blockIdx.x * 8;
    const int i = blockIdx.y * 1024 + threadIdx.x * 4;
    if (i >= npad || i + 3 < j0) return;   // rows past the matrix (npad need not divide by 1024) or above
    const d4_t si = *reinterpret_cast<const d4_t *>(s + i);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int j = j0 + c;
        if (i + 3 < j) break;   // the rest of this thread's rows lie above the diagonal
        const d4_t a = *reinterpret_cast<const d4_t *>(A + i + (int64_t)j * lda);
        const double sj = s[j];
        f4_t f;
#pragma unroll
        for (int e = 0; e < 4; ++e) f[e] = (float)(si[e] * a[e] * sj);
        float *dst = F + i + (int64_t)j * ldf;
        if (i >= j) {
            *reinterpret_cast<f4_t *>(dst) = f;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (i + e >= j) dst[e] = f[e];
        }
    }
}

hipError_t launch_scale_convert(const double *A, int64_t lda, const double *s, int npad, float *F,
                                int64_t ldf, hipStream_t st)
{
    if (npad % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(scale_convert_kernel, dim3(npad / 8, (npad + 1023) / 1024), dim3(256), 0, st, A, lda, s, npad,
                       F, ldf);
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
