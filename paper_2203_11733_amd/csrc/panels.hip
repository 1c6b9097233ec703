// Panel table, right-hand sides and charge sums.
//
// Panel table: the rectangles of the mesh (section 3.1: the boundary split
// into pieces I_j) become one 64-byte record each.  Right-hand side: b_i = 1
// on the main net, 0 elsewhere (eq. "lineareq1"), one column per conductor.
// Charges: Q'_n = eps * sum_{I_j on net n} q_j |I_j| (eq. "electriccharge"),
// where X_j = q_j |I_j| is the unknown of the system, so the sum runs over X.
#include "gbem_internal.h"

namespace gbem {

__global__ void build_panels_kernel(const double *__restrict__ lo, const double *__restrict__ hi,
                                    const int32_t *__restrict__ cond, int n, int n_cond,
                                    Panel *__restrict__ pan, int32_t *__restrict__ bad)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double l[3], h[3];
    for (int k = 0; k < 3; ++k) {
        l[k] = lo[3 * i + k];
        h[k] = hi[3 * i + k];
    }
    int nz = 0, nrm = -1, neg = 0;
    for (int k = 0; k < 3; ++k) {
        if (l[k] == h[k]) {
            ++nz;
            nrm = k;
        } else if (!(l[k] < h[k])) {
            neg = 1;   // also catches NaN
        }
    }
    int c = cond[i];
    if (nz != 1 || neg || c < -1 || c >= n_cond) {
        atomicMax(bad, i + 1);
        nrm = nrm < 0 ? 0 : nrm;
    }
    int t1 = nrm == 0 ? 1 : 0, t2 = nrm == 2 ? 1 : 2;
    Panel p;
    for (int k = 0; k < 3; ++k) p.c[k] = 0.5 * (l[k] + h[k]);
    p.h1 = 0.5 * (h[t1] - l[t1]);
    p.h2 = 0.5 * (h[t2] - l[t2]);
    p.area = (h[t1] - l[t1]) * (h[t2] - l[t2]);
    double e0 = h[0] - l[0], e1 = h[1] - l[1], e2 = h[2] - l[2];
    p.diam2 = __dadd_rn(__dadd_rn(__dmul_rn(e0, e0), __dmul_rn(e1, e1)), __dmul_rn(e2, e2));
    p.nrm = nrm;
    p.cond = c;
    pan[i] = p;
}

hipError_t launch_build_panels(const double *lo, const double *hi, const int32_t *cond, int n,
                               int n_cond, Panel *pan, int32_t *bad, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(build_panels_kernel, dim3((n + 255) / 256), dim3(256), 0, s, lo, hi, cond, n,
                       n_cond, pan, bad);
    return hipGetLastError();
}

__global__ void rhs_kernel(const int32_t *__restrict__ cond, int n, int npad, int m,
                           double *__restrict__ B, int64_t ldb)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int k = blockIdx.y;
    if (i >= npad) return;
    B[i + k * ldb] = (i < n && cond[i] == k) ? 1.0 : 0.0;
}

hipError_t launch_rhs(const int32_t *cond, int n, int npad, int m, double *B, int64_t ldb,
                      hipStream_t s)
{
    hipLaunchKernelGGL(rhs_kernel, dim3((npad + 255) / 256, m), dim3(256), 0, s, cond, n, npad, m, B,
                       ldb);
    return hipGetLastError();
}

// Partial charge sums over chunks of 1024 rows, summed in a fixed order so the
// result does not depend on scheduling:
//   partial[(chunk * m + k) * m + l] = sum_{i in chunk, cond_i = k} X[i, l]
constexpr int kChargeChunk = 1024;

__global__ __launch_bounds__(256) void charge_partials_kernel(const double *__restrict__ X,
                                                              int64_t ldx,
                                                              const int32_t *__restrict__ cond,
                                                              int n, int m,
                                                              double *__restrict__ partial)
{
    __shared__ double red[4];
    const int chunk = blockIdx.x, l = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double x[4];
    int c[4];
    for (int r = 0; r < 4; ++r) {
        int i = chunk * kChargeChunk + r * 256 + tid;
        bool in = i < n;
        x[r] = in ? X[i + l * ldx] : 0.0;
        c[r] = in ? cond[i] : -1;
    }
    for (int k = 0; k < m; ++k) {
        double v = 0.0;
        for (int r = 0; r < 4; ++r) v += (c[r] == k) ? x[r] : 0.0;
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wave] = v;
        __syncthreads();
        if (tid == 0)
            partial[((int64_t)chunk * m + k) * m + l] = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
    }
}

hipError_t launch_charge_partials(const double *X, int64_t ldx, const int32_t *cond, int n, int m,
                                  double *partial, int nchunks, hipStream_t s)
{
    hipLaunchKernelGGL(charge_partials_kernel, dim3(nchunks, m), dim3(256), 0, s, X, ldx, cond, n, m,
                       partial);
    return hipGetLastError();
}

__global__ void charge_finish_kernel(const double *__restrict__ partial, int nchunks, int m,
                                     double scale, double *__restrict__ C)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m * m) return;
    int k = t / m, l = t % m;
    double s = 0.0;
    for (int ch = 0; ch < nchunks; ++ch) s += partial[((int64_t)ch * m + k) * m + l];
    C[k * m + l] = scale * s;
}

hipError_t launch_charge_finish(const double *partial, int nchunks, int m, double scale, double *C,
                                hipStream_t s)
{
    int t = m * m;
    hipLaunchKernelGGL(charge_finish_kernel, dim3((t + 255) / 256), dim3(256), 0, s, partial, nchunks,
                       m, scale, C);
    return hipGetLastError();
}

// Identity in the padded rows/columns [n, npad) of an npad x npad matrix:
// column j = blockIdx.x; rows [n, npad) of every column, and all rows of the
// padded columns.
template <typename T>
__global__ void identity_pad_kernel(T *__restrict__ A, int64_t lda, int n, int npad)
{
    const int j = blockIdx.x;
    const int r0 = j >= n ? 0 : n;
    for (int i = r0 + threadIdx.x; i < npad; i += blockDim.x) A[i + (int64_t)j * lda] = (i == j) ? T(1) : T(0);
}

hipError_t launch_identity_pad(void *A, int64_t lda, int n, int npad, bool f64, hipStream_t s)
{
    if (n == npad) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(identity_pad_kernel<double>, dim3(npad), dim3(256), 0, s, (double *)A, lda, n, npad);
    else
        hipLaunchKernelGGL(identity_pad_kernel<float>, dim3(npad), dim3(256), 0, s, (float *)A, lda, n, npad);
    return hipGetLastError();
}

// out[k] = A[ii[k], jj[k]] (indices validated on the host)
template <typename T>
__global__ void gather_kernel(const T *__restrict__ A, int64_t lda, const int32_t *__restrict__ ii,
                              const int32_t *__restrict__ jj, int64_t m, T *__restrict__ out)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) out[k] = A[ii[k] + (int64_t)jj[k] * lda];
}

template <typename T>
static hipError_t gather(const T *A, int64_t lda, const int32_t *ii, const int32_t *jj, int64_t m, T *out,
                         hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_kernel<T>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, A, lda, ii, jj, m, out);
    return hipGetLastError();
}
hipError_t launch_gather(const double *A, int64_t lda, const int32_t *ii, const int32_t *jj, int64_t m,
                         double *out, hipStream_t s)
{
    return gather(A, lda, ii, jj, m, out, s);
}
hipError_t launch_gather(const float *A, int64_t lda, const int32_t *ii, const int32_t *jj, int64_t m, float *out,
                         hipStream_t s)
{
    return gather(A, lda, ii, jj, m, out, s);
}

}  // namespace gbem
