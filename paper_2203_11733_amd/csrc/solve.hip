// Triangular solves L Y = B, L^T X = Y with M right-hand sides (one per
// conductor, eq. "lineareq1") and the FP64 residual of the refinement.
//
// Solves: one persistent launch per direction.  Workgroup k owns block row k
// (128 rows) of the npad/128 blocks.  It accumulates B_k - sum_j L_kj Y_j as
// the blocks Y_j it depends on are published, applies the stored inverse
// W_k = L_kk^{-1}, writes Y_k and publishes it through a per-block flag
// (release store, agent scope); consumers poll the flag (acquire) before
// reading Y_j.  A workgroup takes its block from an atomic ticket, so block k
// only waits on blocks whose workgroups already run; every wait therefore
// ends, and a bounded poll sets an error word instead of spinning forever.
// Flags carry an epoch that grows with every launch and each launch consumes
// exactly nb tickets, so neither needs clearing between launches.  Arithmetic is FP64; L and W are read
// in their storage type.  The two halves of a workgroup split the 128-long
// inner products; the forward pass reads rows of L (coalesced across lanes),
// the backward pass walks down columns (contiguous per lane).
//
// Residual: R = B - A X with the FP64 matrix (row i of the symmetric A is read
// as column i).  The j range is split over kResSplit workgroups per row block;
// partial sums are added in a fixed order by a second kernel.
#include "gbem_internal.h"

namespace gbem {


__device__ __forceinline__ bool wait_flag(const int32_t *flag, int32_t epoch, int32_t *err, int limit)
{
    int n = 0;
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
        __builtin_amdgcn_s_sleep(2);
        if (++n > limit) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    return true;
}

// Publish this workgroup's block: every thread makes its stores visible at
// agent scope, then one thread raises the flag.
__device__ __forceinline__ void publish(int32_t *flag, int32_t epoch)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flag, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Block index of this workgroup: tickets are handed out in execution order.
// Every workgroup of every launch takes exactly one ticket, so the host knows
// the counter value `base` at the start of a launch.
__device__ __forceinline__ int take_ticket(int32_t *counter, uint32_t base)
{
    __shared__ int t;
    if (threadIdx.x == 0) t = (int)((uint32_t)atomicAdd(counter, 1) - base);
    __syncthreads();
    return t;
}

// Wait (thread 0) for a flag, then make the block's data visible to all waves.
__device__ __forceinline__ void acquire_block(const int32_t *flag, int32_t epoch, int32_t *err, int limit)
{
    __shared__ int ok;
    if (threadIdx.x == 0) ok = wait_flag(flag, epoch, err, limit);
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// ys[t * (MC + 1) + c] = B[row0 + t, c] for c < m, 0 for m <= c < MC
template <int MC>
__device__ __forceinline__ void stage_rows(double *ys, const double *B, int64_t ldb, int row0, int m)
{
    for (int idx = threadIdx.x; idx < kNB * MC; idx += 256) {
        const int t = idx % kNB, c = idx / kNB;
        ys[t * (MC + 1) + c] = c < m ? B[(row0 + t) + (int64_t)c * ldb] : 0.0;
    }
}

// acc[c] -= sum_{t in [t0, t0+64)} M(t) ys[t][c], M(t) = src[t * stride]; loads
// are issued 16 at a time.
template <typename T, int MC, bool SUB>
__device__ __forceinline__ void block_dot(double *acc, const T *src, int64_t stride, const double *ys, int t0)
{
    for (int tb = 0; tb < 64; tb += 16) {
        double l[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) l[u] = (double)src[(int64_t)(tb + u) * stride];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const double *y = ys + (t0 + tb + u) * (MC + 1);
#pragma unroll
            for (int c = 0; c < MC; ++c) acc[c] = SUB ? acc[c] - l[u] * y[c] : acc[c] + l[u] * y[c];
        }
    }
}

// Sum the two halves' accumulators: half 1 hands its values to half 0 via LDS.
template <int MC>
__device__ __forceinline__ void combine_halves(double *acc, double *red, int r, int h)
{
    __syncthreads();
    if (h == 1) {
#pragma unroll
        for (int c = 0; c < MC; ++c) red[r * (MC + 1) + c] = acc[c];
    }
    __syncthreads();
    if (h == 0) {
#pragma unroll
        for (int c = 0; c < MC; ++c) acc[c] += red[r * (MC + 1) + c];
    }
}

// Threads: r = tid % 128 (row of the block), h = tid / 128 (half of the
// 128-long t range).  MC >= m columns, padded with zeros.
template <typename T, int MC>
__global__ __launch_bounds__(256) void fwd_solve_kernel(const T *__restrict__ L, int64_t lda,
                                                        const T *__restrict__ W, double *__restrict__ B,
                                                        int64_t ldb, int m, int nb, int32_t *__restrict__ flags,
                                                        int32_t *__restrict__ counter, uint32_t base,
                                                        int32_t epoch, int32_t *__restrict__ err, int limit)
{
    extern __shared__ double sm[];
    double *ys = sm;                          // 128 x (MC+1)
    double *red = sm + kNB * (MC + 1);        // 128 x (MC+1)
    const int k = take_ticket(counter, base), k0 = k * kNB;
    if (k < 0 || k >= nb) {
        if (threadIdx.x == 0) __hip_atomic_store(err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const int r = threadIdx.x & 127, h = threadIdx.x >> 7;
    double acc[MC];
#pragma unroll
    for (int c = 0; c < MC; ++c) acc[c] = (h == 0 && c < m) ? B[(k0 + r) + (int64_t)c * ldb] : 0.0;
    for (int j = 0; j < k; ++j) {
        acquire_block(flags + j, epoch, err, limit);
        stage_rows<MC>(ys, B, ldb, j * kNB, m);
        __syncthreads();
        // L[k0 + r, j0 + t]: consecutive rows across lanes (coalesced)
        block_dot<T, MC, true>(acc, L + (k0 + r) + ((int64_t)j * kNB + h * 64) * lda, lda, ys, h * 64);
        __syncthreads();
    }
    combine_halves<MC>(acc, red, r, h);
    // Y_k = W_k acc: W[r + t * 128]
    if (h == 0) {
#pragma unroll
        for (int c = 0; c < MC; ++c) ys[r * (MC + 1) + c] = acc[c];
    }
    __syncthreads();
    double y[MC];
#pragma unroll
    for (int c = 0; c < MC; ++c) y[c] = 0.0;
    block_dot<T, MC, false>(y, W + (int64_t)k * kNB * kNB + r + (int64_t)h * 64 * kNB, kNB, ys, h * 64);
    combine_halves<MC>(y, red, r, h);
    if (h == 0) {
#pragma unroll
        for (int c = 0; c < MC; ++c)
            if (c < m) B[(k0 + r) + (int64_t)c * ldb] = y[c];
    }
    publish(flags + k, epoch);
}

template <typename T, int MC>
__global__ __launch_bounds__(256) void bwd_solve_kernel(const T *__restrict__ L, int64_t lda,
                                                        const T *__restrict__ W, double *__restrict__ B,
                                                        int64_t ldb, int m, int nb, int32_t *__restrict__ flags,
                                                        int32_t *__restrict__ counter, uint32_t base,
                                                        int32_t epoch, int32_t *__restrict__ err, int limit)
{
    extern __shared__ double sm[];
    double *xs = sm;                          // 128 x (MC+1)
    double *red = sm + kNB * (MC + 1);        // 128 x (MC+1)
    const int tk = take_ticket(counter, base);
    if (tk < 0 || tk >= nb) {
        if (threadIdx.x == 0) __hip_atomic_store(err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const int k = nb - 1 - tk, k0 = k * kNB;
    const int r = threadIdx.x & 127, h = threadIdx.x >> 7;
    double acc[MC];
#pragma unroll
    for (int c = 0; c < MC; ++c) acc[c] = (h == 0 && c < m) ? B[(k0 + r) + (int64_t)c * ldb] : 0.0;
    for (int j = nb - 1; j > k; --j) {
        acquire_block(flags + j, epoch, err, limit);
        stage_rows<MC>(xs, B, ldb, j * kNB, m);
        __syncthreads();
        // L[j0 + t, k0 + r]: a contiguous run down column k0 + r per thread
        block_dot<T, MC, true>(acc, L + ((int64_t)j * kNB + h * 64) + (int64_t)(k0 + r) * lda, 1, xs, h * 64);
        __syncthreads();
    }
    combine_halves<MC>(acc, red, r, h);
    // X_k = W_k^T acc: W[t + r * 128]
    if (h == 0) {
#pragma unroll
        for (int c = 0; c < MC; ++c) xs[r * (MC + 1) + c] = acc[c];
    }
    __syncthreads();
    double x[MC];
#pragma unroll
    for (int c = 0; c < MC; ++c) x[c] = 0.0;
    block_dot<T, MC, false>(x, W + (int64_t)k * kNB * kNB + (int64_t)r * kNB + h * 64, 1, xs, h * 64);
    combine_halves<MC>(x, red, r, h);
    if (h == 0) {
#pragma unroll
        for (int c = 0; c < MC; ++c)
            if (c < m) B[(k0 + r) + (int64_t)c * ldb] = x[c];
    }
    publish(flags + k, epoch);
}

template <typename T, int MC>
static hipError_t solve_mc(int64_t npad, const T *L, int64_t lda, const T *W, int m, double *B, int64_t ldb,
                           SolveSync &sync, hipStream_t s, Prof *prof)
{
    const int nb = (int)(npad / kNB);
    const size_t smem = (size_t)2 * kNB * (MC + 1) * sizeof(double);
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void *)fwd_solve_kernel<T, MC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)smem)) != hipSuccess ||
        (e = hipFuncSetAttribute((const void *)bwd_solve_kernel<T, MC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)smem)) != hipSuccess)
        return e;
    const int limit = 1 << 26;
    ++sync.epoch;
    const int tok = prof ? prof->start(s) : -1;
    hipLaunchKernelGGL((fwd_solve_kernel<T, MC>), dim3(nb), dim3(256), smem, s, L, lda, W, B, ldb, m, nb,
                       sync.flags_f, sync.err + 1, sync.base_f, sync.epoch, sync.err, limit);
    hipLaunchKernelGGL((bwd_solve_kernel<T, MC>), dim3(nb), dim3(256), smem, s, L, lda, W, B, ldb, m, nb,
                       sync.flags_b, sync.err + 2, sync.base_b, sync.epoch, sync.err, limit);
    if (prof) {
        // L read once per direction (lower half incl. diagonal blocks), W read twice, B read/written
        const double lbytes = (double)npad * (npad + kNB) / 2.0 * sizeof(T);
        prof->stop(tok, GBEM_K_SOLVE, 2.0 * 2.0 * (double)npad * npad / 2.0 * m,
                   2.0 * lbytes + 2.0 * npad * kNB * sizeof(T) + 4.0 * npad * m * 8.0, s, 2);
    }
    e = hipGetLastError();
    if (e == hipSuccess) {   // both launches queued: each consumes exactly nb tickets
        sync.base_f += (uint32_t)nb;
        sync.base_b += (uint32_t)nb;
    }
    return e;
}

template <typename T>
static hipError_t solve_t(int64_t npad, const T *L, int64_t lda, const T *W, int m, double *B, int64_t ldb,
                          SolveSync &sync, hipStream_t s, Prof *prof)
{
    if (m <= 8) return solve_mc<T, 8>(npad, L, lda, W, m, B, ldb, sync, s, prof);
    if (m <= 16) return solve_mc<T, 16>(npad, L, lda, W, m, B, ldb, sync, s, prof);
    if (m <= 32) return solve_mc<T, 32>(npad, L, lda, W, m, B, ldb, sync, s, prof);
    return solve_mc<T, 64>(npad, L, lda, W, m, B, ldb, sync, s, prof);
}

hipError_t chol_solve(int dtype, int64_t npad, const void *L, int64_t lda, const void *Winv, int m, double *B,
                      int64_t ldb, SolveSync &sync, hipStream_t s, Prof *prof)
{
    if (npad % kNB || m > kMaxRhs || m <= 0) return hipErrorInvalidValue;
    if (dtype == GBEM_F64)
        return solve_t<double>(npad, (const double *)L, lda, (const double *)Winv, m, B, ldb, sync, s, prof);
    return solve_t<float>(npad, (const float *)L, lda, (const float *)Winv, m, B, ldb, sync, s, prof);
}

// ------------------------------------------------------------------------
// Residual R = B - A X, split over j.
// ------------------------------------------------------------------------
constexpr int kRRows = 64, kRChunk = 32, kRPerThread = kMaxRhs / 4;

__global__ __launch_bounds__(256) void residual_partial_kernel(const double *__restrict__ A, int64_t lda,
                                                               int npad, const double *__restrict__ X,
                                                               int64_t ldx, int m, int jspan,
                                                               double *__restrict__ P)
{
    __shared__ double as[kRRows][kRChunk + 1];    // as[i][jj] = A[j0 + jj, i0 + i]
    __shared__ double xs[kRChunk][kMaxRhs + 1];   // xs[jj][c] = X[j0 + jj, c]
    const int tid = threadIdx.x, il = tid & 63, g = tid >> 6;
    const int i0 = blockIdx.x * kRRows, s = blockIdx.y;
    const int jb = s * jspan, je = min(npad, jb + jspan);
    double acc[kRPerThread];
#pragma unroll
    for (int q = 0; q < kRPerThread; ++q) acc[q] = 0.0;
    // loader: column i0 + tid/4, 8 contiguous rows
    const int lc = tid >> 2, lr = (tid & 3) * 8;
    for (int j0 = jb; j0 < je; j0 += kRChunk) {
        const double *src = A + (j0 + lr) + (int64_t)(i0 + lc) * lda;
#pragma unroll
        for (int e = 0; e < 8; ++e) as[lc][lr + e] = src[e];
        for (int idx = tid; idx < kRChunk * m; idx += 256) {
            const int jj = idx % kRChunk, c = idx / kRChunk;
            xs[jj][c] = X[(j0 + jj) + (int64_t)c * ldx];
        }
        __syncthreads();
        for (int jj = 0; jj < kRChunk; ++jj) {
            const double a = as[il][jj];
#pragma unroll
            for (int q = 0; q < kRPerThread; ++q) {
                const int c = g + 4 * q;
                if (c < m) acc[q] = __builtin_fma(a, xs[jj][c], acc[q]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < kRPerThread; ++q) {
        const int c = g + 4 * q;
        if (c < m) P[((int64_t)s * m + c) * npad + i0 + il] = acc[q];
    }
}

__global__ void residual_finish_kernel(const double *__restrict__ P, int nsplit, int npad, int m,
                                       const double *__restrict__ B, int64_t ldb, double *__restrict__ R,
                                       int64_t ldr)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
    if (i >= npad) return;
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += P[((int64_t)k * m + c) * npad + i];
    R[i + (int64_t)c * ldr] = B[i + (int64_t)c * ldb] - s;
}

int residual_splits(int npad) { return max(1, min(kResMaxSplit, npad / 2048)); }

hipError_t launch_residual(const double *A, int64_t lda, int npad, const double *X, int64_t ldx, const double *B,
                           int64_t ldb, int m, double *R, int64_t ldr, double *partial, hipStream_t st)
{
    if (npad % kRRows || m > kMaxRhs) return hipErrorInvalidValue;
    const int ns = residual_splits(npad);
    const int jspan = (int)round_up((npad + ns - 1) / ns, kRChunk);
    hipLaunchKernelGGL(residual_partial_kernel, dim3(npad / kRRows, ns), dim3(256), 0, st, A, lda, npad, X, ldx, m,
                       jspan, partial);
    hipLaunchKernelGGL(residual_finish_kernel, dim3((npad + 255) / 256, m), dim3(256), 0, st, partial, ns, npad, m, B,
                       ldb, R, ldr);
    return hipGetLastError();
}

}  // namespace gbem
