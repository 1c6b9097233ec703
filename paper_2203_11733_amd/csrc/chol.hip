// Blocked right-looking Cholesky A = L L^T and the block triangular solves.
//
// A is symmetric positive definite (section 3.2, Theorem 1), so the paper
// solves A X = B by Cholesky.  Matrices here are column-major, lower triangle
// referenced, order npad (a multiple of 128, padded with an identity block).
// Step k of the factorisation, k0 = 128 k, m = npad - k0 - 128:
//   1. diag_kernel: L_kk = chol(A_kk) in LDS, then W_k = L_kk^{-1} in place;
//      L_kk goes back to A, W_k is kept for the solves.
//   2. panel = A[k0+128:, k0:k0+128] W_k^T          (GEMM, MFMA)
//   3. copy the panel into A (and to a 16-bit row-major copy for F16/BF16)
//   4. A[k0+128:, k0+128:] -= panel panel^T, lower tiles only (MFMA)
// dtype F64: FP64 storage, v_mfma_f64_16x16x4; F32: FP32 storage,
// v_mfma_f32_16x16x4f32; F16/BF16: FP32 storage and FP32 steps 1-3, step 4 on
// v_mfma_f32_16x16x32_{f16,bf16} with FP32 accumulation.
#include "gbem_internal.h"

namespace gbem {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));

// ------------------------------------------------------------------------
// Step 1: Cholesky of the 128 x 128 diagonal block in LDS, then its inverse.
// ------------------------------------------------------------------------
constexpr int kLdsLd = kNB + 1;   // column stride of the LDS block

// FACTOR = false: the block already holds L_kk; only W_k is computed.
template <typename T, bool FACTOR>
__global__ __launch_bounds__(1024) void diag_kernel(T *__restrict__ A, int64_t lda,
                                                    T *__restrict__ W, int32_t *__restrict__ info,
                                                    int k0)
{
    extern __shared__ unsigned char smem_raw[];
    T *a = reinterpret_cast<T *>(smem_raw);           // a[c * kLdsLd + r]
    T *x = a + kNB * kLdsLd;                           // 128-entry temporary
    const int tid = threadIdx.x;

    for (int idx = tid; idx < kNB * kNB; idx += 1024) {
        int r = idx % kNB, c = idx / kNB;
        a[c * kLdsLd + r] = (c <= r) ? A[r + c * lda] : T(0);
    }
    __syncthreads();

    // unblocked right-looking Cholesky
    for (int j = 0; FACTOR && j < kNB; ++j) {
        if (tid == 0) {
            T d = a[j * kLdsLd + j];
            if (!(d > T(0))) {
                if (*info == 0) *info = k0 + j + 1;
                d = T(1);
            }
            a[j * kLdsLd + j] = sqrt(d);
        }
        __syncthreads();
        const T inv = T(1) / a[j * kLdsLd + j];
        for (int r = j + 1 + tid; r < kNB; r += 1024) a[j * kLdsLd + r] *= inv;
        __syncthreads();
        const int cnt = kNB - 1 - j;
        for (int e = tid; e < cnt * cnt; e += 1024) {
            int r = j + 1 + e % cnt, c = j + 1 + e / cnt;
            if (c <= r) a[c * kLdsLd + r] -= a[j * kLdsLd + r] * a[j * kLdsLd + c];
        }
        __syncthreads();
    }
    if (FACTOR) {
        for (int idx = tid; idx < kNB * kNB; idx += 1024) {
            int r = idx % kNB, c = idx / kNB;
            if (c <= r) A[r + c * lda] = a[c * kLdsLd + r];
        }
        __syncthreads();
    }

    // in-place inverse of the lower triangular block, last column first:
    // column j of L^{-1} below the diagonal is -(1/l_jj) Linv[j+1:, j+1:] l[j+1:, j]
    for (int j = kNB - 1; j >= 0; --j) {
        const T djj = T(1) / a[j * kLdsLd + j];
        for (int r = j + 1 + tid; r < kNB; r += 1024) x[r] = a[j * kLdsLd + r];
        __syncthreads();
        for (int r = j + 1 + tid; r < kNB; r += 1024) {
            T s = T(0);
            for (int t = j + 1; t <= r; ++t) s += a[t * kLdsLd + r] * x[t];
            a[j * kLdsLd + r] = -djj * s;
        }
        __syncthreads();
        if (tid == 0) a[j * kLdsLd + j] = djj;
        __syncthreads();
    }
    for (int idx = tid; idx < kNB * kNB; idx += 1024) {
        int r = idx % kNB, c = idx / kNB;
        W[r + c * kNB] = (c <= r) ? a[c * kLdsLd + r] : T(0);
    }
}

// ------------------------------------------------------------------------
// GEMM C = A B^T (BETA = 0) or C -= A B^T (BETA = 1), FP64/FP32 operands
// stored column-major.  128 x 128 tile per 256-thread workgroup, 4 waves of
// 64 x 64, each 4 x 4 MFMA 16x16x4 blocks; K chunks of 16 through LDS.
// LOWER: tiles of the lower triangle only (M == N), diagonal tiles store r >= c.
// ------------------------------------------------------------------------
template <typename T> struct Mfma4;
// Output block of one 16x16 MFMA: lane l, register r holds column l % 16 and
// row row(l, r).  The f64 instruction interleaves the rows (l / 16 + 4 r); the
// f32 and 16-bit ones keep four consecutive rows per lane (4 (l / 16) + r).
template <> struct Mfma4<double> {
    typedef d4_t acc_t;
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
    static __device__ __forceinline__ acc_t run(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma4<float> {
    typedef f4_t acc_t;
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
    static __device__ __forceinline__ acc_t run(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

constexpr int kBM = 128, kBK = 16, kLdsPad = 4;

__device__ __forceinline__ void tile_of(int64_t t, bool lower, int tm, int &I, int &J)
{
    if (lower) {
        I = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while ((int64_t)I * (I + 1) / 2 > t) --I;
        while ((int64_t)(I + 1) * (I + 2) / 2 <= t) ++I;
        J = (int)(t - (int64_t)I * (I + 1) / 2);
    } else {
        I = (int)(t % tm);
        J = (int)(t / tm);
    }
}

template <typename T, bool LOWER, bool BETA>
__global__ __launch_bounds__(256) void gemm_nt_kernel(int tm, int K, const T *__restrict__ A,
                                                      int64_t lda, const T *__restrict__ B,
                                                      int64_t ldb, T *__restrict__ C, int64_t ldc)
{
    typedef typename Mfma4<T>::acc_t acc_t;
    __shared__ T As[kBK][kBM + kLdsPad];
    __shared__ T Bs[kBK][kBM + kLdsPad];
    int I, J;
    tile_of(blockIdx.x, LOWER, tm, I, J);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const T *Ab = A + (int64_t)I * kBM;
    const T *Bb = B + (int64_t)J * kBM;

    acc_t acc[4][4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = acc_t{0, 0, 0, 0};

    const int lk = tid >> 4, lr = (tid & 15) * 8;   // loader: column lk, rows lr..lr+7
    for (int k0 = 0; k0 < K; k0 += kBK) {
        const T *pa = Ab + lr + (int64_t)(k0 + lk) * lda;
        const T *pb = Bb + lr + (int64_t)(k0 + lk) * ldb;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            As[lk][lr + e] = pa[e];
            Bs[lk][lr + e] = pb[e];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kBK; kk += 4) {
            T af[4], bf[4];
#pragma unroll
            for (int mi = 0; mi < 4; ++mi) af[mi] = As[kk + (lane >> 4)][wm * 64 + mi * 16 + (lane & 15)];
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) bf[ni] = Bs[kk + (lane >> 4)][wn * 64 + ni * 16 + (lane & 15)];
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = Mfma4<T>::run(af[mi], bf[ni], acc[mi][ni]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
            const int col = J * kBM + wn * 64 + ni * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = I * kBM + wm * 64 + mi * 16 + Mfma4<T>::row(lane, r);
                if (LOWER && I == J && row < col) continue;
                T *pc = C + row + (int64_t)col * ldc;
                *pc = BETA ? *pc - acc[mi][ni][r] : acc[mi][ni][r];
            }
        }
}

// ------------------------------------------------------------------------
// 16-bit trailing update: C (FP32, column-major) -= P P^T with P stored
// row-major in 16 bits (P[r * ldp + k]); v_mfma_f32_16x16x32, FP32 accumulate.
// ------------------------------------------------------------------------
template <typename H> struct Mfma32;
template <> struct Mfma32<__bf16> {
    typedef bf8_t frag_t;
    static __device__ __forceinline__ f4_t run(frag_t a, frag_t b, f4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma32<_Float16> {
    typedef h8_t frag_t;
    static __device__ __forceinline__ f4_t run(frag_t a, frag_t b, f4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

constexpr int kBK16 = 64, kPad16 = 8;

template <typename H>
__global__ __launch_bounds__(256) void syrk16_kernel(int K, const H *__restrict__ P, int64_t ldp,
                                                     float *__restrict__ C, int64_t ldc)
{
    typedef typename Mfma32<H>::frag_t frag_t;
    __shared__ __attribute__((aligned(16))) H As[kBM][kBK16 + kPad16];
    __shared__ __attribute__((aligned(16))) H Bs[kBM][kBK16 + kPad16];
    int I, J;
    tile_of(blockIdx.x, true, 0, I, J);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;

    f4_t acc[4][4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = f4_t{0, 0, 0, 0};

    const int lr = tid >> 1, lk = (tid & 1) * 32;   // loader: row lr, k lk..lk+31
    for (int k0 = 0; k0 < K; k0 += kBK16) {
        const uint4 *pa = reinterpret_cast<const uint4 *>(P + (int64_t)(I * kBM + lr) * ldp + k0 + lk);
        const uint4 *pb = reinterpret_cast<const uint4 *>(P + (int64_t)(J * kBM + lr) * ldp + k0 + lk);
        uint4 *sa = reinterpret_cast<uint4 *>(&As[lr][lk]);
        uint4 *sb = reinterpret_cast<uint4 *>(&Bs[lr][lk]);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            sa[e] = pa[e];
            sb[e] = pb[e];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kBK16; kk += 32) {
            frag_t af[4], bf[4];
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
                af[mi] = *reinterpret_cast<const frag_t *>(&As[wm * 64 + mi * 16 + (lane & 15)][kk + 8 * (lane >> 4)]);
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
                bf[ni] = *reinterpret_cast<const frag_t *>(&Bs[wn * 64 + ni * 16 + (lane & 15)][kk + 8 * (lane >> 4)]);
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = Mfma32<H>::run(af[mi], bf[ni], acc[mi][ni]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
            const int col = J * kBM + wn * 64 + ni * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = I * kBM + wm * 64 + mi * 16 + 4 * (lane >> 4) + r;
                if (I == J && row < col) continue;
                float *pc = C + row + (int64_t)col * ldc;
                *pc = *pc - acc[mi][ni][r];
            }
        }
}

// ------------------------------------------------------------------------
// Step 3: copy the solved panel into A; optionally a 16-bit row-major copy.
// ------------------------------------------------------------------------
template <typename T, typename H>
__global__ void panel_copy_kernel(const T *__restrict__ Pw, int64_t ldw, int m, T *__restrict__ A,
                                  int64_t lda, H *__restrict__ P16)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    int c = blockIdx.y;
    if (r >= m) return;
    T v = Pw[r + (int64_t)c * ldw];
    A[r + (int64_t)c * lda] = v;
    if (P16) P16[(int64_t)r * kNB + c] = (H)(float)v;
}

// ------------------------------------------------------------------------
// Triangular solves with M right-hand sides (B: npad x m, FP64, ld ldb).
// The factor L (type T) and the diagonal inverses W_k (type T) are read in
// their storage precision and used in FP64 arithmetic.
// ------------------------------------------------------------------------
// Shared memory of these kernels is dynamic: kNB x (m + 1) doubles plus,
// for the backward update, a 64 x (kNB + 1) block of L.
constexpr int kRhsPerThread = kMaxRhs / 4;

// B_k <- W_k B_k (forward) or W_k^T B_k (backward); one workgroup, 256 threads.
template <typename T, bool TRANS>
__global__ __launch_bounds__(256) void diag_apply_kernel(const T *__restrict__ W, double *__restrict__ B,
                                                         int64_t ldb, int m)
{
    extern __shared__ double bs[];   // bs[r * (m + 1) + c]
    const int ld = m + 1, tid = threadIdx.x;
    for (int idx = tid; idx < kNB * m; idx += 256) {
        int r = idx % kNB, c = idx / kNB;
        bs[r * ld + c] = B[r + (int64_t)c * ldb];
    }
    __syncthreads();
    for (int idx = tid; idx < kNB * m; idx += 256) {
        int r = idx % kNB, c = idx / kNB;
        double s = 0.0;
        if (!TRANS) {
            for (int t = 0; t <= r; ++t) s += (double)W[r + t * kNB] * bs[t * ld + c];
        } else {
            for (int t = r; t < kNB; ++t) s += (double)W[t + r * kNB] * bs[t * ld + c];
        }
        B[r + (int64_t)c * ldb] = s;
    }
}

// Forward update: B[r, :] -= sum_t L[r, k0+t] Y[t, :] for the 64 rows of this
// workgroup, Y = B[k0:k0+128, :].  Thread (r, g) accumulates columns g, g+4, ...
template <typename T>
__global__ __launch_bounds__(256) void fwd_update_kernel(const T *__restrict__ L, int64_t lda,
                                                         double *__restrict__ B, int64_t ldb,
                                                         int k0, int row0, int m)
{
    extern __shared__ double ys[];   // ys[t * (m + 1) + c]
    const int ld = m + 1, tid = threadIdx.x;
    for (int idx = tid; idx < kNB * m; idx += 256) {
        int r = idx % kNB, c = idx / kNB;
        ys[r * ld + c] = B[(k0 + r) + (int64_t)c * ldb];
    }
    __syncthreads();
    const int r = row0 + blockIdx.x * 64 + (tid & 63), g = tid >> 6;
    double acc[kRhsPerThread];
#pragma unroll
    for (int q = 0; q < kRhsPerThread; ++q) acc[q] = 0.0;
    for (int t = 0; t < kNB; ++t) {
        const double l = (double)L[r + (int64_t)(k0 + t) * lda];
#pragma unroll
        for (int q = 0; q < kRhsPerThread; ++q) {
            int c = g + 4 * q;
            if (c < m) acc[q] += l * ys[t * ld + c];
        }
    }
#pragma unroll
    for (int q = 0; q < kRhsPerThread; ++q) {
        int c = g + 4 * q;
        if (c < m) B[r + (int64_t)c * ldb] -= acc[q];
    }
}

// Backward update: B[c, :] -= sum_t L[k0+t, c] X[t, :] for the 64 rows c < k0
// of this workgroup, X = B[k0:k0+128, :].
template <typename T>
__global__ __launch_bounds__(256) void bwd_update_kernel(const T *__restrict__ L, int64_t lda,
                                                         double *__restrict__ B, int64_t ldb,
                                                         int k0, int m)
{
    extern __shared__ double xs[];           // xs[t * (m + 1) + c]
    const int ld = m + 1, tid = threadIdx.x;
    double *ls = xs + kNB * ld;              // ls[q * (kNB + 1) + t] = L[k0+t, c0+q]
    for (int idx = tid; idx < kNB * m; idx += 256) {
        int r = idx % kNB, c = idx / kNB;
        xs[r * ld + c] = B[(k0 + r) + (int64_t)c * ldb];
    }
    const int c0 = blockIdx.x * 64;
    for (int idx = tid; idx < 64 * kNB; idx += 256) {
        int t = idx % kNB, q = idx / kNB;
        ls[q * (kNB + 1) + t] = (double)L[(k0 + t) + (int64_t)(c0 + q) * lda];
    }
    __syncthreads();
    const int q = tid & 63, g = tid >> 6;
    double acc[kRhsPerThread];
#pragma unroll
    for (int p = 0; p < kRhsPerThread; ++p) acc[p] = 0.0;
    for (int t = 0; t < kNB; ++t) {
        const double l = ls[q * (kNB + 1) + t];
#pragma unroll
        for (int p = 0; p < kRhsPerThread; ++p) {
            int c = g + 4 * p;
            if (c < m) acc[p] += l * xs[t * ld + c];
        }
    }
#pragma unroll
    for (int p = 0; p < kRhsPerThread; ++p) {
        int c = g + 4 * p;
        if (c < m) B[(c0 + q) + (int64_t)c * ldb] -= acc[p];
    }
}

// ------------------------------------------------------------------------
// host drivers
// ------------------------------------------------------------------------
static size_t elem_size(int dtype) { return dtype == GBEM_F64 ? 8 : 4; }

size_t chol_winv_bytes(int dtype, int64_t npad) { return (size_t)npad * kNB * elem_size(dtype); }
size_t chol_panel_bytes(int dtype, int64_t npad) { return (size_t)npad * kNB * elem_size(dtype); }
size_t chol_panel16_bytes(int dtype, int64_t npad)
{
    return (dtype == GBEM_F16 || dtype == GBEM_BF16) ? (size_t)npad * kNB * 2 : 0;
}

template <typename T>
static hipError_t factor_t(int dtype, int64_t npad, T *A, int64_t lda, T *Winv, T *Pw, void *P16,
                           int32_t *info, hipStream_t s)
{
    const int nb = (int)(npad / kNB);
    const size_t smem = (size_t)(kNB * kLdsLd + kNB) * sizeof(T);
    hipError_t e = hipFuncSetAttribute((const void *)diag_kernel<T, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    for (int k = 0; k < nb; ++k) {
        const int64_t k0 = (int64_t)k * kNB;
        T *Akk = A + k0 + k0 * lda;
        hipLaunchKernelGGL((diag_kernel<T, true>), dim3(1), dim3(1024), smem, s, Akk, lda,
                           Winv + (int64_t)k * kNB * kNB, info, (int)k0);
        const int64_t m = npad - k0 - kNB;
        if (m == 0) break;
        const int tm = (int)(m / kBM);
        T *Pan = A + (k0 + kNB) + k0 * lda;
        // panel <- A_panel W_k^T
        hipLaunchKernelGGL((gemm_nt_kernel<T, false, false>), dim3(tm), dim3(256), 0, s, tm, kNB,
                           (const T *)Pan, lda, (const T *)(Winv + (int64_t)k * kNB * kNB),
                           (int64_t)kNB, Pw, (int64_t)npad);
        if (dtype == GBEM_BF16)
            hipLaunchKernelGGL((panel_copy_kernel<T, __bf16>), dim3((unsigned)((m + 255) / 256), kNB),
                               dim3(256), 0, s, (const T *)Pw, (int64_t)npad, (int)m, Pan, lda,
                               (__bf16 *)P16);
        else if (dtype == GBEM_F16)
            hipLaunchKernelGGL((panel_copy_kernel<T, _Float16>), dim3((unsigned)((m + 255) / 256), kNB),
                               dim3(256), 0, s, (const T *)Pw, (int64_t)npad, (int)m, Pan, lda,
                               (_Float16 *)P16);
        else
            hipLaunchKernelGGL((panel_copy_kernel<T, T>), dim3((unsigned)((m + 255) / 256), kNB),
                               dim3(256), 0, s, (const T *)Pw, (int64_t)npad, (int)m, Pan, lda,
                               (T *)nullptr);
        T *Trail = A + (k0 + kNB) + (k0 + kNB) * lda;
        const int64_t ntiles = (int64_t)tm * (tm + 1) / 2;
        if (dtype == GBEM_BF16)
            hipLaunchKernelGGL(syrk16_kernel<__bf16>, dim3((unsigned)ntiles), dim3(256), 0, s, kNB,
                               (const __bf16 *)P16, (int64_t)kNB, (float *)Trail, lda);
        else if (dtype == GBEM_F16)
            hipLaunchKernelGGL(syrk16_kernel<_Float16>, dim3((unsigned)ntiles), dim3(256), 0, s, kNB,
                               (const _Float16 *)P16, (int64_t)kNB, (float *)Trail, lda);
        else
            hipLaunchKernelGGL((gemm_nt_kernel<T, true, true>), dim3((unsigned)ntiles), dim3(256), 0, s,
                               tm, kNB, (const T *)Pw, (int64_t)npad, (const T *)Pw, (int64_t)npad, Trail,
                               lda);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t chol_factor(int dtype, int64_t npad, void *A, int64_t lda, void *Winv, void *panel,
                       void *panel16, int32_t *info, hipStream_t s)
{
    if (npad % kNB) return hipErrorInvalidValue;
    if (dtype == GBEM_F64)
        return factor_t<double>(dtype, npad, (double *)A, lda, (double *)Winv, (double *)panel,
                                nullptr, info, s);
    return factor_t<float>(dtype, npad, (float *)A, lda, (float *)Winv, (float *)panel, panel16,
                           info, s);
}

template <typename T>
static hipError_t solve_t(int64_t npad, const T *L, int64_t lda, const T *Winv, int m, double *B,
                          int64_t ldb, hipStream_t s)
{
    const int nb = (int)(npad / kNB);
    const size_t smem_b = (size_t)kNB * (m + 1) * sizeof(double);
    const size_t smem_l = smem_b + (size_t)64 * (kNB + 1) * sizeof(double);
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void *)diag_apply_kernel<T, false>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem_b)) != hipSuccess ||
        (e = hipFuncSetAttribute((const void *)diag_apply_kernel<T, true>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem_b)) != hipSuccess ||
        (e = hipFuncSetAttribute((const void *)fwd_update_kernel<T>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem_b)) != hipSuccess ||
        (e = hipFuncSetAttribute((const void *)bwd_update_kernel<T>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem_l)) != hipSuccess)
        return e;
    for (int k = 0; k < nb; ++k) {
        const int64_t k0 = (int64_t)k * kNB;
        hipLaunchKernelGGL((diag_apply_kernel<T, false>), dim3(1), dim3(256), smem_b, s,
                           Winv + (int64_t)k * kNB * kNB, B + k0, ldb, m);
        const int64_t rows = npad - k0 - kNB;
        if (rows > 0)
            hipLaunchKernelGGL(fwd_update_kernel<T>, dim3((unsigned)(rows / 64)), dim3(256), smem_b, s, L,
                               lda, B, ldb, (int)k0, (int)(k0 + kNB), m);
    }
    for (int k = nb - 1; k >= 0; --k) {
        const int64_t k0 = (int64_t)k * kNB;
        hipLaunchKernelGGL((diag_apply_kernel<T, true>), dim3(1), dim3(256), smem_b, s,
                           Winv + (int64_t)k * kNB * kNB, B + k0, ldb, m);
        if (k0 > 0)
            hipLaunchKernelGGL(bwd_update_kernel<T>, dim3((unsigned)(k0 / 64)), dim3(256), smem_l, s, L, lda,
                               B, ldb, (int)k0, m);
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t diag_inverses_t(int64_t npad, const T *L, int64_t lda, T *Winv, hipStream_t s)
{
    const size_t smem = (size_t)(kNB * kLdsLd + kNB) * sizeof(T);
    hipError_t e = hipFuncSetAttribute((const void *)diag_kernel<T, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    for (int64_t k0 = 0; k0 < npad; k0 += kNB)
        hipLaunchKernelGGL((diag_kernel<T, false>), dim3(1), dim3(1024), smem, s,
                           const_cast<T *>(L) + k0 + k0 * lda, lda, Winv + k0 * kNB, (int32_t *)nullptr,
                           (int)k0);
    return hipGetLastError();
}

hipError_t chol_diag_inverses(int dtype, int64_t npad, const void *L, int64_t lda, void *Winv,
                              hipStream_t s)
{
    if (npad % kNB) return hipErrorInvalidValue;
    if (dtype == GBEM_F64) return diag_inverses_t<double>(npad, (const double *)L, lda, (double *)Winv, s);
    return diag_inverses_t<float>(npad, (const float *)L, lda, (float *)Winv, s);
}

hipError_t chol_solve(int dtype, int64_t npad, const void *L, int64_t lda, const void *Winv, int m,
                      double *B, int64_t ldb, hipStream_t s)
{
    if (npad % kNB || m > kMaxRhs || m <= 0) return hipErrorInvalidValue;
    if (dtype == GBEM_F64)
        return solve_t<double>(npad, (const double *)L, lda, (const double *)Winv, m, B, ldb, s);
    return solve_t<float>(npad, (const float *)L, lda, (const float *)Winv, m, B, ldb, s);
}

}  // namespace gbem
