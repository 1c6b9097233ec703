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
// Step 1: Cholesky of the 128 x 128 diagonal block in LDS and its inverse.
// The block is processed as 4 x 4 sub-blocks of 32.  For each sub-block
// column s: one wave factors the 32 x 32 diagonal sub-block and inverts it in
// registers (lane r owns row r, values broadcast with v_readlane, no
// barriers); all waves then solve the sub-block rows below against it and
// apply the rank-32 update to the rest.  The inverse of the whole block is
// assembled in place from the sub-block inverses W_ss:
//   W_rs = -W_rr sum_{t=s}^{r-1} L_rt W_ts   (columns s left to right).
// Sub-block inverses wait in the unused upper triangle (transposed) and in a
// 128-entry diagonal array until the end.
// ------------------------------------------------------------------------
constexpr int kLdsLd = kNB + 1;   // column stride of the LDS block: a[c * kLdsLd + r]
constexpr int kSB = 32;

// One wave; lanes 0..31 own rows of the 32 x 32 sub-block at a (column
// stride kLdsLd).  FACTOR: Cholesky in place; then W = L^{-1} is written to
// the strictly upper part (a[r * ld + c] = W[r][c] for c < r) and dW.
// Value of v in lane `src` for the whole wave (v_readlane: no LDS round trip).
__device__ __forceinline__ float lane_bcast(float v, int src)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}
__device__ __forceinline__ double lane_bcast(double v, int src)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(u & 0xffffffffu), src);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), src);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <typename T, bool FACTOR>
__device__ __forceinline__ void chol_inv32(T *a, T *dW, int32_t *info, int grow)
{
    // Branch-free on lane-dependent conditions: every lane runs the same
    // instruction stream and masks with selects.
    const int lane = threadIdx.x & 63;
    const int r = lane & 31;
    T v[kSB], w[kSB];
#pragma clang loop unroll(full)
    for (int c = 0; c < kSB; ++c) {
        const T x = a[c * kLdsLd + r];
        v[c] = (c <= r) ? x : T(0);
    }
    if (FACTOR) {
        int firstbad = -1;   // wave-uniform: the pivot comes from v_readlane
#pragma clang loop unroll(full)
        for (int j = 0; j < kSB; ++j) {
            T piv = lane_bcast(v[j], j);
            if (firstbad < 0 && !(piv > T(0))) firstbad = j;
            piv = (piv > T(0)) ? piv : T(1);
            const T d = sqrt(piv);
            const T rd = T(1) / d;
            const T lj = (r == j) ? d : ((r > j) ? v[j] * rd : v[j]);
            v[j] = lj;
#pragma clang loop unroll(full)
            for (int c = 0; c < kSB; ++c) {
                if (c <= j) continue;
                const T lc = lane_bcast(lj, c);
                v[c] -= (r >= c) ? lj * lc : T(0);
            }
        }
        if (firstbad >= 0 && lane == 0 && *info == 0) *info = grow + firstbad + 1;
        if (lane < kSB) {
#pragma clang loop unroll(full)
            for (int c = 0; c < kSB; ++c)
                if (c <= r) a[c * kLdsLd + r] = v[c];
        }
    }
    // W = L^{-1}: rows of the identity eliminated top to bottom
#pragma clang loop unroll(full)
    for (int c = 0; c < kSB; ++c) w[c] = (c == r) ? T(1) : T(0);
#pragma clang loop unroll(full)
    for (int j = 0; j < kSB; ++j) {
        const T rjj = T(1) / lane_bcast(v[j], j);
        const T vj = v[j];
#pragma clang loop unroll(full)
        for (int c = 0; c < kSB; ++c) {
            if (c > j) continue;
            const T wc = (r == j) ? w[c] * rjj : w[c];   // row j is final after scaling
            const T wjc = lane_bcast(wc, j);
            w[c] = (r > j) ? wc - vj * wjc : wc;
        }
    }
    T wd = T(0);   // w[r] without a dynamic index (keeps w in registers)
#pragma clang loop unroll(full)
    for (int c = 0; c < kSB; ++c) wd = (c == r) ? w[c] : wd;
    if (lane < kSB) {
#pragma clang loop unroll(full)
        for (int c = 0; c < kSB; ++c)
            if (c < r) a[r * kLdsLd + c] = w[c];
        dW[r] = wd;
    }
}

// W_ss[c][t] for the sub-block inverse stored by chol_inv32 (t <= c)
template <typename T>
__device__ __forceinline__ T wsub(const T *a, const T *dW, int s0, int c, int t)
{
    return t == c ? dW[s0 + c] : a[(s0 + c) * kLdsLd + (s0 + t)];
}

template <typename T, bool FACTOR>
__global__ __launch_bounds__(256) void diag_kernel(T *__restrict__ A, int64_t lda, T *__restrict__ W,
                                                   int32_t *__restrict__ info, int k0)
{
    extern __shared__ unsigned char smem_raw[];
    T *a = reinterpret_cast<T *>(smem_raw);   // a[c * kLdsLd + r]
    T *dW = a + kNB * kLdsLd;                 // 128 diagonal entries of the sub-block inverses
    T *tmp = dW + kNB;                        // 32 x 33 scratch
    const int tid = threadIdx.x, wave = tid >> 6;

    for (int idx = tid; idx < kNB * kNB; idx += 256) {
        const int r = idx % kNB, c = idx / kNB;
        a[c * kLdsLd + r] = (c <= r) ? A[r + (int64_t)c * lda] : T(0);
    }
    __syncthreads();

    for (int s = 0; s < kNB / kSB; ++s) {
        const int s0 = s * kSB;
        if (wave == 0) chol_inv32<T, FACTOR>(a + s0 * kLdsLd + s0, dW + s0, info, k0 + s0);
        __syncthreads();
        if (!FACTOR) continue;
        const int r0 = s0 + kSB, nr = kNB - r0;
        if (nr == 0) break;
        // rows below: X[r][c] = sum_{t<=c} A[r][s0+t] W_ss[c][t]  (fixed trip
        // count, masked coefficients)
        constexpr int kMaxOut = (kNB - kSB) * kSB / 256;   // 12
        T x[kMaxOut];
#pragma unroll
        for (int q = 0; q < kMaxOut; ++q) {
            const int idx = tid + 256 * q;
            const bool on = idx < nr * kSB;
            const int r = r0 + (on ? idx % nr : 0), c = on ? idx / nr : 0;
            const T dwc = dW[s0 + c];
            T acc = T(0);
#pragma unroll 8
            for (int t = 0; t < kSB; ++t) {
                const T wct = a[(s0 + c) * kLdsLd + (s0 + t)];   // W_ss[c][t] for t < c
                const T coef = (t < c) ? wct : ((t == c) ? dwc : T(0));
                acc += a[(s0 + t) * kLdsLd + r] * coef;
            }
            x[q] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kMaxOut; ++q) {
            const int idx = tid + 256 * q;
            if (idx < nr * kSB) {
                const int r = r0 + idx % nr, c = idx / nr;
                a[(s0 + c) * kLdsLd + r] = x[q];
            }
        }
        __syncthreads();
        // trailing update of the lower part, 2 x 2 outputs per work item
        const int nb2 = nr / 2;
        for (int idx = tid; idx < nb2 * nb2; idx += 256) {
            const int bi = idx % nb2, bj = idx / nb2;
            if (bj > bi) continue;
            const int r = r0 + 2 * bi, c = r0 + 2 * bj;
            T c00 = 0, c01 = 0, c10 = 0, c11 = 0;
            for (int t = 0; t < kSB; ++t) {
                const T* col = a + (s0 + t) * kLdsLd;
                const T xr0 = col[r], xr1 = col[r + 1], xc0 = col[c], xc1 = col[c + 1];
                c00 += xr0 * xc0;
                c01 += xr0 * xc1;
                c10 += xr1 * xc0;
                c11 += xr1 * xc1;
            }
            a[c * kLdsLd + r] -= c00;
            a[c * kLdsLd + r + 1] -= c10;
            if (c + 1 <= r) a[(c + 1) * kLdsLd + r] -= c01;
            a[(c + 1) * kLdsLd + r + 1] -= c11;
        }
        __syncthreads();
    }
    if (FACTOR) {
        for (int idx = tid; idx < kNB * kNB; idx += 256) {
            const int r = idx % kNB, c = idx / kNB;
            if (c <= r) A[r + (int64_t)c * lda] = a[c * kLdsLd + r];
        }
    }
    // Sub-block inverses complete in LDS: W_ss[c][t] = a[(s0+c)*ld + s0+t]
    // for t <= c (the L diagonal, already written back, is overwritten).
    __syncthreads();
    if (tid < kNB) a[tid * kLdsLd + tid] = dW[tid];
    __syncthreads();
    // blocked inverse in place (off-diagonal sub-blocks, columns left to right)
    for (int s = 0; s < kNB / kSB - 1; ++s) {
        const int s0 = s * kSB;
        for (int rb = s + 1; rb < kNB / kSB; ++rb) {
            const int q0 = rb * kSB;
            // tmp = sum_{t=s}^{rb-1} L[rb][t] W[t][s]
            for (int idx = tid; idx < kSB * kSB; idx += 256) {
                const int i = idx % kSB, j = idx / kSB;
                T acc = T(0);
#pragma unroll 8
                for (int u = 0; u < kSB; ++u) {   // t = s: W_ss lower triangular
                    const T wuj = a[(s0 + u) * kLdsLd + s0 + j];
                    acc += a[(s0 + u) * kLdsLd + q0 + i] * (u >= j ? wuj : T(0));
                }
                for (int tb = s + 1; tb < rb; ++tb) {
#pragma unroll 8
                    for (int u = 0; u < kSB; ++u)
                        acc += a[(tb * kSB + u) * kLdsLd + q0 + i] * a[(s0 + j) * kLdsLd + tb * kSB + u];
                }
                tmp[j * (kSB + 1) + i] = acc;
            }
            __syncthreads();
            // W[rb][s] = -W_rr tmp
            for (int idx = tid; idx < kSB * kSB; idx += 256) {
                const int i = idx % kSB, j = idx / kSB;
                T acc = T(0);
#pragma unroll 8
                for (int u = 0; u < kSB; ++u) {
                    const T wiu = a[(q0 + i) * kLdsLd + q0 + u];
                    acc += (u <= i ? wiu : T(0)) * tmp[j * (kSB + 1) + u];
                }
                a[(s0 + j) * kLdsLd + q0 + i] = -acc;
            }
            __syncthreads();
        }
    }
    // diagonal sub-blocks (stored transposed) and the zero upper triangle
    for (int idx = tid; idx < kNB * kNB; idx += 256) {
        const int r = idx % kNB, c = idx / kNB;
        const T lo_part = a[c * kLdsLd + r], diag_part = a[r * kLdsLd + c];
        const bool same = (r / kSB) == (c / kSB);
        W[r + c * kNB] = (c > r) ? T(0) : (same ? diag_part : lo_part);
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
// host drivers
// ------------------------------------------------------------------------
static size_t diag_smem_bytes(size_t es) { return (size_t)(kNB * kLdsLd + kNB + kSB * (kSB + 1)) * es; }
static size_t elem_size(int dtype) { return dtype == GBEM_F64 ? 8 : 4; }

size_t chol_winv_bytes(int dtype, int64_t npad) { return (size_t)npad * kNB * elem_size(dtype); }
size_t chol_panel_bytes(int dtype, int64_t npad) { return (size_t)npad * kNB * elem_size(dtype); }
size_t chol_panel16_bytes(int dtype, int64_t npad)
{
    return (dtype == GBEM_F16 || dtype == GBEM_BF16) ? (size_t)npad * kNB * 2 : 0;
}

template <typename T>
static hipError_t factor_t(int dtype, int64_t npad, T *A, int64_t lda, T *Winv, T *Pw, void *P16,
                           int32_t *info, hipStream_t s, Prof *prof)
{
    const double es = (double)sizeof(T);
    const double eo = (dtype == GBEM_F16 || dtype == GBEM_BF16) ? 2.0 : es;   // trailing-update operand size
    const int nb = (int)(npad / kNB);
    const size_t smem = diag_smem_bytes(sizeof(T));
    hipError_t e = hipFuncSetAttribute((const void *)diag_kernel<T, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    for (int k = 0; k < nb; ++k) {
        const int64_t k0 = (int64_t)k * kNB;
        T *Akk = A + k0 + k0 * lda;
        int tok = prof ? prof->start(s) : -1;
        hipLaunchKernelGGL((diag_kernel<T, true>), dim3(1), dim3(256), smem, s, Akk, lda,
                           Winv + (int64_t)k * kNB * kNB, info, (int)k0);
        if (prof) prof->stop(tok, GBEM_K_DIAG, 2.0 * kNB * kNB * kNB / 3.0, 3.0 * kNB * kNB * es, s);
        const int64_t m = npad - k0 - kNB;
        if (m == 0) break;
        const int tm = (int)(m / kBM);
        T *Pan = A + (k0 + kNB) + k0 * lda;
        // panel <- A_panel W_k^T
        tok = prof ? prof->start(s) : -1;
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
        if (prof)
            prof->stop(tok, GBEM_K_TRSM, 2.0 * m * kNB * kNB,
                       (double)m * kNB * (3.0 * es + (eo < es ? eo : 0.0)) + kNB * kNB * es, s, 2);
        T *Trail = A + (k0 + kNB) + (k0 + kNB) * lda;
        const int64_t ntiles = (int64_t)tm * (tm + 1) / 2;
        tok = prof ? prof->start(s) : -1;
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
        if (prof) {
            const double tile_el = (double)ntiles * kBM * kBM;
            prof->stop(tok, GBEM_K_SYRK, 2.0 * tile_el * kNB, 2.0 * tile_el * es + (double)m * kNB * eo, s);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t chol_factor(int dtype, int64_t npad, void *A, int64_t lda, void *Winv, void *panel,
                       void *panel16, int32_t *info, hipStream_t s, Prof *prof)
{
    if (npad % kNB) return hipErrorInvalidValue;
    if (dtype == GBEM_F64)
        return factor_t<double>(dtype, npad, (double *)A, lda, (double *)Winv, (double *)panel,
                                nullptr, info, s, prof);
    return factor_t<float>(dtype, npad, (float *)A, lda, (float *)Winv, (float *)panel, panel16,
                           info, s, prof);
}

template <typename T>
static hipError_t diag_inverses_t(int64_t npad, const T *L, int64_t lda, T *Winv, hipStream_t s)
{
    const size_t smem = diag_smem_bytes(sizeof(T));
    hipError_t e = hipFuncSetAttribute((const void *)diag_kernel<T, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    for (int64_t k0 = 0; k0 < npad; k0 += kNB)
        hipLaunchKernelGGL((diag_kernel<T, false>), dim3(1), dim3(256), smem, s,
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

}  // namespace gbem
