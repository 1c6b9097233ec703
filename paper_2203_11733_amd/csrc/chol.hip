// Blocked right-looking Cholesky A = L L^T.
//
// A is symmetric positive definite (section 3.2, Theorem 1), so the paper
// solves A X = B by Cholesky.  Matrices here are column-major, lower triangle
// referenced, order npad (a multiple of the outer panel width, padded with
// an identity block).  Outer panels of ow = 256 or 512 columns (the wider
// panels halve the trailing matrix's read-modify-write traffic and pay off
// once the trailing updates outweigh the panel work), each made of
// 128-wide column blocks j:
//   diag_kernel / diag_block: L_jj = chol(A_jj) and W_j = L_jj^{-1} in LDS
//     (W_j is kept: the panel solves and the triangular solves use it)
//   panel_step_kernel j: update of column block j by blocks 0..j-1 of the
//     panel, panel solve X = A W_j^T in place (MFMA), and the next diagonal
//     block
//   outer update of the columns beyond the panel, A -= X X^T over lower tiles
//     (MFMA), with one panel of look-ahead on a second stream
// dtype F64: FP64 storage, v_mfma_f64_16x16x4; F32: FP32 storage,
// v_mfma_f32_16x16x4f32; F16/BF16: FP32 storage and FP32 panel work, the
// outer update on v_mfma_f32_16x16x32_{f16,bf16} with FP32 accumulation from a
// 16-bit row-major copy of the panel.
#include "gbem_internal.h"

#include <atomic>
#include <cstdlib>
#include <type_traits>

namespace gbem {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef unsigned int u4_t __attribute__((ext_vector_type(4)));   // 16-byte chunk

// ------------------------------------------------------------------------
// MFMA 16x16x4 (f64 / f32) with its output layout.  Operand fragments: lane l
// supplies A[l % 16][k = l / 16] and B[k = l / 16][l % 16].  Output: lane l,
// register q holds column l % 16 and row row(l, q); the f64 instruction
// interleaves the rows (l / 16 + 4 q), the f32 one keeps four consecutive rows
// per lane (4 (l / 16) + q).
// ------------------------------------------------------------------------
template <typename T> struct Mfma4;
template <> struct Mfma4<double> {
    typedef d4_t acc_t;
    static constexpr bool kConsecutiveRows = false;
    static __device__ __forceinline__ int row(int lane, int q) { return (lane >> 4) + 4 * q; }
    static __device__ __forceinline__ acc_t run(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma4<float> {
    typedef f4_t acc_t;
    static constexpr bool kConsecutiveRows = true;
    static __device__ __forceinline__ int row(int lane, int q) { return 4 * (lane >> 4) + q; }
    static __device__ __forceinline__ acc_t run(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// ------------------------------------------------------------------------
// Step 1: Cholesky of the 128 x 128 diagonal block and its inverse, one
// workgroup, everything in LDS.  The lower triangle is held as 36 blocks of
// 16 x 16 (column-major, 256 elements each, block (R, S) at R (R + 1) / 2 + S).
// Column of blocks s:
//   a. one wave factors the 16 x 16 diagonal block ("leaf") and inverts it;
//      lanes own rows, values move between lanes with DPP row broadcasts
//   b. the blocks below are solved against it: X_Rs = A_Rs W_ss^T (MFMA)
//   c. the trailing blocks are updated, A_RT -= X_Rs X_Ts^T (MFMA); wave 0
//      updates the next diagonal block first and goes on to factor it while
//      the other waves finish the update
// The inverse W = L^{-1} is then built block row by block row:
//   W_rs = -W_rr (L_rs W_ss + sum_{s<t<r} L_rt W_ts),
// all columns s of a block row at once, in place of L_rs.
// ------------------------------------------------------------------------
constexpr int kLB = 16;                          // leaf block
constexpr int kNL = kNB / kLB;                   // 8 block rows
constexpr int kNBlk = kNL * (kNL + 1) / 2;       // 36 lower blocks
__device__ __forceinline__ int blk(int R, int S) { return (R * (R + 1) / 2 + S) * (kLB * kLB); }

// value of v in lane c of this lane's row of 16 (DPP row_newbcast)
template <typename T>
__device__ __forceinline__ T rowbc(T v, int c)
{
    switch (c) {
    case 0: return __builtin_amdgcn_mov_dpp(v, 0x150, 0xF, 0xF, true);
    case 1: return __builtin_amdgcn_mov_dpp(v, 0x151, 0xF, 0xF, true);
    case 2: return __builtin_amdgcn_mov_dpp(v, 0x152, 0xF, 0xF, true);
    case 3: return __builtin_amdgcn_mov_dpp(v, 0x153, 0xF, 0xF, true);
    case 4: return __builtin_amdgcn_mov_dpp(v, 0x154, 0xF, 0xF, true);
    case 5: return __builtin_amdgcn_mov_dpp(v, 0x155, 0xF, 0xF, true);
    case 6: return __builtin_amdgcn_mov_dpp(v, 0x156, 0xF, 0xF, true);
    case 7: return __builtin_amdgcn_mov_dpp(v, 0x157, 0xF, 0xF, true);
    case 8: return __builtin_amdgcn_mov_dpp(v, 0x158, 0xF, 0xF, true);
    case 9: return __builtin_amdgcn_mov_dpp(v, 0x159, 0xF, 0xF, true);
    case 10: return __builtin_amdgcn_mov_dpp(v, 0x15A, 0xF, 0xF, true);
    case 11: return __builtin_amdgcn_mov_dpp(v, 0x15B, 0xF, 0xF, true);
    case 12: return __builtin_amdgcn_mov_dpp(v, 0x15C, 0xF, 0xF, true);
    case 13: return __builtin_amdgcn_mov_dpp(v, 0x15D, 0xF, 0xF, true);
    case 14: return __builtin_amdgcn_mov_dpp(v, 0x15E, 0xF, 0xF, true);
    default: return __builtin_amdgcn_mov_dpp(v, 0x15F, 0xF, 0xF, true);
    }
}

// Sum of x over the four 16-lane row groups of the wave, in every group
// (v_permlane16_swap exchanges rows 0 <-> 1 and 2 <-> 3 of two registers,
// v_permlane32_swap the two halves; both sums are formed in the same order in
// every group, so all groups hold the same value).
__device__ __forceinline__ float group_sum(float x)
{
    const unsigned u = __builtin_bit_cast(unsigned, x);
    const auto p = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    const float y = __builtin_bit_cast(float, (unsigned)p[0]) + __builtin_bit_cast(float, (unsigned)p[1]);
    const unsigned v = __builtin_bit_cast(unsigned, y);
    const auto q = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return __builtin_bit_cast(float, (unsigned)q[0]) + __builtin_bit_cast(float, (unsigned)q[1]);
}

// FP32 leaf factorisation and inverse with the work split over the four row
// groups of the wave (lane = 16 g + r; group g owns the columns c = 4 k + g):
// column c is the input column minus sum_{t<c} L_rt L_ct, each group summing
// its own columns t and the groups' sums added with group_sum (left-looking),
// then scaled by the pivot taken inside the owning group.  The substitution
// for W = L^{-1} likewise updates W's columns 4 k + g in group g, with column
// c of L sent to every group.  About 20 % faster than the replicated leaf
// below on gfx950 (3.8 vs 4.8 thousand cycles); the FP64 leaf stays
// replicated (its 64-bit swaps and divisions make the split version slower).
__device__ __forceinline__ void leaf16_split(float *Lb, float *Wb, int32_t *info, int grow)
{
    typedef float T;
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    T a[4], l[4], w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        a[k] = Lb[(4 * k + g) * kLB + r];
        l[k] = T(0);
        w[k] = (4 * k + g == r) ? T(1) : T(0);
    }
    int firstbad = -1;
    T rr = T(0);
#pragma clang loop unroll(full)
    for (int c = 0; c < kLB; ++c) {
        const int gc = c & 3, kc = c >> 2;
        T x = T(0);
#pragma unroll
        for (int k = 0; k < (c + 3) / 4; ++k) x += l[k] * rowbc(l[k], c);   // columns not yet done hold 0
        const T y = a[kc] - group_sum(x);   // column c after its updates (group gc)
        T piv = rowbc(y, c);
        const bool bad = !(piv > T(0));
        firstbad = (firstbad < 0 && bad && g == gc) ? c : firstbad;
        piv = bad ? T(1) : piv;
        const T rdc = __builtin_amdgcn_rsqf(piv);   // refined in FP64 later: hardware rsq (~1 ulp)
        const T d = piv * rdc;
        const T lc = r > c ? y * rdc : (r == c ? d : T(0));
        if (g == gc) l[kc] = lc;
        // substitution step c: rows below c subtract L_rc / L_cc times row c
        const T lr = group_sum(g == gc ? lc : T(0));   // column c in every group
        const T inv = __builtin_amdgcn_rcpf(rowbc(lr, c));
        rr = r == c ? inv : rr;
        const T coef = r > c ? lr * inv : T(0);
#pragma unroll
        for (int k = 0; k <= c / 4; ++k) w[k] -= coef * rowbc(w[k], c);
    }
    // first non-positive pivot over the four groups
    int fb = -1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int f = __builtin_amdgcn_readlane(firstbad, 16 * q);
        fb = (f >= 0 && (fb < 0 || f < fb)) ? f : fb;
    }
    if (fb >= 0 && lane == 0 && *info == 0) *info = grow + fb + 1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        Lb[(4 * k + g) * kLB + r] = l[k];
        Wb[(4 * k + g) * kLB + r] = w[k] * rr;
    }
}

// One wave; lane r (mod 16) owns row r of the 16 x 16 block Lb (column-major,
// lower triangle valid).  FACTOR: Cholesky in place (upper part written as
// zero).  Then Wb = L^{-1} (lower, zero above).  Branch-free on lane-dependent
// values: the rows of 16 lanes hold identical copies.
template <typename T, bool FACTOR>
__device__ __forceinline__ void leaf16(T *Lb, T *Wb, int32_t *info, int grow)
{
    if constexpr (FACTOR && sizeof(T) == 4) {
        leaf16_split(Lb, Wb, info, grow);
        return;
    }
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    T v[kLB], rd[kLB];
#pragma clang loop unroll(full)
    for (int c = 0; c < kLB; ++c) v[c] = Lb[c * kLB + r];
    if (FACTOR) {
        int firstbad = -1;
#pragma clang loop unroll(full)
        for (int j = 0; j < kLB; ++j) {
            T piv = rowbc(v[j], j);
            firstbad = (firstbad < 0 && !(piv > T(0))) ? j : firstbad;
            piv = (piv > T(0)) ? piv : T(1);
            T d;
            if constexpr (sizeof(T) == 4) {   // FP32 factors are refined in FP64: hardware rsq (~1 ulp)
                rd[j] = __builtin_amdgcn_rsqf(piv);
                d = piv * rd[j];
            } else {
                d = sqrt(piv);
                rd[j] = T(1) / d;
            }
            const T lj = (r == j) ? d : v[j] * rd[j];   // rows above j: unused
            v[j] = lj;
#pragma clang loop unroll(full)
            for (int c = j + 1; c < kLB; ++c) v[c] -= lj * rowbc(lj, c);
        }
        if (firstbad >= 0 && lane == 0 && *info == 0) *info = grow + firstbad + 1;
    } else {
#pragma clang loop unroll(full)
        for (int j = 0; j < kLB; ++j) {
            if constexpr (sizeof(T) == 4) rd[j] = __builtin_amdgcn_rcpf(rowbc(v[j], j));
            else rd[j] = T(1) / rowbc(v[j], j);
        }
    }
    // W = L^{-1}: row j of W is (raw row j) / L_jj; rows below subtract
    // L_rj / L_jj times the raw row j.
    T w[kLB];
#pragma clang loop unroll(full)
    for (int c = 0; c < kLB; ++c) w[c] = (c == r) ? T(1) : T(0);
#pragma clang loop unroll(full)
    for (int j = 0; j < kLB; ++j) {
        const T coef = (r > j) ? v[j] * rd[j] : T(0);
#pragma clang loop unroll(full)
        for (int c = 0; c <= j; ++c) w[c] -= coef * rowbc(w[c], j);
    }
    T rr = T(0);
#pragma clang loop unroll(full)
    for (int j = 0; j < kLB; ++j) rr = (r == j) ? rd[j] : rr;
    if (lane < kLB) {
#pragma clang loop unroll(full)
        for (int c = 0; c < kLB; ++c) {
            if (FACTOR) Lb[c * kLB + r] = (c <= r) ? v[c] : T(0);
            Wb[c * kLB + r] = w[c] * rr;
        }
    }
}

// acc (16 x 16, MFMA output layout, transposed: see bstore) += op(P) op(Q),
// op(P) = TA ? P^T : P, op(Q) = TB ? Q^T : Q; P, Q 16 x 16 column-major in
// LDS.  The MFMA computes the transposed product (operands swapped) so that
// lane l's outputs lie in row l % 16: stores are contiguous.
template <typename T, bool TA, bool TB>
__device__ __forceinline__ void bmm(typename Mfma4<T>::acc_t &acc, const T *P, const T *Q, int lane)
{
    const int i = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int k0 = 0; k0 < kLB; k0 += 4) {
        const int k = k0 + kq;
        const T qa = TB ? Q[k * kLB + i] : Q[i * kLB + k];   // op(Q)[k][i]
        const T pb = TA ? P[i * kLB + k] : P[k * kLB + i];   // op(P)[i][k]
        acc = Mfma4<T>::run(qa, pb, acc);
    }
}
// element (row, col) of the block held by lane l, register q
template <typename T>
__device__ __forceinline__ int bidx(int lane, int q) { return Mfma4<T>::row(lane, q) * kLB + (lane & 15); }

// One 128 x 128 diagonal block by the whole workgroup (256 threads); lds:
// diag_smem_bytes(sizeof(T)) bytes of LDS.
template <typename T, bool FACTOR>
__device__ __forceinline__ void diag_block(T *__restrict__ A, int64_t lda, T *__restrict__ W,
                                           int32_t *__restrict__ info, int k0, unsigned char *lds)
{
    typedef typename Mfma4<T>::acc_t acc_t;
    T *L = reinterpret_cast<T *>(lds);           // 36 blocks
    T *Wd = L + kNBlk * kLB * kLB;               // 8 diagonal inverse blocks
    T *Tw = Wd + kNL * kLB * kLB;                // one 16 x 16 scratch block per wave
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    // load the lower blocks: thread = column c, 64 rows h*64.., 16-byte chunks
    constexpr int VE = 16 / sizeof(T);           // elements per chunk
    constexpr int NCH = 64 / VE;                 // chunks per thread
    typedef u4_t v16_t;
    const int c = tid >> 1, h = tid & 1;
    const int cb = c / kLB;
    {
        v16_t buf[NCH];
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
            const int r0 = h * 64 + q * VE;
            if (r0 + VE - 1 >= cb * kLB) buf[q] = *reinterpret_cast<const v16_t *>(A + r0 + (int64_t)c * lda);
        }
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
            const int r0 = h * 64 + q * VE;
            const int rb = r0 / kLB;
            if (rb < cb) continue;
            T *dst = L + blk(rb, cb) + (c % kLB) * kLB + (r0 % kLB);
            if (rb > cb || r0 >= c) {
                *reinterpret_cast<v16_t *>(dst) = buf[q];
            } else {
                // zero the rows above the diagonal with a bit mask on the whole chunk
                u4_t m;
#pragma unroll
                for (int e = 0; e < 4; ++e) m[e] = (r0 + e * 4 / (int)sizeof(T) >= c) ? ~0u : 0u;
                *reinterpret_cast<v16_t *>(dst) = buf[q] & m;
            }
        }
    }
    __syncthreads();

    if (FACTOR) {
        if (wave == 0) leaf16<T, true>(L + blk(0, 0), Wd, info, k0);
        __syncthreads();
        for (int s = 0; s + 1 < kNL; ++s) {
            // b. X_Rs = A_Rs W_ss^T
            for (int R = s + 1 + wave; R < kNL; R += 4) {
                acc_t acc = acc_t{0, 0, 0, 0};
                bmm<T, false, true>(acc, L + blk(R, s), Wd + s * kLB * kLB, lane);
                T *dst = L + blk(R, s);
#pragma unroll
                for (int q = 0; q < 4; ++q) dst[bidx<T>(lane, q)] = acc[q];
            }
            __syncthreads();
            // c. A_RT -= X_Rs X_Ts^T; wave 0: next diagonal block, then its leaf
            if (wave == 0) {
                acc_t acc = acc_t{0, 0, 0, 0};
                const T *X = L + blk(s + 1, s);
                bmm<T, false, true>(acc, X, X, lane);
                T *dst = L + blk(s + 1, s + 1);
#pragma unroll
                for (int q = 0; q < 4; ++q) dst[bidx<T>(lane, q)] -= acc[q];
                __builtin_amdgcn_wave_barrier();
                leaf16<T, true>(L + blk(s + 1, s + 1), Wd + (s + 1) * kLB * kLB, info, k0 + (s + 1) * kLB);
            } else {
                const int n = kNL - 1 - s;                 // trailing block rows
                int idx = 0;
                for (int R = s + 1; R < kNL; ++R)
                    for (int T2 = s + 1; T2 <= R; ++T2) {
                        if (R == s + 1 && T2 == s + 1) continue;
                        if (idx++ % 3 != wave - 1) continue;
                        acc_t acc = acc_t{0, 0, 0, 0};
                        bmm<T, false, true>(acc, L + blk(R, s), L + blk(T2, s), lane);
                        T *dst = L + blk(R, T2);
#pragma unroll
                        for (int q = 0; q < 4; ++q) dst[bidx<T>(lane, q)] -= acc[q];
                    }
                (void)n;
            }
            __syncthreads();
        }
        // L back to global memory, lower triangle only
        for (int q = 0; q < NCH; ++q) {
            const int r0 = h * 64 + q * VE;
            const int rb = r0 / kLB;
            if (rb < cb || r0 + VE - 1 < c) continue;
            const T *src = L + blk(rb, cb) + (c % kLB) * kLB + (r0 % kLB);
            T *dst = A + r0 + (int64_t)c * lda;
            if (r0 >= c) {
                *reinterpret_cast<v16_t *>(dst) = *reinterpret_cast<const v16_t *>(src);
            } else {
#pragma unroll
                for (int u = 0; u < VE; ++u)
                    if (r0 + u >= c) dst[u] = src[u];
            }
        }
    } else {
        // inverses of the given diagonal blocks, two per wave
        leaf16<T, false>(L + blk(wave, wave), Wd + wave * kLB * kLB, nullptr, 0);
        leaf16<T, false>(L + blk(wave + 4, wave + 4), Wd + (wave + 4) * kLB * kLB, nullptr, 0);
        __syncthreads();
    }

    // inverse, block row by block row; wave w takes the columns s = w, w + 4
    for (int r = 1; r < kNL; ++r) {
        acc_t res[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int s = wave + 4 * u;
            res[u] = acc_t{0, 0, 0, 0};
            if (s >= r) continue;
            acc_t acc = acc_t{0, 0, 0, 0};
            bmm<T, false, false>(acc, L + blk(r, s), Wd + s * kLB * kLB, lane);
            for (int t = s + 1; t < r; ++t) bmm<T, false, false>(acc, L + blk(r, t), L + blk(t, s), lane);
            T *tw = Tw + wave * kLB * kLB;
#pragma unroll
            for (int q = 0; q < 4; ++q) tw[bidx<T>(lane, q)] = acc[q];
            __builtin_amdgcn_wave_barrier();
            bmm<T, false, false>(res[u], Wd + r * kLB * kLB, tw, lane);
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int s = wave + 4 * u;
            if (s >= r) continue;
            T *dst = L + blk(r, s);
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[bidx<T>(lane, q)] = -res[u][q];
        }
        __syncthreads();
    }

    // W (128 x 128, column-major, ld 128), zero above the diagonal
    for (int q = 0; q < NCH; ++q) {
        const int r0 = h * 64 + q * VE;
        const int rb = r0 / kLB;
        v16_t out = v16_t{0, 0, 0, 0};
        if (rb >= cb) {
            const T *src = (rb == cb ? Wd + cb * kLB * kLB : L + blk(rb, cb)) + (c % kLB) * kLB + (r0 % kLB);
            out = *reinterpret_cast<const v16_t *>(src);
        }
        *reinterpret_cast<v16_t *>(W + r0 + (int64_t)c * kNB) = out;
    }
}

template <typename T, bool FACTOR>
__global__ __launch_bounds__(256) void diag_kernel(T *__restrict__ A, int64_t lda, T *__restrict__ W,
                                                   int32_t *__restrict__ info, int k0)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    // several independent blocks (inverse only): block b of the grid
    diag_block<T, FACTOR>(A + (int64_t)blockIdx.x * kNB * (lda + 1), lda, W + (int64_t)blockIdx.x * kNB * kNB, info,
                          k0 + blockIdx.x * kNB, smem_raw);
}

// ------------------------------------------------------------------------
// GEMM on 128 x 128 tiles: C -= A B^T (SUB) or C = A B^T, with A (M x K) and
// B (N x K) column-major (rows contiguous).  256 threads = 4 waves of 64 x 64,
// each 4 x 4 MFMA 16x16x4 blocks (f64 or f32).  K runs in chunks of 16 through
// two LDS buffers; the next chunk is loaded into registers (16-byte loads)
// while the MFMAs work on the current one.
// Tiles: kTri = lower triangle of a square tile grid (linear index); kRect =
// tm x tn grid.  MASK: the C origin lies on the matrix diagonal; tiles above
// it are skipped and diagonal tiles keep rows >= columns only.
// A may alias C (the in-place panel solve): a tile reads all of its A rows
// before its epilogue writes them, and no other tile touches those rows.
// ------------------------------------------------------------------------
constexpr int kBM = 128, kBK = 16;
// outer panel width for a matrix of order npad
// (measured on the MI355X in mixed mode: 512 wins from order ~16k up, e.g.
// 26.7 vs 28.2 ms at 20k panels; 256 below, where the panel chain dominates)
// (the autotuner's cache may move the threshold: chol_shape in tune.cpp)
static int outer_width(int dtype, int64_t npad) { return chol_shape(dtype, npad).outer_width; }
constexpr int kLdsLd = kBM + 16;   // LDS row stride: the four k-rows of a fragment load hit distinct banks
constexpr int kRect = 0, kTri = 1;

// Workgroup b -> tile (I, J).  Workgroups are handed to the 8 XCDs in turn
// (b % 8); each XCD gets a contiguous range of the tile order, so the tiles it
// runs at the same time share operand rows in its L2.  kTri orders the lower
// triangle in groups of 8 tile rows: within a group, column by column, so a
// window of consecutive tiles touches about 8 row blocks of each operand.
__device__ __forceinline__ int64_t tri_group_start(int64_t g) { return 32 * g * (g - 1) + 36 * g; }

__device__ __forceinline__ void tile_of(int64_t b, int mode, int tm, int &I, int &J)
{
    if (mode == kTri) {
        const int64_t n = (int64_t)tm * (tm + 1) / 2, q = n / 8, r = n % 8, x = b % 8, k = b / 8;
        const int64_t v = (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
        int64_t g = v > 0 ? (int64_t)((sqrt(16.0 + 128.0 * (double)v) - 4.0) / 64.0) : 0;
        while (g > 0 && tri_group_start(g) > v) --g;
        while (8 * (g + 1) < tm && tri_group_start(g + 1) <= v) ++g;
        const int I0 = (int)(8 * g), Gg = min(8, tm - I0);
        int64_t w = v - tri_group_start(g);
        if (w < (int64_t)I0 * Gg) {
            I = I0 + (int)(w % Gg);
            J = (int)(w / Gg);
            return;
        }
        w -= (int64_t)I0 * Gg;
        int c = I0;
        while (w >= I0 + Gg - c) {
            w -= I0 + Gg - c;
            ++c;
        }
        I = c + (int)w;
        J = c;
    } else {
        I = (int)(b % tm);
        J = (int)(b / tm);
    }
}

template <typename T>
static size_t gemm_smem_bytes() { return (size_t)2 * 2 * kBK * kLdsLd * sizeof(T); }

// Epilogue: the old C values a wave needs are read with all loads in flight
// at once (f32: prefetched before the K loop; f64: two batches), never one
// read-modify-write at a time.  f64 runs the MFMA with the operands swapped
// (it produces C^T), so that lane l's outputs lie in row l % 16 and every
// access covers 16 consecutive rows.
// Q16 (f32 only; 1: bf16, 2: f16): the tile is also written, rounded to 16
// bits, row-major into Q (row stride qld): tile row R goes to Q row R + qrow
// (skipped below qmin), tile column c to Q column qcol + c.  The tile is
// transposed through LDS so that Q is written 16 bytes at a time.
// One 128 x 128 tile (I, J) by the whole workgroup; smem: gemm_smem_bytes<T>()
// bytes of LDS.  MASK: the tile lies on or below the diagonal of C's origin
// (I >= J), diagonal tiles keep rows >= columns.
template <typename T, bool MASK, bool SUB, int Q16 = 0>
__device__ __forceinline__ void gemm_tile(int I, int J, int K, const T *A, int64_t lda, const T *B, int64_t ldb,
                                          T *C, int64_t ldc, void *Q, int qrow, int qcol, unsigned char *smem_raw,
                                          int qld = 0, int qmin = 0)
{
    typedef typename Mfma4<T>::acc_t acc_t;
    constexpr int LD = kLdsLd;
    constexpr bool kF32 = Mfma4<T>::kConsecutiveRows;
    constexpr bool kOld = SUB || MASK;            // old C values needed
    T *lds = reinterpret_cast<T *>(smem_raw);   // [buf][operand][k][row]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const T *Ab = A + (int64_t)I * kBM;
    const T *Bb = B + (int64_t)J * kBM;
    const bool diag_tile = MASK && I == J;
    const int row0 = I * kBM + wm * 64, col0 = J * kBM + wn * 64;

    f4_t cpre[4][4];
    if constexpr (kF32 && kOld) {
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) {
                const int row = row0 + mi * 16 + 4 * (lane >> 4), col = col0 + ni * 16 + (lane & 15);
                cpre[mi][ni] = *reinterpret_cast<const f4_t *>(C + row + (int64_t)col * ldc);
            }
    }

    acc_t acc[4][4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = acc_t{0, 0, 0, 0};

    const int lk = tid >> 4, lr = (tid & 15) * 8;   // loader: column lk, rows lr..lr+7
    typedef u4_t v16_t;
    constexpr int NV = 8 * sizeof(T) / 16;          // 16-byte chunks per 8 elements
    v16_t ra[NV], rb[NV];
#define GEMM_LOAD(k0)                                                                                \
    do {                                                                                             \
        const v16_t *pa = reinterpret_cast<const v16_t *>(Ab + lr + (int64_t)((k0) + lk) * lda);     \
        const v16_t *pb = reinterpret_cast<const v16_t *>(Bb + lr + (int64_t)((k0) + lk) * ldb);     \
        _Pragma("unroll") for (int e = 0; e < NV; ++e)                                               \
        {                                                                                            \
            ra[e] = pa[e];                                                                           \
            rb[e] = pb[e];                                                                           \
        }                                                                                            \
    } while (0)
#define GEMM_STORE(buf)                                                                              \
    do {                                                                                             \
        v16_t *sa = reinterpret_cast<v16_t *>(lds + (((buf) * 2 + 0) * kBK + lk) * LD + lr);         \
        v16_t *sb = reinterpret_cast<v16_t *>(lds + (((buf) * 2 + 1) * kBK + lk) * LD + lr);         \
        _Pragma("unroll") for (int e = 0; e < NV; ++e)                                               \
        {                                                                                            \
            sa[e] = ra[e];                                                                           \
            sb[e] = rb[e];                                                                           \
        }                                                                                            \
    } while (0)
    const int nk = K / kBK;
    GEMM_LOAD(0);
    GEMM_STORE(0);
    __syncthreads();
    for (int kc = 0; kc < nk; ++kc) {
        if (kc + 1 < nk) GEMM_LOAD((kc + 1) * kBK);
        const T *As = lds + ((kc & 1) * 2 + 0) * kBK * LD;
        const T *Bs = lds + ((kc & 1) * 2 + 1) * kBK * LD;
#pragma unroll
        for (int kk = 0; kk < kBK; kk += 4) {
            T af[4], bf[4];
#pragma unroll
            for (int mi = 0; mi < 4; ++mi) af[mi] = As[(kk + (lane >> 4)) * LD + wm * 64 + mi * 16 + (lane & 15)];
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) bf[ni] = Bs[(kk + (lane >> 4)) * LD + wn * 64 + ni * 16 + (lane & 15)];
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
                    acc[mi][ni] = kF32 ? Mfma4<T>::run(af[mi], bf[ni], acc[mi][ni])
                                       : Mfma4<T>::run(bf[ni], af[mi], acc[mi][ni]);
        }
        if (kc + 1 < nk) GEMM_STORE((kc + 1) & 1);
        __syncthreads();
    }
#undef GEMM_LOAD
#undef GEMM_STORE

    if constexpr (kF32) {
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) {
                const int row = row0 + mi * 16 + 4 * (lane >> 4), col = col0 + ni * 16 + (lane & 15);
                f4_t v;
                if constexpr (kOld) v = cpre[mi][ni];
                else v = f4_t{0, 0, 0, 0};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float x = SUB ? v[q] - (float)acc[mi][ni][q] : (float)acc[mi][ni][q];
                    v[q] = (!diag_tile || row + q >= col) ? x : v[q];
                }
                *reinterpret_cast<f4_t *>(C + row + (int64_t)col * ldc) = v;
                if constexpr (Q16 != 0) {
                    typedef typename std::conditional<Q16 == 1, __bf16, _Float16>::type H;
                    H *t16 = reinterpret_cast<H *>(smem_raw);   // LDS is free after the K loop
                    const int rl = row - I * kBM, cl = col - J * kBM;
#pragma unroll
                    for (int q = 0; q < 4; ++q) t16[(rl + q) * (kBM + 8) + cl] = (H)v[q];
                }
            }
        if constexpr (Q16 != 0) {
            typedef typename std::conditional<Q16 == 1, __bf16, _Float16>::type H;
            const H *t16 = reinterpret_cast<const H *>(smem_raw);
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = tid + 256 * u, rl = idx >> 4, cc = (idx & 15) * 8;
                const int64_t qr = (int64_t)I * kBM + rl + qrow;
                if (qr >= qmin)
                    *reinterpret_cast<u4_t *>(reinterpret_cast<H *>(Q) + qr * qld + qcol + J * kBM + cc) =
                        *reinterpret_cast<const u4_t *>(t16 + rl * (kBM + 8) + cc);
            }
        }
    } else {
        // f64, C^T in the accumulators: row = row0 + mi*16 + lane%16,
        // col = col0 + ni*16 + row(lane, q)
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            T old[2][4][4];
            if constexpr (kOld) {
#pragma unroll
                for (int m2 = 0; m2 < 2; ++m2)
#pragma unroll
                    for (int ni = 0; ni < 4; ++ni)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int row = row0 + (half * 2 + m2) * 16 + (lane & 15);
                            const int col = col0 + ni * 16 + Mfma4<T>::row(lane, q);
                            old[m2][ni][q] = C[row + (int64_t)col * ldc];
                        }
            }
#pragma unroll
            for (int m2 = 0; m2 < 2; ++m2)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int mi = half * 2 + m2;
                        const int row = row0 + mi * 16 + (lane & 15);
                        const int col = col0 + ni * 16 + Mfma4<T>::row(lane, q);
                        if (diag_tile && row < col) continue;
                        const T a = acc[mi][ni][q];
                        C[row + (int64_t)col * ldc] = SUB ? old[m2][ni][q] - a : a;
                    }
        }
    }
}

template <typename T, int MODE, bool MASK, bool SUB, int Q16 = 0>
__global__ __launch_bounds__(256, 2) void gemm_kernel(int tm, int K, const T *A, int64_t lda, const T *B,
                                                   int64_t ldb, T *C, int64_t ldc, void *Q = nullptr, int qrow = 0,
                                                   int qcol = 0)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    int I, J;
    tile_of(blockIdx.x, MODE, tm, I, J);
    if (MASK && I < J) return;
    gemm_tile<T, MASK, SUB, Q16>(I, J, K, A, lda, B, ldb, C, ldc, Q, qrow, qcol, smem_raw);
}

// ------------------------------------------------------------------------
// Factorisation of one outer panel (ow columns from P0, ns = ow/128 column
// blocks) after its diagonal block 0 is factored, in one launch.  P = the
// panel's top-left corner; workgroup I owns row block q = I + 1 (rows
// 128 q ..) and walks the panel's columns j = 0 .. min(q, ns) - 1:
//   - j > 0: A[q, j] -= X[q, 0..j-1] X[j, 0..j-1]^T     (K = 128 j), once row
//     block j has published its columns 0..j-1;
//   - panel solve in place, X[q, j] = A[q, j] W_j^T    (W_j = L_jj^{-1}), once
//     W_j is published (W_0 comes from the launch before);
//   - q < ns (a diagonal block of the panel): after its columns it publishes
//     them, updates A[q, q] with them and factors it (L_qq, W_q), then
//     publishes W_q.
// So while one workgroup factors diagonal block q, the others already apply
// column q's update.  Row blocks are handed out by an atomic ticket in
// execution order, so a workgroup only ever waits for lower row blocks whose
// workgroups already run: every wait ends (also beside other kernels that
// hold CUs); each is bounded and sets the error word pf[0] instead of
// spinning on.  pf[2 ns + 1] is the ticket counter; the workgroup with the
// last ticket resets it for the next launch on the stream.  pf[1 + q] / pf[1 + ns + q]: "columns of
// row block q" / "W_q" flags, holding the launch's epoch when published
// (release after the stores, acquire after the flag: agent scope, since the
// workgroups sit on different XCDs).  For 16-bit trailing updates the solve
// also writes the 16-bit copy of the rows below the panel: row-major Q with
// row stride qld, panel row 128 q + r (q >= ns) to Q row 128 q + r - 128 ns +
// qoff, column block j to Q columns qcol0 + 128 j ...
// ------------------------------------------------------------------------
__device__ __forceinline__ bool panel_wait(const int32_t *flag, int32_t epoch, int32_t *err, int limit)
{
    __shared__ int ok;
    if (threadIdx.x == 0) {
        int n = 0;
        while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
            __builtin_amdgcn_s_sleep(2);
            if (++n > limit) break;
        }
        ok = n <= limit;
        if (!ok) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok;
}
__device__ __forceinline__ void panel_publish(int32_t *flag, int32_t epoch)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flag, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T, int Q16>
__global__ __launch_bounds__(256) void panel_kernel(T *P, int64_t lda, int ns, T *W, int32_t *info, int kn0, void *Q,
                                                    int qoff, int qcol0, int qld, int32_t *pf, int32_t epoch,
                                                    int limit)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    __shared__ int ticket;
    if (threadIdx.x == 0) {
        ticket = atomicAdd(pf + 2 * ns + 1, 1);
        if (ticket == (int)gridDim.x - 1) __hip_atomic_store(pf + 2 * ns + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (ticket < 0 || ticket >= (int)gridDim.x) {   // counter not reset: report, do nothing
        if (threadIdx.x == 0) __hip_atomic_store(pf, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const int q = ticket + 1;
    const int64_t r0 = (int64_t)kNB * q;   // first row of the block within the panel
    const int nc = min(q, ns);
    T *D = P + r0 + r0 * lda;   // diagonal block q (factored here when q < ns)
    // FP64: diagonal block q's update (K = 128 q, on one workgroup) is split so
    // that only its last column block follows W_{q-1} (C2, same GPU: 94.5 ->
    // 91.5 ms per extraction); FP32: one update after the loop (the split
    // measured 0.6 ms slower there)
    constexpr bool kSplitD = sizeof(T) == 8;
    for (int j = 0; j < nc; ++j) {
        T *C = P + r0 + (int64_t)kNB * j * lda;
        if (kSplitD && j > 0 && j == q - 1 && q < ns) {
            // the part of diagonal block q's update from column blocks 0..q-2
            // (final already), ahead of the waits for block q-1
            gemm_tile<T, true, true, 0>(0, 0, kNB * (q - 1), P + r0, lda, P + r0, lda, D, lda, nullptr, 0, 0,
                                        smem_raw);
            __syncthreads();
        }
        if (j > 0) {
            if (!panel_wait(pf + 1 + j, epoch, pf, limit)) return;
            gemm_tile<T, false, true, 0>(0, 0, kNB * j, P + r0, lda, P + (int64_t)kNB * j, lda, C, lda, nullptr, 0, 0,
                                         smem_raw);
            __syncthreads();   // this workgroup's updated block is complete and visible to it
            if (!panel_wait(pf + 1 + ns + j, epoch, pf, limit)) return;
        }
        gemm_tile<T, false, false, Q16>(0, 0, kNB, C, lda, W + (int64_t)kNB * j * kNB, kNB, C, lda, Q,
                                        (int)(r0 - kNB * ns) + qoff, qcol0 + kNB * j, smem_raw, qld, qoff);
        __syncthreads();
    }
    if (q >= ns) return;
    panel_publish(pf + 1 + q, epoch);   // columns 0..q-1 of row block q
    if (kSplitD && q >= 2) {   // the rest of the update: column block q-1
        const T *Pq = P + r0 + (int64_t)kNB * (q - 1) * lda;
        gemm_tile<T, true, true, 0>(0, 0, kNB, Pq, lda, Pq, lda, D, lda, nullptr, 0, 0, smem_raw);
    } else {
        gemm_tile<T, true, true, 0>(0, 0, kNB * q, P + r0, lda, P + r0, lda, D, lda, nullptr, 0, 0, smem_raw);
    }
    __syncthreads();
    diag_block<T, true>(D, lda, W + (int64_t)kNB * q * kNB, info, kn0 + kNB * q, smem_raw);
    panel_publish(pf + 1 + ns + q, epoch);   // W_q and L_qq
}

// ------------------------------------------------------------------------
// 16-bit outer trailing update: C (FP32, column-major) -= Q Q^T, Q stored
// row-major in 16 bits with K contiguous (Q[r * ldq + k]);
// v_mfma_f32_16x16x32_{bf16,f16}, FP32 accumulation.  Same tiling, modes and
// double-buffered K chunks (64) as gemm_kernel.
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

// LDS rows of a K chunk are 128 bytes (eight 16-byte pieces) without
// padding; piece p of row r is stored in place p ^ (r & 7).  The fragment
// reads (16 consecutive rows, one piece per lane group) then run without
// bank conflicts, which a 144-byte padded row stride does not achieve on
// gfx950 (measured 125 against 182 B/clk per CU); the loader's stores run at
// the same rate in both layouts.
constexpr int kBK16 = 64;
static size_t syrk16_smem_bytes() { return (size_t)2 * 2 * kBM * kBK16 * 2; }

// DIAG0: the launch that updates the next outer panel's columns (MODE
// kRect, C at that panel's diagonal) also factors the panel's first diagonal
// block: the workgroup of tile (0, 0) runs diag_block on it after its own
// update (W into Wd, pivot status into info, global row k0), so the
// factorisation overlaps the rest of the update instead of following it.
template <typename H, int MODE, int NK, bool DIAG0 = false>
__global__ __launch_bounds__(256) void syrk16_kernel(int tm, int K, const H *__restrict__ QA,
                                                     const H *__restrict__ QB, int64_t ldq,
                                                     float *__restrict__ C, int64_t ldc, float *Wd = nullptr,
                                                     int32_t *info = nullptr, int k0 = 0)
{
    typedef typename Mfma32<H>::frag_t frag_t;
    constexpr int LD = kBK16;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    H *lds = reinterpret_cast<H *>(smem_raw);   // [buf][operand][row][k]
    int I, J;
    tile_of(blockIdx.x, MODE, tm, I, J);
    if (I < J) return;                          // C origin on the diagonal in every use
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;

    f4_t acc[4][4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = f4_t{0, 0, 0, 0};

    // K = 64 NK in chunks of 64, fully unrolled.  Two register buffers keep
    // each chunk's loads two MFMA phases ahead of its use (one phase is far
    // shorter than the memory latency); the old C values are requested two
    // chunks before the end.  Loads complete in order, so C goes last.
    static_assert(NK >= 2 && NK % 2 == 0, "an even number of chunks");
    const int lr = tid >> 1, lk = (tid & 1) * 32;   // loader: row lr, k lk..lk+31 of a chunk
    u4_t r0[2][4], r1[2][4];                        // [operand][piece], even / odd chunks
#define S16_LOAD(R, c)                                                                               \
    do {                                                                                             \
        const u4_t *pa = reinterpret_cast<const u4_t *>(QA + (int64_t)(I * kBM + lr) * ldq + (c) * kBK16 + lk); \
        const u4_t *pb = reinterpret_cast<const u4_t *>(QB + (int64_t)(J * kBM + lr) * ldq + (c) * kBK16 + lk); \
        _Pragma("unroll") for (int e = 0; e < 4; ++e)                                                \
        {                                                                                            \
            R[0][e] = pa[e];                                                                         \
            R[1][e] = pb[e];                                                                         \
        }                                                                                            \
    } while (0)
#define S16_STORE(R, buf)                                                                            \
    do {                                                                                             \
        u4_t *sa = reinterpret_cast<u4_t *>(lds + (((buf) * 2 + 0) * kBM + lr) * LD);              \
        u4_t *sb = reinterpret_cast<u4_t *>(lds + (((buf) * 2 + 1) * kBM + lr) * LD);              \
        _Pragma("unroll") for (int e = 0; e < 4; ++e)                                                \
        {                                                                                            \
            sa[(lk / 8 + e) ^ (lr & 7)] = R[0][e];                                                   \
            sb[(lk / 8 + e) ^ (lr & 7)] = R[1][e];                                                   \
        }                                                                                            \
    } while (0)
    auto mma = [&](int buf) __attribute__((always_inline)) {
        const H *As = lds + (buf * 2 + 0) * kBM * LD;
        const H *Bs = lds + (buf * 2 + 1) * kBM * LD;
#pragma unroll
        for (int kk = 0; kk < kBK16; kk += 32) {
            frag_t af[4], bf[4];
            // row & 7 == lane & 7 for every fragment row
            const int pk = 8 * (((kk / 8) + (lane >> 4)) ^ (lane & 7));
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
                af[mi] = *reinterpret_cast<const frag_t *>(As + (wm * 64 + mi * 16 + (lane & 15)) * LD + pk);
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
                bf[ni] = *reinterpret_cast<const frag_t *>(Bs + (wn * 64 + ni * 16 + (lane & 15)) * LD + pk);
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = Mfma32<H>::run(af[mi], bf[ni], acc[mi][ni]);
        }
    };
    S16_LOAD(r0, 0);
    S16_LOAD(r1, 1);
    S16_STORE(r0, 0);
    __syncthreads();
    f4_t cpre[4][4];   // old C values
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        if (c + 2 < NK) {
            if (c % 2 == 0) S16_LOAD(r0, c + 2);
            else S16_LOAD(r1, c + 2);
        }
        if (c == NK - 2) {
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni) {
                    const int col = J * kBM + wn * 64 + ni * 16 + (lane & 15);
                    const int row = I * kBM + wm * 64 + mi * 16 + 4 * (lane >> 4);
                    cpre[mi][ni] = *reinterpret_cast<const f4_t *>(C + row + (int64_t)col * ldc);
                }
        }
        mma(c % 2);
        if (c + 1 < NK) {
            if ((c + 1) % 2 == 0) S16_STORE(r0, 0);
            else S16_STORE(r1, 1);
            __syncthreads();
        }
    }
#undef S16_LOAD
#undef S16_STORE
    const bool diag_tile = I == J;   // uniform over the workgroup
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
            const int col = J * kBM + wn * 64 + ni * 16 + (lane & 15);
            const int row = I * kBM + wm * 64 + mi * 16 + 4 * (lane >> 4);
            f4_t v = cpre[mi][ni];
            if (!diag_tile) {
                v -= acc[mi][ni];
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = row + q >= col ? v[q] - acc[mi][ni][q] : v[q];
            }
            *reinterpret_cast<f4_t *>(C + row + (int64_t)col * ldc) = v;
        }
    if constexpr (DIAG0) {
        if (I == 0 && J == 0) {   // uniform over the workgroup
            // the block this workgroup just wrote: stores complete and visible
            // (release), every wave done, then loads past the stale L1 lines
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            diag_block<float, true>(C, ldc, Wd, info, k0, smem_raw);
        }
    }
}

// ------------------------------------------------------------------------
// host drivers
// ------------------------------------------------------------------------
static size_t diag_smem_bytes(size_t es) { return (size_t)(kNBlk + kNL + 4) * kLB * kLB * es; }
static size_t elem_size(int dtype) { return dtype == GBEM_F64 ? 8 : 4; }

size_t chol_winv_bytes(int dtype, int64_t npad) { return (size_t)npad * kNB * elem_size(dtype); }
size_t chol_panel_bytes(int, int64_t) { return 64; }
// Outer panels per super-panel of the 16-bit factorisation (the trailing
// matrix beyond a super-panel is updated once, with K = that many panels).
// Measured at the three-layer bus (order 59,904, mixed): 4 panels (K = 2048)
// 199.8 ms per extraction against 217.2 ms with 2 (trailing update 109.5 vs
// 130.4 ms, the look-ahead updates 36.2 vs 20.2 ms); at the crossing bus
// (order 21,504) 2 panels stay ahead (25.25 vs 25.71 ms), the look-ahead
// chain weighing more there.  Default thresholds and the autotuner's cache:
// chol_shape (tune.cpp).
static int super_panels(int dtype, int64_t npad) { return chol_shape(dtype, npad).super_panels; }
size_t chol_panel16_bytes(int dtype, int64_t npad)
{
    // two super-panels in flight (look-ahead): ping-pong buffers of npad rows
    // x (super-panel width) 16-bit values
    return (dtype == GBEM_F16 || dtype == GBEM_BF16)
               ? (size_t)2 * npad * super_panels(dtype, npad) * outer_width(dtype, npad) * 2
               : 0;
}

template <typename T, int MODE, bool MASK, bool SUB, int Q16 = 0>
static hipError_t launch_gemm(int tm, int ntiles, int K, const T *A, int64_t lda, const T *B, int64_t ldb, T *C,
                              int64_t ldc, hipStream_t s, void *Q = nullptr, int qrow = 0, int qcol = 0)
{
    const size_t smem = gemm_smem_bytes<T>();
    hipError_t e = hipFuncSetAttribute((const void *)gemm_kernel<T, MODE, MASK, SUB, Q16>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((gemm_kernel<T, MODE, MASK, SUB, Q16>), dim3(ntiles), dim3(256), smem, s, tm, K, A, lda, B,
                       ldb, C, ldc, Q, qrow, qcol);
    return hipGetLastError();
}

// Wd != nullptr: also factor the first diagonal block (DIAG0, kRect only)
template <typename H, int MODE, int NK, bool D0>
static hipError_t launch_syrk16_nk(int tm, int ntiles, int K, const H *QA, const H *QB, int64_t ldq, float *C,
                                   int64_t ldc, hipStream_t s, float *Wd, int32_t *info, int k0)
{
    const size_t smem = std::max(syrk16_smem_bytes(), D0 ? diag_smem_bytes(sizeof(float)) : (size_t)0);
    const void *fn = (const void *)syrk16_kernel<H, MODE, NK, D0>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((syrk16_kernel<H, MODE, NK, D0>), dim3(ntiles), dim3(256), smem, s, tm, K, QA, QB, ldq, C,
                       ldc, Wd, info, k0);
    return hipGetLastError();
}
template <typename H, int MODE, bool D0>
static hipError_t launch_syrk16_k(int tm, int ntiles, int K, const H *QA, const H *QB, int64_t ldq, float *C,
                                  int64_t ldc, hipStream_t s, float *Wd, int32_t *info, int k0)
{
    switch (K) {
    case 256: return launch_syrk16_nk<H, MODE, 4, D0>(tm, ntiles, K, QA, QB, ldq, C, ldc, s, Wd, info, k0);
    case 512: return launch_syrk16_nk<H, MODE, 8, D0>(tm, ntiles, K, QA, QB, ldq, C, ldc, s, Wd, info, k0);
    case 768: return launch_syrk16_nk<H, MODE, 12, D0>(tm, ntiles, K, QA, QB, ldq, C, ldc, s, Wd, info, k0);
    case 1024: return launch_syrk16_nk<H, MODE, 16, D0>(tm, ntiles, K, QA, QB, ldq, C, ldc, s, Wd, info, k0);
    case 1536: return launch_syrk16_nk<H, MODE, 24, D0>(tm, ntiles, K, QA, QB, ldq, C, ldc, s, Wd, info, k0);
    case 2048: return launch_syrk16_nk<H, MODE, 32, D0>(tm, ntiles, K, QA, QB, ldq, C, ldc, s, Wd, info, k0);
    default: return hipErrorInvalidValue;
    }
}
template <typename H, int MODE>
static hipError_t launch_syrk16(int tm, int ntiles, int K, const H *QA, const H *QB, int64_t ldq, float *C,
                                int64_t ldc, hipStream_t s, float *Wd = nullptr, int32_t *info = nullptr, int k0 = 0)
{
    if constexpr (MODE == kRect) {
        if (Wd) return launch_syrk16_k<H, MODE, true>(tm, ntiles, K, QA, QB, ldq, C, ldc, s, Wd, info, k0);
    } else if (Wd) {
        return hipErrorInvalidValue;
    }
    return launch_syrk16_k<H, MODE, false>(tm, ntiles, K, QA, QB, ldq, C, ldc, s, nullptr, nullptr, 0);
}

// Factor the outer panel at P0 (ow columns, rows P0 .. npad): diagonal
// block 0 (unless the update of the panel's columns already factored it),
// then the rest of the panel in one launch.  info[1 .. 1 + 2 ns]:
// error word and flags of panel_kernel.
static std::atomic<int32_t> g_panel_epoch{0};
// Q16 placement (16-bit updates): see panel_kernel (qoff, qcol0, qld)
template <typename T, int Q16T>
static hipError_t launch_panel(int64_t npad, int ow, T *A, int64_t lda, T *Winv, void *Q16, int32_t *info,
                               int64_t P0, hipStream_t s, Prof *prof, bool diag0_done, int qoff = 0, int qcol0 = 0,
                               int qld = 0)
{
    const double es = (double)sizeof(T);
    const int ns = ow / kNB;
    if (ns > kMaxPanelBlocks) return hipErrorInvalidValue;
    const size_t smem = std::max(gemm_smem_bytes<T>(), diag_smem_bytes(sizeof(T)));
    hipError_t e = hipFuncSetAttribute((const void *)panel_kernel<T, Q16T>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    int tok;
    if (!diag0_done) {
        tok = prof ? prof->start(s, GBEM_K_DIAG) : -1;
        hipLaunchKernelGGL((diag_kernel<T, true>), dim3(1), dim3(256), diag_smem_bytes(sizeof(T)), s,
                           A + P0 + P0 * lda, lda, Winv + P0 * kNB, info, (int)P0);
        if (prof) prof->stop(tok, GBEM_K_DIAG, 2.0 * kNB * kNB * kNB / 3.0, 3.0 * kNB * kNB * es, s);
    }
    const int64_t m = npad - P0 - kNB;   // rows below diagonal block 0
    if (m <= 0) return hipGetLastError();
    const int32_t epoch = ++g_panel_epoch;
    tok = prof ? prof->start(s, GBEM_K_TRSM) : -1;
    hipLaunchKernelGGL((panel_kernel<T, Q16T>), dim3((unsigned)(m / kNB)), dim3(256), smem, s, A + P0 + P0 * lda,
                       lda, ns, Winv + P0 * kNB, info, (int)P0, Q16, qoff, qcol0, qld > 0 ? qld : ow, info + 1,
                       epoch, 1 << 22);
    if (prof) {
        double fl = 0.0, by = 0.0;
        for (int j = 0; j < ns; ++j) {
            const double mj = (double)(m - (int64_t)kNB * j);
            fl += 2.0 * mj * kNB * kNB * (j + 1) + (j + 1 < ns ? 2.0 * kNB * kNB * kNB * (j + 1.0 + 1.0 / 3.0) : 0.0);
            by += (2.0 + j) * mj * kNB * es + 3.0 * kNB * kNB * es + (Q16 ? 2.0 * mj * kNB : 0.0);
        }
        prof->stop(tok, GBEM_K_TRSM, fl, by, s);
    }
    return hipGetLastError();
}

// diag0_done: the first diagonal block was factored by the launch that
// updated the panel's columns
template <typename T>
static hipError_t factor_panel(int dtype, int64_t npad, int ow, T *A, int64_t lda, T *Winv, void *Q16,
                               int32_t *info, int p, hipStream_t s, Prof *prof, bool diag0_done = false,
                               int qoff = 0, int qcol0 = 0, int qld = 0)
{
    const int64_t P0 = (int64_t)p * ow;
    if (Q16 && dtype == GBEM_BF16)
        return launch_panel<T, 1>(npad, ow, A, lda, Winv, Q16, info, P0, s, prof, diag0_done, qoff, qcol0, qld);
    if (Q16 && dtype == GBEM_F16)
        return launch_panel<T, 2>(npad, ow, A, lda, Winv, Q16, info, P0, s, prof, diag0_done, qoff, qcol0, qld);
    return launch_panel<T, 0>(npad, ow, A, lda, Winv, nullptr, info, P0, s, prof, diag0_done);
}

// Outer update of columns [c0, c0 + ncols) of the trailing matrix with the
// outer panel at P0 (ow columns, FP32 or FP64 storage): C = A[c0.., c0..]
// (origin on the diagonal), rows m = npad - c0.  TRI when the block is square.
template <typename T>
static hipError_t outer_update(int64_t npad, int ow, T *A, int64_t lda, int64_t P0, int64_t c0, int64_t ncols,
                               hipStream_t s, Prof *prof, int cls)
{
    const int64_t m = npad - c0;
    const int tm = (int)(m / kBM), tn = (int)(ncols / kBM);
    const bool tri = ncols == m;
    const int ntiles = tri ? tm * (tm + 1) / 2 : tm * tn;
    T *C = A + c0 + c0 * lda;
    const double es = (double)sizeof(T);
    const double tiles_el = tri ? (double)tm * (tm + 1) / 2 * kBM * kBM : (double)m * ncols;
    const int tok = prof ? prof->start(s, cls) : -1;
    const T *Q = A + c0 + P0 * lda;   // L[c0:, P0:P0+ow], column-major
    hipError_t e = tri ? launch_gemm<T, kTri, true, true>(tm, ntiles, ow, Q, lda, Q, lda, C, lda, s)
                       : launch_gemm<T, kRect, true, true>(tm, ntiles, ow, Q, lda, Q, lda, C, lda, s);
    if (prof) prof->stop(tok, cls, 2.0 * tiles_el * ow, 2.0 * tiles_el * es + (double)m * ow * es, s);
    return e;
}

// 16-bit update of columns [c0, c0 + ncols) of the trailing matrix (origin
// on the diagonal, rows m = npad - c0): C -= Q Q^T with Q the 16-bit copy of
// the panel columns used (row-major, row stride ldq, K values per row, first
// row = global row c0).  TRI when the block is square; Wd: the launch also
// factors the diagonal block at C's origin (rectangular grid only).
static hipError_t update16(int dtype, int64_t npad, float *A, int64_t lda, const void *Q, int64_t ldq, int K,
                           int64_t c0, int64_t ncols, hipStream_t s, Prof *prof, int cls, float *Wd = nullptr,
                           int32_t *info = nullptr)
{
    const int64_t m = npad - c0;
    const bool tri = ncols == m && !Wd;
    const int tm = (int)(m / kBM), tn = (int)(ncols / kBM);
    const int ntiles = tri ? tm * (tm + 1) / 2 : tm * tn;
    float *C = A + c0 + c0 * lda;
    const double tiles_el = tri ? (double)tm * (tm + 1) / 2 * kBM * kBM : (double)m * ncols;
    const int tok = prof ? prof->start(s, cls) : -1;
    hipError_t e;
    if (dtype == GBEM_BF16) {
        const __bf16 *q = (const __bf16 *)Q;
        e = tri ? launch_syrk16<__bf16, kTri>(tm, ntiles, K, q, q, ldq, C, lda, s)
                : launch_syrk16<__bf16, kRect>(tm, ntiles, K, q, q, ldq, C, lda, s, Wd, info, (int)c0);
    } else {
        const _Float16 *q = (const _Float16 *)Q;
        e = tri ? launch_syrk16<_Float16, kTri>(tm, ntiles, K, q, q, ldq, C, lda, s)
                : launch_syrk16<_Float16, kRect>(tm, ntiles, K, q, q, ldq, C, lda, s, Wd, info, (int)c0);
    }
    if (prof) {
        double fl = 2.0 * tiles_el * K, by = 2.0 * tiles_el * 4.0 + (double)m * K * 2.0;
        if (Wd) fl += 2.0 * kNB * kNB * kNB / 3.0, by += 3.0 * kNB * kNB * 4.0;   // the diagonal block
        prof->stop(tok, cls, fl, by, s);
    }
    return e;
}

// Cholesky with 16-bit trailing updates on super-panels of P ow-wide outer
// panels (P = super_panels: 1, 2 or 4): the trailing matrix beyond a
// super-panel is updated once with K = P ow (its FP32 read-modify-write
// traffic falls as 1 / P against one update per panel), while the panel
// factorisations keep ow-wide panels.  The look-ahead chain carries more
// update work per panel as P grows (P = 1: one update per panel); the tile
// shape table picks P per matrix order.  Super-panel s = panels P s .. P s + P - 1 (the last may
// have fewer), columns from P0_s = P s ow.  Its 16-bit copy Q_s (ping-pong
// buffer s & 1, row stride P ow) holds global row R_s + i in row i, R_s =
// P0_s + ow: panel P s + j in columns [j ow, (j + 1) ow) from row j ow on.
//   side stream, super-panel s + 1 (after main finished its update with
//   super-panel s - 1): its columns -= Q_s Q_s^T (K = P ow; the same launch
//   factors the first diagonal block), factor its first panel; then for each
//   further panel j of it, the panel's columns -= the Q_{s+1} columns of
//   panels 0 .. j - 1 (K = j ow, first diagonal block in the same launch),
//   and factor it;
//   main stream (after the side stream factored super-panel s): the columns
//   beyond super-panel s + 1 -= Q_s Q_s^T (K = P ow, lower triangle).
static hipError_t factor16_t(int dtype, int64_t npad, float *A, int64_t lda, float *Winv, void *Q16, int32_t *info,
                             hipStream_t s, hipStream_t side, std::vector<hipEvent_t> &ev, Prof *prof)
{
    const int ow = outer_width(dtype, npad), P = super_panels(dtype, npad), sw = P * ow;
    const int nbo = (int)(npad / ow);
    const int nsp = (nbo + P - 1) / P;
    hipError_t e = hipFuncSetAttribute((const void *)diag_kernel<float, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)diag_smem_bytes(sizeof(float)));
    if (e != hipSuccess) return e;
    while ((int)ev.size() < 2 * nsp + 2) {   // evP[0..nsp), evB[0..nsp]
        hipEvent_t x;
        if ((e = hipEventCreateWithFlags(&x, hipEventDisableTiming | hipEventDisableSystemFence)) != hipSuccess) return e;
        ev.push_back(x);
    }
    auto qbuf = [&](int sp) -> _Float16 * {   // 16-bit element type only sizes the pointer arithmetic
        return (_Float16 *)Q16 + (size_t)(sp & 1) * npad * sw;
    };
    auto panels_in = [&](int sp) { return std::min(P, nbo - P * sp); };
    // factor super-panel sp; its first panel's columns are up to date and,
    // when d0, its first diagonal block already factored
    auto factor_sp = [&](int sp, bool d0) -> hipError_t {
        const int p0 = P * sp;
        _Float16 *q = qbuf(sp);
        hipError_t r;
        if ((r = factor_panel<float>(dtype, npad, ow, A, lda, Winv, q, info, p0, side, prof, d0, 0, 0, sw)) !=
            hipSuccess)
            return r;
        for (int j = 1; j < panels_in(sp); ++j) {
            // panel p0 + j's columns with panels p0 .. p0 + j - 1 (Q rows from
            // global row cj), first diagonal block in the same launch
            const int64_t cj = (int64_t)(p0 + j) * ow;
            if ((r = update16(dtype, npad, A, lda, q + (size_t)(j - 1) * ow * sw, sw, j * ow, cj, ow, side, prof,
                              GBEM_K_PANEL, Winv + cj * kNB, info)) != hipSuccess)
                return r;
            if ((r = factor_panel<float>(dtype, npad, ow, A, lda, Winv, q, info, p0 + j, side, prof, true, j * ow,
                                         j * ow, sw)) != hipSuccess)
                return r;
        }
        return hipSuccess;
    };
    hipEvent_t *evP = ev.data(), *evB = ev.data() + nsp + 1;
    if ((e = hipEventRecord(evB[nsp], s)) != hipSuccess) return e;   // inputs of this call are ready
    if ((e = hipStreamWaitEvent(side, evB[nsp], 0)) != hipSuccess) return e;
    if ((e = factor_sp(0, false)) != hipSuccess) return e;
    if ((e = hipEventRecord(evP[0], side)) != hipSuccess) return e;
    for (int sp = 0; sp + 1 < nsp; ++sp) {
        const int64_t P0n = (int64_t)P * (sp + 1) * ow;   // first column of super-panel sp + 1
        const int64_t Rs = (int64_t)(P * sp + 1) * ow;    // row 0 of Q_sp
        // side: super-panel sp + 1's columns with super-panel sp (K = P ow), then factor it
        if (sp > 0 && (e = hipStreamWaitEvent(side, evB[sp - 1], 0)) != hipSuccess) return e;
        if ((e = update16(dtype, npad, A, lda, qbuf(sp) + (P0n - Rs) * sw, sw, sw, P0n,
                          (int64_t)panels_in(sp + 1) * ow, side, prof, GBEM_K_PANEL, Winv + P0n * kNB, info)) !=
            hipSuccess)
            return e;
        if ((e = factor_sp(sp + 1, true)) != hipSuccess) return e;
        if ((e = hipEventRecord(evP[sp + 1], side)) != hipSuccess) return e;
        // main: the columns beyond super-panel sp + 1 with super-panel sp
        const int64_t c0 = P0n + (int64_t)panels_in(sp + 1) * ow;
        if (c0 < npad) {
            if ((e = hipStreamWaitEvent(s, evP[sp], 0)) != hipSuccess) return e;
            if ((e = update16(dtype, npad, A, lda, qbuf(sp) + (c0 - Rs) * sw, sw, sw, c0, npad - c0, s, prof,
                              GBEM_K_SYRK)) != hipSuccess)
                return e;
        }
        if ((e = hipEventRecord(evB[sp], s)) != hipSuccess) return e;
    }
    if ((e = hipStreamWaitEvent(s, evP[nsp - 1], 0)) != hipSuccess) return e;
    return hipGetLastError();
}

// Right-looking Cholesky with ow-wide outer panels and one panel of
// look-ahead (FP32 and FP64 storage, trailing updates in the storage type):
// the side stream updates the next panel's columns and factors it while the
// main stream applies the rest of the outer update.
template <typename T>
static hipError_t factor_t(int dtype, int64_t npad, T *A, int64_t lda, T *Winv, int32_t *info, hipStream_t s,
                           hipStream_t side, std::vector<hipEvent_t> &ev, Prof *prof)
{
    const int ow = outer_width(dtype, npad);
    const int nbo = (int)(npad / ow);
    hipError_t e = hipFuncSetAttribute((const void *)diag_kernel<T, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)diag_smem_bytes(sizeof(T)));
    if (e != hipSuccess) return e;
    while ((int)ev.size() < 2 * nbo + 2) {   // evP[0..nbo), evB[0..nbo]
        hipEvent_t x;
        if ((e = hipEventCreateWithFlags(&x, hipEventDisableTiming | hipEventDisableSystemFence)) != hipSuccess) return e;
        ev.push_back(x);
    }
    // Side stream: the latency-critical chain (update of the next panel's
    // columns, then its factorisation).  Main stream: the rest of each outer
    // update.  Events: evP[K] = panel K factored (side -> main), evB[K] =
    // main's update with panel K done (main -> side, needed before the side
    // stream updates the columns of panel K+2).
    hipEvent_t *evP = ev.data(), *evB = ev.data() + nbo + 1;
    if ((e = hipEventRecord(evB[nbo], s)) != hipSuccess) return e;   // inputs of this call are ready
    if ((e = hipStreamWaitEvent(side, evB[nbo], 0)) != hipSuccess) return e;
    if ((e = factor_panel<T>(dtype, npad, ow, A, lda, Winv, nullptr, info, 0, side, prof)) != hipSuccess) return e;
    if ((e = hipEventRecord(evP[0], side)) != hipSuccess) return e;
    for (int K = 0; K + 1 < nbo; ++K) {
        const int64_t P0 = (int64_t)K * ow;
        // side: (a) panel K+1's columns with panel K, then factor panel K+1
        if (K > 0 && (e = hipStreamWaitEvent(side, evB[K - 1], 0)) != hipSuccess) return e;
        if ((e = outer_update<T>(npad, ow, A, lda, P0, P0 + ow, ow, side, prof, GBEM_K_PANEL)) != hipSuccess)
            return e;
        if ((e = factor_panel<T>(dtype, npad, ow, A, lda, Winv, nullptr, info, K + 1, side, prof)) != hipSuccess)
            return e;
        if ((e = hipEventRecord(evP[K + 1], side)) != hipSuccess) return e;
        // main: (b) the columns beyond panel K+1 with panel K
        const int64_t c0 = P0 + 2 * ow;
        if (c0 < npad) {
            if ((e = hipStreamWaitEvent(s, evP[K], 0)) != hipSuccess) return e;
            if ((e = outer_update<T>(npad, ow, A, lda, P0, c0, npad - c0, s, prof, GBEM_K_SYRK)) != hipSuccess)
                return e;
        }
        if ((e = hipEventRecord(evB[K], s)) != hipSuccess) return e;
    }
    if ((e = hipStreamWaitEvent(s, evP[nbo - 1], 0)) != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t chol_factor(int dtype, int64_t npad, void *A, int64_t lda, void *Winv, void *, void *panel16,
                       int32_t *info, hipStream_t s, hipStream_t side, std::vector<hipEvent_t> &ev, Prof *prof)
{
    if (npad % outer_width(dtype, npad)) return hipErrorInvalidValue;
    if (dtype == GBEM_F64)
        return factor_t<double>(dtype, npad, (double *)A, lda, (double *)Winv, info, s, side, ev, prof);
    if (dtype == GBEM_F16 || dtype == GBEM_BF16)
        return factor16_t(dtype, npad, (float *)A, lda, (float *)Winv, panel16, info, s, side, ev, prof);
    return factor_t<float>(dtype, npad, (float *)A, lda, (float *)Winv, info, s, side, ev, prof);
}

template <typename T>
static hipError_t diag_inverses_t(int64_t npad, const T *L, int64_t lda, T *Winv, hipStream_t s)
{
    const size_t smem = diag_smem_bytes(sizeof(T));
    hipError_t e = hipFuncSetAttribute((const void *)diag_kernel<T, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    // the diagonal blocks are independent: one workgroup each
    hipLaunchKernelGGL((diag_kernel<T, false>), dim3((unsigned)(npad / kNB)), dim3(256), smem, s,
                       const_cast<T *>(L), lda, Winv, (int32_t *)nullptr, 0);
    return hipGetLastError();
}

hipError_t chol_diag_inverses(int dtype, int64_t npad, const void *L, int64_t lda, void *Winv,
                              hipStream_t s)
{
    if (npad % kNB) return hipErrorInvalidValue;
    if (dtype == GBEM_F64) return diag_inverses_t<double>(npad, (const double *)L, lda, (double *)Winv, s);
    return diag_inverses_t<float>(npad, (const float *)L, lda, (float *)Winv, s);
}

hipError_t launch_gram_f64(int64_t nrows, int64_t K, const double *P, int64_t ldp, double *C, int64_t ldc,
                           bool subtract, hipStream_t s)
{
    if (nrows % kBM || K % kBK || nrows <= 0 || K <= 0) return hipErrorInvalidValue;
    const int tm = (int)(nrows / kBM);
    if (subtract)
        return launch_gemm<double, kTri, true, true>(tm, tm * (tm + 1) / 2, (int)K, P, ldp, P, ldp, C, ldc, s);
    return launch_gemm<double, kTri, true, false>(tm, tm * (tm + 1) / 2, (int)K, P, ldp, P, ldp, C, ldc, s);
}

}  // namespace gbem
