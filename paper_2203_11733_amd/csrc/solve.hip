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
// as column i).  The j range is split over several workgroups per row block;
// partial sums are added in a fixed order by a second kernel.
#include <type_traits>

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

// ------------------------------------------------------------------------
// FP32 storage (the low-precision factors): the same persistent scheme with
// the block products on MFMA (v_mfma_f32_16x16x4f32, FP32 accumulation; the
// solve only has to match the precision of the factor, the FP64 refinement
// supplies the rest).  With D_k = L_kk and W_k = D_k^{-1}:
//   forward   Y_k = W_k (B_k - sum_{j<k-2} L_kj Y_j) - M2_k Y_{k-2} - M_k Y_{k-1},
//             M_k = W_k L_{k,k-1},  M2_k = W_k L_{k,k-2};
//   backward  X_k = W_k^T (Y_k - sum_{j>k+2} L_jk^T X_j) - N2_k^T X_{k+2} - N_k^T X_{k+1},
//             N_k = L_{k+1,k} W_k,  N2_k = L_{k+2,k} W_k.
// The four products are formed once per factor (solve_prep).  A workgroup
// finishes the W_k product while its block's second-to-last dependency is
// being computed, applies M2_k / N2_k while the last one is, and after the
// last has arrived only one 128 x 128 product remains (measured at order
// 59,904 with 48 right-hand sides: with W_k applied after the second-to-last
// dependency, a workgroup entered its final wait 3.6 us after the block it
// waits for was published, against 1.8 us from publication to arrival).  One
// workgroup per block solves every right-hand side (MC = 16 NCB >= m
// columns), so L is streamed once per direction whatever the conductor
// count.  Per workgroup:
//   - W_k and M_k / N_k wait in registers from the start, M2_k / N2_k are
//     loaded into the L-tile registers after the last L block; each goes
//     through the LDS tile buffer once the dependency stream is over; the L
//     blocks stream through that buffer, the next one loaded into registers
//     while the MFMAs work on the current one;
//   - each wave owns 32 rows of the block, so the products need no
//     cross-wave reduction;
//   - a finished block is published as 64-bit words (value bits, epoch) with
//     agent-scope atomic stores (they bypass the non-coherent per-XCD L2);
//     consumers load the words with agent-scope atomic loads and re-load the
//     ones whose epoch is stale.  Data and readiness travel together, so there
//     is no separate flag and no store-completion wait before one.
// Word layout of a published block (128 x MC values): word
// ((R NCB + cb) 4 + q) 64 + l holds row 16 R + 4 (l / 16) + q, column
// 16 cb + l % 16 (the MFMA output layout of the producing wave, so each store
// instruction covers 512 contiguous bytes).
// LDS: the left operand A(i, t) of the block products (the L block, W_k,
// M_k, M2_k, or their transposes) as tile[i * TLD + t], and two right-operand
// buffers Y(t, n) as ys[n * YLD + t]: both contiguous in the summation index
// t, so one 16-byte read gives a lane the operands of four MFMAs (lane group
// g takes t = 16 s + 4 g .. 16 s + 4 g + 3 in step s; 7.2 against 8.8
// thousand cycles per 128 x 128 x 48 product with one 4-byte read per
// operand and MFMA).  Strides of 132 words put the 16-byte reads of eight
// consecutive lanes on distinct banks.
// ------------------------------------------------------------------------
template <bool FWD, int NCB> struct SolveCfg {
    static constexpr int MC = 16 * NCB;               // right-hand sides per workgroup
    static constexpr int RB = 2;                      // 16-row blocks per wave
    static constexpr int NW = MC / 2;                 // published words per thread (128 MC / 256)
    static constexpr int TLD = 132;                   // LDS tile row stride
    static constexpr int YLD = 132;                   // right-operand column stride
    static constexpr size_t kTileBytes = (size_t)kNB * TLD * 4;
    static constexpr size_t kYBytes = (size_t)MC * YLD * 4;
    static constexpr size_t kSmem = kTileBytes + 2 * kYBytes;
};
typedef float f4s_t __attribute__((ext_vector_type(4)));
typedef unsigned int u4s_t __attribute__((ext_vector_type(4)));

// 128 x 128 block at P (column-major, ld) -> registers: thread = column
// c = tid % 128, rows h*64 .. h*64+63 (h = tid / 128) as 16-byte chunks
__device__ __forceinline__ void tile_load(u4s_t (&tr)[16], const float *P, int64_t ld)
{
    const int c = threadIdx.x & 127, h = threadIdx.x >> 7;
    const u4s_t *src = reinterpret_cast<const u4s_t *>(P + h * 64 + (int64_t)c * ld);
#pragma unroll
    for (int q = 0; q < 16; ++q) tr[q] = src[q];
}
// Registers of tile_load -> the LDS tile, A(i, t) = tile[i * TLD + t].
// FWD (A = L_kj, W_k, M_k, M2_k: the loaded column is t): transposing 4-byte
// stores, a wave's lanes on 64 consecutive columns of one row (distinct
// banks).  BWD (A = L_jk^T, W_k^T, N_k^T, N2_k^T: the loaded column is i):
// the column as it is, in 16-byte stores (eight consecutive columns per
// store cycle, distinct banks at the stride of 132 words).
template <bool FWD, int TLD>
__device__ __forceinline__ void tile_store(float *tile, const u4s_t (&tr)[16])
{
    const int c = threadIdx.x & 127, h = threadIdx.x >> 7;
    if constexpr (FWD) {
#pragma unroll
        for (int q = 0; q < 16; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) tile[(h * 64 + 4 * q + e) * TLD + c] = __uint_as_float(tr[q][e]);
    } else {
        u4s_t *dst = reinterpret_cast<u4s_t *>(tile + c * TLD + h * 64);
#pragma unroll
        for (int q = 0; q < 16; ++q) dst[q] = tr[q];
    }
}

// acc[rb][cb] += A(i, t) Y(t, n) over t = 0..127 for the wave's rows
// i = 32 w + 16 rb + .. and columns n = 16 cb + ..; A(i, t) = tile[i*TLD + t],
// Y(t, n) = ys[n*YLD + t].  MFMA j of step s contracts t = 16 s + 4 g + j
// over the lane groups g (any order of the sum over t is the same product).
template <bool FWD, int NCB>
__device__ __forceinline__ void tile_product(f4s_t (&acc)[2][NCB], const float *tile, const float *ys)
{
    typedef SolveCfg<FWD, NCB> C;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r = lane & 15, g4 = 4 * (lane >> 4);
    const float *ap0 = tile + ((w * C::RB + 0) * 16 + r) * C::TLD + g4;
    const float *ap1 = tile + ((w * C::RB + 1) * 16 + r) * C::TLD + g4;
    const float *bp = ys + r * C::YLD + g4;
#pragma unroll 2
    for (int k16 = 0; k16 < kNB; k16 += 16) {
        const f4s_t a0 = *reinterpret_cast<const f4s_t *>(ap0 + k16);
        const f4s_t a1 = *reinterpret_cast<const f4s_t *>(ap1 + k16);
        f4s_t b[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) b[cb] = *reinterpret_cast<const f4s_t *>(bp + cb * 16 * C::YLD + k16);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                acc[0][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[j], b[cb][j], acc[0][cb], 0, 0, 0);
                acc[1][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[j], b[cb][j], acc[1][cb], 0, 0, 0);
            }
    }
}

// Issue the loads of this thread's words (w = tid + 256 u) of a published block.
template <int NW>
__device__ __forceinline__ void pub_issue(uint64_t (&wd)[NW], const uint64_t *blk)
{
    const uint64_t *p = blk + threadIdx.x;
#pragma unroll
    for (int u = 0; u < NW; ++u) wd[u] = __hip_atomic_load(p + 256 * u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Complete the loads of a block: when some word is stale, one thread polls
// word 0 until it carries `tag` (a waiting workgroup then adds one load per
// poll to the memory system, not the whole block), after which the stale
// words are re-loaded until all carry `tag`.  Bounded; returns the same value
// in every thread (false after a timeout, with the error word set).
template <int NW>
__device__ __forceinline__ bool pub_complete(uint64_t (&wd)[NW], const uint64_t *blk, uint32_t tag, int32_t *err,
                                             int limit)
{
    const uint64_t *p = blk + threadIdx.x;
    bool good = true;
#pragma unroll
    for (int u = 0; u < NW; ++u) good = good && (uint32_t)(wd[u] >> 32) == tag;
    if (!__syncthreads_or(!good)) return true;
    if (threadIdx.x == 0) {
        for (int n = 0; n < limit; ++n) {
            if ((uint32_t)(__hip_atomic_load(blk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 32) == tag) break;
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
    for (int n = 0;; ++n) {
#pragma unroll
        for (int u = 0; u < NW; ++u)
            if ((uint32_t)(wd[u] >> 32) != tag)
                wd[u] = __hip_atomic_load(p + 256 * u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = true;
#pragma unroll
        for (int u = 0; u < NW; ++u) good = good && (uint32_t)(wd[u] >> 32) == tag;
        if (good || n >= limit) break;
        __builtin_amdgcn_s_sleep(2);
    }
    if (!good) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return !__syncthreads_or(!good);
}
// The same for the blocks a workgroup's last two products wait on (the
// solve's critical path): every thread re-loads its own stale words until
// they carry `tag`, which takes one memory round trip after publication
// instead of two.  Two workgroups wait on a block this way, so the extra
// polling traffic is two blocks per round trip.
template <int NW>
__device__ __forceinline__ bool pub_complete_direct(uint64_t (&wd)[NW], const uint64_t *blk, uint32_t tag,
                                                    int32_t *err, int limit)
{
    const uint64_t *p = blk + threadIdx.x;
    bool good = true;
    for (int n = 0;; ++n) {
        good = true;
#pragma unroll
        for (int u = 0; u < NW; ++u) good = good && (uint32_t)(wd[u] >> 32) == tag;
        if (good || n >= limit) break;
#pragma unroll
        for (int u = 0; u < NW; ++u)
            if ((uint32_t)(wd[u] >> 32) != tag)
                wd[u] = __hip_atomic_load(p + 256 * u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!good) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return !__syncthreads_or(!good);
}
// words -> ys[col * YLD + row] (FP32): word t + 256 u is (R, cb) = (u / NCB,
// u % NCB), q = wave, l = lane
template <bool FWD, int NCB>
__device__ __forceinline__ void pub_to_lds(float *ys, const uint64_t (&wd)[SolveCfg<FWD, NCB>::NW])
{
    typedef SolveCfg<FWD, NCB> C;
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
#pragma unroll
    for (int u = 0; u < C::NW; ++u) {
        const int R = u / NCB, cb = u % NCB;
        ys[(cb * 16 + (lane & 15)) * C::YLD + R * 16 + 4 * (lane >> 4) + q] = __uint_as_float((uint32_t)wd[u]);
    }
}

// One workgroup per block (every right-hand side).  Ticket t -> block t in
// solve order; Y holds the published words, block k at Y + k * 128 * MC.
template <bool FWD, int NCB>
__global__ __launch_bounds__(256) void tsolve32_kernel(const float *__restrict__ L, int64_t lda,
                                                       const float *__restrict__ W, const float *__restrict__ S,
                                                       const float *__restrict__ S2, double *B, int64_t ldb,
                                                       uint64_t *Y, int m, int nb,
                                                       int32_t *__restrict__ counter, uint32_t base, uint32_t tag,
                                                       int32_t *err, int limit)
{
    typedef SolveCfg<FWD, NCB> C;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    float *tile = reinterpret_cast<float *>(smem_raw);                     // L blocks, then W_k, then M_k / N_k
    float *ys0 = reinterpret_cast<float *>(smem_raw + C::kTileBytes);
    float *ys1 = reinterpret_cast<float *>(smem_raw + C::kTileBytes + C::kYBytes);
    const int tk = take_ticket(counter, base);
    if (tk < 0 || tk >= nb) {
        if (threadIdx.x == 0) __hip_atomic_store(err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // solve order: FWD blocks 0, 1, ..; BWD blocks nb-1, nb-2, ..
    const int k = FWD ? tk : nb - 1 - tk, k0 = k * kNB;
    const int cnt = tk;                      // blocks this one depends on
    const int nn = cnt > 1 ? cnt - 2 : 0;    // all but the last two of them
    constexpr int BW = kNB * C::MC;          // words per published block
    auto jof = [&](int idx) { return FWD ? idx : nb - 1 - idx; };
    auto pblk = [&](int idx) { return Y + (int64_t)jof(idx) * BW; };
    auto lsrc = [&](int idx) {   // L_kj (FWD) or L_jk (BWD) of the idx-th dependency
        const int j = jof(idx);
        return FWD ? L + k0 + (int64_t)j * kNB * lda : L + (int64_t)j * kNB + (int64_t)k0 * lda;
    };
    // element (rb, q) of this thread: row within the block; column 16 cb + lane % 16
    auto erow = [&](int rb, int q) { return (wave * C::RB + rb) * 16 + 4 * (lane >> 4) + q; };
    const int col = lane & 15;

    double bk[C::RB][NCB][4];
#pragma unroll
    for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                bk[rb][cb][q] = cb * 16 + col < m ? B[(k0 + erow(rb, q)) + (int64_t)(cb * 16 + col) * ldb] : 0.0;

    u4s_t tr[16], wr[16], sr[16];
    tile_load(wr, W + (int64_t)k * kNB * kNB, kNB);
    if (cnt > 0) tile_load(sr, S + (int64_t)k * kNB * kNB, kNB);
    if (nn > 0) tile_load(tr, lsrc(0), lda);

    f4s_t acc[2][NCB];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = f4s_t{0.f, 0.f, 0.f, 0.f};
    uint64_t wd[C::NW];
    if (nn > 0) {
        pub_issue<C::NW>(wd, pblk(0));
        if (!pub_complete<C::NW>(wd, pblk(0), tag, err, limit)) return;
        pub_to_lds<FWD, NCB>(ys0, wd);
        tile_store<FWD, C::TLD>(tile, tr);
        if (nn > 1) tile_load(tr, lsrc(1), lda);
        __syncthreads();
        for (int idx = 0; idx < nn; ++idx) {
            const bool more = idx + 1 < nn;
            if (more) pub_issue<C::NW>(wd, pblk(idx + 1));
            tile_product<FWD, NCB>(acc, tile, (idx & 1) ? ys1 : ys0);
            if (!more) break;
            if (!pub_complete<C::NW>(wd, pblk(idx + 1), tag, err, limit)) return;
            __syncthreads();
            tile_store<FWD, C::TLD>(tile, tr);
            pub_to_lds<FWD, NCB>(((idx + 1) & 1) ? ys1 : ys0, wd);
            if (idx + 2 < nn) tile_load(tr, lsrc(idx + 2), lda);
            __syncthreads();
        }
    }
    __syncthreads();   // the last product is done with tile, ys0 and ys1
    // M2_k / N2_k into the registers the L tiles used; waited for after the
    // W_k product
    if (cnt > 1) tile_load(tr, S2 + (int64_t)k * kNB * kNB, kNB);
    // Z = W_k (B_k - acc): the difference goes through LDS as the right operand
#pragma unroll
    for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                ys0[(cb * 16 + col) * C::YLD + erow(rb, q)] = (float)(bk[rb][cb][q] - (double)acc[rb][cb][q]);
            acc[rb][cb] = f4s_t{0.f, 0.f, 0.f, 0.f};
        }
    tile_store<FWD, C::TLD>(tile, wr);
    // the next dependency to arrive (the second-to-last, else the last), completed after the product
    if (cnt > 0) pub_issue<C::NW>(wd, pblk(cnt > 1 ? cnt - 2 : cnt - 1));
    __syncthreads();
    tile_product<FWD, NCB>(acc, tile, ys0);
    if (cnt > 1) {
        // Z -= M2_k Y_{k-2} (FWD) or N2_k^T X_{k+2} (BWD), while Y_{k-1} / X_{k+1} is computed
        __syncthreads();   // every wave is done with W_k in the tile
        tile_store<FWD, C::TLD>(tile, tr);
        if (!pub_complete_direct<C::NW>(wd, pblk(cnt - 2), tag, err, limit)) return;
        pub_to_lds<FWD, NCB>(ys1, wd);
        pub_issue<C::NW>(wd, pblk(cnt - 1));   // the last dependency, completed after this product
        __syncthreads();
        f4s_t acc2[2][NCB];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc2[rb][cb] = f4s_t{0.f, 0.f, 0.f, 0.f};
        tile_product<FWD, NCB>(acc2, tile, ys1);
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] -= acc2[rb][cb];
    }
    if (cnt > 0) {
        // Y_k = Z - M_k Y_{k-1} (FWD) or X_k = Z - N_k^T X_{k+1} (BWD)
        __syncthreads();   // every wave is done with the tile (W_k or M2_k) and with ys1
        tile_store<FWD, C::TLD>(tile, sr);
        if (!pub_complete_direct<C::NW>(wd, pblk(cnt - 1), tag, err, limit)) return;
        pub_to_lds<FWD, NCB>(ys1, wd);
        __syncthreads();
        f4s_t acc2[2][NCB];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc2[rb][cb] = f4s_t{0.f, 0.f, 0.f, 0.f};
        tile_product<FWD, NCB>(acc2, tile, ys1);
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] -= acc2[rb][cb];
    }
    // publish, then the FP64 result
    uint64_t *yk = Y + (int64_t)k * BW;
#pragma unroll
    for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                __hip_atomic_store(yk + (((wave * C::RB + rb) * NCB + cb) * 4 + q) * 64 + lane,
                                   ((uint64_t)tag << 32) | __float_as_uint(acc[rb][cb][q]), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (cb * 16 + col < m) B[(k0 + erow(rb, q)) + (int64_t)(cb * 16 + col) * ldb] = (double)acc[rb][cb][q];
}

// Products with the diagonal-block inverses for the FP32 solves, in four
// npad x 128 slots of S: M_k = W_k L_{k,k-1} (slot 0, k = 1 .. nb-1),
// N_k = L_{k+1,k} W_k (slot 1, k = 0 .. nb-2), M2_k = W_k L_{k,k-2}
// (slot 2, k = 2 .. nb-1), N2_k = L_{k+2,k} W_k (slot 3, k = 0 .. nb-3);
// block k of a slot at offset 128 k * 128.  One workgroup per product
// (blockIdx.y = slot), both operands in LDS, 8 x 8 outputs per thread on
// FP32 FMAs.
constexpr int kPLd = kNB + 4;
__global__ __launch_bounds__(256) void solve_prep_kernel(const float *__restrict__ L, int64_t lda,
                                                         const float *__restrict__ W, float *__restrict__ S,
                                                         int64_t npad)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    float *As = reinterpret_cast<float *>(smem_raw);   // As[t * kPLd + i] = A(i, t)
    float *Bs = As + kNB * kPLd;                       // Bs[t * kPLd + c] = B(t, c)
    const int slot = blockIdx.y, d = 1 + (slot >> 1);   // d: block distance of the L factor
    const bool second = slot & 1;                        // L block on the left (N_k, N2_k)
    if ((int64_t)(blockIdx.x + d) * kNB >= npad) return; // slots 2, 3 hold one product fewer
    const int k = second ? blockIdx.x : blockIdx.x + d;
    const int64_t k0 = (int64_t)k * kNB;
    const float *Wk = W + k0 * kNB;
    const float *A = second ? L + (k0 + d * kNB) + k0 * lda : Wk;
    const int64_t ldA = second ? lda : kNB;
    const float *Bm = second ? Wk : L + k0 + (k0 - d * kNB) * lda;
    const int64_t ldB = second ? kNB : lda;
    float *out = S + slot * npad * kNB + k0 * kNB;
    const int tid = threadIdx.x;
    {
        const int c = tid >> 1, h = tid & 1;
        for (int r = h * 64; r < h * 64 + 64; r += 4) {
            const f4s_t a = *reinterpret_cast<const f4s_t *>(A + r + (int64_t)c * ldA);
            *reinterpret_cast<f4s_t *>(As + c * kPLd + r) = a;
            const f4s_t b = *reinterpret_cast<const f4s_t *>(Bm + r + (int64_t)c * ldB);
#pragma unroll
            for (int e = 0; e < 4; ++e) Bs[(r + e) * kPLd + c] = b[e];
        }
    }
    __syncthreads();
    const int ti = (tid & 15) * 8, tc = (tid >> 4) * 8;
    float acc[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = 0.f;
    for (int t = 0; t < kNB; ++t) {
        const f4s_t a0 = *reinterpret_cast<const f4s_t *>(As + t * kPLd + ti);
        const f4s_t a1 = *reinterpret_cast<const f4s_t *>(As + t * kPLd + ti + 4);
        const f4s_t b0 = *reinterpret_cast<const f4s_t *>(Bs + t * kPLd + tc);
        const f4s_t b1 = *reinterpret_cast<const f4s_t *>(Bs + t * kPLd + tc + 4);
        const float a[8] = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
        const float b[8] = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        f4s_t o0, o1;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            o0[i] = acc[i][j];
            o1[i] = acc[i + 4][j];
        }
        *reinterpret_cast<f4s_t *>(out + (int64_t)(tc + j) * kNB + ti) = o0;
        *reinterpret_cast<f4s_t *>(out + (int64_t)(tc + j) * kNB + ti + 4) = o1;
    }
}

template <int NCB>
static hipError_t solve32_n(int64_t npad, const float *L, int64_t lda, const float *W, int m, double *B, int64_t ldb,
                            SolveSync &sync, hipStream_t s, Prof *prof)
{
    const int nb = (int)(npad / kNB);
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void *)tsolve32_kernel<true, NCB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)SolveCfg<true, NCB>::kSmem)) != hipSuccess ||
        (e = hipFuncSetAttribute((const void *)tsolve32_kernel<false, NCB>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)SolveCfg<false, NCB>::kSmem)) !=
            hipSuccess)
        return e;
    const int limit = 1 << 22;
    ++sync.epoch;
    const uint32_t tag = (uint32_t)sync.epoch;
    uint64_t *Yf = sync.pub, *Yb = sync.pub + (size_t)npad * kMaxPub;
    const unsigned grid = (unsigned)nb;
    const int tok = prof ? prof->start(s, GBEM_K_SOLVE) : -1;
    const float *sub = sync.sub;   // M, N, M2, N2: npad x 128 floats each
    hipLaunchKernelGGL((tsolve32_kernel<true, NCB>), dim3(grid), dim3(256), (SolveCfg<true, NCB>::kSmem), s, L, lda, W,
                       sub, sub + 2 * npad * kNB, B, ldb, Yf, m, nb, sync.err + 1, sync.base_f, tag, sync.err, limit);
    hipLaunchKernelGGL((tsolve32_kernel<false, NCB>), dim3(grid), dim3(256), (SolveCfg<false, NCB>::kSmem), s, L, lda,
                       W, sub + npad * kNB, sub + 3 * npad * kNB, B, ldb, Yb, m, nb, sync.err + 2, sync.base_b, tag,
                       sync.err, limit);
    if (prof) {
        // L once per direction, W, M/N and M2/N2 per block, B read/written, published blocks read by every later block
        const double lbytes = (double)npad * (npad + kNB) / 2.0 * 4.0;
        const double pub = (double)nb * (nb - 1) / 2.0 * kNB * 16 * NCB * 8.0;
        prof->stop(tok, GBEM_K_SOLVE, 2.0 * 2.0 * (double)npad * npad / 2.0 * m,
                   2.0 * lbytes + 6.0 * npad * kNB * 4.0 + 4.0 * npad * m * 8.0 + 2.0 * pub, s, 2);
    }
    e = hipGetLastError();
    if (e == hipSuccess) {   // each launch consumes exactly grid tickets
        sync.base_f += grid;
        sync.base_b += grid;
    }
    return e;
}

static hipError_t solve32(int64_t npad, const float *L, int64_t lda, const float *W, int m, double *B, int64_t ldb,
                          SolveSync &sync, hipStream_t s, Prof *prof)
{
    if (m <= 16) return solve32_n<1>(npad, L, lda, W, m, B, ldb, sync, s, prof);
    if (m <= 32) return solve32_n<2>(npad, L, lda, W, m, B, ldb, sync, s, prof);
    if (m <= 48) return solve32_n<3>(npad, L, lda, W, m, B, ldb, sync, s, prof);
    return solve32_n<4>(npad, L, lda, W, m, B, ldb, sync, s, prof);
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
    const int tok = prof ? prof->start(s, GBEM_K_SOLVE) : -1;
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
    const float *Lf = (const float *)L, *Wf = (const float *)Winv;
    if (sync.prep_of != L || sync.prep_npad != npad) return hipErrorInvalidValue;   // solve_prep first
    return solve32(npad, Lf, lda, Wf, m, B, ldb, sync, s, prof);
}

hipError_t chol_solve_prep(int dtype, int64_t npad, const void *L, int64_t lda, const void *Winv,
                           SolveSync &sync, hipStream_t s)
{
    if (npad % kNB) return hipErrorInvalidValue;
    sync.prep_of = nullptr;
    if (dtype == GBEM_F64) return hipSuccess;
    const int nb = (int)(npad / kNB);
    if (nb > 1) {
        const size_t smem = (size_t)2 * kNB * kPLd * 4;
        hipError_t e = hipFuncSetAttribute((const void *)solve_prep_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(solve_prep_kernel, dim3(nb - 1, 4), dim3(256), smem, s, (const float *)L, lda,
                           (const float *)Winv, sync.sub, npad);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    sync.prep_of = L;
    sync.prep_npad = npad;
    return hipSuccess;
}

// ------------------------------------------------------------------------
// Residual R = B - A X, split over j.  Row i of the symmetric A is read as
// column i (contiguous in j).  A workgroup takes 128 values of i (32 per
// wave) and a range of j in chunks of 32; each wave multiplies on
// v_mfma_f64_16x16x4f64.  The summation index is permuted so that lane l
// (k-slot q = l / 16) takes the 8 consecutive j = j0 + 8q .. j0 + 8q + 7 of
// a chunk: four 16-byte loads of A (column i0 + l % 16) straight into
// registers, one chunk ahead of their use, and four 16-byte LDS reads of X
// (column c0 + l % 16).  The workgroup stages each X chunk in LDS once for
// its four waves (double-buffered, loaded one chunk ahead) instead of every
// wave holding it in registers, so two waves fit on each SIMD (three-layer
// bus, 48 columns: 8.1 against 9.2 ms per residual with X in registers at
// one wave per SIMD; A two chunks ahead at one wave per SIMD: 9.6 ms).
// With X as the first operand the outputs of lane l lie in row
// i0 + l % 16, so partial sums are stored 16 rows at a time.
// ------------------------------------------------------------------------
constexpr int kRRows = 128, kRChunk = 32, kRXld = kRChunk + 2;   // X chunk row stride in LDS (doubles)
typedef double d4r_t __attribute__((ext_vector_type(4)));
typedef double d2r_t __attribute__((ext_vector_type(2)));

template <int MC>
__global__ __launch_bounds__(256, 2) void residual_partial_kernel(const double *__restrict__ A, int64_t lda,
                                                               int npad, const double *__restrict__ X,
                                                               int64_t ldx, int m, int jspan,
                                                               double *__restrict__ P)
{
    constexpr int CB = MC / 16;
    constexpr int NXP = MC / 16;   // 16-byte pieces of an X chunk per thread (MC columns x 16 pieces / 256)
    extern __shared__ __attribute__((aligned(16))) double xs_raw[];   // [2][MC][kRXld]
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q = lane >> 4, li = lane & 15;
    const int i0 = blockIdx.x * kRRows + w * 32, s = blockIdx.y;
    const int jb = s * jspan, je = min(npad, jb + jspan);
    const int nch = je > jb ? (je - jb) / kRChunk : 0;   // npad, jb and jspan are multiples of 32
    d4r_t acc[2][CB];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = d4r_t{0, 0, 0, 0};
    if (nch > 0) {   // uniform over the workgroup; an empty range leaves zero partials
        d2r_t ra[2][2][4];   // [buffer][row block][16-byte piece]
        d2r_t xg[NXP];       // the next X chunk on its way to LDS
        auto loadA = [&](d2r_t (&r)[2][4], int c) __attribute__((always_inline)) {
            const int j = jb + c * kRChunk + 8 * q;
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                const d2r_t *pa = reinterpret_cast<const d2r_t *>(A + j + (int64_t)(i0 + rb * 16 + li) * lda);
#pragma unroll
                for (int e = 0; e < 4; ++e) r[rb][e] = pa[e];
            }
        };
        auto loadX = [&](int c) __attribute__((always_inline)) {
#pragma unroll
            for (int u = 0; u < NXP; ++u) {
                const int p = threadIdx.x + 256 * u, col = p >> 4, jj = (p & 15) * 2;
                xg[u] = col < m ? *reinterpret_cast<const d2r_t *>(X + jb + c * kRChunk + jj + (int64_t)col * ldx)
                                : d2r_t{0, 0};
            }
        };
        auto storeX = [&](int buf) __attribute__((always_inline)) {
            double *xs = xs_raw + buf * MC * kRXld;
#pragma unroll
            for (int u = 0; u < NXP; ++u) {
                const int p = threadIdx.x + 256 * u;
                *reinterpret_cast<d2r_t *>(xs + (p >> 4) * kRXld + (p & 15) * 2) = xg[u];
            }
        };
        auto mult = [&](const d2r_t (&r)[2][4], int buf) __attribute__((always_inline)) {
            const double *xs = xs_raw + buf * MC * kRXld + li * kRXld + 8 * q;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                d2r_t xf[CB];
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) xf[cb] = *reinterpret_cast<const d2r_t *>(xs + cb * 16 * kRXld + 2 * e);
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb)
                            acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(xf[cb][h], r[rb][e][h], acc[rb][cb], 0, 0, 0);
            }
        };
        // chunk c: A in ra[c % 2] (loaded one chunk ahead), X in LDS buffer c & 1
        auto step = [&](auto cur, int c) __attribute__((always_inline)) {
            constexpr int B = decltype(cur)::value;
            if (c + 1 < nch) loadA(ra[B ^ 1], c + 1);
            mult(ra[B], c & 1);
            if (c + 1 < nch) {
                storeX((c + 1) & 1);   // its last readers finished before the previous barrier
                if (c + 2 < nch) loadX(c + 2);
            }
            __syncthreads();
        };
        loadA(ra[0], 0);
        loadX(0);
        storeX(0);
        if (nch > 1) loadX(1);
        __syncthreads();
        for (int c = 0; c < nch; c += 2) {
            step(std::integral_constant<int, 0>{}, c);
            if (c + 1 >= nch) break;
            step(std::integral_constant<int, 1>{}, c + 1);
        }
    }
    // lane l, register r: row i0 + rb*16 + l%16, column cb*16 + l/16 + 4r
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = cb * 16 + q + 4 * r;
                if (c < m) P[((int64_t)s * m + c) * npad + i0 + rb * 16 + li] = acc[rb][cb][r];
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
    if (npad % kRRows || m > kMaxRhs || m <= 0) return hipErrorInvalidValue;
    const int ns = residual_splits(npad);
    const int jspan = (int)round_up((npad + ns - 1) / ns, kRChunk);
    const dim3 grid(npad / kRRows, ns);
    const int mc = m <= 16 ? 16 : m <= 32 ? 32 : m <= 48 ? 48 : 64;   // the instance launched below
    const size_t smem = (size_t)2 * mc * kRXld * 8;
    if (m <= 16)
        hipLaunchKernelGGL(residual_partial_kernel<16>, grid, dim3(256), smem, st, A, lda, npad, X, ldx, m, jspan, partial);
    else if (m <= 32)
        hipLaunchKernelGGL(residual_partial_kernel<32>, grid, dim3(256), smem, st, A, lda, npad, X, ldx, m, jspan, partial);
    else if (m <= 48)   // FP64 MFMA work grows with the padded width: 48 saves a quarter against 64
        hipLaunchKernelGGL(residual_partial_kernel<48>, grid, dim3(256), smem, st, A, lda, npad, X, ldx, m, jspan, partial);
    else
        hipLaunchKernelGGL(residual_partial_kernel<64>, grid, dim3(256), smem, st, A, lda, npad, X, ldx, m, jspan, partial);
    hipLaunchKernelGGL(residual_finish_kernel, dim3((npad + 255) / 256, m), dim3(256), 0, st, partial, ns, npad, m, B,
                       ldb, R, ldr);
    return hipGetLastError();
}

}  // namespace gbem
