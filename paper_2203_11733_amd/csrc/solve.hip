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
//   forward   Y_k = W_k (B_k - sum_{j<k-1} L_kj Y_j) - M_k Y_{k-1},
//             M_k = W_k L_{k,k-1};
//   backward  X_k = W_k^T (Y_k - sum_{j>k+1} L_jk^T X_j) - N_k^T X_{k+1},
//             N_k = L_{k+1,k} W_k.
// M_k and N_k are formed once per factor (solve_prep), so after the block a
// workgroup waits for last has arrived only one 128 x 128 product remains;
// everything else overlaps the wait.  One workgroup per block solves every
// right-hand side (MC = 16 NCB >= m columns), so L is streamed once per
// direction whatever the conductor count.  Per workgroup:
//   - W_k and M_k / N_k wait in registers from the start and go through the
//     LDS tile buffer once the dependency stream is over; the L blocks stream
//     through that buffer, the next one loaded into registers while the MFMAs
//     work on the current one;
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
// LDS: the tile (row stride TLD: FWD 144, BWD 132, conflict-free fragment
// reads in either orientation) and two 128 x MC right-operand buffers (row
// stride YLD: the four rows a fragment read touches fall on distinct banks).
// ------------------------------------------------------------------------
template <bool FWD, int NCB> struct SolveCfg {
    static constexpr int MC = 16 * NCB;               // right-hand sides per workgroup
    static constexpr int RB = 2;                      // 16-row blocks per wave
    static constexpr int NW = MC / 2;                 // published words per thread (128 MC / 256)
    static constexpr int TLD = FWD ? 144 : 132;       // LDS tile stride
    static constexpr int YLD = MC == 64 ? 80 : (MC == 32 ? 48 : MC);   // right-operand stride
    static constexpr size_t kTileBytes = (size_t)kNB * TLD * 4;
    static constexpr size_t kYBytes = (size_t)kNB * YLD * 4;
    static constexpr size_t kSmem = kTileBytes + 2 * kYBytes;
};
typedef float f4s_t __attribute__((ext_vector_type(4)));
typedef unsigned int u4s_t __attribute__((ext_vector_type(4)));

// 128 x 128 block at P (column-major, ld) -> registers: thread = column c,
// rows h*64 .. h*64+63 as 16-byte chunks
__device__ __forceinline__ void tile_load(u4s_t (&tr)[16], const float *P, int64_t ld)
{
    const int c = threadIdx.x >> 1, h = threadIdx.x & 1;
    const u4s_t *src = reinterpret_cast<const u4s_t *>(P + h * 64 + (int64_t)c * ld);
#pragma unroll
    for (int q = 0; q < 16; ++q) tr[q] = src[q];
}
template <int TLD>
__device__ __forceinline__ void tile_store(float *tile, const u4s_t (&tr)[16])
{
    const int c = threadIdx.x >> 1, h = threadIdx.x & 1;
    u4s_t *dst = reinterpret_cast<u4s_t *>(tile + c * TLD + h * 64);
#pragma unroll
    for (int q = 0; q < 16; ++q) dst[q] = tr[q];
}

// acc[rb][cb] += A(i, t) Y(t, n) over t = 0..127 for the wave's rows
// i = 32 w + 16 rb + ..; A(i, t) = tile[t*TLD + i] (FWD: L_kj, W_k, M_k) or
// tile[i*TLD + t] (BWD: L_jk^T, W_k^T, N_k^T); Y(t, n) = ys[t*YLD + n],
// n = 16 cb + ..
template <bool FWD, int NCB>
__device__ __forceinline__ void tile_product(f4s_t (&acc)[2][NCB], const float *tile, const float *ys)
{
    typedef SolveCfg<FWD, NCB> C;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll 4
    for (int kk = 0; kk < kNB; kk += 4) {
        const int t = kk + (lane >> 4);
        float b[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) b[cb] = ys[t * C::YLD + cb * 16 + (lane & 15)];
#pragma unroll
        for (int rb = 0; rb < C::RB; ++rb) {
            const int i = (w * C::RB + rb) * 16 + (lane & 15);
            const float a = FWD ? tile[t * C::TLD + i] : tile[i * C::TLD + t];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
                acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[cb], acc[rb][cb], 0, 0, 0);
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
// words -> ys[row * YLD + col] (FP32): word t + 256 u is (R, cb) = (u / NCB,
// u % NCB), q = wave, l = lane
template <bool FWD, int NCB>
__device__ __forceinline__ void pub_to_lds(float *ys, const uint64_t (&wd)[SolveCfg<FWD, NCB>::NW])
{
    typedef SolveCfg<FWD, NCB> C;
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
#pragma unroll
    for (int u = 0; u < C::NW; ++u) {
        const int R = u / NCB, cb = u % NCB;
        ys[(R * 16 + 4 * (lane >> 4) + q) * C::YLD + cb * 16 + (lane & 15)] = __uint_as_float((uint32_t)wd[u]);
    }
}

// One workgroup per block (every right-hand side).  Ticket t -> block t in
// solve order; Y holds the published words, block k at Y + k * 128 * MC.
template <bool FWD, int NCB>
__global__ __launch_bounds__(256) void tsolve32_kernel(const float *__restrict__ L, int64_t lda,
                                                       const float *__restrict__ W, const float *__restrict__ S,
                                                       double *B, int64_t ldb, uint64_t *Y, int m, int nb,
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
    const int nn = cnt > 0 ? cnt - 1 : 0;    // all but the last of them
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
        tile_store<C::TLD>(tile, tr);
        if (nn > 1) tile_load(tr, lsrc(1), lda);
        __syncthreads();
        for (int idx = 0; idx < nn; ++idx) {
            const bool more = idx + 1 < nn;
            if (more) pub_issue<C::NW>(wd, pblk(idx + 1));
            tile_product<FWD, NCB>(acc, tile, (idx & 1) ? ys1 : ys0);
            if (!more) break;
            if (!pub_complete<C::NW>(wd, pblk(idx + 1), tag, err, limit)) return;
            __syncthreads();
            tile_store<C::TLD>(tile, tr);
            pub_to_lds<FWD, NCB>(((idx + 1) & 1) ? ys1 : ys0, wd);
            if (idx + 2 < nn) tile_load(tr, lsrc(idx + 2), lda);
            __syncthreads();
        }
    }
    __syncthreads();   // the last product is done with tile, ys0 and ys1
    // Z = W_k (B_k - acc): the difference goes through LDS as the right operand
#pragma unroll
    for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                ys0[erow(rb, q) * C::YLD + cb * 16 + col] = (float)(bk[rb][cb][q] - (double)acc[rb][cb][q]);
            acc[rb][cb] = f4s_t{0.f, 0.f, 0.f, 0.f};
        }
    tile_store<C::TLD>(tile, wr);
    if (cnt > 0) pub_issue<C::NW>(wd, pblk(cnt - 1));   // the last dependency, completed after the product
    __syncthreads();
    tile_product<FWD, NCB>(acc, tile, ys0);
    if (cnt > 0) {
        // Y_k = Z - M_k Y_{k-1} (FWD) or X_k = Z - N_k^T X_{k+1} (BWD)
        __syncthreads();   // every wave is done with W_k in the tile
        tile_store<C::TLD>(tile, sr);
        if (!pub_complete<C::NW>(wd, pblk(cnt - 1), tag, err, limit)) return;
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

// M_k = W_k L_{k,k-1} (k = 1 .. nb-1, slot k of S) and N_k = L_{k+1,k} W_k
// (k = 0 .. nb-2, slot k of S + npad * 128).  One workgroup per product,
// both operands in LDS, 8 x 8 outputs per thread on FP32 FMAs.
constexpr int kPLd = kNB + 4;
__global__ __launch_bounds__(256) void solve_prep_kernel(const float *__restrict__ L, int64_t lda,
                                                         const float *__restrict__ W, float *__restrict__ S,
                                                         int64_t npad)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    float *As = reinterpret_cast<float *>(smem_raw);   // As[t * kPLd + i] = A(i, t)
    float *Bs = As + kNB * kPLd;                       // Bs[t * kPLd + c] = B(t, c)
    const bool second = blockIdx.y == 1;
    const int k = second ? blockIdx.x : blockIdx.x + 1;
    const int64_t k0 = (int64_t)k * kNB;
    const float *Wk = W + k0 * kNB;
    const float *A = second ? L + (k0 + kNB) + k0 * lda : Wk;
    const int64_t ldA = second ? lda : kNB;
    const float *Bm = second ? Wk : L + k0 + (k0 - kNB) * lda;
    const int64_t ldB = second ? kNB : lda;
    float *out = S + (second ? npad * kNB : 0) + k0 * kNB;
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
    hipLaunchKernelGGL((tsolve32_kernel<true, NCB>), dim3(grid), dim3(256), (SolveCfg<true, NCB>::kSmem), s, L, lda, W,
                       (const float *)sync.sub, B, ldb, Yf, m, nb, sync.err + 1, sync.base_f, tag, sync.err, limit);
    hipLaunchKernelGGL((tsolve32_kernel<false, NCB>), dim3(grid), dim3(256), (SolveCfg<false, NCB>::kSmem), s, L, lda,
                       W, (const float *)sync.sub + npad * kNB, B, ldb, Yb, m, nb, sync.err + 2, sync.base_b, tag,
                       sync.err, limit);
    if (prof) {
        // L once per direction, W and M/N per block, B read/written, published blocks read by every later block
        const double lbytes = (double)npad * (npad + kNB) / 2.0 * 4.0;
        const double pub = (double)nb * (nb - 1) / 2.0 * kNB * 16 * NCB * 8.0;
        prof->stop(tok, GBEM_K_SOLVE, 2.0 * 2.0 * (double)npad * npad / 2.0 * m,
                   2.0 * lbytes + 4.0 * npad * kNB * 4.0 + 4.0 * npad * m * 8.0 + 2.0 * pub, s, 2);
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
        hipLaunchKernelGGL(solve_prep_kernel, dim3(nb - 1, 2), dim3(256), smem, s, (const float *)L, lda,
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
// wave) and a range of j; each wave multiplies on v_mfma_f64_16x16x4f64
// without LDS or barriers: the summation index is permuted so that lane l
// (k-slot q = l / 16) reads the 8 consecutive j = j0 + 8q .. j0 + 8q + 7 of
// a 32-long chunk as four 16-byte loads, from A (column i0 + l % 16) and from
// X (column c0 + l % 16) alike; the next chunk is loaded while the current
// one is multiplied.  With X as the first operand the outputs of lane l lie
// in row i0 + l % 16, so partial sums are stored 16 rows at a time.
// ------------------------------------------------------------------------
constexpr int kRRows = 128, kRChunk = 32;
typedef double d4r_t __attribute__((ext_vector_type(4)));
typedef double d2r_t __attribute__((ext_vector_type(2)));

template <int MC>
__global__ __launch_bounds__(256) void residual_partial_kernel(const double *__restrict__ A, int64_t lda,
                                                               int npad, const double *__restrict__ X,
                                                               int64_t ldx, int m, int jspan,
                                                               double *__restrict__ P)
{
    constexpr int CB = MC / 16;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q = lane >> 4, li = lane & 15;
    const int i0 = blockIdx.x * kRRows + w * 32, s = blockIdx.y;
    const int jb = s * jspan, je = min(npad, jb + jspan);
    d4r_t acc[2][CB];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = d4r_t{0, 0, 0, 0};
    if (jb >= je) {
        // empty range: zero partials keep the fixed-order sum exact
    } else {
        d2r_t ra[2][2][4], rx[2][CB][4];   // [buffer][block][16-byte piece]
        auto load = [&](int buf, int j0) __attribute__((always_inline)) {
            const int j = j0 + 8 * q;
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                const d2r_t *pa = reinterpret_cast<const d2r_t *>(A + j + (int64_t)(i0 + rb * 16 + li) * lda);
#pragma unroll
                for (int e = 0; e < 4; ++e) ra[buf][rb][e] = pa[e];
            }
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const int c = cb * 16 + li;
                if (c < m) {
                    const d2r_t *px = reinterpret_cast<const d2r_t *>(X + j + (int64_t)c * ldx);
#pragma unroll
                    for (int e = 0; e < 4; ++e) rx[buf][cb][e] = px[e];
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) rx[buf][cb][e] = d2r_t{0, 0};
                }
            }
        };
        auto mult = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb)
                            acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(rx[buf][cb][e][h], ra[buf][rb][e][h],
                                                                               acc[rb][cb], 0, 0, 0);
        };
        load(0, jb);
        // two chunks per trip: the register buffers are indexed by constants
        for (int j0 = jb; j0 < je; j0 += 2 * kRChunk) {
            if (j0 + kRChunk < je) load(1, j0 + kRChunk);
            mult(0);
            if (j0 + kRChunk >= je) break;
            if (j0 + 2 * kRChunk < je) load(0, j0 + 2 * kRChunk);
            mult(1);
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
    if (m <= 16)
        hipLaunchKernelGGL(residual_partial_kernel<16>, grid, dim3(256), 0, st, A, lda, npad, X, ldx, m, jspan, partial);
    else if (m <= 32)
        hipLaunchKernelGGL(residual_partial_kernel<32>, grid, dim3(256), 0, st, A, lda, npad, X, ldx, m, jspan, partial);
    else if (m <= 48)   // FP64 MFMA work grows with the padded width: 48 saves a quarter against 64
        hipLaunchKernelGGL(residual_partial_kernel<48>, grid, dim3(256), 0, st, A, lda, npad, X, ldx, m, jspan, partial);
    else
        hipLaunchKernelGGL(residual_partial_kernel<64>, grid, dim3(256), 0, st, A, lda, npad, X, ldx, m, jspan, partial);
    hipLaunchKernelGGL(residual_finish_kernel, dim3((npad + 255) / 256, m), dim3(256), 0, st, partial, ns, npad, m, B,
                       ldb, R, ldr);
    return hipGetLastError();
}

}  // namespace gbem
