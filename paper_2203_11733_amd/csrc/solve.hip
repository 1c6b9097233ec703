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
// supplies the rest).  Per workgroup:
//   - 128 x 128 tiles of L (then W_k) stream through one LDS tile; the next
//     tile is loaded into registers while the MFMAs work on the current one;
//   - published blocks are read and written with agent-scope atomic loads and
//     stores (they bypass the non-coherent per-XCD L2), so publishing needs
//     only the completion of those stores before the flag, and consuming needs
//     no cache invalidation;
//   - a published block k implies that every block before it (in solve
//     order) is published, so one observed flag covers all earlier blocks.
// Waves split the 128-long inner dimension (and the rows when MC = 64); their
// partial sums are added through LDS once per block row.
// ------------------------------------------------------------------------
template <int MC, bool FWD> struct SolveCfg {
    static constexpr int CB = MC / 16;                 // 16-column blocks of the RHS
    static constexpr int NKG = MC <= 32 ? 4 : 2;      // wave groups over the inner dimension
    static constexpr int NRG = 4 / NKG;               // wave groups over the rows
    static constexpr int RB = 8 / NRG;                // 16-row blocks per wave
    static constexpr int KW = kNB / NKG;              // inner range per wave
    static constexpr int TLD = FWD ? 144 : 132;       // LDS tile stride (conflict-free fragment reads)
    static constexpr int YLD = MC == 16 ? 16 : (MC == 32 ? 48 : 80);
    static constexpr int RLD = MC + 4;                // partial-sum stride
    static constexpr int EPT = kNB * MC / 256;        // (row, column) elements per thread
    static constexpr size_t kTileBytes = (size_t)kNB * 144 * 4;
    static constexpr size_t kSmem = kTileBytes + (size_t)2 * kNB * YLD * 4 + 64;
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

// acc[rb][cb] += A(i, t) Y(t, n) over this wave's inner range; A(i, t) =
// tile[t*TLD + i] (FWD: L_kj, W_k) or tile[i*TLD + t] (BWD: L_jk^T, W_k^T)
template <int MC, bool FWD, int RB, int CB>
__device__ __forceinline__ void tile_product(f4s_t (&acc)[RB][CB], const float *tile, const float *ys)
{
    typedef SolveCfg<MC, FWD> C;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int rg = w % C::NRG, kg = w / C::NRG;
#pragma unroll 4
    for (int kk = 0; kk < C::KW; kk += 4) {
        const int t = kg * C::KW + kk + (lane >> 4);
        float b[C::CB];
#pragma unroll
        for (int cb = 0; cb < C::CB; ++cb) b[cb] = ys[t * C::YLD + cb * 16 + (lane & 15)];
#pragma unroll
        for (int rb = 0; rb < C::RB; ++rb) {
            const int i = (rg * C::RB + rb) * 16 + (lane & 15);
            const float a = FWD ? tile[t * C::TLD + i] : tile[i * C::TLD + t];
#pragma unroll
            for (int cb = 0; cb < C::CB; ++cb)
                acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[cb], acc[rb][cb], 0, 0, 0);
        }
    }
}

// partial sums of all waves -> red (reusing the tile), then each thread adds
// the groups for its elements e = tid + 256 u: row e % 128, column e / 128
template <int MC, bool FWD, int EPT, int RB, int CB>
__device__ __forceinline__ void reduce_partials(float (&out)[EPT], f4s_t (&acc)[RB][CB], float *red)
{
    typedef SolveCfg<MC, FWD> C;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int rg = w % C::NRG, kg = w / C::NRG;
#pragma unroll
    for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < C::CB; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = (rg * C::RB + rb) * 16 + 4 * (lane >> 4) + q, n = cb * 16 + (lane & 15);
                red[(kg * kNB + row) * C::RLD + n] = acc[rb][cb][q];
            }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < C::EPT; ++u) {
        const int e = threadIdx.x + 256 * u, row = e % kNB, n = e / kNB;
        float s = 0.f;
#pragma unroll
        for (int g = 0; g < C::NKG; ++g) s += red[(g * kNB + row) * C::RLD + n];
        out[u] = s;
    }
}

template <int MC, bool FWD>
__global__ __launch_bounds__(256) void tsolve32_kernel(const float *__restrict__ L, int64_t lda,
                                                       const float *__restrict__ W, double *B, int64_t ldb, int m,
                                                       int nb, int32_t *flags, int32_t *__restrict__ counter,
                                                       uint32_t base, int32_t epoch, int32_t *err, int limit)
{
    typedef SolveCfg<MC, FWD> C;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    float *tile = reinterpret_cast<float *>(smem_raw);
    float *ysb = reinterpret_cast<float *>(smem_raw + C::kTileBytes);   // two Y buffers
    int *ready_s = reinterpret_cast<int *>(smem_raw + C::kTileBytes + (size_t)2 * kNB * C::YLD * 4);
    const int tk = take_ticket(counter, base);
    if (tk < 0 || tk >= nb) {
        if (threadIdx.x == 0) __hip_atomic_store(err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    // solve order: FWD blocks 0, 1, ..; BWD blocks nb-1, nb-2, ..
    const int k = FWD ? tk : nb - 1 - tk, k0 = k * kNB;
    const int cnt = tk;                                  // blocks this one depends on
    auto jof = [&](int idx) { return FWD ? idx : nb - 1 - idx; };
    // block of the matrix multiplying Y_j: FWD L[k, j] at (k0, j0); BWD L[j, k] at (j0, k0)
    auto lblock = [&](int j) -> const float * {
        return FWD ? L + k0 + (int64_t)j * kNB * lda : L + (int64_t)j * kNB + (int64_t)k0 * lda;
    };
    const float *Wk = W + (int64_t)k * kNB * kNB;

    // right-hand side of this block (read once, FP64)
    double bk[C::EPT];
#pragma unroll
    for (int u = 0; u < C::EPT; ++u) {
        const int e = threadIdx.x + 256 * u, row = e % kNB, n = e / kNB;
        bk[u] = n < m ? B[(k0 + row) + (int64_t)n * ldb] : 0.0;
    }

    // wait until the idx-th block in solve order is published (thread 0
    // polls; the observed index is shared through LDS)
    int ready = -1;
    auto ensure_ready = [&](int idx) -> bool {
        if (idx <= ready) return true;
        if (threadIdx.x == 0) {
            int got = -2;
            if (wait_flag(flags + jof(idx), epoch, err, limit)) {
                got = idx;
                // blocks are published in solve order: probe further ahead
                // (all loads in flight at once) and keep the newest published
                int32_t f[8];
#pragma unroll
                for (int p = 0; p < 8; ++p) {
                    const int q = min(cnt - 1, idx + (1 << (p + 1)) - 1);
                    f[p] = __hip_atomic_load(flags + jof(q), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
#pragma unroll
                for (int p = 0; p < 8; ++p)
                    if (f[p] == epoch) got = max(got, min(cnt - 1, idx + (1 << (p + 1)) - 1));
            }
            *ready_s = got;
        }
        __syncthreads();
        ready = *ready_s;
        return ready >= idx;
    };
    // Y_j (FP64, published) -> registers
    auto y_load = [&](double (&yr)[C::EPT], int j) {
#pragma unroll
        for (int u = 0; u < C::EPT; ++u) {
            const int e = threadIdx.x + 256 * u, row = e % kNB, n = e / kNB;
            yr[u] = n < m ? __hip_atomic_load(B + (j * kNB + row) + (int64_t)n * ldb, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT)
                          : 0.0;
        }
    };
    auto y_store = [&](float *ys, const double (&yr)[C::EPT]) {
#pragma unroll
        for (int u = 0; u < C::EPT; ++u) {
            const int e = threadIdx.x + 256 * u, row = e % kNB, n = e / kNB;
            ys[row * C::YLD + n] = (float)yr[u];
        }
    };

    f4s_t acc[C::RB][C::CB];
#pragma unroll
    for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < C::CB; ++cb) acc[rb][cb] = f4s_t{0.f, 0.f, 0.f, 0.f};

    u4s_t tr[16];
    double yr[C::EPT];
    bool ok = true;
    if (cnt > 0) {
        tile_load(tr, lblock(jof(0)), lda);
        ok = ensure_ready(0);
        if (ok) y_load(yr, jof(0));
        tile_store<C::TLD>(tile, tr);
        y_store(ysb, yr);
        tile_load(tr, cnt > 1 ? lblock(jof(1)) : Wk, cnt > 1 ? lda : (int64_t)kNB);
        __syncthreads();
        for (int idx = 0; idx < cnt && ok; ++idx) {
            const bool more = idx + 1 < cnt;
            // the next Y block: loaded ahead of the product when already
            // published, else waited for after it
            const bool early = more && idx + 1 <= ready;
            if (early) y_load(yr, jof(idx + 1));
            tile_product<MC, FWD>(acc, tile, ysb + (idx & 1) * kNB * C::YLD);
            if (more && !early) {
                ok = ensure_ready(idx + 1);
                if (ok) y_load(yr, jof(idx + 1));
            }
            __syncthreads();
            tile_store<C::TLD>(tile, tr);
            if (more) {
                y_store(ysb + ((idx + 1) & 1) * kNB * C::YLD, yr);
                if (idx + 2 < cnt) tile_load(tr, lblock(jof(idx + 2)), lda);
                else tile_load(tr, Wk, kNB);
            }
            __syncthreads();
        }
        if (!ok) return;   // error word set; the host reports it
        // tile holds L of the last block or W_k: W_k is in tr when cnt > 0
    } else {
        tile_load(tr, Wk, kNB);
    }
    // r = B_k - sum_j (...) Y_j  -> ys[0]
    float part[C::EPT];
    __syncthreads();
    reduce_partials<MC, FWD>(part, acc, tile);
    float *ys = ysb;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < C::EPT; ++u) {
        const int e = threadIdx.x + 256 * u, row = e % kNB, n = e / kNB;
        ys[row * C::YLD + n] = (float)(bk[u] - (double)part[u]);
    }
    tile_store<C::TLD>(tile, tr);   // W_k
    __syncthreads();
#pragma unroll
    for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < C::CB; ++cb) acc[rb][cb] = f4s_t{0.f, 0.f, 0.f, 0.f};
    tile_product<MC, FWD>(acc, tile, ys);
    __syncthreads();
    reduce_partials<MC, FWD>(part, acc, tile);
#pragma unroll
    for (int u = 0; u < C::EPT; ++u) {
        const int e = threadIdx.x + 256 * u, row = e % kNB, n = e / kNB;
        if (n < m)
            __hip_atomic_store(B + (k0 + row) + (int64_t)n * ldb, (double)part[u], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    // the stores above complete before the flag is raised
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flags + k, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int MC>
static hipError_t solve32_mc(int64_t npad, const float *L, int64_t lda, const float *W, int m, double *B,
                             int64_t ldb, SolveSync &sync, hipStream_t s, Prof *prof)
{
    const int nb = (int)(npad / kNB);
    const size_t smem = SolveCfg<MC, true>::kSmem;
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void *)tsolve32_kernel<MC, true>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem)) != hipSuccess ||
        (e = hipFuncSetAttribute((const void *)tsolve32_kernel<MC, false>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)SolveCfg<MC, false>::kSmem)) !=
            hipSuccess)
        return e;
    const int limit = 1 << 26;
    const size_t smem_b = SolveCfg<MC, false>::kSmem;
    ++sync.epoch;
    const int tok = prof ? prof->start(s, GBEM_K_SOLVE) : -1;
    hipLaunchKernelGGL((tsolve32_kernel<MC, true>), dim3(nb), dim3(256), smem, s, L, lda, W, B, ldb, m, nb,
                       sync.flags_f, sync.err + 1, sync.base_f, sync.epoch, sync.err, limit);
    hipLaunchKernelGGL((tsolve32_kernel<MC, false>), dim3(nb), dim3(256), smem_b, s, L, lda, W, B, ldb, m, nb,
                       sync.flags_b, sync.err + 2, sync.base_b, sync.epoch, sync.err, limit);
    if (prof) {
        const double lbytes = (double)npad * (npad + kNB) / 2.0 * 4.0;
        prof->stop(tok, GBEM_K_SOLVE, 2.0 * 2.0 * (double)npad * npad / 2.0 * m,
                   2.0 * lbytes + 2.0 * npad * kNB * 4.0 + 4.0 * npad * m * 8.0, s, 2);
    }
    e = hipGetLastError();
    if (e == hipSuccess) {
        sync.base_f += (uint32_t)nb;
        sync.base_b += (uint32_t)nb;
    }
    return e;
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
    if (m <= 16) return solve32_mc<16>(npad, Lf, lda, Wf, m, B, ldb, sync, s, prof);
    if (m <= 32) return solve32_mc<32>(npad, Lf, lda, Wf, m, B, ldb, sync, s, prof);
    return solve32_mc<64>(npad, Lf, lda, Wf, m, B, ldb, sync, s, prof);
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
    else
        hipLaunchKernelGGL(residual_partial_kernel<64>, grid, dim3(256), 0, st, A, lda, npad, X, ldx, m, jspan, partial);
    hipLaunchKernelGGL(residual_finish_kernel, dim3((npad + 255) / 256, m), dim3(256), 0, st, partial, ns, npad, m, B,
                       ldb, R, ldr);
    return hipGetLastError();
}

}  // namespace gbem
