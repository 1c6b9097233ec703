// Near/far classification of panel pairs (j <= i) into a CSR list.
//
// The paper evaluates every matrix entry by the section 3.4 reductions; this
// library evaluates only near pairs that way and uses Gauss quadrature for the
// rest.  The split:
//   d_k   = max(0, lo_j[k] - hi_i[k], lo_i[k] - hi_j[k])
//   sep2  = (d_0^2 + d_1^2) + d_2^2
//   diam2 = (e_0^2 + e_1^2) + e_2^2,  e_k = hi[k] - lo[k]
//   near  iff sep2 < eta2 * max(diam2_i, diam2_j)
// Every operation is a correctly rounded IEEE operation in this fixed order
// (this file is compiled with -ffp-contract=off), so the list is bit-exact.
#include "gbem_internal.h"

namespace gbem {

__device__ __forceinline__ double diam2_of(const double *l, const double *h)
{
    double e0 = h[0] - l[0], e1 = h[1] - l[1], e2 = h[2] - l[2];
    return (e0 * e0 + e1 * e1) + e2 * e2;
}

__device__ __forceinline__ bool is_near(const double *li, const double *hi_, double di,
                                        const double *lj, const double *hj, double dj, double eta2)
{
    double d[3];
    for (int k = 0; k < 3; ++k) {
        double g1 = lj[k] - hi_[k], g2 = li[k] - hj[k];
        double g = g1 > g2 ? g1 : g2;
        d[k] = g > 0.0 ? g : 0.0;
    }
    double sep2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    double dm = di > dj ? di : dj;
    return sep2 < eta2 * dm;
}

// Counts near j in [0, i] for every row i and keeps the test results as bit
// masks: mask[i * nw + c] bit b <=> column 64 c + b is near (nw = ceil(n /
// 64) words per row; words past i / 64 are not written).  Workgroup: 64 rows
// x 256 columns of the lower triangle (grid: column blocks x row blocks;
// blocks wholly above the diagonal return); a thread keeps its column's box
// and diameter, the rows' come from LDS; each wave's ballot is one mask word,
// its popcount goes to cnt[i] by an integer atomic (cnt zeroed first).
__global__ __launch_bounds__(256) void near_count_kernel(const double *__restrict__ lo,
                                                         const double *__restrict__ hi, int n,
                                                         double eta2, int64_t *__restrict__ cnt,
                                                         uint64_t *__restrict__ mask)
{
    __shared__ double rl[64][3], rh[64][3], rd[64];
    const int c0 = blockIdx.x * 256, i0 = blockIdx.y * 64;
    if (c0 > i0 + 63) return;   // uniform
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rows = min(64, n - i0);
    if (tid < rows) {
        double l[3], h[3];
        for (int k = 0; k < 3; ++k) {
            l[k] = lo[3 * (i0 + tid) + k];
            h[k] = hi[3 * (i0 + tid) + k];
            rl[tid][k] = l[k];
            rh[tid][k] = h[k];
        }
        rd[tid] = diam2_of(l, h);
    }
    const int j = c0 + tid;
    const bool colok = j < n;
    double lj[3] = {0.0, 0.0, 0.0}, hj[3] = {0.0, 0.0, 0.0}, dj = 0.0;
    if (colok) {
        for (int k = 0; k < 3; ++k) {
            lj[k] = lo[3 * j + k];
            hj[k] = hi[3 * j + k];
        }
        dj = diam2_of(lj, hj);
    }
    __syncthreads();
    const int64_t nw = (n + 63) / 64;
    const int w0 = c0 + 64 * wave;   // first column of this wave's word
    for (int r = 0; r < rows; ++r) {
        const int i = i0 + r;
        const double li[3] = {rl[r][0], rl[r][1], rl[r][2]}, hi_[3] = {rh[r][0], rh[r][1], rh[r][2]};
        const bool nr = colok && j <= i && is_near(li, hi_, rd[r], lj, hj, dj, eta2);
        const uint64_t bits = __ballot(nr);
        if (lane == 0 && w0 <= i) {
            mask[(int64_t)i * nw + w0 / 64] = bits;
            if (bits) atomicAdd((unsigned long long *)(cnt + i), (unsigned long long)__popcll(bits));
        }
    }
}
hipError_t launch_near_count(const double *lo, const double *hi, int n, double eta2, int64_t *cnt,
                             uint64_t *mask, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipError_t e = hipMemsetAsync(cnt, 0, sizeof(int64_t) * n, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(near_count_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)((n + 63) / 64)), dim3(256), 0,
                       s, lo, hi, n, eta2, cnt, mask);
    return hipGetLastError();
}
// Exclusive scan of n counts into row_ptr[0..n] (single workgroup, in order).
__global__ __launch_bounds__(1024) void scan_kernel(const int64_t *__restrict__ cnt, int n,
                                                    int64_t *__restrict__ row_ptr)
{
    __shared__ int64_t buf[1024];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        int i = base + threadIdx.x;
        int64_t v = i < n ? cnt[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        // Hillis-Steele inclusive scan
        for (int off = 1; off < 1024; off <<= 1) {
            int64_t t = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < n) row_ptr[i] = carry + buf[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += buf[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) row_ptr[n] = carry;
}

hipError_t launch_exclusive_scan(const int64_t *cnt, int n, int64_t *row_ptr, hipStream_t s)
{
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, cnt, n, row_ptr);
    return hipGetLastError();
}

// One wave per row: the columns of row i in ascending order, read from the
// masks of near_count (popcounts, a prefix sum over the wave's 64 words,
// then each lane writes the set bits of its word), and the row index.
__global__ __launch_bounds__(256) void near_fill_kernel(const uint64_t *__restrict__ mask, int n,
                                                        const int64_t *__restrict__ row_ptr,
                                                        int32_t *__restrict__ row, int32_t *__restrict__ col)
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;   // whole wave
    const int64_t nw = (n + 63) / 64;
    const int words = i / 64 + 1;
    int64_t out = row_ptr[i];
    for (int g = 0; g < words; g += 64) {
        const int w = g + lane;
        uint64_t bits = w < words ? mask[(int64_t)i * nw + w] : 0ull;
        const int pc = __popcll(bits);
        int incl = pc;   // inclusive prefix over the lanes
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(incl, off, 64);
            if (lane >= off) incl += t;
        }
        int64_t o = out + incl - pc;
        while (bits) {
            const int b = __ffsll((long long)bits) - 1;
            bits &= bits - 1;
            col[o] = 64 * w + b;
            row[o] = i;
            ++o;
        }
        out += __shfl(incl, 63, 64);
    }
}
hipError_t launch_near_fill(const uint64_t *mask, int n, const int64_t *row_ptr, int32_t *row, int32_t *col,
                            hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(near_fill_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, mask, n, row_ptr, row, col);
    return hipGetLastError();
}
}  // namespace gbem
