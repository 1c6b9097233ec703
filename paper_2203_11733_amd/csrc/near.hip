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

// One workgroup per row i; counts near j in [0, i] and keeps the test
// results as bit masks: mask[i * nw + c] bit b <=> column 64 c + b is near
// (nw = ceil(n / 64) words per row; words past i / 64 are not written).
__global__ __launch_bounds__(256) void near_count_kernel(const double *__restrict__ lo,
                                                         const double *__restrict__ hi, int n,
                                                         double eta2, int64_t *__restrict__ cnt,
                                                         uint64_t *__restrict__ mask)
{
    __shared__ int64_t red[4];
    const int i = blockIdx.x;
    double li[3], hi_[3];
    for (int k = 0; k < 3; ++k) {
        li[k] = lo[3 * i + k];
        hi_[k] = hi[3 * i + k];
    }
    const double di = diam2_of(li, hi_);
    const int64_t nw = (n + 63) / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t c = 0;
    for (int base = 0; base <= i; base += 256) {   // uniform trip count: every lane reaches the ballot
        const int j = base + threadIdx.x;
        bool nr = false;
        if (j <= i) {
            double lj[3], hj[3];
            for (int k = 0; k < 3; ++k) {
                lj[k] = lo[3 * j + k];
                hj[k] = hi[3 * j + k];
            }
            nr = is_near(li, hi_, di, lj, hj, diam2_of(lj, hj), eta2);
        }
        c += nr ? 1 : 0;
        const uint64_t bits = __ballot(nr);
        const int w0 = base + 64 * wave;   // first column of this wave's word
        if (lane == 0 && w0 <= i) mask[(int64_t)i * nw + w0 / 64] = bits;
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) cnt[i] = red[0] + red[1] + red[2] + red[3];
}

hipError_t launch_near_count(const double *lo, const double *hi, int n, double eta2, int64_t *cnt,
                             uint64_t *mask, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(near_count_kernel, dim3(n), dim3(256), 0, s, lo, hi, n, eta2, cnt, mask);
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
