// Far-field assembly: a_ij = 1/(4 pi) sum_{a,b} w_a w_b / |x_a - y_b| over a
// p x p tensor Gauss-Legendre rule on each panel (weights normalised to sum 1),
// the quadrature form of eq. "matrix" (section 3.1) for well separated pairs.
// The near kernel overwrites near entries afterwards.
//
// Work per pair is p^4 evaluations of 1/r.  For axis-aligned panels the
// squared distance separates: index a (b) runs along the first in-plane axis
// of I_i (I_j) that both panels share, c (d) along the rest, and
//   parallel:   r^2 = (d1 + h1i x_a - h1j x_b)^2 + [(d2 + h2i x_c - h2j x_d)^2 + dn^2]
//   orthogonal: r^2 = (ds + hsi x_a - hsj x_b)^2 + [(dq + hqi x_c)^2 + (dp - hpj x_d)^2]
// so with S1[ab] and S2[cd] precomputed (2 p^2 values) each evaluation is one
// add, one reciprocal square root and one FMA.  Centre differences are formed
// in FP64 and only then rounded to the arithmetic type T.
//
// Tiling: one 256-thread workgroup per 64 x 64 tile of the lower triangle
// (tile row >= tile column).  Thread t owns row i = t % 64 and columns
// j = t / 64 + 4 m; a wave's 64 lanes write 64 consecutive doubles of a
// column (A is column-major).  The mirrored (upper) tile goes through LDS so
// that its stores are coalesced too; A is bitwise symmetric.  Rows/columns
// in [n, npad) get the identity.
#include "gbem_internal.h"

namespace gbem {

template <typename T> __device__ __forceinline__ T rsqrt_t(T x);

template <> __device__ __forceinline__ float rsqrt_t<float>(float x)
{
    return __builtin_amdgcn_rsqf(x);
}

// Hardware reciprocal square root refined by one Newton step
// y <- y (3 - x y^2) / 2, which squares its relative error: the hardware
// value is within 2^-24.2 of 1/sqrt(x) on gfx950 and the refined one within
// 4.2e-15 (measured over 4e7 arguments spanning 40 binades), far below what
// the far rule's quadrature error or the entries' 5e-12 parity bar resolve.
// (Two steps cost four more instructions per evaluation: 12.5 against 8.5.)
template <> __device__ __forceinline__ double rsqrt_t<double>(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    return (0.5 * y) * __builtin_fma(-x * y, y, 3.0);
}

// fused multiply-add in the arithmetic type itself (the plain builtin is the
// double one and would widen FP32 operands)
template <typename T> __device__ __forceinline__ T fma_t(T a, T b, T c);
template <> __device__ __forceinline__ float fma_t<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double fma_t<double>(double a, double b, double c)
{
    return __builtin_fma(a, b, c);
}

template <typename T> __device__ __forceinline__ T node(const GaussRule &g, int a);
template <> __device__ __forceinline__ float node<float>(const GaussRule &g, int a) { return g.xf[a]; }
template <> __device__ __forceinline__ double node<double>(const GaussRule &g, int a) { return g.x[a]; }
template <typename T> __device__ __forceinline__ T wprod(const GaussRule &g, int k);
template <> __device__ __forceinline__ float wprod<float>(const GaussRule &g, int k) { return g.wwf[k]; }
template <> __device__ __forceinline__ double wprod<double>(const GaussRule &g, int k) { return g.ww[k]; }

// component k of the centre without dynamic indexing of a private array
__device__ __forceinline__ double cc(const Panel &p, int k)
{
    return k == 0 ? p.c[0] : (k == 1 ? p.c[1] : p.c[2]);
}

template <int P, typename T>
__device__ __forceinline__ T far_pair(const Panel &pi, const Panel &pj, const GaussRule &g)
{
    T S1[P * P], S2[P * P];
    const int ni = pi.nrm, nj = pj.nrm;
    if (ni == nj) {
        const int t1 = ni == 0 ? 1 : 0, t2 = ni == 2 ? 1 : 2;
        const T d1 = (T)(cc(pi, t1) - cc(pj, t1));
        const T d2 = (T)(cc(pi, t2) - cc(pj, t2));
        const T dn = (T)(cc(pi, ni) - cc(pj, ni));
        const T dn2 = dn * dn;
        const T h1i = (T)pi.h1, h1j = (T)pj.h1, h2i = (T)pi.h2, h2j = (T)pj.h2;
#pragma unroll
        for (int a = 0; a < P; ++a)
#pragma unroll
            for (int b = 0; b < P; ++b) {
                T u = d1 + h1i * node<T>(g, a) - h1j * node<T>(g, b);
                S1[a * P + b] = u * u;
                T v = d2 + h2i * node<T>(g, a) - h2j * node<T>(g, b);
                S2[a * P + b] = v * v + dn2;
            }
    } else {
        const int sx = 3 - ni - nj;
        const int t1i = ni == 0 ? 1 : 0, t1j = nj == 0 ? 1 : 0;
        const T hsi = (T)(t1i == sx ? pi.h1 : pi.h2), hqi = (T)(t1i == sx ? pi.h2 : pi.h1);
        const T hsj = (T)(t1j == sx ? pj.h1 : pj.h2), hpj = (T)(t1j == sx ? pj.h2 : pj.h1);
        const T ds = (T)(cc(pi, sx) - cc(pj, sx));
        const T dq = (T)(cc(pi, nj) - cc(pj, nj));
        const T dp = (T)(cc(pi, ni) - cc(pj, ni));
        T U[P], V[P];
#pragma unroll
        for (int a = 0; a < P; ++a) {
            T q = dq + hqi * node<T>(g, a);
            U[a] = q * q;
            T p = dp - hpj * node<T>(g, a);
            V[a] = p * p;
        }
#pragma unroll
        for (int a = 0; a < P; ++a)
#pragma unroll
            for (int b = 0; b < P; ++b) {
                T u = ds + hsi * node<T>(g, a) - hsj * node<T>(g, b);
                S1[a * P + b] = u * u;
                S2[a * P + b] = U[a] + V[b];
            }
    }
    // orders above 4 only unroll the inner pair of loops (code size)
    constexpr int UO = P <= 4 ? P : 1;
    T acc = 0;
#pragma unroll UO
    for (int a = 0; a < P; ++a)
#pragma unroll UO
        for (int b = 0; b < P; ++b) {
            const T s1 = S1[a * P + b];
            T in = 0;
#pragma unroll
            for (int c = 0; c < P; ++c)
#pragma unroll
                for (int d = 0; d < P; ++d)
                    in = fma_t<T>(wprod<T>(g, c * P + d), rsqrt_t<T>(s1 + S2[c * P + d]), in);
            acc = fma_t<T>(wprod<T>(g, a * P + b), in, acc);
        }
    return acc;
}

// F != nullptr: also F[i + j ldf] = (float)(sc_i a_ij sc_j) for the lower tile
template <int P, typename T>
__global__ __launch_bounds__(256) void far_tile_kernel(const Panel *__restrict__ pan, int n,
                                                       int ntile, GaussRule g,
                                                       double *__restrict__ A, int64_t lda,
                                                       float *__restrict__ F, int64_t ldf,
                                                       const double *__restrict__ sc)
{
    __shared__ Panel pj_s[kFarTile];
    __shared__ double tile[kFarTile][kFarTile + 1];
    __shared__ double scj[kFarTile];   // column scales of F

    // lower-triangle tile (I, J), I >= J, from the linear block index
    const int64_t t = blockIdx.x;
    int I = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((int64_t)I * (I + 1) / 2 > t) --I;
    while ((int64_t)(I + 1) * (I + 2) / 2 <= t) ++I;
    const int J = (int)(t - (int64_t)I * (I + 1) / 2);

    const int tid = threadIdx.x;
    const int il = tid & 63, jg = tid >> 6;
    const int i = I * kFarTile + il;
    const int j0 = J * kFarTile;

    if (tid < kFarTile) {
        int j = j0 + tid;
        if (j < n) pj_s[tid] = pan[j];
        if (F) scj[tid] = sc[j];   // j < npad
    }
    Panel pi;
    if (i < n) pi = pan[i];
    __syncthreads();

    const double inv4pi = 0.25 / M_PI;
    for (int m = 0; m < kFarTile / 4; ++m) {
        const int jl = jg + 4 * m;
        const int j = j0 + jl;
        double v;
        if (i >= n || j >= n) {
            v = (i == j) ? 1.0 : 0.0;
        } else if (I == J && jl > il) {
            v = 0.0;   // filled from the mirrored entry
        } else {
            v = (double)far_pair<P, T>(pi, pj_s[jl], g) * inv4pi;
        }
        tile[il][jl] = v;
    }
    __syncthreads();
    // lower tile (rows i, columns j)
    const double si = F ? sc[i] : 0.0;
    for (int m = 0; m < kFarTile / 4; ++m) {
        const int jl = jg + 4 * m;
        double v = (I == J && jl > il) ? tile[jl][il] : tile[il][jl];
        A[(int64_t)(I * kFarTile + il) + (int64_t)(j0 + jl) * lda] = v;
        if (F && (I != J || jl <= il)) F[(int64_t)i + (int64_t)(j0 + jl) * ldf] = (float)(si * v * scj[jl]);
    }
    // mirrored tile (rows j, columns i); the diagonal tile is already complete
    if (I != J) {
        for (int m = 0; m < kFarTile / 4; ++m) {
            const int ilm = jg + 4 * m;   // column index within the mirrored tile
            A[(int64_t)(j0 + il) + (int64_t)(I * kFarTile + ilm) * lda] = tile[ilm][il];
        }
    }
}

template <typename T>
static hipError_t launch_far_t(const Panel *pan, int n, int npad, int p, const GaussRule &g,
                               double *A, int64_t lda, hipStream_t s, float *F, int64_t ldf, const double *sc)
{
    const int ntile = npad / kFarTile;
    const int64_t nblk = (int64_t)ntile * (ntile + 1) / 2;
    dim3 grid((unsigned)nblk), block(256);
#define FAR_CASE(PP)                                                                                           \
    case PP:                                                                                                   \
        hipLaunchKernelGGL((far_tile_kernel<PP, T>), grid, block, 0, s, pan, n, ntile, g, A, lda, F, ldf, sc); \
        break;
    switch (p) {
    FAR_CASE(1)
    FAR_CASE(2)
    FAR_CASE(3)
    FAR_CASE(4)
    FAR_CASE(5)
    FAR_CASE(6)
    FAR_CASE(8)
    default: return hipErrorInvalidValue;
    }
#undef FAR_CASE
    return hipGetLastError();
}

hipError_t launch_far(const Panel *pan, int n, int npad, int p, const GaussRule &rule,
                      int far_dtype, double *A, int64_t lda, hipStream_t s, float *F, int64_t ldf,
                      const double *sc)
{
    if (npad % kFarTile) return hipErrorInvalidValue;
    if ((F == nullptr) != (sc == nullptr)) return hipErrorInvalidValue;
    if (far_dtype == GBEM_F32) return launch_far_t<float>(pan, n, npad, p, rule, A, lda, s, F, ldf, sc);
    return launch_far_t<double>(pan, n, npad, p, rule, A, lda, s, F, ldf, sc);
}

}  // namespace gbem
