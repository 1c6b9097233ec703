// Galerkin-exact entries of the near pairs (and the diagonal), FP64.
//
// a_ij = 1/(4 pi |I_i||I_j|) Int_{I_i} Int_{I_j} 1/|x-y| (section 3.1, eq.
// "matrix").  Section 3.4 integrates the quadruple integral analytically along
// the in-plane directions (corner operator D) and numerically along whatever is
// left.  Here every case is closed: the double integral over two intervals of a
// function of the coordinate difference is a corner sum of a second
// antiderivative, and over one interval with a fixed point a corner sum of a
// first antiderivative, so with R = sqrt(.):
//
// Parallel rectangles, plane offset w (w = 0 covers coplanar pairs and the
// diagonal):  Int = sum_{corners} (+-) F(u, v, w), u, v the corner differences
// along the two in-plane axes, d^2/du^2 d^2/dv^2 F = 1/R:
//   F = (u^2-w^2)/2 v ln(v+R) + (v^2-w^2)/2 u ln(u+R) - u v w atan(uv/(wR))
//       - R (u^2 + v^2 - 2 w^2)/6
// Orthogonal rectangles (section 3.4, eq. "orthogonal"): s = difference along
// the shared axis (second antiderivative), p = offset of a point of I_j from the
// plane of I_i, q = offset of a point of I_i from the plane of I_j (first
// antiderivatives), d^2/ds^2 d/dp d/dq K = 1/R:
//   K = p q s ln(s+R) + q (3s^2 - q^2)/6 ln(p+R) + p (3s^2 - p^2)/6 ln(q+R)
//       - s/2 (q^2 atan(ps/(qR)) + p^2 atan(qs/(pR))) - s^3/6 atan(pq/(sR)) - pqR/3
// Both reduce to the paper's G1 - G2 (eqs. int1/int2) and G3 (eq. int4) along
// the way; they were checked by symbolic differentiation and against brute
// force.  Logarithms of z + R with z < 0 use ln(rho^2) - ln(R - z) to avoid
// cancellation; a log whose prefactor vanishes contributes 0 (x ln x -> 0).
//
// The 16-term corner sums cancel: the terms grow like D^3 while the integral
// is about |I_i||I_j|/D, so FP64 loses about kappa = D^4 / (|I_i| |I_j|)
// (D = centre distance + half diameters).  When kappa > 1e3 and the smaller
// panel lies at least 1.5 of its longest side away from the other one, the
// pair is integrated semi-analytically instead: a 10 x 10 Gauss rule (8 x 8
// when the gap is at least two sides) over the smaller panel of the
// closed-form potential of the larger rectangle,
//   Int_J 1/|x-y| dy = sum_{corners} (+-) [u ln(v+R) + v ln(u+R) - w atan(uv/(wR))],
// whose corner sum only loses (D/side)^2.  The potential is analytic near the
// smaller panel (its singular set, the larger rectangle, is >= 1.5 sides
// away), so the Gauss rule converges geometrically: along an axis of half
// width h the nearest singularity sits at least g / h >= 3 half widths off
// (g the gap), Bernstein ellipse parameter rho >= 3 + sqrt(10) = 6.2, error
// ~ rho^(-2n): 10 points give 1.6e-16; from g >= 2 sides, rho >= 8.1 and 8
// points give 3.5e-15 with 36 % fewer evaluations.
#include "gbem_internal.h"

#include <type_traits>

namespace gbem {

// ln(z + sqrt(z^2 + rho2)), R = sqrt(z^2 + rho2) given.
__device__ __forceinline__ double ln_z_plus_r(double z, double rho2, double R)
{
    if (z >= 0.0) return (z + R) > 0.0 ? log(z + R) : 0.0;
    if (rho2 <= 0.0) return 0.0;
    return log(rho2) - log(R - z);
}

__device__ double corner_parallel(double u, double v, double w)
{
    double u2 = u * u, v2 = v * v, w2 = w * w;
    double R = sqrt(u2 + v2 + w2);
    if (R == 0.0) return 0.0;
    double t = 0.0;
    double a = 0.5 * (u2 - w2) * v;
    if (a != 0.0) t += a * ln_z_plus_r(v, u2 + w2, R);
    double b = 0.5 * (v2 - w2) * u;
    if (b != 0.0) t += b * ln_z_plus_r(u, v2 + w2, R);
    if (w != 0.0 && u != 0.0 && v != 0.0) t -= u * v * w * atan(u * v / (w * R));
    t -= R * (u2 + v2 - 2.0 * w2) * (1.0 / 6.0);
    return t;
}

__device__ double corner_orthogonal(double s, double p, double q)
{
    double s2 = s * s, p2 = p * p, q2 = q * q;
    double R = sqrt(s2 + p2 + q2);
    if (R == 0.0) return 0.0;
    double t = 0.0;
    double a = p * q * s;
    if (a != 0.0) t += a * ln_z_plus_r(s, p2 + q2, R);
    double b = q * (3.0 * s2 - q2) * (1.0 / 6.0);
    if (b != 0.0) t += b * ln_z_plus_r(p, s2 + q2, R);
    double c = p * (3.0 * s2 - p2) * (1.0 / 6.0);
    if (c != 0.0) t += c * ln_z_plus_r(q, s2 + p2, R);
    if (s != 0.0) {
        if (q != 0.0 && p != 0.0) t -= 0.5 * s * q2 * atan(p * s / (q * R));
        if (p != 0.0 && q != 0.0) t -= 0.5 * s * p2 * atan(q * s / (p * R));
        if (p != 0.0 && q != 0.0) t -= s2 * s * (1.0 / 6.0) * atan(p * q / (s * R));
    }
    t -= p * q * R * (1.0 / 3.0);
    return t;
}

// u ln(v+R) + v ln(u+R) - w atan(uv/(wR)): d/du d/dv of it is 1/R.
__device__ __forceinline__ double corner_potential(double u, double v, double w)
{
    const double u2 = u * u, v2 = v * v, w2 = w * w;
    const double R = sqrt(u2 + v2 + w2);
    if (R == 0.0) return 0.0;
    double t = 0.0;
    if (u != 0.0) t += u * ln_z_plus_r(v, u2 + w2, R);
    if (v != 0.0) t += v * ln_z_plus_r(u, v2 + w2, R);
    if (w != 0.0 && u != 0.0 && v != 0.0) t -= w * atan(u * v / (w * R));
    return t;
}

// Int_{I_i} Int_{I_j} 1/|x-y| for axis-aligned rectangles given by lo/hi.
__device__ double pair_integral_closed(const double *li, const double *hi_, int ni,
                                       const double *lj, const double *hj, int nj)
{
    double g = 0.0;
    if (ni == nj) {
        const int t1 = ni == 0 ? 1 : 0, t2 = ni == 2 ? 1 : 2;
        const double w = li[ni] - lj[ni];
        const double x1[2] = {li[t1], hi_[t1]}, x2[2] = {li[t2], hi_[t2]};
        const double y1[2] = {lj[t1], hj[t1]}, y2[2] = {lj[t2], hj[t2]};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                const double u = x1[a] - y1[b];
                for (int c = 0; c < 2; ++c)
                    for (int d = 0; d < 2; ++d) {
                        const double v = x2[c] - y2[d];
                        const double f = corner_parallel(u, v, w);
                        g += ((a + b + c + d) & 1) ? -f : f;
                    }
            }
        return g;
    }
    const int sx = 3 - ni - nj;
    const double X = li[ni], Y = lj[nj];
    const double xs[2] = {li[sx], hi_[sx]}, ys[2] = {lj[sx], hj[sx]};
    const double pp[2] = {lj[ni] - X, hj[ni] - X};   // I_j along the normal of I_i
    const double qq[2] = {li[nj] - Y, hi_[nj] - Y};  // I_i along the normal of I_j
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const double s = xs[a] - ys[b];
            for (int c = 0; c < 2; ++c)
                for (int d = 0; d < 2; ++d) {
                    const double f = corner_orthogonal(s, pp[c], qq[d]);
                    // -sign(a) sign(b) for the difference axis, sign(c) sign(d)
                    // for the two single axes (sign = +1 upper, -1 lower)
                    g += ((a + b + c + d) & 1) ? f : -f;
                }
        }
    return g;
}

// Route of one pair: true = semi-analytic with panel `small_is_i` as the
// Gauss side (see the header comment for the rule).
// wide: the gap is at least two longest sides of the smaller panel
__device__ bool use_semi(const double *li, const double *hi_, const double *lj, const double *hj,
                         bool &small_is_i, bool *wide = nullptr)
{
    double ei[3], ej[3], gap2 = 0.0, cd2 = 0.0, di2 = 0.0, dj2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        ei[k] = hi_[k] - li[k];
        ej[k] = hj[k] - lj[k];
        const double g = fmax(0.0, fmax(lj[k] - hi_[k], li[k] - hj[k]));
        gap2 += g * g;
        const double d = 0.5 * (li[k] + hi_[k]) - 0.5 * (lj[k] + hj[k]);
        cd2 += d * d;
        di2 += ei[k] * ei[k];
        dj2 += ej[k] * ej[k];
    }
    const double D = sqrt(cd2) + 0.5 * (sqrt(di2) + sqrt(dj2));
    const double mi = fmax(ei[0], fmax(ei[1], ei[2])), mj = fmax(ej[0], fmax(ej[1], ej[2]));
    // area = product of the two non-zero extents = (sum of pairwise products)
    const double ai = ei[0] * ei[1] + ei[1] * ei[2] + ei[0] * ei[2];
    const double aj = ej[0] * ej[1] + ej[1] * ej[2] + ej[0] * ej[2];
    const double D2 = D * D;
    if (D2 * D2 <= 1e3 * ai * aj) return false;
    small_is_i = ai <= aj;
    const double ms = small_is_i ? mi : mj;
    if (wide) *wide = gap2 >= 4.0 * ms * ms;
    return gap2 >= 2.25 * ms * ms;
}

// Gauss rule of the semi-analytic route (set before each launch; the same
// values every time)
__constant__ NearRule c_near;

// component k of a 3-vector without a dynamic index (keeps it in registers)
__device__ __forceinline__ double comp(const double *v, int k) { return k == 0 ? v[0] : (k == 1 ? v[1] : v[2]); }

// Pass 1: one thread per near pair.  Pairs on the closed-form route are
// evaluated here; semi-analytic pairs are queued (wave-aggregated slots) for
// pass 2, so that their 100-point rule does not stall the closed-form lanes
// of the same wave.
__global__ __launch_bounds__(256) void near_eval_kernel(const double *__restrict__ lo,
                                                        const double *__restrict__ hi,
                                                        const Panel *__restrict__ pan,
                                                        const int32_t *__restrict__ row,
                                                        const int32_t *__restrict__ col,
                                                        int64_t nnz, double *__restrict__ A,
                                                        int64_t lda, int32_t *__restrict__ semi_list,
                                                        int32_t *__restrict__ semi_count, float *__restrict__ F,
                                                        int64_t ldf, const double *__restrict__ sc)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = t < nnz;
    int i = 0, j = 0;
    double li[3], hi_[3], lj[3], hj[3];
    bool semi = false, small_is_i = true;
    if (live) {
        i = row[t];
        j = col[t];
        for (int k = 0; k < 3; ++k) {
            li[k] = lo[3 * i + k];
            hi_[k] = hi[3 * i + k];
            lj[k] = lo[3 * j + k];
            hj[k] = hi[3 * j + k];
        }
        semi = use_semi(li, hi_, lj, hj, small_is_i);
    }
    const unsigned long long ballot = __ballot(semi);
    if (ballot) {
        const int lane = threadIdx.x & 63;
        int base = 0;
        if (lane == __ffsll((long long)ballot) - 1) base = atomicAdd(semi_count, __popcll(ballot));
        base = __shfl(base, __ffsll((long long)ballot) - 1);
        if (semi) semi_list[base + __popcll(ballot & ((1ull << lane) - 1))] = (int32_t)t;
    }
    if (!live || semi) return;
    const double G = pair_integral_closed(li, hi_, pan[i].nrm, lj, hj, pan[j].nrm);
    const double a = G / (4.0 * M_PI * pan[i].area * pan[j].area);
    A[i + j * lda] = a;
    A[j + i * lda] = a;
    if (F) F[i + j * ldf] = (float)(sc[i] * a * sc[j]);   // j <= i
}

// Pass 2: one wave per queued pair.  The 100 (or 64) Gauss points x 4 corners
// of the rectangle potential are spread over the lanes and summed by a fixed
// butterfly, so the value does not depend on scheduling.
__global__ __launch_bounds__(256) void near_semi_kernel(const double *__restrict__ lo,
                                                        const double *__restrict__ hi,
                                                        const Panel *__restrict__ pan,
                                                        const int32_t *__restrict__ row,
                                                        const int32_t *__restrict__ col,
                                                        const int32_t *__restrict__ semi_list,
                                                        const int32_t *__restrict__ semi_count,
                                                        double *__restrict__ A, int64_t lda, float *__restrict__ F,
                                                        int64_t ldf, const double *__restrict__ sc)
{
    const int lane = threadIdx.x & 63;
    const int nwaves = gridDim.x * (blockDim.x >> 6);
    const int count = *semi_count;
    for (int p = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); p < count; p += nwaves) {
        const int64_t t = semi_list[p];
        const int i = row[t], j = col[t];
        double li[3], hi_[3], lj[3], hj[3];
        for (int k = 0; k < 3; ++k) {
            li[k] = lo[3 * i + k];
            hi_[k] = hi[3 * i + k];
            lj[k] = lo[3 * j + k];
            hj[k] = hi[3 * j + k];
        }
        bool small_is_i = true, wide = false;
        (void)use_semi(li, hi_, lj, hj, small_is_i, &wide);   // uniform over the wave
        double ls[3], hs[3], lb[3], hb[3];
        for (int k = 0; k < 3; ++k) {
            ls[k] = small_is_i ? li[k] : lj[k];
            hs[k] = small_is_i ? hi_[k] : hj[k];
            lb[k] = small_is_i ? lj[k] : li[k];
            hb[k] = small_is_i ? hj[k] : hi_[k];
        }
        const int ns = small_is_i ? pan[i].nrm : pan[j].nrm, nb = small_is_i ? pan[j].nrm : pan[i].nrm;
        const int t1 = ns == 0 ? 1 : 0, t2 = ns == 2 ? 1 : 2;
        const double c1 = 0.5 * (comp(ls, t1) + comp(hs, t1)), h1 = 0.5 * (comp(hs, t1) - comp(ls, t1));
        const double c2 = 0.5 * (comp(ls, t2) + comp(hs, t2)), h2 = 0.5 * (comp(hs, t2) - comp(ls, t2));
        const double xn = comp(ls, ns);
        const int b1 = nb == 0 ? 1 : 0, b2 = nb == 2 ? 1 : 2;
        const double lbn = comp(lb, nb);
        double acc = 0.0;
        auto sum = [&](auto order, const double *gx, const double *gw) __attribute__((always_inline)) {
            constexpr int NO = decltype(order)::value;
            for (int e = lane; e < NO * NO * 4; e += 64) {
                const int pt = e >> 2, a = pt / NO, b = pt % NO, ca = (e >> 1) & 1, cc = e & 1;
                const double xa = c1 + h1 * gx[a], xb = c2 + h2 * gx[b];
                // point x: coordinate ns = xn, t1 = xa, t2 = xb
                double x[3];
                for (int k = 0; k < 3; ++k) x[k] = k == ns ? xn : (k == t1 ? xa : xb);
                const double w = comp(x, nb) - lbn;
                const double u = (ca ? comp(hb, b1) : comp(lb, b1)) - comp(x, b1);
                const double v = (cc ? comp(hb, b2) : comp(lb, b2)) - comp(x, b2);
                const double f = corner_potential(u, v, w);
                acc += gw[a] * gw[b] * (((ca + cc) & 1) ? -f : f);
            }
        };
        if (wide) sum(std::integral_constant<int, kNearOrderWide>(), c_near.x8, c_near.w8);
        else sum(std::integral_constant<int, kNearOrder>(), c_near.x, c_near.w);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) {
            const double a = acc * (4.0 * h1 * h2) / (4.0 * M_PI * pan[i].area * pan[j].area);
            A[i + j * lda] = a;
            A[j + i * lda] = a;
            if (F) F[i + j * ldf] = (float)(sc[i] * a * sc[j]);   // j <= i
        }
    }
}

// sc[i] = a_ii^(-1/2): the same closed form and expression as near_eval_kernel
// for the pair (i, i) (diagonal pairs are near and never semi-analytic: their
// gap is 0), so the value matches the diagonal the near pass writes.
__global__ __launch_bounds__(256) void self_scale_kernel(const double *__restrict__ lo,
                                                         const double *__restrict__ hi,
                                                         const Panel *__restrict__ pan, int n, int npad,
                                                         double *__restrict__ sc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    if (i >= n) {
        sc[i] = 1.0;   // identity padding
        return;
    }
    double li[3], hi_[3];
    for (int k = 0; k < 3; ++k) {
        li[k] = lo[3 * i + k];
        hi_[k] = hi[3 * i + k];
    }
    const double G = pair_integral_closed(li, hi_, pan[i].nrm, li, hi_, pan[i].nrm);
    const double a = G / (4.0 * M_PI * pan[i].area * pan[i].area);
    sc[i] = 1.0 / sqrt(a);
}

hipError_t launch_self_scale(const double *lo, const double *hi, const Panel *pan, int n, int npad, double *sc,
                             hipStream_t s)
{
    hipLaunchKernelGGL(self_scale_kernel, dim3((unsigned)((npad + 255) / 256)), dim3(256), 0, s, lo, hi, pan, n,
                       npad, sc);
    return hipGetLastError();
}

// Gauss rules of the semi-analytic reductions into constant memory (from a
// host copy: outside any captured region, since a captured copy would read
// the host buffer again at every replay)
hipError_t near_eval_upload_rule(hipStream_t s)
{
    NearRule g;
    gauss_legendre(kNearOrder, g.x, g.w);
    gauss_legendre(kNearOrderWide, g.x8, g.w8);
    return hipMemcpyToSymbolAsync(HIP_SYMBOL(c_near), &g, sizeof(g), 0, hipMemcpyHostToDevice, s);
}

hipError_t launch_near_eval(const double *lo, const double *hi, const Panel *pan,
                            const int32_t *row, const int32_t *col, int64_t nnz, double *A,
                            int64_t lda, int32_t *semi_buf, hipStream_t s, float *F, int64_t ldf,
                            const double *sc, bool upload_rule)
{
    if ((F == nullptr) != (sc == nullptr)) return hipErrorInvalidValue;
    if (nnz <= 0) return hipSuccess;
    hipError_t e = hipSuccess;
    if (upload_rule && (e = near_eval_upload_rule(s)) != hipSuccess) return e;
    int32_t *count = semi_buf, *list = semi_buf + 64;
    if ((e = launch_fill_i32(count, 1, 0, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(near_eval_kernel, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, lo, hi,
                       pan, row, col, nnz, A, lda, list, count, F, ldf, sc);
    const int64_t waves = std::min<int64_t>(nnz, 4096);
    hipLaunchKernelGGL(near_semi_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, lo, hi, pan, row, col,
                       list, count, A, lda, F, ldf, sc);
    return hipGetLastError();
}

}  // namespace gbem
