// Multi-dielectric case (section 4): the double-layer integrals Q_ik of
// section 4.2, the region-by-region Galerkin system of section 4.1 and the
// pieces of its solve.
//
// Q_ik = Int_{I_i} Int_{I_k} <x - y, n_k> / (4 pi |x - y|^3) dG(y) dG(x), the
// normal of I_k along + its normal axis.
//   far pairs (the near list's complement): the inner integral over the flat
//   rectangle I_k in closed form (its solid angle at x over 4 pi: sum over the
//   corners of s_x s_y atan(u v / (h r)), h the height of x over the plane of
//   I_k, evaluated as one atan2), the outer one n x n Gauss-Legendre over
//   I_i with n = 6 at the near threshold down to 2 at 40 diameters (within
//   about 1e-13 |I_i| of the exact value); one thread per pair.
//   near pairs: all four integrations in closed form, one thread per ordered
//   pair.  Section 4.2 integrates the kernel analytically along all but one
//   coordinate (corner differences D of antiderivatives) and leaves a single
//   1-D integral; that last integral is elementary too, so each near entry is
//   a 16-term corner sum:
//     parallel panels, separation b = x_n - y_n != 0, offsets p1, p2 along
//     the two shared in-plane axes:
//       K(p1, p2) = b (p1 atanh(p1/R) + p2 atanh(p2/R) - R)
//                   + p1 p2 atan(p1 p2 / (b R)),   R = |(p1, p2, b)|;
//     orthogonal panels, w = height of x over the plane of I_k (along an
//     in-plane axis of I_i), p = offset along the shared axis, q = offset
//     along the normal of I_i (an in-plane axis of I_k):
//       L(p, q, w) = q R / 2 + (w^2 - p^2) / 2 asinh(q / |(p, w)|)
//                    - p q asinh(p / |(q, w)|) + p w atan(p q / (w R)).
//     Terms whose coefficient vanishes are dropped (their limits are 0), so
//     touching and T-junction pairs need no special case.
// Coplanar pairs (both normals on one axis, one plane) give 0 (section 4.2).
#include "gbem_internal.h"

namespace gbem {

namespace {
constexpr double kInv4Pi = 0.07957747154594767;   // 1 / (4 pi)

// centre coordinate k of a panel record (selects, no dynamic indexing)
__device__ __forceinline__ double pc(const Panel &p, int k) { return k == 0 ? p.c[0] : (k == 1 ? p.c[1] : p.c[2]); }
// lower/upper corner coordinate k of a panel record
__device__ __forceinline__ double plo(const Panel &p, int k, int t1, int t2)
{
    return k == t1 ? pc(p, k) - p.h1 : (k == t2 ? pc(p, k) - p.h2 : pc(p, k));
}
__device__ __forceinline__ double phi(const Panel &p, int k, int t1, int t2)
{
    return k == t1 ? pc(p, k) + p.h1 : (k == t2 ? pc(p, k) + p.h2 : pc(p, k));
}
__device__ __forceinline__ void inplane(int nrm, int &t1, int &t2)
{
    t1 = nrm == 0 ? 1 : 0;
    t2 = nrm == 2 ? 1 : 2;
}
struct P3 {
    double x, y, z;
};
__device__ __forceinline__ double comp(const P3 &p, int k) { return k == 0 ? p.x : (k == 1 ? p.y : p.z); }
// the point with coordinate va along axis t1, vb along t2 and vn along the third
__device__ __forceinline__ P3 place(int t1, int t2, double va, double vb, double vn)
{
    P3 p;
    p.x = t1 == 0 ? va : (t2 == 0 ? vb : vn);
    p.y = t1 == 1 ? va : (t2 == 1 ? vb : vn);
    p.z = t1 == 2 ? va : (t2 == 2 ? vb : vn);
    return p;
}

// The source panel in its own frame: extents along its two in-plane axes and
// the plane coordinate.
struct Source {
    int nrm, t1, t2;
    double x1, x2, y1, y2, z;
};
__device__ __forceinline__ Source source_of(const Panel &p)
{
    Source s;
    s.nrm = p.nrm;
    inplane(p.nrm, s.t1, s.t2);
    s.x1 = pc(p, s.t1) - p.h1;
    s.x2 = pc(p, s.t1) + p.h1;
    s.y1 = pc(p, s.t2) - p.h2;
    s.y2 = pc(p, s.t2) + p.h2;
    s.z = pc(p, s.nrm);
    return s;
}

// Int over I_k of q*(x, y) dG(y) at x (normal of I_k along +): the solid angle
// Omega over 4 pi, Omega = sum over the corners of s_x s_y atan(u v / (h r)),
// for points x from which the rectangle subtends |Omega| < pi (every far pair:
// the solid angle there is below 1/8).  The four atan terms are the arguments
// of (h r_ab +- i u_a v_b), whose real parts carry the common sign of h, so
// their sum is the argument of the product of the four factors (the positive
// scale h^4 r_11 r_12 r_21 r_22 drops out): one atan2 and no division.
// h |(u, v, h)| from the hardware reciprocal square root with one Newton
// step (within about 4e-15 relative); the solid angle takes it as a scale of
// a whole factor, so the error stays at that level in Omega
__device__ __forceinline__ double h_times_r(double h, double q)
{
    double y = __builtin_amdgcn_rsq(q);
    y = (0.5 * y) * __builtin_fma(-q * y, y, 3.0);
    return h * (q * y);
}

__device__ __forceinline__ double dl_potential_far(const Source &s, const P3 &x)
{
    const double h = comp(x, s.nrm) - s.z;
    if (h == 0.0) return 0.0;
    const double px = comp(x, s.t1), py = comp(x, s.t2);
    const double u2 = s.x2 - px, u1 = s.x1 - px, v2 = s.y2 - py, v1 = s.y1 - py;
    const double h2 = h * h;
    const double a = h_times_r(h, u2 * u2 + v2 * v2 + h2), b = u2 * v2;    // + atan(u2 v2 / (h r))
    const double c = h_times_r(h, u1 * u1 + v1 * v1 + h2), d = u1 * v1;    // + atan(u1 v1 / (h r))
    const double e = h_times_r(h, u2 * u2 + v1 * v1 + h2), f = -u2 * v1;   // - atan(u2 v1 / (h r))
    const double g = h_times_r(h, u1 * u1 + v2 * v2 + h2), k = -u1 * v2;   // - atan(u1 v2 / (h r))
    const double re1 = a * c - b * d, im1 = a * d + b * c;
    const double re2 = e * g - f * k, im2 = e * k + f * g;
    return atan2(re1 * im2 + im1 * re2, re1 * re2 - im1 * im2) * kInv4Pi;
}

__device__ __forceinline__ bool coplanar(const Panel &a, const Panel &b)
{
    return a.nrm == b.nrm && pc(a, a.nrm) == pc(b, b.nrm);
}
}  // namespace

// Gauss-Legendre rules of 2..6 points per direction for the far pairs (nodes
// on [-1, 1] and halved weights, rule n at offset (n - 2)(n + 1) / 2), written
// by launch_double_layer from the library's own rule generator.
__constant__ double kFarX[20], kFarW[20];

__device__ __forceinline__ double half_extent(const Panel &p, int k)
{
    int t1, t2;
    inplane(p.nrm, t1, t2);
    return k == t1 ? p.h1 : (k == t2 ? p.h2 : 0.0);
}

// Points per direction of the far rule on the target, from the gap between
// the two panels' boxes over the larger diameter (rho): the rule's error,
// measured against the closed form of both integrals at the worst
// orientations, stays below about 1e-13 |I_i| with 6 points from rho = 2 (the
// near threshold), 5 from 3, 4 from 5, 3 from 12 and 2 from 40.
__device__ __forceinline__ int far_points(const Panel &T, const Panel &S)
{
    double g2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double g = fmax(0.0, fabs(pc(T, k) - pc(S, k)) - (half_extent(T, k) + half_extent(S, k)));
        g2 = fma(g, g, g2);
    }
    const double d2 = fmax(T.diam2, S.diam2);
    return g2 >= 1600.0 * d2 ? 2 : g2 >= 144.0 * d2 ? 3 : g2 >= 25.0 * d2 ? 4 : g2 >= 9.0 * d2 ? 5 : 6;
}

// Q[i + k ldq] for every pair with the far rule (near pairs are overwritten
// by dl_near_kernel).  Block: 256 targets i for one source k at a time.
__global__ __launch_bounds__(256) void dl_far_kernel(const Panel *__restrict__ pan, int n, double *__restrict__ Q,
                                                     int64_t ldq)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const Panel pi = pan[i];
    int t1, t2;
    inplane(pi.nrm, t1, t2);
    const double c1 = pc(pi, t1), c2 = pc(pi, t2), cn = pc(pi, pi.nrm);
    for (int k = blockIdx.y; k < n; k += gridDim.y) {
        const Panel pk = pan[k];
        double q = 0.0;
        if (!coplanar(pi, pk)) {
            const Source s = source_of(pk);
            const int np = far_points(pi, pk), off = (np - 2) * (np + 1) / 2;
            for (int a = 0; a < np; ++a) {
                const double xa = c1 + pi.h1 * kFarX[off + a], wa = kFarW[off + a];
                double qa = 0.0;
                for (int b = 0; b < np; ++b) {
                    const P3 x = place(t1, t2, xa, c2 + pi.h2 * kFarX[off + b], cn);
                    qa = fma(kFarW[off + b], dl_potential_far(s, x), qa);
                }
                q = fma(wa, qa, q);
            }
            q *= pi.area;
        }
        Q[i + (int64_t)k * ldq] = q;
    }
}

// Double antiderivatives of the kernel (see the header), zero where their
// coefficient vanishes.
__device__ __forceinline__ double k_parallel(double p1, double p2, double b)
{
    const double R = sqrt(p1 * p1 + p2 * p2 + b * b);
    double t = -R;
    if (p1 != 0.0) t += p1 * atanh(p1 / R);
    if (p2 != 0.0) t += p2 * atanh(p2 / R);
    t *= b;
    if (p1 != 0.0 && p2 != 0.0) t += p1 * p2 * atan(p1 * p2 / (b * R));
    return t;
}
__device__ __forceinline__ double l_orthogonal(double p, double q, double w)
{
    const double R = sqrt(p * p + q * q + w * w);
    double t = 0.5 * q * R;
    if (q != 0.0 && w * w != p * p) t += 0.5 * (w * w - p * p) * asinh(q / sqrt(p * p + w * w));
    if (q != 0.0 && p != 0.0) t -= q * p * asinh(p / sqrt(q * q + w * w));
    if (p != 0.0 && q != 0.0 && w != 0.0) t += p * w * atan(p * q / (w * R));
    return t;
}

// Near pairs: pairs (row[e], col[e]) of the near list (col <= row) in both
// orders, one thread per ordered pair (thread 2 e + order), closed form.
__global__ __launch_bounds__(256) void dl_near_kernel(const Panel *__restrict__ pan, const int32_t *__restrict__ row,
                                                      const int32_t *__restrict__ col, int64_t nnz,
                                                      double *__restrict__ Q, int64_t ldq)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t e = g >> 1;
    if (e >= nnz) return;
    const int r = row[e], c = col[e];
    if (r == c && (g & 1)) return;   // the diagonal once
    const int ti = (g & 1) ? c : r, sk = (g & 1) ? r : c;
    const Panel T = pan[ti], S = pan[sk];
    double sum = 0.0;
    if (!coplanar(T, S)) {
        int t1, t2, u1, u2;
        inplane(T.nrm, t1, t2);
        inplane(S.nrm, u1, u2);
        if (T.nrm == S.nrm) {
            // int over x in [xa, xb], y in [ya, yb] of f(x - y) = sum of the
            // corners (xb - ya) + (xa - yb) - (xa - ya) - (xb - yb) of its
            // double antiderivative
            const double b = pc(T, T.nrm) - pc(S, S.nrm);
            const double xa1 = plo(T, t1, t1, t2), xb1 = phi(T, t1, t1, t2);
            const double ya1 = plo(S, t1, u1, u2), yb1 = phi(S, t1, u1, u2);
            const double xa2 = plo(T, t2, t1, t2), xb2 = phi(T, t2, t1, t2);
            const double ya2 = plo(S, t2, u1, u2), yb2 = phi(S, t2, u1, u2);
            const double P1[4] = {xb1 - ya1, xa1 - yb1, xa1 - ya1, xb1 - yb1};
            const double P2[4] = {xb2 - ya2, xa2 - yb2, xa2 - ya2, xb2 - yb2};
#pragma unroll
            for (int m1 = 0; m1 < 4; ++m1)
#pragma unroll
                for (int m2 = 0; m2 < 4; ++m2) {
                    const double sg = ((m1 < 2) == (m2 < 2)) ? 1.0 : -1.0;
                    sum += sg * k_parallel(P1[m1], P2[m2], b);
                }
        } else {
            // height axis hc (normal of S, in the plane of T), shared axis hb,
            // and T's normal ha (in the plane of S)
            const int hc = S.nrm, ha = T.nrm, hb = 3 - S.nrm - T.nrm;
            const double sz = pc(S, hc), tz = pc(T, ha);
            const double W[2] = {phi(T, hc, t1, t2) - sz, plo(T, hc, t1, t2) - sz};
            const double xa = plo(T, hb, t1, t2), xb = phi(T, hb, t1, t2);
            const double ya = plo(S, hb, u1, u2), yb = phi(S, hb, u1, u2);
            const double P[4] = {xb - ya, xa - yb, xa - ya, xb - yb};
            const double Qv[2] = {tz - plo(S, ha, u1, u2), tz - phi(S, ha, u1, u2)};
#pragma unroll
            for (int mw = 0; mw < 2; ++mw)
#pragma unroll
                for (int mp = 0; mp < 4; ++mp)
#pragma unroll
                    for (int mq = 0; mq < 2; ++mq) {
                        const double sg = ((mw == 0) == (mq == 0)) == (mp < 2) ? 1.0 : -1.0;
                        sum += sg * l_orthogonal(P[mp], Qv[mq], W[mw]);
                    }
        }
        sum *= kInv4Pi;
    }
    Q[ti + (int64_t)sk * ldq] = sum;
}

hipError_t launch_double_layer(const Panel *pan, int n, const int32_t *row, const int32_t *col, int64_t nnz,
                               double *Q, int64_t ldq, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    double x[20], w[20];
    for (int p = 2, off = 0; p <= 6; off += p, ++p) gauss_legendre(p, x + off, w + off);
    hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(kFarX), x, sizeof x, 0, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyToSymbolAsync(HIP_SYMBOL(kFarW), w, sizeof w, 0, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dl_far_kernel, dim3((n + 255) / 256, std::min(n, 65535)), dim3(256), 0, s, pan, n, Q, ldq);
    e = hipGetLastError();
    if (e != hipSuccess || nnz == 0) return e;
    hipLaunchKernelGGL(dl_near_kernel, dim3((unsigned)((2 * nnz + 255) / 256)), dim3(256), 0, s, pan, row, col, nnz,
                       Q, ldq);
    return hipGetLastError();
}

// ---------------------------------------------------------------- system
// Row r = (region eq_reg[r], panel eq_pan[r]) of the Galerkin system (eq_reg
// -1: a gap row between two regions' row ranges, left zero), column k
// a panel of that region's boundary (orientation: the region's outward normal
// is -e_n when it lies on the + side of panel k, +e_n otherwise):
//   u unknown at k (Neumann, interface):       M[r, u_slot[k]] = 1/2 |I_i| [k = i] + s Q_ik
//   q unknown at k (conductor, Dirichlet, interface): M[r, q_slot[k]] = -f G_ik,
//     f = 1, or for an interface panel seen from its + side region
//     -eps_minus / eps_plus (the unknown is the - side region's q)
// Every (row, slot) is written by one thread, into M and its transpose Mt.
// G = A |I_i| |I_k| (A: the single-layer entries with their 1 / (|I_i| |I_k|)
// normalisation).
__global__ __launch_bounds__(256) void dl_system_kernel(const Panel *__restrict__ pan, int n,
                                                        const double *__restrict__ A, int64_t lda,
                                                        const double *__restrict__ Q, int64_t ldq,
                                                        const int32_t *__restrict__ kind, const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ rm, const double *__restrict__ eps,
                                                        const int32_t *__restrict__ eq_reg,
                                                        const int32_t *__restrict__ eq_pan,
                                                        const int32_t *__restrict__ u_slot,
                                                        const int32_t *__restrict__ q_slot, int nu,
                                                        double *__restrict__ M, double *__restrict__ Mt, int64_t ldm)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    for (int r = blockIdx.y; r < nu; r += gridDim.y) {
        const int a = eq_reg[r], i = eq_pan[r];
        if (a < 0 || (rp[k] != a && rm[k] != a)) continue;   // a < 0: a gap row (all zero)
        const double sgn = rp[k] == a ? -1.0 : 1.0;
        if (u_slot[k] >= 0) {
            const double coef = (k == i ? 0.5 * pan[i].area : 0.0) + sgn * Q[i + (int64_t)k * ldq];
            M[r + (int64_t)u_slot[k] * ldm] = coef;
            Mt[u_slot[k] + (int64_t)r * ldm] = coef;
        }
        if (q_slot[k] >= 0) {
            double f = 1.0;
            if (kind[k] == 3 && rp[k] == a) f = -eps[rm[k]] / eps[rp[k]];
            const double g = -f * A[i + (int64_t)k * lda] * pan[i].area * pan[k].area;
            M[r + (int64_t)q_slot[k] * ldm] = g;
            Mt[q_slot[k] + (int64_t)r * ldm] = g;
        }
    }
}

// Right-hand side of main net m (column m of B, and -B beside it): the known
// potential 1 on the panels of conductor m moved to the right,
// b_r = -sum over those panels k of the region of row r of
// (1/2 |I_i| [k = i] + s Q_ik); the net's panels in order.
__global__ __launch_bounds__(256) void dl_rhs_kernel(const Panel *__restrict__ pan, const double *__restrict__ Q,
                                                     int64_t ldq, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ rm,
                                                     const int32_t *__restrict__ eq_reg,
                                                     const int32_t *__restrict__ eq_pan,
                                                     const int32_t *__restrict__ cp_ptr,
                                                     const int32_t *__restrict__ cp_idx, int nu,
                                                     double *__restrict__ B, double *__restrict__ Bneg, int64_t ldb)
{
    const int r = blockIdx.x * 256 + threadIdx.x, m = blockIdx.y;
    if (r >= nu) return;
    const int a = eq_reg[r], i = eq_pan[r];
    if (a < 0) {   // a gap row
        B[r + (int64_t)m * ldb] = 0.0;
        Bneg[r + (int64_t)m * ldb] = 0.0;
        return;
    }
    double b = 0.0;
    for (int t = cp_ptr[m]; t < cp_ptr[m + 1]; ++t) {
        const int k = cp_idx[t];
        if (rp[k] != a && rm[k] != a) continue;
        const double sgn = rp[k] == a ? -1.0 : 1.0;
        b -= (k == i ? 0.5 * pan[i].area : 0.0) + sgn * Q[i + (int64_t)k * ldq];
    }
    B[r + (int64_t)m * ldb] = b;
    Bneg[r + (int64_t)m * ldb] = -b;
}

// C[k * m_main + m] = scale * sum over the panels of conductor k of eps q |I|,
// the region's q (along its outward normal, into the conductor) from column m
// of X.  One workgroup per (k, m): strided partial sums, then a fixed-order
// tree, so the result does not depend on timing.
__global__ __launch_bounds__(256) void dl_charge_kernel(const Panel *__restrict__ pan, const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ rm,
                                                        const double *__restrict__ eps,
                                                        const int32_t *__restrict__ q_slot,
                                                        const int32_t *__restrict__ cp_ptr,
                                                        const int32_t *__restrict__ cp_idx,
                                                        const double *__restrict__ X, int64_t ldx, int m_main,
                                                        double scale, double *__restrict__ C)
{
    __shared__ double red[4];
    const int k = blockIdx.x, m = blockIdx.y;
    double s = 0.0;
    for (int t = cp_ptr[k] + (int)threadIdx.x; t < cp_ptr[k + 1]; t += 256) {
        const int i = cp_idx[t];
        const int a = rp[i] >= 0 ? rp[i] : rm[i];
        s += eps[a] * X[q_slot[i] + (int64_t)m * ldx] * pan[i].area;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) C[k * m_main + m] = scale * ((red[0] + red[1]) + (red[2] + red[3]));
}

__global__ void dl_negate_kernel(double *__restrict__ A, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) A[i] = -A[i];
}

hipError_t launch_dl_negate(double *A, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(dl_negate_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1 << 16)), dim3(256), 0, s,
                       A, n);
    return hipGetLastError();
}

__global__ void dl_sub_kernel(double *__restrict__ X, int64_t ldx, const double *__restrict__ D, int64_t ldd, int rows)
{
    const int i = blockIdx.x * 256 + threadIdx.x, c = blockIdx.y;
    if (i < rows) X[i + (int64_t)c * ldx] -= D[i + (int64_t)c * ldd];
}

hipError_t launch_dl_system(const Panel *pan, int n, const double *A, int64_t lda, const double *Q, int64_t ldq,
                            const int32_t *kind, const int32_t *rp, const int32_t *rm, const double *eps,
                            const int32_t *eq_reg, const int32_t *eq_pan, const int32_t *u_slot,
                            const int32_t *q_slot, const int32_t *cp_ptr, const int32_t *cp_idx, int nu, int m_main,
                            double *M, double *Mt, int64_t ldm, double *B, double *Bneg, int64_t ldb, hipStream_t s)
{
    if (n <= 0 || nu <= 0 || m_main <= 0 || m_main > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(dl_system_kernel, dim3((n + 255) / 256, std::min(nu, 65535)), dim3(256), 0, s, pan, n, A, lda,
                       Q, ldq, kind, rp, rm, eps, eq_reg, eq_pan, u_slot, q_slot, nu, M, Mt, ldm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dl_rhs_kernel, dim3((nu + 255) / 256, m_main), dim3(256), 0, s, pan, Q, ldq, rp, rm, eq_reg,
                       eq_pan, cp_ptr, cp_idx, nu, B, Bneg, ldb);
    return hipGetLastError();
}

hipError_t launch_dl_charges(const Panel *pan, const int32_t *rp, const int32_t *rm, const double *eps,
                             const int32_t *q_slot, const int32_t *cp_ptr, const int32_t *cp_idx, const double *X,
                             int64_t ldx, int m_main, double scale, double *C, hipStream_t s)
{
    if (m_main <= 0 || m_main > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(dl_charge_kernel, dim3(m_main, m_main), dim3(256), 0, s, pan, rp, rm, eps, q_slot, cp_ptr,
                       cp_idx, X, ldx, m_main, scale, C);
    return hipGetLastError();
}

hipError_t launch_dl_sub(double *X, int64_t ldx, const double *D, int64_t ldd, int rows, int m, hipStream_t s)
{
    if (rows <= 0 || m <= 0) return hipSuccess;
    hipLaunchKernelGGL(dl_sub_kernel, dim3((rows + 255) / 256, m), dim3(256), 0, s, X, ldx, D, ldd, rows);
    return hipGetLastError();
}

}  // namespace gbem
