/*
 * CPU FP64 oracle for the Galerkin single-layer capacitance method
 * (arXiv 2203.11733, "GBEM", single-dielectric case, section 3).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference the GPU
 * library is checked against.  Only the tests, the smoke check and the bench's
 * CPU-baseline leg may load it.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * What it computes (section 3.1, eqs. "matrix", "lineareq1", "electriccharge"):
 *   a_ij = 1/(4 pi |I_i||I_j|) * Int_{I_i} Int_{I_j} 1/|x-y| dGamma(y) dGamma(x)
 * for axis-aligned rectangular panels I_i.  Near pairs (and the diagonal) are
 * integrated the way section 3.4 describes: analytic reduction of the
 * quadruple integral, closed form for coplanar pairs (eqs. int1/int2), and
 * one-dimensional numerical integrals for parallel-offset pairs (eq. int3) and
 * orthogonal pairs (eqs. int4/int5).  Far pairs use a tensor Gauss-Legendre
 * rule of order p per panel direction, the far-field rule of the method.
 *
 * Readings of garbled or silent passages (all listed in the design notes):
 *  - eq. int3: the weight of the one-dimensional reduction is the trapezoid
 *    w(t) = min(t, dx, dy, dx+dy-t) on [0, dx+dy]; the printed limits are
 *    inconsistent.
 *  - eq. int5: the last term enters with a minus sign; it follows from
 *    2f = d/dx(x f) + d/dy(y f) - (a - a^2/R) for f = a ln(a+R).
 *  - section 3.4 corner operator D: the fourth argument is -y_{1d}; all
 *    reductions use the corner form sum(+-) F(x_corner - y_corner).
 *  - near/far split (not in the paper): near iff the squared Euclidean distance
 *    between the closed rectangles is < eta^2 * max(diam_i^2, diam_j^2).
 *  - coplanar: same normal axis and bit-identical plane coordinate.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (see build_oracle.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre rule on [-1,1] by Newton iteration on P_n.                 */
/* ------------------------------------------------------------------------ */
static void legendre_eval(int n, double x, double *pn, double *dpn)
{
    /* three-term recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1} */
    double p0 = 1.0, p1 = x;
    if (n == 0) { *pn = 1.0; *dpn = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
    }
    *pn = p1;
    /* P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1) */
    *dpn = n * (x * p1 - p0) / (x * x - 1.0);
}

void oracle_gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(ORACLE_PI * (i + 0.75) / (n + 0.5));
        double pn, dpn;
        for (int it = 0; it < 100; ++it) {
            legendre_eval(n, z, &pn, &dpn);
            double dz = pn / dpn;
            z -= dz;
            if (fabs(dz) < 1e-17) break;
        }
        legendre_eval(n, z, &pn, &dpn);
        /* ascending order */
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dpn * dpn);
    }
}

/* ------------------------------------------------------------------------ */
/* Adaptive one-dimensional quadrature: 16-point Gauss on [a,b] compared with */
/* 16-point Gauss on both halves; bisect until they agree.                   */
/* ------------------------------------------------------------------------ */
/* The near-pair reductions run in x87 extended precision (long double, 64-bit
 * significand): the corner sums cancel up to (D/h)^4 of their magnitude for
 * panels of very different sizes, and the extra 11 bits keep the rounded FP64
 * result accurate. */
typedef long double real;
typedef real (*fun1d)(real t, const real *par);

static real g16x[16], g16w[16];
static int g16_ready = 0;

static void legendre_eval_l(int n, real x, real *pn, real *dpn)
{
    real p0 = 1.0L, p1 = x;
    for (int k = 1; k < n; ++k) {
        real p2 = ((2.0L * k + 1.0L) * x * p1 - k * p0) / (k + 1.0L);
        p0 = p1;
        p1 = p2;
    }
    *pn = p1;
    *dpn = n * (x * p1 - p0) / (x * x - 1.0L);
}

static void ensure_g16(void)
{
    if (!g16_ready) {
        const int n = 16;
        for (int i = 0; i < n; ++i) {
            real z = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
            real pn, dpn;
            for (int it = 0; it < 100; ++it) {
                legendre_eval_l(n, z, &pn, &dpn);
                real dz = pn / dpn;
                z -= dz;
                if (fabsl(dz) < 1e-21L) break;
            }
            legendre_eval_l(n, z, &pn, &dpn);
            g16x[n - 1 - i] = z;
            g16w[n - 1 - i] = 2.0L / ((1.0L - z * z) * dpn * dpn);
        }
        g16_ready = 1;
    }
}

static real gauss16(fun1d f, const real *par, real a, real b)
{
    real m = 0.5L * (a + b), h = 0.5L * (b - a), s = 0.0L;
    for (int k = 0; k < 16; ++k) s += g16w[k] * f(m + h * g16x[k], par);
    return s * h;
}

/* Recursive bisection with the same tolerance on every piece.  Rounding noise
 * of a piece shrinks with its length while the tolerance does not, so the
 * refinement ends even where the integrand's own rounding noise is above the
 * tolerance of the whole interval; *budget bounds the work in any case. */
static real adapt_rec(fun1d f, const real *par, real a, real b, real whole, real tol, int depth,
                      long *budget)
{
    real m = 0.5L * (a + b);
    real left = gauss16(f, par, a, m), right = gauss16(f, par, m, b);
    real both = left + right;
    *budget -= 32;
    if (depth >= 40 || *budget <= 0 || fabsl(both - whole) <= tol) return both;
    return adapt_rec(f, par, a, m, left, tol, depth + 1, budget) +
           adapt_rec(f, par, m, b, right, tol, depth + 1, budget);
}

/* 16-point Gauss estimate of the integral of |f| over [a,b] */
static real gauss16_abs(fun1d f, const real *par, real a, real b)
{
    real m = 0.5L * (a + b), h = 0.5L * (b - a), s = 0.0L;
    for (int k = 0; k < 16; ++k) s += g16w[k] * fabsl(f(m + h * g16x[k], par));
    return s * fabsl(h);
}

/* Integral of f over [a,b] to about 1e-18 of the integral of |f| (estimated
 * from the first 16-point sum). */
static real integrate(fun1d f, const real *par, real a, real b)
{
    if (a == b) return 0.0L;
    ensure_g16();
    real mag = gauss16_abs(f, par, a, b);
    if (mag == 0.0L) return 0.0L;
    long budget = 400000;
    return adapt_rec(f, par, a, b, gauss16(f, par, a, b), 1e-18L * mag, 0, &budget);
}

/* ln(z + sqrt(z^2 + r2)) without cancellation when z < 0; r2 = the sum of the
 * other squared coordinates.  Returns 0 when the argument is exactly 0, for use
 * only where the prefactor vanishes there (limit x ln x -> 0). */
static real log_z_plus_r(real z, real r2)
{
    real R = sqrtl(z * z + r2);
    if (z >= 0.0L) {
        real s = z + R;
        return s > 0.0L ? logl(s) : 0.0L;
    }
    if (r2 <= 0.0L) return 0.0L;
    return logl(r2) - logl(R - z);
}

/* ------------------------------------------------------------------------ */
/* Coplanar pairs (b = 0): closed form of eqs. int1 and int2.                */
/* After the analytic reduction along the first in-plane axis the integrand */
/* is a ln(a + sqrt(a^2 + u^2)) - sqrt(a^2 + u^2); G1 and G2 are its second  */
/* antiderivatives in u (u = difference along the second in-plane axis).     */
/* ------------------------------------------------------------------------ */
static real G1(real a, real u)
{
    real r2a = a * a, r2u = u * u;
    real R = sqrtl(r2a + r2u);
    real t = 0.0L;
    if (a != 0.0L && u != 0.0L) t += 0.5L * a * r2u * log_z_plus_r(a, r2u);
    t -= 0.75L * a * r2u;
    t -= 0.5L * r2a * R;
    if (a != 0.0L && u != 0.0L) t += r2a * u * log_z_plus_r(u, r2a);
    return t;
}

static real G2(real a, real u)
{
    real r2a = a * a, r2u = u * u;
    real R = sqrtl(r2a + r2u);
    real t = (r2u + r2a) * R / 6.0L;
    if (a != 0.0L && u != 0.0L) t += 0.5L * r2a * u * log_z_plus_r(u, r2a);
    t -= 0.5L * r2a * R;
    return t;
}

/* Sign of a corner of the difference operator D along one axis shared by both
 * panels: the double integral of g(x - y) over [xd,xu] x [yd,yu] equals
 * sum over corners of -s(x) s(y) H(x_c - y_c), H'' = g, s(upper)=+1, s(lower)=-1. */
static real coplanar_integral(const double x1[2], const double x2[2],
                              const double y1[2], const double y2[2])
{
    real g = 0.0L;
    for (int al = 0; al < 2; ++al)
        for (int be = 0; be < 2; ++be)
            for (int ga = 0; ga < 2; ++ga)
                for (int de = 0; de < 2; ++de) {
                    real sg = ((al + be + ga + de) & 1) ? -1.0L : 1.0L;
                    real a = (real)x1[al] - (real)y1[be];
                    real u = (real)x2[ga] - (real)y2[de];
                    g += sg * (G1(a, u) - G2(a, u));
                }
    return g;
}

/* ------------------------------------------------------------------------ */
/* Parallel pairs with offset b != 0: reduce the first in-plane axis         */
/* analytically (H(s) = s ln(s+R) - R, R = sqrt(s^2 + tau^2 + b^2)), then the */
/* double integral over the second axis to one dimension with the trapezoid  */
/* weight of eq. int3.                                                        */
/* ------------------------------------------------------------------------ */
static real par_integrand(real t, const real *par)
{
    /* par: s, b2, tau0, dx, dy */
    real s = par[0], b2 = par[1], tau = t + par[2], dx = par[3], dy = par[4];
    real w = t;
    real dmin = dx < dy ? dx : dy;
    if (dmin < w) w = dmin;
    if (dx + dy - t < w) w = dx + dy - t;
    if (w <= 0.0L) return 0.0L;
    real r2 = tau * tau + b2;
    real R = sqrtl(s * s + r2);
    real h = -R;
    if (s != 0.0L) h += s * log_z_plus_r(s, r2);
    return w * h;
}

static real parallel_offset_integral(const double x1[2], const double x2[2],
                                     const double y1[2], const double y2[2], double b)
{
    real dx = (real)x2[1] - x2[0], dy = (real)y2[1] - y2[0];
    real dmin = dx < dy ? dx : dy, dmax = dx < dy ? dy : dx;
    real g = 0.0L;
    for (int al = 0; al < 2; ++al)
        for (int be = 0; be < 2; ++be) {
            real sg = (al == be) ? -1.0L : 1.0L;   /* -s(x)s(y) */
            real par[5];
            par[0] = (real)x1[al] - (real)y1[be];
            par[1] = (real)b * (real)b;
            par[2] = (real)x2[0] - (real)y2[1];
            par[3] = dx;
            par[4] = dy;
            real v = integrate(par_integrand, par, 0.0L, dmin) +
                     integrate(par_integrand, par, dmin, dmax) +
                     integrate(par_integrand, par, dmax, dx + dy);
            g += sg * v;
        }
    return g;
}

/* ------------------------------------------------------------------------ */
/* Orthogonal pairs: eqs. int4 and int5 (last term with a minus sign).       */
/* With a = s (difference along the shared axis), x in [xd,xu] and y in      */
/* [yd,yu] the two out-of-plane offsets, R = sqrt(a^2 + x^2 + y^2):           */
/*   I_R  = Int Int R dy dx = Int [G3(x,y)]_{y=yd}^{yu} dx                   */
/*   I_L  = Int Int a ln(a+R) dy dx                                          */
/*        = 1/2 [Int (y a) ln(a+R) dx]_y + 1/2 [Int (x a) ln(a+R) dy]_x       */
/*          - 1/2 ( [a x y]_{x,y} - [Int a^2 ln(y+R) dx]_y )                  */
/* and the wanted double integral of H = a ln(a+R) - R is I_L - I_R.          */
/* ------------------------------------------------------------------------ */
static real f_g3(real x, const real *par)
{
    /* par: a, y ; G3(x,y) = y/2 R + (x^2 + a^2)/2 ln(y + R) */
    real a = par[0], y = par[1];
    real r2 = x * x + a * a;
    real R = sqrtl(r2 + y * y);
    real t = 0.5L * y * R;
    if (r2 != 0.0L) t += 0.5L * r2 * log_z_plus_r(y, r2);
    return t;
}

static real f_yaln(real x, const real *par)
{
    /* par: a, y ; y a ln(a + R) */
    real a = par[0], y = par[1];
    if (a == 0.0L || y == 0.0L) return 0.0L;
    return y * a * log_z_plus_r(a, x * x + y * y);
}

static real f_a2lny(real x, const real *par)
{
    /* par: a, y ; a^2 ln(y + R) */
    real a = par[0], y = par[1];
    if (a == 0.0L) return 0.0L;
    return a * a * log_z_plus_r(y, x * x + a * a);
}

static real orth_double(real a, real xd, real xu, real yd, real yu)
{
    real par[2];
    real IR = 0.0L, IL = 0.0L;
    /* I_R */
    par[0] = a; par[1] = yu; IR += integrate(f_g3, par, xd, xu);
    par[1] = yd;             IR -= integrate(f_g3, par, xd, xu);
    if (a != 0.0L) {
        real t1 = 0.0L, t2 = 0.0L, t3, t4 = 0.0L;
        par[0] = a; par[1] = yu; t1 += integrate(f_yaln, par, xd, xu);
        par[1] = yd;             t1 -= integrate(f_yaln, par, xd, xu);
        /* x a ln(a+R) integrated over y at x = xu, xd (same function with roles swapped) */
        par[1] = xu;             t2 += integrate(f_yaln, par, yd, yu);
        par[1] = xd;             t2 -= integrate(f_yaln, par, yd, yu);
        t3 = a * (xu * yu - xu * yd - xd * yu + xd * yd);
        par[1] = yu;             t4 += integrate(f_a2lny, par, xd, xu);
        par[1] = yd;             t4 -= integrate(f_a2lny, par, xd, xu);
        IL = 0.5L * t1 + 0.5L * t2 - 0.5L * (t3 - t4);
    }
    return IL - IR;
}

/* panel i spans the shared axis (xs) and the normal axis of j (xq) at X (its
 * own plane); panel j spans the shared axis (ys) and the normal axis of i (yp)
 * at Y. */
static real orthogonal_integral(const double xs[2], const double xq[2], double X,
                                const double ys[2], const double yp[2], double Y)
{
    real g = 0.0L;
    for (int al = 0; al < 2; ++al)
        for (int be = 0; be < 2; ++be) {
            real sg = (al == be) ? -1.0L : 1.0L;
            real a = (real)xs[al] - (real)ys[be];
            /* x <-> offset of the point of panel i along j's normal: xq - Y
               y <-> offset of the point of panel j along i's normal: yp - X */
            g += sg * orth_double(a, (real)xq[0] - Y, (real)xq[1] - Y, (real)yp[0] - X, (real)yp[1] - X);
        }
    return g;
}

/* ------------------------------------------------------------------------ */
/* Panels                                                                    */
/* ------------------------------------------------------------------------ */
int normal_axis(const double *lo, const double *hi)
{
    for (int k = 0; k < 3; ++k)
        if (lo[k] == hi[k]) return k;
    return -1;
}

/* exact double integral Int_{I_i} Int_{I_j} 1/|x-y| (no 1/4pi, no areas) */
double oracle_pair_integral_exact(const double *lo_i, const double *hi_i,
                                  const double *lo_j, const double *hi_j)
{
    int ni = normal_axis(lo_i, hi_i), nj = normal_axis(lo_j, hi_j);
    if (ni < 0 || nj < 0) return NAN;
    if (ni == nj) {
        int t1 = (ni + 1) % 3, t2 = (ni + 2) % 3;
        double x1[2] = {lo_i[t1], hi_i[t1]}, x2[2] = {lo_i[t2], hi_i[t2]};
        double y1[2] = {lo_j[t1], hi_j[t1]}, y2[2] = {lo_j[t2], hi_j[t2]};
        double b = lo_i[ni] - lo_j[ni];
        if (b == 0.0) return (double)coplanar_integral(x1, x2, y1, y2);
        return (double)parallel_offset_integral(x1, x2, y1, y2, b);
    }
    int s = 3 - ni - nj;
    double xs[2] = {lo_i[s], hi_i[s]}, xq[2] = {lo_i[nj], hi_i[nj]};
    double ys[2] = {lo_j[s], hi_j[s]}, yp[2] = {lo_j[ni], hi_j[ni]};
    return (double)orthogonal_integral(xs, xq, lo_i[ni], ys, yp, lo_j[nj]);
}

double oracle_panel_area(const double *lo, const double *hi)
{
    int n = normal_axis(lo, hi);
    int t1 = n == 0 ? 1 : 0, t2 = n == 2 ? 1 : 2;
    return (hi[t1] - lo[t1]) * (hi[t2] - lo[t2]);
}

/* Tensor Gauss-Legendre rule of order p on both panels; returns the weighted
 * mean sum_{a,b} w_a w_b / |x_a - y_b| with weights that sum to 1 on each
 * panel, so that the far-field a_ij is this value divided by 4 pi. */
double oracle_pair_gauss_mean(const double *lo_i, const double *hi_i,
                              const double *lo_j, const double *hi_j, int p)
{
    double gx[16], gw[16];
    if (p < 1 || p > 16) return NAN;
    oracle_gauss_legendre(p, gx, gw);
    double xi[256][3], wi[256], yj[256][3], wj[256];
    const double *plo[2] = {lo_i, lo_j}, *phi[2] = {hi_i, hi_j};
    for (int side = 0; side < 2; ++side) {
        const double *lo = plo[side], *hi = phi[side];
        int n = normal_axis(lo, hi);
        int t1 = n == 0 ? 1 : 0, t2 = n == 2 ? 1 : 2;
        int m = 0;
        for (int a = 0; a < p; ++a)
            for (int c = 0; c < p; ++c) {
                double pt[3];
                pt[n] = lo[n];
                pt[t1] = 0.5 * (lo[t1] + hi[t1]) + 0.5 * (hi[t1] - lo[t1]) * gx[a];
                pt[t2] = 0.5 * (lo[t2] + hi[t2]) + 0.5 * (hi[t2] - lo[t2]) * gx[c];
                double w = 0.25 * gw[a] * gw[c];
                if (side == 0) { memcpy(xi[m], pt, sizeof pt); wi[m] = w; }
                else           { memcpy(yj[m], pt, sizeof pt); wj[m] = w; }
                ++m;
            }
    }
    double s = 0.0;
    for (int a = 0; a < p * p; ++a)
        for (int b = 0; b < p * p; ++b) {
            double dx = xi[a][0] - yj[b][0], dy = xi[a][1] - yj[b][1], dz = xi[a][2] - yj[b][2];
            s += wi[a] * wj[b] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Near/far classification (not in the paper; the method's near/far split).  */
/*   d_k  = max(0, lo_j[k] - hi_i[k], lo_i[k] - hi_j[k])                     */
/*   sep2 = (d_0^2 + d_1^2) + d_2^2                                          */
/*   diam2 = (e_0^2 + e_1^2) + e_2^2,  e_k = hi[k] - lo[k]                   */
/*   near  iff  sep2 < eta2 * max(diam2_i, diam2_j),  eta2 = eta*eta         */
/* ------------------------------------------------------------------------ */
static double diam2(const double *lo, const double *hi)
{
    double e0 = hi[0] - lo[0], e1 = hi[1] - lo[1], e2 = hi[2] - lo[2];
    return (e0 * e0 + e1 * e1) + e2 * e2;
}

int oracle_is_near(const double *lo_i, const double *hi_i,
                   const double *lo_j, const double *hi_j, double eta2)
{
    double d[3];
    for (int k = 0; k < 3; ++k) {
        double g1 = lo_j[k] - hi_i[k], g2 = lo_i[k] - hi_j[k];
        double g = g1 > g2 ? g1 : g2;
        d[k] = g > 0.0 ? g : 0.0;
    }
    double sep2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    double di = diam2(lo_i, hi_i), dj = diam2(lo_j, hi_j);
    double dm = di > dj ? di : dj;
    return sep2 < eta2 * dm;
}

/* CSR of near pairs j <= i (diagonal included), columns ascending.
 * row_ptr has n+1 entries.  If col is NULL only row_ptr is filled.  Returns the
 * number of near pairs. */
int64_t oracle_near_csr(int n, const double *lo, const double *hi, double eta,
                        int64_t *row_ptr, int32_t *col)
{
    double eta2 = eta * eta;
    int64_t *cnt = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    #pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int j = 0; j <= i; ++j)
            c += oracle_is_near(lo + 3 * i, hi + 3 * i, lo + 3 * j, hi + 3 * j, eta2);
        cnt[i] = c;
    }
    row_ptr[0] = 0;
    for (int i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[i];
    free(cnt);
    if (col) {
        #pragma omp parallel for schedule(dynamic, 16)
        for (int i = 0; i < n; ++i) {
            int64_t k = row_ptr[i];
            for (int j = 0; j <= i; ++j)
                if (oracle_is_near(lo + 3 * i, hi + 3 * i, lo + 3 * j, hi + 3 * j, eta2))
                    col[k++] = j;
        }
    }
    return row_ptr[n];
}

/* one matrix entry a_ij of eq. "matrix" under the method's near/far rule */
double oracle_entry(const double *lo_i, const double *hi_i,
                    const double *lo_j, const double *hi_j, int p, double eta)
{
    if (oracle_is_near(lo_i, hi_i, lo_j, hi_j, eta * eta)) {
        double g = oracle_pair_integral_exact(lo_i, hi_i, lo_j, hi_j);
        return g / (4.0 * ORACLE_PI * oracle_panel_area(lo_i, hi_i) * oracle_panel_area(lo_j, hi_j));
    }
    return oracle_pair_gauss_mean(lo_i, hi_i, lo_j, hi_j, p) / (4.0 * ORACLE_PI);
}

/* dense symmetric A (row-major n x n); entry (i,j), i >= j, is evaluated with
 * panel i as the first argument and mirrored to (j,i) */
void oracle_assemble(int n, const double *lo, const double *hi, int p, double eta, double *A)
{
    ensure_g16();
    #pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double v = oracle_entry(lo + 3 * i, hi + 3 * i, lo + 3 * j, hi + 3 * j, p, eta);
            A[(int64_t)i * n + j] = v;
            A[(int64_t)j * n + i] = v;
        }
}

/* sampled entries (rows ii[k], cols jj[k]) */
void oracle_entries(const double *lo, const double *hi, int64_t m, const int32_t *ii,
                    const int32_t *jj, int p, double eta, double *out)
{
    ensure_g16();
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < m; ++k) {
        int i = ii[k], j = jj[k];
        if (i < j) { int t = i; i = j; j = t; }
        out[k] = oracle_entry(lo + 3 * i, hi + 3 * i, lo + 3 * j, hi + 3 * j, p, eta);
    }
}

/* ------------------------------------------------------------------------ */
/* Mesher: boxes -> rectangles.                                              */
/* Edge splits:                                                              */
/*   uniform(h):  n = max(1, ceil(L/h - 1e-9)), e_k = lo + ((hi-lo)*k)/n     */
/*   graded(hmin, g, hmax): cells c_0 = hmin, c_{k+1} = c_k*g taken from     */
/*     both ends while c_k <= hmax and the running sum stays <= L/2; the     */
/*     middle [a,b] is split uniformly into max(1, ceil((L-2S)/hmax - 1e-9)) */
/*     cells (none if L-2S == 0).                                            */
/* Panel order: boxes as given; faces -x,+x,-y,+y,-z,+z; within a face the   */
/* lower in-plane axis is the outer loop.                                    */
/* ------------------------------------------------------------------------ */
static int split_edge(double lo, double hi, int kind, const double *prm, double *e)
{
    double L = hi - lo;
    if (kind == 0) {
        int n = (int)ceil(L / prm[0] - 1e-9);
        if (n < 1) n = 1;
        if (e) {
            for (int k = 0; k < n; ++k) e[k] = lo + (L * k) / n;
            e[n] = hi;
        }
        return n;
    }
    double hmin = prm[0], g = prm[1], hmax = prm[2];
    double half = 0.5 * L, S = 0.0, c = hmin;
    double cells[256];
    int kg = 0;
    while (c <= hmax && S + c <= half && kg < 256) {
        cells[kg++] = c;
        S = S + c;
        c = c * g;
    }
    double rem = L - 2.0 * S;
    int nmid = 0;
    if (rem > 0.0) {
        nmid = (int)ceil(rem / hmax - 1e-9);
        if (nmid < 1) nmid = 1;
    }
    int n = 2 * kg + nmid;
    if (e) {
        double right[257];
        right[0] = hi;
        for (int k = 0; k < kg; ++k) right[k + 1] = right[k] - cells[k];
        e[0] = lo;
        for (int k = 0; k < kg; ++k) e[k + 1] = e[k] + cells[k];
        double a = e[kg], b = right[kg];
        for (int m = 1; m < nmid; ++m) e[kg + m] = a + ((b - a) * m) / nmid;
        if (nmid > 0) e[kg + nmid] = b;
        for (int k = kg - 1; k >= 0; --k) e[2 * kg + nmid - k] = right[k];
    }
    return n;
}

/* returns the panel count; fills lo/hi/cond when they are not NULL.
 * kind 0 = uniform (prm[0] = h), 1 = graded (prm = hmin, growth, hmax) */
int64_t oracle_mesh(int nbox, const double *blo, const double *bhi, const int32_t *bcond,
                    int kind, const double *prm, double *lo, double *hi, int32_t *cond)
{
    int64_t np = 0;
    for (int b = 0; b < nbox; ++b) {
        int nk[3];
        double *E[3];
        for (int k = 0; k < 3; ++k) {
            nk[k] = split_edge(blo[3 * b + k], bhi[3 * b + k], kind, prm, NULL);
            E[k] = (double *)malloc(sizeof(double) * (nk[k] + 1));
            split_edge(blo[3 * b + k], bhi[3 * b + k], kind, prm, E[k]);
        }
        for (int f = 0; f < 6; ++f) {
            int n = f / 2;
            double plane = (f & 1) ? bhi[3 * b + n] : blo[3 * b + n];
            int t1 = n == 0 ? 1 : 0, t2 = n == 2 ? 1 : 2;
            for (int a = 0; a < nk[t1]; ++a)
                for (int c = 0; c < nk[t2]; ++c) {
                    if (lo) {
                        double *l = lo + 3 * np, *h = hi + 3 * np;
                        l[n] = plane; h[n] = plane;
                        l[t1] = E[t1][a]; h[t1] = E[t1][a + 1];
                        l[t2] = E[t2][c]; h[t2] = E[t2][c + 1];
                        cond[np] = bcond[b];
                    }
                    ++np;
                }
        }
        for (int k = 0; k < 3; ++k) free(E[k]);
    }
    return np;
}
