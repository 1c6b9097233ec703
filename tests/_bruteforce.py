"""Independent brute-force values of Int_{I_i} Int_{I_j} 1/|x-y| for test pins.

These routes share nothing with the oracle's section 3.4 reductions:
  * parallel panels: the two in-plane double integrals of a function of the
    coordinate differences collapse to convolution (trapezoid) weights, leaving
    a 2-D integral of w1(s) w2(t) / sqrt(s^2 + t^2 + b^2), done numerically by
    mpmath's tanh-sinh rule split at every kink;
  * orthogonal panels: the shared axis gives one convolution weight w(s); the
    other two directions are the potential of a rectangle at height s, whose
    textbook closed form is the corner sum of
        p ln(q + R) + q ln(p + R) - s atan(p q / (s R));
    the remaining 1-D integral over s is done by mpmath;
  * separated pairs: plain high-order tensor Gauss-Legendre (numpy) in 4-D.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np


def _normal(lo, hi):
    z = [k for k in range(3) if lo[k] == hi[k]]
    assert len(z) == 1
    return z[0]


def _conv_weight(a0, a1, b0, b1):
    """weight w(s) = |{x in [a0,a1] : x - s in [b0,b1]}| and its kinks"""
    def w(s):
        lo = max(a0, s + b0)
        hi = min(a1, s + b1)
        return max(mp.mpf(0), hi - lo)
    kinks = sorted({a0 - b1, a0 - b0, a1 - b1, a1 - b0})
    return w, kinks


def pair_integral_mp(lo_i, hi_i, lo_j, hi_j, dps: int = 20) -> float:
    mp.mp.dps = dps
    lo_i = [mp.mpf(float(v)) for v in lo_i]
    hi_i = [mp.mpf(float(v)) for v in hi_i]
    lo_j = [mp.mpf(float(v)) for v in lo_j]
    hi_j = [mp.mpf(float(v)) for v in hi_j]
    ni, nj = _normal(lo_i, hi_i), _normal(lo_j, hi_j)
    if ni == nj:
        t1, t2 = [k for k in range(3) if k != ni]
        b = lo_i[ni] - lo_j[ni]
        w1, k1 = _conv_weight(lo_i[t1], hi_i[t1], lo_j[t1], hi_j[t1])
        w2, k2 = _conv_weight(lo_i[t2], hi_i[t2], lo_j[t2], hi_j[t2])
        pts1 = sorted(set(k1 + ([mp.mpf(0)] if k1[0] < 0 < k1[-1] else [])))
        pts2 = sorted(set(k2 + ([mp.mpf(0)] if k2[0] < 0 < k2[-1] else [])))
        f = lambda s, t: w1(s) * w2(t) / mp.sqrt(s * s + t * t + b * b)
        return float(mp.quad(f, pts1, pts2))
    s_ax = 3 - ni - nj
    w, ks = _conv_weight(lo_i[s_ax], hi_i[s_ax], lo_j[s_ax], hi_j[s_ax])
    # p: offset along ni of the points of panel j from the plane of panel i
    p0, p1 = lo_j[ni] - lo_i[ni], hi_j[ni] - lo_i[ni]
    # q: offset along nj of the points of panel i from the plane of panel j
    q0, q1 = lo_i[nj] - lo_j[nj], hi_i[nj] - lo_j[nj]

    def prim(s, p, q):
        R = mp.sqrt(s * s + p * p + q * q)
        v = mp.mpf(0)
        if p != 0:
            v += p * mp.log(q + R) if q + R > 0 else 0
        if q != 0:
            v += q * mp.log(p + R) if p + R > 0 else 0
        if s != 0 and p != 0 and q != 0:
            v -= s * mp.atan(p * q / (s * R))
        return v

    def rect_potential(s):
        return (prim(s, p1, q1) - prim(s, p0, q1) - prim(s, p1, q0) + prim(s, p0, q0))

    pts = sorted(set(ks + ([mp.mpf(0)] if ks[0] < 0 < ks[-1] else [])))
    return float(mp.quad(lambda s: w(s) * rect_potential(s), pts))


def pair_integral_gauss4d(lo_i, hi_i, lo_j, hi_j, n: int = 24) -> float:
    """Plain n^4-point tensor Gauss for well separated pairs."""
    x, w = np.polynomial.legendre.leggauss(n)

    def nodes(lo, hi):
        nrm = _normal(lo, hi)
        t1, t2 = [k for k in range(3) if k != nrm]
        pts = np.zeros((n, n, 3))
        pts[..., nrm] = lo[nrm]
        pts[..., t1] = (0.5 * (lo[t1] + hi[t1]) + 0.5 * (hi[t1] - lo[t1]) * x)[:, None]
        pts[..., t2] = (0.5 * (lo[t2] + hi[t2]) + 0.5 * (hi[t2] - lo[t2]) * x)[None, :]
        wt = np.outer(w, w) * 0.25 * (hi[t1] - lo[t1]) * (hi[t2] - lo[t2])
        return pts.reshape(-1, 3), wt.reshape(-1)

    xa, wa = nodes(np.asarray(lo_i, float), np.asarray(hi_i, float))
    yb, wb = nodes(np.asarray(lo_j, float), np.asarray(hi_j, float))
    d = xa[:, None, :] - yb[None, :, :]
    r = np.sqrt((d * d).sum(-1))
    return float(wa @ (1.0 / r) @ wb)
