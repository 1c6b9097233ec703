"""Multi-dielectric case of arXiv 2203.11733 (section 4), test infrastructure only.

In each dielectric region Omega_a the potential satisfies Laplace's equation
with u = 1 on the main net, u = 0 on the other nets and the Dirichlet
boundary, du/dn = 0 on the Neumann boundary, and on an interface between
Omega_a and Omega_b u_a = u_b and eps_a q_a = -eps_b q_b (section 2.1, q the
normal derivative along each region's outward normal).  Green's identity
gives, for x on the boundary of Omega_a (eq. "representation", sigma = 1/2):

    1/2 u_a(x) + Int_{dOmega_a} q*(x, y) u_a(y) dG(y) = Int_{dOmega_a} u*(x, y) q_a(y) dG(y),
    u* = 1 / (4 pi |x - y|),   q* = <x - y, n_y> / (4 pi |x - y|^3),

with n_y the outward normal of Omega_a.  Integrated over each panel I_i with
u and q constant per panel (section 4.1):

    1/2 |I_i| u_i + sum_k Q_ik u_k = sum_j G_ij q_j,
    G_ij = Int_{I_i} Int_{I_j} u*,   Q_ik = Int_{I_i} Int_{I_k} q*   (section 4.2).

This module writes that out directly:
  * Q_ik: the inner integral over I_k in closed form (q* integrated over a
    flat rectangle is the solid angle it subtends at x over 4 pi, with the
    sign of the normal), the outer one over I_i by tensor Gauss-Legendre on
    a recursively bisected I_i until two levels agree;
  * G_ij: the oracle's exact single-layer pair integral (section 3.4);
  * one equation per (region, panel of its boundary), unknowns q on conductor
    and Dirichlet panels, u on Neumann panels, (u, q_a) on interface panels
    (q_b = -eps_a / eps_b q_a), solved densely by LAPACK (numpy.linalg.solve);
  * the charge on a conductor, sum over its panels of eps q |I_j| (q along the
    region's outward normal, which points into the conductor), times eps0 and
    the length unit, one main net per solve.

Panels are axis-aligned rectangles (lo, hi, exactly one zero extent, the
normal axis); each carries the regions on its + and - side along that axis
(-1: none, i.e. inside a conductor or outside the domain) and a kind.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as _o

CONDUCTOR, DIRICHLET, NEUMANN, INTERFACE = 0, 1, 2, 3


def _axes(lo, hi):
    ext = np.asarray(hi, dtype=np.float64) - np.asarray(lo, dtype=np.float64)
    nrm = int(np.flatnonzero(ext == 0.0)[0])
    t1, t2 = [k for k in range(3) if k != nrm]
    return nrm, t1, t2


def solid_angle_rect(px, py, h, x1, x2, y1, y2):
    """Signed solid angle subtended at (px, py, h) by the rectangle
    [x1, x2] x [y1, y2] of the plane h = 0, with the plane's normal along +h:
    Int Int h / (u^2 + v^2 + h^2)^(3/2) du dv over the rectangle, whose
    antiderivative in u and v is atan(u v / (h sqrt(u^2 + v^2 + h^2))).  Zero
    for h = 0 (a point in the plane).  Vectorised over the point."""
    px, py, h = np.broadcast_arrays(np.asarray(px, float), np.asarray(py, float), np.asarray(h, float))
    out = np.zeros(px.shape)
    nz = h != 0.0
    if not np.any(nz):
        return out
    X, Y, H = px[nz], py[nz], h[nz]
    s = np.zeros(X.shape)
    for xa, sx in ((x2, 1.0), (x1, -1.0)):
        for yb, sy in ((y2, 1.0), (y1, -1.0)):
            u, v = xa - X, yb - Y
            r = np.sqrt(u * u + v * v + H * H)
            s += sx * sy * np.arctan(u * v / (H * r))
    out[nz] = s
    return out


def double_layer_potential(x, lo_k, hi_k):
    """Int_{I_k} q*(x, y) dG(y) for the normal of I_k along + its normal axis,
    at points x (n x 3): <x - y, n> / (4 pi |x - y|^3) integrated over the
    rectangle, i.e. the solid angle at x over 4 pi."""
    nrm, t1, t2 = _axes(lo_k, hi_k)
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    h = x[:, nrm] - lo_k[nrm]
    return solid_angle_rect(x[:, t1], x[:, t2], h, lo_k[t1], hi_k[t1], lo_k[t2], hi_k[t2]) / (4.0 * math.pi)


_GL = {}


def _gl(n):
    if n not in _GL:
        _GL[n] = np.polynomial.legendre.leggauss(n)
    return _GL[n]


def _rect_nodes(lo, hi, t1, t2, n):
    """Nodes (n*n x 3) and weights of the n x n tensor Gauss-Legendre rule on
    a rectangle's in-plane extent."""
    x, w = _gl(n)
    a1, b1, a2, b2 = lo[t1], hi[t1], lo[t2], hi[t2]
    u = 0.5 * (a1 + b1) + 0.5 * (b1 - a1) * x
    v = 0.5 * (a2 + b2) + 0.5 * (b2 - a2) * x
    U, V = np.meshgrid(u, v, indexing="ij")
    pts = np.zeros((n * n, 3))
    pts[:, :] = lo
    pts[:, t1] = U.ravel()
    pts[:, t2] = V.ravel()
    return pts, np.outer(w, w).ravel() * 0.25 * (b1 - a1) * (b2 - a2)


def _rect_gauss(f, lo, hi, t1, t2, n):
    """Tensor Gauss-Legendre (n x n) of f over the rectangle's in-plane extent."""
    pts, W = _rect_nodes(lo, hi, t1, t2, n)
    return float(np.dot(W, f(pts)))


def double_layer_pair(lo_i, hi_i, lo_k, hi_k, tol=1e-12, n=8, depth=14):
    """Q_ik = Int_{I_i} Int_{I_k} q*(x, y) dG(y) dG(x), the normal of I_k along
    + its normal axis.  The outer integral: Gauss on I_i against the sum over
    its four quarters, recursing where they differ by more than tol |I_i|
    (the inner integral is bounded, so the recursion ends at the edges where
    I_i meets the plane of I_k).  The four quarters' rules are evaluated in
    one call of the inner integral."""
    lo_i = np.asarray(lo_i, float)
    hi_i = np.asarray(hi_i, float)
    lo_k = np.asarray(lo_k, float)
    hi_k = np.asarray(hi_k, float)
    nrm_i, t1, t2 = _axes(lo_i, hi_i)
    nrm_k = _axes(lo_k, hi_k)[0]
    if nrm_i == nrm_k and lo_i[nrm_i] == lo_k[nrm_k]:
        return 0.0                       # coplanar: <x - y, n_y> = 0 (section 4.2)
    f = lambda pts: double_layer_potential(pts, lo_k, hi_k)
    area = (hi_i[t1] - lo_i[t1]) * (hi_i[t2] - lo_i[t2])

    def rec(lo, hi, whole, d):
        m1 = 0.5 * (lo[t1] + hi[t1])
        m2 = 0.5 * (lo[t2] + hi[t2])
        quarters = []
        for a1, b1 in ((lo[t1], m1), (m1, hi[t1])):
            for a2, b2 in ((lo[t2], m2), (m2, hi[t2])):
                ql, qh = lo.copy(), hi.copy()
                ql[t1], qh[t1], ql[t2], qh[t2] = a1, b1, a2, b2
                quarters.append((ql, qh))
        nodes = [_rect_nodes(ql, qh, t1, t2, n) for ql, qh in quarters]
        vals = f(np.concatenate([p for p, _ in nodes])).reshape(4, n * n)
        parts = [float(np.dot(w, v)) for (_, w), v in zip(nodes, vals)]
        s = sum(parts)
        sub = (hi[t1] - lo[t1]) * (hi[t2] - lo[t2])
        if abs(s - whole) <= tol * area * max(sub / area, 1e-3) or d >= depth:
            return s
        return sum(rec(ql, qh, p, d + 1) for (ql, qh), p in zip(quarters, parts))

    return rec(lo_i.copy(), hi_i.copy(), _rect_gauss(f, lo_i, hi_i, t1, t2, n), 0)


def double_layer_matrix(lo, hi, sep=4.0):
    """Q (n x n) of a mesh, normals along + each panel's normal axis.  Pairs
    whose distance exceeds sep times the larger diameter take a single 8 x 8
    Gauss rule on I_i (the inner integral is then smooth); the others the
    adaptive rule of double_layer_pair."""
    lo = np.asarray(lo, float).reshape(-1, 3)
    hi = np.asarray(hi, float).reshape(-1, 3)
    n = lo.shape[0]
    Q = np.zeros((n, n))
    diam = np.sqrt(((hi - lo) ** 2).sum(1))
    for i in range(n):
        nrm_i, t1, t2 = _axes(lo[i], hi[i])
        for k in range(n):
            if i == k:
                continue                 # a panel and itself are coplanar
            gap = np.maximum(0.0, np.maximum(lo[k] - hi[i], lo[i] - hi[k]))
            if math.sqrt(float((gap ** 2).sum())) > sep * max(diam[i], diam[k]):
                nrm_k = _axes(lo[k], hi[k])[0]
                if nrm_i == nrm_k and lo[i][nrm_i] == lo[k][nrm_k]:
                    continue
                Q[i, k] = _rect_gauss(lambda p: double_layer_potential(p, lo[k], hi[k]), lo[i], hi[i], t1, t2, 8)
            else:
                Q[i, k] = double_layer_pair(lo[i], hi[i], lo[k], hi[k])
    return Q


def single_layer_matrix(lo, hi):
    """G_ij = Int Int 1 / (4 pi |x - y|), exactly (the oracle's section 3.4 pair integrals)."""
    lo = np.asarray(lo, float).reshape(-1, 3)
    hi = np.asarray(hi, float).reshape(-1, 3)
    n = lo.shape[0]
    G = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1):
            G[i, j] = G[j, i] = _o.pair_integral(lo[i], hi[i], lo[j], hi[j]) / (4.0 * math.pi)
    return G


def extract(lo, hi, kind, cond, reg_plus, reg_minus, eps_r, n_conductors: int, length_unit_m: float,
            single_layer=None):
    """Maxwell capacitance matrix (n_conductors x n_conductors, F) of a
    multi-dielectric mesh.  kind: CONDUCTOR (cond = net id), DIRICHLET
    (grounded outer boundary), NEUMANN (du/dn = 0), INTERFACE; reg_plus /
    reg_minus: region on the + / - side of the panel's normal axis (-1 none);
    eps_r: relative permittivity per region.  Column k: main net k at 1.
    single_layer: None for the exact G_ij, or (p, eta) for G_ij as section 3.4
    computes it (exact near pairs, p x p Gauss far pairs: the oracle's
    assemble, times the two panel areas)."""
    lo = np.asarray(lo, float).reshape(-1, 3)
    hi = np.asarray(hi, float).reshape(-1, 3)
    kind = np.asarray(kind, int)
    cond = np.asarray(cond, int)
    rp = np.asarray(reg_plus, int)
    rm = np.asarray(reg_minus, int)
    n = lo.shape[0]
    area = np.array([float(np.prod([hi[i][t] - lo[i][t] for t in _axes(lo[i], hi[i])[1:]])) for i in range(n)])
    if single_layer is None:
        G = single_layer_matrix(lo, hi)
    else:
        G = _o.assemble(lo, hi, *single_layer) * np.outer(area, area)
    Q = double_layer_matrix(lo, hi)
    n_reg = int(max(rp.max(), rm.max())) + 1
    # unknown slots: q of conductor / Dirichlet / interface panels (interface:
    # q along the outward normal of its minus-side region, see below); u of
    # Neumann and interface panels
    q_slot = -np.ones(n, int)
    u_slot = -np.ones(n, int)
    nu = 0
    for i in range(n):
        if kind[i] in (CONDUCTOR, DIRICHLET, INTERFACE):
            q_slot[i] = nu
            nu += 1
        if kind[i] in (NEUMANN, INTERFACE):
            u_slot[i] = nu
            nu += 1
    # equations: one per (region, boundary panel of it)
    rows = [(a, i) for a in range(n_reg) for i in range(n) if rp[i] == a or rm[i] == a]
    if len(rows) != nu:
        raise ValueError(f"{len(rows)} equations for {nu} unknowns: check the panel kinds and regions")
    eps = np.asarray(eps_r, float)
    C = np.zeros((n_conductors, n_conductors))
    # outward normal of region a at panel i: -e_n if a is on the + side, +e_n if on the - side
    s = lambda a, i: -1.0 if rp[i] == a else 1.0
    for main in range(n_conductors):
        M = np.zeros((nu, nu))
        b = np.zeros(nu)
        for r, (a, i) in enumerate(rows):
            members = np.flatnonzero((rp == a) | (rm == a))
            # left side: 1/2 |I_i| u_i + sum_k Q^a_ik u_k (known u to the right side)
            for k in members:
                coef = (0.5 * area[i] if k == i else 0.0) + s(a, k) * Q[i, k]
                if coef == 0.0:
                    continue
                if kind[k] == CONDUCTOR:
                    b[r] -= coef * (1.0 if cond[k] == main else 0.0)
                elif kind[k] == DIRICHLET:
                    pass
                else:
                    M[r, u_slot[k]] += coef
            # right side: sum_j G_ij q^a_j, moved to the left
            for j in members:
                if kind[j] == NEUMANN:
                    continue
                if kind[j] == INTERFACE:
                    # unknown q = q of the minus-side region (outward normal +e_n);
                    # the plus-side region's q is -eps_minus / eps_plus of it
                    f = 1.0 if rm[j] == a else -eps[rm[j]] / eps[rp[j]]
                    M[r, q_slot[j]] -= f * G[i, j]
                else:
                    M[r, q_slot[j]] -= G[i, j]
        x = np.linalg.solve(M, b)
        for i in range(n):
            if kind[i] == CONDUCTOR:
                a = rp[i] if rp[i] >= 0 else rm[i]
                C[cond[i], main] += eps[a] * x[q_slot[i]] * area[i]
    return C * _o.EPS0 * length_unit_m


__all__ = ["CONDUCTOR", "DIRICHLET", "NEUMANN", "INTERFACE", "solid_angle_rect", "double_layer_potential",
           "double_layer_pair", "double_layer_matrix", "single_layer_matrix", "extract"]
