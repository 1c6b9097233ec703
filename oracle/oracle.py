"""Python driver of the CPU FP64 oracle (test infrastructure only).

Computes, for a mesh of axis-aligned rectangular panels with a conductor id each
(arXiv 2203.11733, section 3.1):
  1. A_ij = 1/(4 pi |I_i||I_j|) Int Int 1/|x-y|            (eq. "matrix")
     near pairs by the section 3.4 reductions, far pairs by p x p Gauss
  2. B_ik = 1 if panel i belongs to conductor k              (eq. "lineareq1", b)
  3. A X = B by Cholesky; A is symmetric positive definite   (section 3.2, Theorem 1)
  4. C_kl = eps_r eps0 l * sum_{i in k} X_il                 (eq. "electriccharge")
The pair integrals, mesher and near/far test live in gbem_oracle.c; the
Cholesky factorisation is LAPACK's (scipy.linalg.cho_factor / cho_solve).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import build_oracle

EPS0 = 8.8541878128e-12

_LIB = None
_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.POINTER(ctypes.c_int64)


def _lib():
    global _LIB
    if _LIB is None:
        path = build_oracle.build()
        lib = ctypes.CDLL(path)
        lib.oracle_gauss_legendre.argtypes = [ctypes.c_int, _d, _d]
        lib.oracle_pair_integral_exact.argtypes = [_d, _d, _d, _d]
        lib.oracle_pair_integral_exact.restype = ctypes.c_double
        lib.oracle_pair_gauss_mean.argtypes = [_d, _d, _d, _d, ctypes.c_int]
        lib.oracle_pair_gauss_mean.restype = ctypes.c_double
        lib.oracle_panel_area.argtypes = [_d, _d]
        lib.oracle_panel_area.restype = ctypes.c_double
        lib.oracle_is_near.argtypes = [_d, _d, _d, _d, ctypes.c_double]
        lib.oracle_is_near.restype = ctypes.c_int
        lib.oracle_near_csr.argtypes = [ctypes.c_int, _d, _d, ctypes.c_double, _i64, _i32]
        lib.oracle_near_csr.restype = ctypes.c_int64
        lib.oracle_entry.argtypes = [_d, _d, _d, _d, ctypes.c_int, ctypes.c_double]
        lib.oracle_entry.restype = ctypes.c_double
        lib.oracle_assemble.argtypes = [ctypes.c_int, _d, _d, ctypes.c_int, ctypes.c_double, _d]
        lib.oracle_entries.argtypes = [_d, _d, ctypes.c_int64, _i32, _i32, ctypes.c_int,
                                       ctypes.c_double, _d]
        lib.oracle_mesh.argtypes = [ctypes.c_int, _d, _d, _i32, ctypes.c_int, _d, _d, _d, _i32]
        lib.oracle_mesh.restype = ctypes.c_int64
        _LIB = lib
    return _LIB


def _p(a, t=_d):
    return a.ctypes.data_as(t)


def _vec(x):
    return np.ascontiguousarray(x, dtype=np.float64).reshape(3)


# ---------------------------------------------------------------- quadrature
def gauss_legendre(n: int):
    """n-point Gauss-Legendre nodes and weights on [-1, 1], ascending."""
    x = np.zeros(n)
    w = np.zeros(n)
    _lib().oracle_gauss_legendre(n, _p(x), _p(w))
    return x, w


# ---------------------------------------------------------------- pair integrals
def pair_integral(lo_i, hi_i, lo_j, hi_j) -> float:
    """Int_{I_i} Int_{I_j} 1/|x-y| dy dx by the section 3.4 reductions (no 1/4pi)."""
    a, b, c, d = (_vec(v) for v in (lo_i, hi_i, lo_j, hi_j))
    return _lib().oracle_pair_integral_exact(_p(a), _p(b), _p(c), _p(d))


def pair_gauss_mean(lo_i, hi_i, lo_j, hi_j, p: int) -> float:
    """p x p tensor Gauss mean of 1/|x-y| (weights summing to 1 on each panel)."""
    a, b, c, d = (_vec(v) for v in (lo_i, hi_i, lo_j, hi_j))
    return _lib().oracle_pair_gauss_mean(_p(a), _p(b), _p(c), _p(d), p)


def panel_area(lo, hi) -> float:
    a, b = _vec(lo), _vec(hi)
    return _lib().oracle_panel_area(_p(a), _p(b))


def is_near(lo_i, hi_i, lo_j, hi_j, eta: float) -> bool:
    a, b, c, d = (_vec(v) for v in (lo_i, hi_i, lo_j, hi_j))
    return bool(_lib().oracle_is_near(_p(a), _p(b), _p(c), _p(d), eta * eta))


def entry(lo_i, hi_i, lo_j, hi_j, p: int = 3, eta: float = 2.0) -> float:
    """One matrix entry a_ij under the method's near/far rule."""
    a, b, c, d = (_vec(v) for v in (lo_i, hi_i, lo_j, hi_j))
    return _lib().oracle_entry(_p(a), _p(b), _p(c), _p(d), p, eta)


# ---------------------------------------------------------------- mesh
def mesh_boxes(blo, bhi, bcond, rule):
    """Boxes -> panels (lo, hi, cond), deterministic order (see gbem_oracle.c)."""
    blo = np.ascontiguousarray(blo, dtype=np.float64).reshape(-1, 3)
    bhi = np.ascontiguousarray(bhi, dtype=np.float64).reshape(-1, 3)
    bcond = np.ascontiguousarray(bcond, dtype=np.int32).reshape(-1)
    if rule[0] == "uniform":
        kind, prm = 0, np.array([rule[1], 0.0, 0.0])
    elif rule[0] == "graded":
        kind, prm = 1, np.array([rule[1], rule[2], rule[3]], dtype=np.float64)
    else:
        raise ValueError(rule)
    lib = _lib()
    nb = blo.shape[0]
    null_d, null_i = ctypes.cast(None, _d), ctypes.cast(None, _i32)
    n = lib.oracle_mesh(nb, _p(blo), _p(bhi), _p(bcond, _i32), kind, _p(prm), null_d, null_d, null_i)
    lo = np.zeros((n, 3))
    hi = np.zeros((n, 3))
    cond = np.zeros(n, dtype=np.int32)
    lib.oracle_mesh(nb, _p(blo), _p(bhi), _p(bcond, _i32), kind, _p(prm), _p(lo), _p(hi),
                    _p(cond, _i32))
    return lo, hi, cond


def mesh_layout(layout):
    blo, bhi, bcond = layout.arrays()
    return mesh_boxes(blo, bhi, bcond, layout.rule)


# ---------------------------------------------------------------- near list
def near_csr(lo, hi, eta: float):
    """CSR (row_ptr int64[n+1], col int32[nnz]) of near pairs j <= i, ascending."""
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    n = lo.shape[0]
    rp = np.zeros(n + 1, dtype=np.int64)
    lib = _lib()
    lib.oracle_near_csr(n, _p(lo), _p(hi), eta, _p(rp, _i64), ctypes.cast(None, _i32))
    col = np.zeros(int(rp[-1]), dtype=np.int32)
    lib.oracle_near_csr(n, _p(lo), _p(hi), eta, _p(rp, _i64), _p(col, _i32))
    return rp, col


# ---------------------------------------------------------------- matrix
def assemble(lo, hi, p: int = 3, eta: float = 2.0) -> np.ndarray:
    """Dense symmetric A (n x n, FP64)."""
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    n = lo.shape[0]
    A = np.empty((n, n))
    _lib().oracle_assemble(n, _p(lo), _p(hi), p, eta, _p(A))
    return A


def entries(lo, hi, ii, jj, p: int = 3, eta: float = 2.0) -> np.ndarray:
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    ii = np.ascontiguousarray(ii, dtype=np.int32)
    jj = np.ascontiguousarray(jj, dtype=np.int32)
    out = np.empty(ii.shape[0])
    _lib().oracle_entries(_p(lo), _p(hi), ii.shape[0], _p(ii, _i32), _p(jj, _i32), p, eta, _p(out))
    return out


# ---------------------------------------------------------------- solve + charges
def rhs(cond, n_conductors: int) -> np.ndarray:
    """B_ik = 1 if panel i lies on conductor k (b of eq. "lineareq1" per main net)."""
    cond = np.asarray(cond)
    B = np.zeros((cond.shape[0], n_conductors))
    for k in range(n_conductors):
        B[cond == k, k] = 1.0
    return B


def solve(A, B):
    """Cholesky solve A X = B (LAPACK dpotrf/dpotrs)."""
    import scipy.linalg as sla
    c, low = sla.cho_factor(A, lower=True, check_finite=False)
    return sla.cho_solve((c, low), B, check_finite=False)


def solve_inplace(A, B):
    """Cholesky solve A X = B for orders whose dense matrix is too large for a
    second copy: LAPACK potrf/potrs as PyTorch's CPU build ships them (MKL),
    factoring A (symmetric, C-contiguous, n x n) in place.  (scipy's bundled
    OpenBLAS potrf fails on this host for orders above about 30,000.)
    A C-contiguous symmetric matrix read column by column is itself; on
    return A holds the Cholesky factor L (lower, zero above).  Returns X."""
    import torch
    assert A.flags.c_contiguous and A.dtype == np.float64 and A.shape[0] == A.shape[1]
    T = torch.from_numpy(A)                       # shares A's memory
    info = torch.empty((), dtype=torch.int32)
    torch.linalg.cholesky_ex(T, out=(T, info))    # in place: out is the input's own storage
    if int(info) != 0:
        raise np.linalg.LinAlgError(f"potrf: info = {int(info)}")
    Bt = torch.from_numpy(np.ascontiguousarray(np.asarray(B, dtype=np.float64).reshape(A.shape[0], -1)))
    return torch.cholesky_solve(Bt, T).numpy().copy()


def charges(X, cond, n_conductors: int, eps_r: float, length_unit_m: float) -> np.ndarray:
    """C_kl = eps_r eps0 l * sum_{i on conductor k} X_il, summed exactly (math.fsum)."""
    cond = np.asarray(cond)
    C = np.zeros((n_conductors, n_conductors))
    scale = eps_r * EPS0 * length_unit_m
    for k in range(n_conductors):
        rows = X[cond == k]
        for l in range(n_conductors):
            C[k, l] = scale * math.fsum(rows[:, l].tolist())
    return C


def extract_panels(lo, hi, cond, n_conductors: int, eps_r: float, length_unit_m: float,
                   p: int = 3, eta: float = 2.0, return_matrix: bool = False):
    """Whole path on a given mesh: returns the Maxwell capacitance matrix (F)."""
    A = assemble(lo, hi, p, eta)
    B = rhs(cond, n_conductors)
    X = solve(A, B)
    C = charges(X, cond, n_conductors, eps_r, length_unit_m)
    if return_matrix:
        return C, A, X
    return C


def extract(layout, p: int = 3, eta: float = 2.0, return_matrix: bool = False):
    lo, hi, cond = mesh_layout(layout)
    return extract_panels(lo, hi, cond, layout.n_conductors, layout.eps_r, layout.length_unit_m,
                          p, eta, return_matrix)


__all__ = ["EPS0", "gauss_legendre", "pair_integral", "pair_gauss_mean", "panel_area", "is_near",
           "entry", "mesh_boxes", "mesh_layout", "near_csr", "assemble", "entries", "rhs",
           "solve", "solve_inplace", "charges", "extract_panels", "extract"]
