"""Pins of the CPU oracle against values fixed by the paper or by mathematics.

Each check is independent of the oracle's own route (the section 3.4
reductions): textbook closed forms, library routines, brute force by other
reductions, exact scaling laws, physics invariants and the paper's printed
numbers (section 5, Table 2).
"""
import json
import math
import os

import numpy as np
import pytest

import gbem_inputs as gi
import oracle
from tests import _bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SELF_UNIT = 4.0 * math.log(1.0 + math.sqrt(2.0)) - 4.0 / 3.0 * (math.sqrt(2.0) - 1.0)


# ----------------------------------------------------------- quadrature rule
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 12, 16])
def test_gauss_legendre_matches_library(n):
    x, w = oracle.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(x, xr, rtol=0, atol=2e-15)
    np.testing.assert_allclose(w, wr, rtol=0, atol=2e-15)
    # exact for polynomials of degree 2n-1
    for deg in range(2 * n):
        exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
        assert abs(np.dot(w, x ** deg) - exact) < 1e-14


# ----------------------------------------------------------- pair integrals
@pytest.mark.parametrize("h", [1.0, 0.1, 0.37])
def test_self_square_closed_form(h):
    """Self integral of an h x h square: h^3 (4 ln(1+sqrt2) - 4/3 (sqrt2 - 1))."""
    for axis in range(3):
        lo = np.zeros(3)
        hi = np.full(3, h)
        hi[axis] = 0.0
        got = oracle.pair_integral(lo, hi, lo, hi)
        assert got == pytest.approx(SELF_UNIT * h ** 3, rel=2e-15)


def test_self_rectangle_textbook_reduction():
    """a x b rectangle: 4 Int_0^a Int_0^b (a-u)(b-v)/sqrt(u^2+v^2) (mpmath)."""
    import mpmath as mp
    mp.mp.dps = 20
    a, b = 2.0, 0.5
    ref = 4 * mp.quad(lambda u, v: (a - u) * (b - v) / mp.sqrt(u * u + v * v), [0, a], [0, b])
    got = oracle.pair_integral((0, 0, 0), (a, b, 0), (0, 0, 0), (a, b, 0))
    assert got == pytest.approx(float(ref), rel=1e-14)


NEAR_CASES = [
    # (lo_i, hi_i, lo_j, hi_j), description
    (((0, 0, 0), (1, 0, 1), (0, 0, 0), (1, 1, 0)), "orthogonal, shared edge"),
    (((0, 0.5, 1), (1, 0.5, 2), (0.3, -1, 0), (1.8, 1, 0)), "orthogonal, separated"),
    (((0, 0, 0), (0.3, 0, 0.7), (0.1, 0.2, -0.4), (0.5, 0.9, -0.4)), "orthogonal, offset"),
    (((0, 0, 0), (1, 1, 0), (1, 0, 0), (2, 1, 0)), "coplanar, shared edge"),
    (((0, 0, 0), (1, 1, 0), (1, 1, 0), (2, 2, 0)), "coplanar, shared corner"),
    (((0, 0, 0.2), (2, 1, 0.2), (0.5, -0.3, 0), (1.2, 0.4, 0)), "parallel offset"),
    (((0, 0, 0), (1, 1, 0), (0.2, 0.3, 0), (0.6, 0.5, 0)), "coplanar, contained"),
]


@pytest.mark.parametrize("case,desc", NEAR_CASES, ids=[c[1] for c in NEAR_CASES])
def test_near_pairs_vs_bruteforce(case, desc):
    got = oracle.pair_integral(*case)
    ref = bf.pair_integral_mp(*case, dps=17)
    assert got == pytest.approx(ref, rel=5e-14)


# Pairs of very different sizes (a 0.05 or 0.01 panel against a 4 x 4 one, as
# a fine bar panel against a coarse enclosure panel): the 16-term corner sum
# of the coplanar closed form cancels about (D/h)^4 of its magnitude, which the
# oracle's extended-precision arithmetic must absorb.  Reference: mpmath at 25
# digits by the convolution-weight route.
RATIO_CASES = [
    (((0, 0, 0), (0.05, 0.05, 0), (0.3, -2, 0), (4.3, 2, 0)), "coplanar separated, ratio 80"),
    (((4, 0, 0), (4.05, 0.05, 0), (0, -2, 0), (4, 2, 0)), "coplanar partial shared edge, ratio 80"),
    (((4, 0, 0), (4.01, 0.01, 0), (0, -2, 0), (4, 2, 0)), "coplanar partial shared edge, ratio 400"),
    (((1.0, 0.2, 1.0), (1.05, 0.25, 1.0), (0, -2, 0), (4, 2, 0)), "parallel above, ratio 80"),
    (((4.1, 0.0, 0.0), (4.15, 0.0, 0.05), (0, -2, 0), (4, 2, 0)), "orthogonal beside, ratio 80"),
    (((2.0, 0.0, 0.0), (2.05, 0.0, 0.05), (0, -2, 0), (4, 2, 0)), "orthogonal standing on, ratio 80"),
]


@pytest.mark.parametrize("case,desc", RATIO_CASES, ids=[c[1] for c in RATIO_CASES])
def test_large_size_ratio_pairs_vs_bruteforce(case, desc):
    got = oracle.pair_integral(*case)
    ref = bf.pair_integral_mp(*case, dps=25)
    assert got == pytest.approx(ref, rel=1e-13)
    # both orders of the pair
    assert oracle.pair_integral(case[2], case[3], case[0], case[1]) == pytest.approx(ref, rel=1e-13)


def test_pair_symmetry_and_invariance():
    """Int Int is symmetric in (I_i, I_j) and invariant under translation and mirroring."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        lo_i = rng.uniform(-1, 1, 3)
        hi_i = lo_i + rng.uniform(0.1, 1, 3)
        lo_j = rng.uniform(-1, 1, 3)
        hi_j = lo_j + rng.uniform(0.1, 1, 3)
        ni, nj = rng.integers(0, 3, 2)
        hi_i[ni] = lo_i[ni]
        hi_j[nj] = lo_j[nj]
        if ni == nj and lo_i[ni] == lo_j[ni]:
            continue
        g = oracle.pair_integral(lo_i, hi_i, lo_j, hi_j)
        assert oracle.pair_integral(lo_j, hi_j, lo_i, hi_i) == pytest.approx(g, rel=1e-12)
        t = rng.uniform(-3, 3, 3)
        assert oracle.pair_integral(lo_i + t, hi_i + t, lo_j + t, hi_j + t) == pytest.approx(g, rel=1e-11)
        # mirror x -> -x swaps lo/hi on that axis
        m = np.array([-1.0, 1.0, 1.0])
        li, hi2 = np.minimum(lo_i * m, hi_i * m), np.maximum(lo_i * m, hi_i * m)
        lj, hj2 = np.minimum(lo_j * m, hi_j * m), np.maximum(lo_j * m, hi_j * m)
        assert oracle.pair_integral(li, hi2, lj, hj2) == pytest.approx(g, rel=1e-11)


def test_separated_pair_vs_tensor_gauss():
    case = ((0, 0, 0), (1, 1, 0), (3, 0.5, 0.7), (4, 1.5, 0.7))
    assert oracle.pair_integral(*case) == pytest.approx(bf.pair_integral_gauss4d(*case), rel=1e-12)
    case = ((0, 0, 0), (1, 0, 1), (2.5, 0.5, -0.5), (3.0, 1.7, -0.5))
    assert oracle.pair_integral(*case) == pytest.approx(bf.pair_integral_gauss4d(*case), rel=1e-12)


# ----------------------------------------------------------- far-field rule
def test_far_rule_p1_is_centroid():
    lo_i, hi_i = np.array([0, 0, 0.0]), np.array([1, 0.5, 0.0])
    lo_j, hi_j = np.array([3, 1, 0.0]), np.array([3, 2, 1.0])
    ci, cj = 0.5 * (lo_i + hi_i), 0.5 * (lo_j + hi_j)
    assert oracle.pair_gauss_mean(lo_i, hi_i, lo_j, hi_j, 1) == pytest.approx(
        1.0 / np.linalg.norm(ci - cj), rel=1e-15)


def test_far_rule_converges_to_integral():
    case = ((0, 0, 0), (1, 1, 0), (2.2, 0.3, 0.4), (2.2, 1.1, 1.6))
    exact = oracle.pair_integral(*case)
    area = oracle.panel_area(case[0], case[1]) * oracle.panel_area(case[2], case[3])
    errs = [abs(oracle.pair_gauss_mean(*case, p) * area - exact) / exact for p in (1, 2, 3, 4, 8)]
    assert errs[-1] < 1e-10
    assert all(errs[k + 1] < errs[k] for k in range(len(errs) - 1))


def test_entry_uses_near_rule_for_touching_pairs():
    lo, hi = (0, 0, 0), (1, 1, 0)
    a = oracle.entry(lo, hi, lo, hi, p=3, eta=2.0)
    assert a == pytest.approx(SELF_UNIT / (4 * math.pi), rel=1e-15)


# ----------------------------------------------------------- near/far test
def test_near_classification_cases():
    sq = ((0, 0, 0), (1, 1, 0))
    assert oracle.is_near(*sq, *sq, 2.0)
    assert oracle.is_near(*sq, (1, 0, 0), (2, 1, 0), 0.5)       # touching: distance 0
    # distance^2 = 2 exactly, threshold eta^2 * diam^2 = 1 * 2: not near (strict)
    assert not oracle.is_near(*sq, (2, 2, 0), (3, 3, 0), 1.0)
    assert oracle.is_near(*sq, (1.999, 2, 0), (2.999, 3, 0), 1.0)
    # the larger panel's diameter sets the threshold
    big = ((0, 0, 5), (4, 4, 5))
    assert oracle.is_near(*sq, *big, 1.0) == oracle.is_near(*big, *sq, 1.0)
    assert oracle.is_near(*sq, *big, 1.0)     # distance 5 < 1 * sqrt(32)


def test_near_csr_structure():
    L = gi.two_plates(h=0.25)
    lo, hi, cond = oracle.mesh_layout(L)
    rp, col = oracle.near_csr(lo, hi, 2.0)
    n = lo.shape[0]
    for i in range(n):
        c = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0) and c[-1] == i and np.all(c <= i)
        for j in range(i + 1):
            assert (j in set(c.tolist())) == oracle.is_near(lo[i], hi[i], lo[j], hi[j], 2.0)


# ----------------------------------------------------------- mesher
def test_mesh_counts():
    assert oracle.mesh_layout(gi.two_plates())[0].shape[0] == 480
    assert oracle.mesh_layout(gi.crossing_bus())[0].shape[0] == 21420
    assert oracle.mesh_layout(gi.three_layer_bus())[0].shape[0] == 59904


@pytest.mark.parametrize("layout", [gi.two_plates(), gi.crossing_bus(), gi.crossing_bars_in_box()],
                         ids=["two_plates", "crossing_bus", "bars_in_box"])
def test_mesh_tiles_box_surfaces(layout):
    lo, hi, cond = oracle.mesh_layout(layout)
    ext = hi - lo
    assert np.all((ext == 0).sum(1) == 1) and np.all(ext >= 0)
    area = sum(oracle.panel_area(lo[k], hi[k]) for k in range(lo.shape[0]))
    surf = 0.0
    for blo, bhi, _ in layout.boxes:
        d = np.subtract(bhi, blo)
        surf += 2 * (d[0] * d[1] + d[1] * d[2] + d[0] * d[2])
    assert area == pytest.approx(surf, rel=1e-12)
    for k, (blo, bhi, c) in enumerate(layout.boxes):
        on = cond == c
        assert np.all(lo[on] >= np.array(blo) - 1e-12) and np.all(hi[on] <= np.array(bhi) + 1e-12)


def test_graded_edge_rule():
    """0.1-long edges: 3 graded cells per end + 1 middle; 2-long edges: 7 + 59 + 7."""
    L = gi.crossing_bus()
    lo, hi, cond = oracle.mesh_layout(L)
    on = (cond == 0) & (lo[:, 2] == 0.0) & (hi[:, 2] == 0.0)   # bottom face of wire 0
    xs = np.unique(np.concatenate([lo[on, 0], hi[on, 0]]))
    ys = np.unique(np.concatenate([lo[on, 1], hi[on, 1]]))
    assert len(xs) - 1 == 73 and len(ys) - 1 == 7
    dx = np.diff(xs)
    np.testing.assert_allclose(dx[:7], 0.01 * 1.2 ** np.arange(7), rtol=1e-12)
    np.testing.assert_allclose(dx[-7:], (0.01 * 1.2 ** np.arange(7))[::-1], rtol=1e-12)


# ----------------------------------------------------------- capacitance
@pytest.fixture(scope="module")
def c1():
    L = gi.two_plates()
    lo, hi, cond = oracle.mesh_layout(L)
    C, A, X = oracle.extract_panels(lo, hi, cond, 2, L.eps_r, L.length_unit_m, 3, 2.0, True)
    return L, lo, hi, cond, C, A, X


def test_matrix_symmetric_positive_definite(c1):
    L, lo, hi, cond, C, A, X = c1
    assert np.array_equal(A, A.T)
    ev = np.linalg.eigvalsh(A)
    assert ev[0] > 0
    B = oracle.rhs(cond, 2)
    assert np.linalg.norm(A @ X - B) / np.linalg.norm(B) < 1e-12


def test_maxwell_invariants(c1):
    C = c1[4]
    assert abs(C[0, 1] - C[1, 0]) <= 1e-10 * abs(C).max()
    assert C[0, 0] > 0 and C[1, 1] > 0 and C[0, 1] < 0
    assert np.all(C.sum(1) > 0)                           # free space
    assert np.all(np.linalg.eigvalsh(0.5 * (C + C.T)) > 0)
    assert C[0, 0] == pytest.approx(C[1, 1], rel=1e-9)    # mirror-symmetric pair


def test_parallel_plate_estimate(c1):
    """-C12 exceeds eps A/d (fringing adds) but stays of that order: 1 < ratio < 1.6."""
    C = c1[4]
    L = c1[0]
    eA_d = L.eps_r * oracle.EPS0 * 1e-12 / 0.2e-6
    r = -C[0, 1] / eA_d
    assert 1.0 < r < 1.6


def test_parallel_plate_limit():
    """The ratio -C12 d / (eps A) falls towards 1 as the gap shrinks."""
    ratios = []
    for d in (0.2, 0.1, 0.05):
        L = gi.parallel_plates(w=1.0, d=d, t=0.05, h=0.05)
        C = oracle.extract(L)
        ratios.append(-C[0, 1] * d * 1e-6 / (oracle.EPS0 * 1e-12))
    assert ratios[0] > ratios[1] > ratios[2] > 1.0
    assert ratios[2] < 1.25


def test_scale_and_permittivity_laws():
    base = gi.two_plates(h=0.25)
    C = oracle.extract(base)
    s = 2.0
    scaled = gi.Layout("scaled", [(tuple(s * v for v in lo), tuple(s * v for v in hi), c)
                                   for lo, hi, c in base.boxes], 2, ("uniform", 0.25 * s), base.eps_r)
    np.testing.assert_allclose(oracle.extract(scaled), s * C, rtol=1e-12)
    vac = gi.two_plates(h=0.25, eps_r=1.0)
    np.testing.assert_allclose(oracle.extract(vac) * base.eps_r, C, rtol=1e-14)


def test_permutation_invariance():
    L = gi.two_plates(h=0.25)
    lo, hi, cond = oracle.mesh_layout(L)
    C = oracle.extract_panels(lo, hi, cond, 2, L.eps_r, L.length_unit_m)
    perm = np.random.default_rng(1).permutation(lo.shape[0])
    Cp = oracle.extract_panels(lo[perm], hi[perm], cond[perm], 2, L.eps_r, L.length_unit_m)
    np.testing.assert_allclose(Cp, C, rtol=1e-12)


def test_unit_cube_lower_bound_and_convergence():
    """Galerkin capacitance of the unit cube rises towards 0.660678 * 4 pi eps0 a
    (73.510 aF) from below as the mesh is refined (exact-mode integration)."""
    ref = 0.660678 * 4 * math.pi * oracle.EPS0 * 1e-6
    c = [oracle.extract(gi.unit_cube(h), p=8, eta=4.0)[0, 0] for h in (0.5, 0.25, 0.125)]
    assert c[0] < c[1] < c[2] < ref
    assert (ref - c[2]) / ref < 0.01


def test_table2_window():
    """Section 5, Table 2: the paper's GBEM values lie within 5 % of the
    comparator; the oracle at its own mesh does too (permittivity read as 1)."""
    with open(os.path.join(GOLDEN, "table2_crossing_bars.json")) as f:
        g = json.load(f)
    L = gi.crossing_bars_in_box()
    bars = L.boxes[:2]
    encl = L.boxes[2:]
    parts = [oracle.mesh_boxes([b[0] for b in bars], [b[1] for b in bars], [b[2] for b in bars],
                               ("graded", 0.05, 1.3, 0.25)),
             oracle.mesh_boxes([b[0] for b in encl], [b[1] for b in encl], [b[2] for b in encl],
                               ("graded", 0.4, 1.4, 4.0))]
    lo = np.concatenate([p[0] for p in parts])
    hi = np.concatenate([p[1] for p in parts])
    cond = np.concatenate([p[2] for p in parts])
    C = oracle.extract_panels(lo, hi, cond, 2, 1.0, 1e-6) * 1e18
    cmp_ = g["comparator"]
    tol = g["claimed_accuracy"]
    for key, val in (("C11", C[0, 0]), ("C12", C[0, 1]), ("C21", C[1, 0]), ("C22", C[1, 1])):
        assert abs(val - cmp_[key]) <= tol * abs(cmp_[key]), (key, val)
    # and within 5 % of the paper's own finest GBEM row
    row = g["gbem"][-1]
    for key, val in (("C11", C[0, 0]), ("C12", C[0, 1]), ("C22", C[1, 1])):
        assert abs(val - row[key]) <= 0.05 * abs(row[key]), (key, val)


def test_inplace_solve_is_the_library_cholesky(c1):
    """The in-place solve used for orders too large for a second copy (the
    stored result of the three-layer bus) is LAPACK's Cholesky as well: on the
    C1 matrix it reproduces scipy's cho_factor/cho_solve, and it leaves the
    factor L (L L^T = A) in the matrix's memory."""
    import scipy.linalg as sla
    L, lo, hi, cond, C, A, X = c1
    B = oracle.rhs(cond, 2)
    X0 = sla.cho_solve(sla.cho_factor(A, lower=True), B)
    A2 = np.ascontiguousarray(A.copy())
    X1 = oracle.solve_inplace(A2, B)
    assert np.abs(X1 - X0).max() <= 1e-12 * np.abs(X0).max()
    Lf = np.tril(A2)
    assert np.abs(np.triu(A2, 1)).max() == 0.0
    assert np.abs(Lf @ Lf.T - A).max() <= 1e-12 * np.abs(A).max()
