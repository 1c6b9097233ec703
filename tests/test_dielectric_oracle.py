"""Pins of the multi-dielectric oracle (section 4 of arXiv 2203.11733).

None of them re-types the oracle's formulas: the solid angle against the
textbook on-axis value of a rectangle, the double-layer integrals against
Gauss's theorem on a closed box and against brute-force 4-D Gauss, the
coplanar zero the paper states (section 4.2), and whole extractions against
the closed-form capacitance of a two-slab capacitor, a mirror symmetry and
the permittivity scaling."""
import math
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import gbem_inputs as gi  # noqa: E402
from oracle import dielectric as od  # noqa: E402
from oracle import oracle as oo  # noqa: E402


def say(*a):
    print(*a, flush=True)


def test_solid_angle_on_axis():
    """A 2a x 2b rectangle seen from height h on its axis subtends
    4 atan(a b / (h sqrt(a^2 + b^2 + h^2))); just above its interior 2 pi,
    just below -2 pi, in its plane 0."""
    for a, b, h in ((0.5, 0.5, 1.0), (1.0, 0.25, 0.3), (2.0, 3.0, 7.0)):
        ref = 4.0 * math.atan(a * b / (h * math.sqrt(a * a + b * b + h * h)))
        got = float(od.solid_angle_rect(0.0, 0.0, h, -a, a, -b, b)[()])
        assert got == pytest.approx(ref, rel=1e-14)
        assert float(od.solid_angle_rect(0.0, 0.0, -h, -a, a, -b, b)[()]) == pytest.approx(-ref, rel=1e-14)
    assert float(od.solid_angle_rect(0.1, 0.2, 1e-12, -1, 1, -1, 1)[()]) == pytest.approx(2 * math.pi, rel=1e-9)
    assert float(od.solid_angle_rect(0.1, 0.2, 0.0, -1, 1, -1, 1)[()]) == 0.0


def _box_panels(lo, hi, n):
    """Panels of a box surface, n x n per face, each with its outward sign
    (+1 when the outward normal is + along the panel's normal axis)."""
    P = []
    for nrm in range(3):
        t1, t2 = [k for k in range(3) if k != nrm]
        for plane, sgn in ((lo[nrm], -1.0), (hi[nrm], 1.0)):
            for i in range(n):
                for j in range(n):
                    a = [0.0] * 3
                    b = [0.0] * 3
                    a[nrm] = b[nrm] = plane
                    a[t1] = lo[t1] + (hi[t1] - lo[t1]) * i / n
                    b[t1] = lo[t1] + (hi[t1] - lo[t1]) * (i + 1) / n
                    a[t2] = lo[t2] + (hi[t2] - lo[t2]) * j / n
                    b[t2] = lo[t2] + (hi[t2] - lo[t2]) * (j + 1) / n
                    P.append((np.array(a), np.array(b), sgn))
    return P


def _area(lo, hi):
    e = hi - lo
    return float(np.prod(e[e != 0]))


def test_gauss_theorem_on_a_closed_box():
    """Int over a closed surface of q*(x, y) with outward normals is -1/2 at a
    smooth point of the surface and 0 outside it (the identity behind
    sigma = 1/2 in eq. "representation"), so summing Q_ik over the panels k of
    a box gives -|I_i| / 2 for a panel I_i on the box and 0 for a panel
    outside it."""
    box = _box_panels(np.array([0.0, 0.0, 0.0]), np.array([1.0, 0.6, 0.8]), 2)
    for i in (0, 5, 13, 22):
        lo_i, hi_i, _ = box[i]
        s = sum(sgn * od.double_layer_pair(lo_i, hi_i, lo_k, hi_k) for lo_k, hi_k, sgn in box)
        say(f"  on the box, panel {i}: {s:.15f} vs {-0.5 * _area(lo_i, hi_i):.15f}")
        assert s == pytest.approx(-0.5 * _area(lo_i, hi_i), abs=1e-9 * _area(lo_i, hi_i))
    for lo_i, hi_i in (([1.3, 0.1, 0.2], [1.3, 0.5, 0.6]), ([0.2, 0.0, 1.1], [0.9, 0.6, 1.1]),
                       ([-0.5, -0.2, 0.4], [0.4, -0.2, 1.5])):
        lo_i, hi_i = np.array(lo_i), np.array(hi_i)
        s = sum(sgn * od.double_layer_pair(lo_i, hi_i, lo_k, hi_k) for lo_k, hi_k, sgn in box)
        say(f"  outside the box: {s:.3e}")
        assert abs(s) <= 1e-9 * _area(lo_i, hi_i)


def _brute(lo_i, hi_i, lo_k, hi_k, n=24):
    """Tensor Gauss of q* over both panels (normal of I_k along +)."""
    x, w = np.polynomial.legendre.leggauss(n)

    def pts(lo, hi):
        e = hi - lo
        nrm = int(np.flatnonzero(e == 0)[0])
        t1, t2 = [k for k in range(3) if k != nrm]
        u = 0.5 * (lo[t1] + hi[t1]) + 0.5 * e[t1] * x
        v = 0.5 * (lo[t2] + hi[t2]) + 0.5 * e[t2] * x
        U, V = np.meshgrid(u, v, indexing="ij")
        P = np.zeros((n * n, 3))
        P[:] = lo
        P[:, t1], P[:, t2] = U.ravel(), V.ravel()
        return P, np.outer(w, w).ravel() * 0.25 * e[t1] * e[t2], nrm
    X, WX, _ = pts(lo_i, hi_i)
    Y, WY, nk = pts(lo_k, hi_k)
    d = X[:, None, :] - Y[None, :, :]
    r = np.sqrt((d * d).sum(-1))
    q = d[:, :, nk] / (4 * math.pi * r ** 3)
    return float(WX @ q @ WY)


@pytest.mark.parametrize("case", [
    (([0, 0, 0], [1, 1, 0]), ([2.5, 0.3, 1.0], [3.1, 1.2, 1.0])),        # parallel, separated
    (([0, 0, 0], [1, 0, 1]), ([2.0, 1.5, 0.2], [2.7, 2.5, 0.2])),        # orthogonal, separated
    (([0, 0, 0], [0, 1, 2]), ([1.5, -1, 3.0], [2.5, 2, 3.0])),           # orthogonal, other axes
], ids=["parallel", "orthogonal", "orthogonal2"])
def test_separated_pairs_vs_bruteforce(case):
    (a, b), (c, d) = case
    a, b, c, d = (np.array(v, float) for v in (a, b, c, d))
    got = od.double_layer_pair(a, b, c, d)
    ref = _brute(a, b, c, d)
    assert got == pytest.approx(ref, rel=1e-10)


def test_coplanar_pairs_vanish():
    """Section 4.2: for parallel panels in one plane (b = x3 - y3 = 0) Q = 0."""
    assert od.double_layer_pair([0, 0, 0], [1, 1, 0], [1, 0, 0], [2, 1, 0]) == 0.0
    assert od.double_layer_pair([0, 0, 0], [1, 1, 0], [3, 4, 0], [5, 5, 0]) == 0.0


def test_two_slab_capacitor_converges_to_series_formula():
    """Two dielectric slabs between plates with Neumann side walls: the field
    is one-dimensional, C = eps0 L^2 / (d1/eps1 + d2/eps2).  The piecewise
    constant Galerkin solution converges to it (errors 39 %, 13 %, 6.5 % at
    2, 4, 6 panels across), with C12 = C21 approached and C11 = -C21 (all flux
    of net 0 ends on net 1)."""
    L, d1, d2, e = 1.0, 0.3, 0.7, [4.0, 1.0]
    exact = oo.EPS0 * 1e-6 * L * L / (d1 / e[0] + d2 / e[1])
    errs = []
    for nxy, nz in ((2, 1), (4, 2), (6, 3)):
        C = od.extract(*gi.two_slab_capacitor(L, d1, d2, nxy, nz, e).args())
        errs.append(C[0, 0] / exact - 1.0)
        say(f"  {nxy} x {nz}: C00 / exact - 1 = {errs[-1]:.4f}, C01 / C10 = {C[0, 1] / C[1, 0]:.6f}")
        assert C[0, 0] > 0 and C[1, 0] < 0
        assert abs(C[0, 0] + C[1, 0]) <= 2e-3 * C[0, 0]
    assert errs[0] > errs[1] > errs[2] > 0
    assert errs[1] < 0.14 and errs[2] < 0.07
    assert errs[0] / errs[1] > 2.5 and errs[1] / errs[2] > 1.8


def test_two_slab_mirror_and_scaling():
    """The mirrored capacitor (slabs swapped, plates swapped) gives the same C
    with the nets exchanged, and scaling every permittivity scales C."""
    L, d1, d2 = 1.0, 0.3, 0.7
    C = od.extract(*gi.two_slab_capacitor(L, d1, d2, 3, 2, [4.0, 1.0]).args())
    # mirror z -> H - z: swap the roles (net 0 <-> net 1, region 0 <-> region 1)
    Cm = od.extract(*gi.two_slab_capacitor(L, d2, d1, 3, 2, [1.0, 4.0]).args())
    assert Cm[1, 1] == pytest.approx(C[0, 0], rel=1e-10)
    assert Cm[0, 0] == pytest.approx(C[1, 1], rel=1e-10)
    assert Cm[0, 1] == pytest.approx(C[1, 0], rel=1e-10)
    C2 = od.extract(*gi.two_slab_capacitor(L, d1, d2, 3, 2, [8.0, 2.0]).args())
    assert np.allclose(C2, 2.0 * C, rtol=1e-12, atol=0)
