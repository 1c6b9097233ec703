"""Partition rule and per-main-net extraction (test infrastructure only).

Follows section 3.3 of arXiv 2203.11733: the discretisation error of a piece
I_j scales with its area times the tangential derivative of the surface
charge density (Proposition 2), and far from the main net that derivative
falls with the cube of the distance (eq. "electric_derivative").  For one main
net the boundary is therefore split into rectangles I with

    |I| <= p4                          if d(I, main net) <= p5,
    |I| <= p4 * p3 * (d / p5)**3       otherwise,

p4 = p1 on boundary facing the main net and p4 = p1 * p2 on boundary turned
away from it.  The capacitances of the main net are the charges on all nets
with the main net at potential 1 and every other boundary at 0 (section 3.2),
so each main net gets its own mesh and its own solve.

Where the paper is silent this module takes these readings (stated once, used
by the tests as the definition):
  * d is the Euclidean distance from I to the nearest box of the main net;
  * the faces of the main net, and of any box that strictly contains the main
    net's bounding box, face it; another face faces it when some box of the
    main net reaches strictly beyond the face's plane on its outer side;
  * a rectangle over its bound is halved across its longer side (the lower of
    its two in-plane axes on a tie) at lo + (hi - lo) * 0.5, and the halves
    are refined depth first, lower half first;
  * arithmetic is plain IEEE double: d2 = sum over x, y, z of g * g (g the
    per-axis gap, 0 where the extents overlap), minimum over the net's boxes,
    d = sqrt(d2); bound = p4 if d <= p5 else p4 * p3 * (r * r * r), r = d / p5;
    area = (hi1 - lo1) * (hi2 - lo2).
Output order: boxes as given; faces -x, +x, -y, +y, -z, +z.

Section 5's Table 2 prints C12 = C21 at every mesh size, which per-main-net
meshes do not give at 74 or 183 panels (the other net is meshed coarsely in
each).  Its reading here: one mesh refined around every conductor at once
(main_net = ALL_NETS: the union of all conductor boxes is the main net), so
one symmetric system yields every column and C is symmetric.

Pure Python (no shared code with the GPU library); meant for meshes of up to
a few thousand panels.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as _o


def _in_plane(nrm: int):
    return (1, 2) if nrm == 0 else ((0, 2) if nrm == 1 else (0, 1))


def _dist2_to_net(net, lo, hi) -> float:
    best = math.inf
    for nl, nh in net:
        d2 = 0.0
        for k in range(3):
            if nl[k] > hi[k]:
                g = nl[k] - hi[k]
            elif lo[k] > nh[k]:
                g = lo[k] - nh[k]
            else:
                g = 0.0
            d2 = d2 + g * g
        if d2 < best:
            best = d2
    return best


def area_bound(net, lo, hi, p4: float, p3: float, p5: float) -> float:
    """Largest admissible area of the rectangle lo..hi (section 3.3)."""
    d = math.sqrt(_dist2_to_net(net, lo, hi))
    if d <= p5:
        return p4
    r = d / p5
    return p4 * p3 * (r * r * r)


def faces_main_net(box_lo, box_hi, on_net: bool, net, nrm: int, upper: bool) -> bool:
    """Whether the face (normal axis nrm, upper or lower side of the box) faces
    the main net (reading above)."""
    if on_net:
        return True
    nlo = [min(b[0][k] for b in net) for k in range(3)]
    nhi = [max(b[1][k] for b in net) for k in range(3)]
    if all(box_lo[k] < nlo[k] and nhi[k] < box_hi[k] for k in range(3)):
        return True
    plane = box_hi[nrm] if upper else box_lo[nrm]
    if upper:
        return any(b[1][nrm] > plane for b in net)
    return any(b[0][nrm] < plane for b in net)


ALL_NETS = -2   # main_net value: every conductor together is the main net


def _on_main(c: int, main_net: int) -> bool:
    return c >= 0 if main_net == ALL_NETS else c == main_net


def mesh_partition(blo, bhi, bcond, main_net: int, p1: float, p2: float, p3: float, p5: float):
    """Boxes -> panels (lo, hi, cond) for one main net, or for all conductors
    together (main_net = ALL_NETS: distance to the nearest conductor box, every
    conductor face facing), one mesh for every column of C."""
    blo = [tuple(float(v) for v in row) for row in np.asarray(blo, dtype=np.float64).reshape(-1, 3)]
    bhi = [tuple(float(v) for v in row) for row in np.asarray(bhi, dtype=np.float64).reshape(-1, 3)]
    bcond = [int(c) for c in np.asarray(bcond).reshape(-1)]
    net = [(blo[b], bhi[b]) for b in range(len(blo)) if _on_main(bcond[b], main_net)]
    if not net:
        raise ValueError("no box on the main net")
    out_lo, out_hi, out_c = [], [], []

    def refine(nrm, plane, a0, a1, b0, b1, p4, c):
        t1, t2 = _in_plane(nrm)
        lo = [0.0] * 3
        hi = [0.0] * 3
        lo[nrm] = hi[nrm] = plane
        lo[t1], hi[t1], lo[t2], hi[t2] = a0, a1, b0, b1
        w1, w2 = a1 - a0, b1 - b0
        if w1 * w2 <= area_bound(net, lo, hi, p4, p3, p5):
            out_lo.append(lo)
            out_hi.append(hi)
            out_c.append(c)
            return
        if w1 >= w2:
            m = a0 + (a1 - a0) * 0.5
            refine(nrm, plane, a0, m, b0, b1, p4, c)
            refine(nrm, plane, m, a1, b0, b1, p4, c)
        else:
            m = b0 + (b1 - b0) * 0.5
            refine(nrm, plane, a0, a1, b0, m, p4, c)
            refine(nrm, plane, a0, a1, m, b1, p4, c)

    for b in range(len(blo)):
        for f in range(6):
            nrm, upper = f // 2, bool(f & 1)
            plane = bhi[b][nrm] if upper else blo[b][nrm]
            facing = faces_main_net(blo[b], bhi[b], _on_main(bcond[b], main_net), net, nrm, upper)
            p4 = p1 if facing else p1 * p2
            t1, t2 = _in_plane(nrm)
            refine(nrm, plane, blo[b][t1], bhi[b][t1], blo[b][t2], bhi[b][t2], p4, bcond[b])
    return (np.array(out_lo, dtype=np.float64).reshape(-1, 3), np.array(out_hi, dtype=np.float64).reshape(-1, 3),
            np.array(out_c, dtype=np.int32))


def extract_partitioned(blo, bhi, bcond, n_conductors: int, eps_r: float, length_unit_m: float,
                        p1: float, p2: float, p3: float, p5: float, p: int = 3, eta: float = 2.0):
    """Column k of C from the mesh of main net k (charges on every net per volt
    on net k).  Returns (C, panels per mesh)."""
    C = np.zeros((n_conductors, n_conductors))
    panels = []
    for k in range(n_conductors):
        lo, hi, cond = mesh_partition(blo, bhi, bcond, k, p1, p2, p3, p5)
        Ck = _o.extract_panels(lo, hi, cond, n_conductors, eps_r, length_unit_m, p, eta)
        C[:, k] = Ck[:, k]
        panels.append(lo.shape[0])
    return C, panels


def extract_shared(blo, bhi, bcond, n_conductors: int, eps_r: float, length_unit_m: float,
                   p1: float, p2: float, p3: float, p5: float, p: int = 3, eta: float = 2.0):
    """All of C from one mesh refined around every conductor (the reading of
    section 5's Table 2, whose coupling columns agree at every size).
    Returns (C, panel count)."""
    lo, hi, cond = mesh_partition(blo, bhi, bcond, ALL_NETS, p1, p2, p3, p5)
    return _o.extract_panels(lo, hi, cond, n_conductors, eps_r, length_unit_m, p, eta), lo.shape[0]


__all__ = ["ALL_NETS", "area_bound", "faces_main_net", "mesh_partition", "extract_partitioned", "extract_shared"]
