"""Per-main-net meshes of layered multi-dielectric layouts (test infrastructure only).

Section 4.1 of arXiv 2203.11733 keeps the section 3.3 partition for the
boundary elements on conductors and on the outer boundary and changes it for
the dielectric interfaces, whose unknowns include the potential: far from the
main net the tangential derivative of the potential falls with the square of
the distance, so an interface piece I may grow as d**2 instead of d**3:

    conductors, outer boundary:  |I| <= p4 within p5,  p4 * p3 * (d / p5)**3 beyond
    interfaces:                  |I| <= p4 within p5,  p4 * p3 * (d / l)**2 beyond

Readings (the paper leaves them open):
  * l is p5, the length that normalises d in the section 3.3 rule;
  * p4 = p1 on interfaces and on the outer boundary (it encloses the main net),
    p1 or p1 * p2 on conductor faces as in the section 3.3 reading of
    oracle.partition (facing the main net or turned away from it);
  * d, the bisection (longer side first, lower half first) and the IEEE
    arithmetic of the bound are those of oracle.partition.
A layered layout is a box domain cut along z into layers, with conductor boxes
each strictly inside one layer; the domain's bottom, top and side faces are
Dirichlet or Neumann.  Panel order: conductor boxes as given (faces -x, +x,
-y, +y, -z, +z), bottom, top, the side walls layer by layer (-x, +x, -y, +y),
the interfaces from the bottom up.

Pure Python, no code shared with the GPU library.
"""
from __future__ import annotations

import math

import numpy as np

from . import dielectric as od
from .partition import _dist2_to_net, faces_main_net


def bound(net, lo, hi, p4: float, p3: float, p5: float, power: int) -> float:
    """Largest admissible area of lo..hi: power 3 for conductors and the outer
    boundary (section 3.3), 2 for interfaces (section 4.1)."""
    d = math.sqrt(_dist2_to_net(net, lo, hi))
    if d <= p5:
        return p4
    r = d / p5
    return p4 * p3 * (r * r * r if power == 3 else r * r)


def mesh(layout, main_net: int, p1: float, p2: float, p3: float, p5: float):
    """Panels of a gbem_inputs.DielectricLayout for one main net:
    (lo, hi, kind, conductor, region_plus, region_minus)."""
    blo = [tuple(float(v) for v in b) for b in layout.box_lo]
    bhi = [tuple(float(v) for v in b) for b in layout.box_hi]
    nets = [int(c) for c in layout.box_net]
    z = [float(v) for v in layout.z_layer]
    nl = len(z) - 1
    dlo = [float(v) for v in layout.domain_lo]
    dhi = [float(v) for v in layout.domain_hi]
    net = [(blo[b], bhi[b]) for b in range(len(blo)) if nets[b] == main_net]
    if not net:
        raise ValueError("no box on the main net")
    layer = []
    for b in range(len(blo)):
        inside = [a for a in range(nl) if z[a] < blo[b][2] and bhi[b][2] < z[a + 1]]
        if len(inside) != 1:
            raise ValueError(f"box {b} is not strictly inside one layer")
        layer.append(inside[0])
    rows = []   # (lo, hi, kind, net, region_plus, region_minus)

    def refine(nrm, plane, a0, a1, b0, b1, p4, power, tag):
        t1, t2 = (1, 2) if nrm == 0 else ((0, 2) if nrm == 1 else (0, 1))
        lo = [0.0] * 3
        hi = [0.0] * 3
        lo[nrm] = hi[nrm] = plane
        lo[t1], hi[t1], lo[t2], hi[t2] = a0, a1, b0, b1
        w1, w2 = a1 - a0, b1 - b0
        if w1 * w2 <= bound(net, lo, hi, p4, p3, p5, power):
            rows.append((lo, hi) + tag)
            return
        if w1 >= w2:
            m = a0 + (a1 - a0) * 0.5
            refine(nrm, plane, a0, m, b0, b1, p4, power, tag)
            refine(nrm, plane, m, a1, b0, b1, p4, power, tag)
        else:
            m = b0 + (b1 - b0) * 0.5
            refine(nrm, plane, a0, a1, b0, m, p4, power, tag)
            refine(nrm, plane, a0, a1, m, b1, p4, power, tag)

    for b in range(len(blo)):
        for f in range(6):
            nrm, upper = f // 2, bool(f & 1)
            plane = bhi[b][nrm] if upper else blo[b][nrm]
            p4 = p1 if faces_main_net(blo[b], bhi[b], nets[b] == main_net, net, nrm, upper) else p1 * p2
            t1, t2 = (1, 2) if nrm == 0 else ((0, 2) if nrm == 1 else (0, 1))
            # the dielectric lies outside the box
            tag = (od.CONDUCTOR, nets[b], layer[b] if upper else -1, -1 if upper else layer[b])
            refine(nrm, plane, blo[b][t1], bhi[b][t1], blo[b][t2], bhi[b][t2], p4, 3, tag)
    refine(2, dlo[2], dlo[0], dhi[0], dlo[1], dhi[1], p1, 3, (layout.bottom_kind, -1, 0, -1))
    refine(2, dhi[2], dlo[0], dhi[0], dlo[1], dhi[1], p1, 3, (layout.top_kind, -1, -1, nl - 1))
    for a in range(nl):
        for nrm in (0, 1):
            t = 1 - nrm
            for upper in (False, True):
                plane = dhi[nrm] if upper else dlo[nrm]
                refine(nrm, plane, dlo[t], dhi[t], z[a], z[a + 1], p1, 3,
                       (layout.side_kind, -1, -1 if upper else a, a if upper else -1))
    for a in range(1, nl):
        refine(2, z[a], dlo[0], dhi[0], dlo[1], dhi[1], p1, 2, (od.INTERFACE, -1, a, a - 1))
    cols = list(zip(*rows))
    return (np.array(cols[0], np.float64), np.array(cols[1], np.float64), np.array(cols[2], np.int32),
            np.array(cols[3], np.int32), np.array(cols[4], np.int32), np.array(cols[5], np.int32))


def extract(layout, p1: float, p2: float, p3: float, p5: float, single_layer=(3, 2.0)):
    """Column k of C from the mesh of main net k.  Returns (C, panels per mesh)."""
    m = layout.n_conductors
    C = np.zeros((m, m))
    panels = []
    for k in range(m):
        lo, hi, kind, cond, rp, rm = mesh(layout, k, p1, p2, p3, p5)
        Ck = od.extract(lo, hi, kind, cond, rp, rm, layout.eps_r, m, layout.length_unit_m, single_layer)
        C[:, k] = Ck[:, k]
        panels.append(lo.shape[0])
    return C, panels


__all__ = ["bound", "mesh", "extract"]
