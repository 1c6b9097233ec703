"""Seeded synthetic layouts shared by the GPU path's tests/bench and the CPU oracle.

This module only describes geometry: lists of axis-aligned boxes with a conductor
id each, plus the meshing rule to apply.  It holds none of the method's
arithmetic (no integrals, no solve); both the library and the oracle mesh these
boxes with their own code.  The multi-dielectric layouts at the end are given
panel by panel instead (uniform grids on each face, with the kind and the
regions on both sides), since that entry point takes panels.

A box is ``(lo, hi, cond)`` with ``lo``/``hi`` 3-tuples in micrometres.
``cond`` is the conductor index 0..M-1, or -1 for a grounded boundary that is
part of the boundary integral equation but not reported (the paper's Dirichlet
outer boundary, section 2.1 / 3.1).

Mesh rules (numbers are in the box's length unit):
  ("uniform", h)                  every box edge of length L is split into
                                  n = max(1, ceil(L/h - 1e-9)) equal cells
  ("graded", h_min, growth, h_max) edge-graded split: cells h_min, h_min*growth,
                                  ... from both ends while a cell is <= h_max and
                                  the run from one end stays <= L/2; the middle
                                  is split uniformly into
                                  max(1, ceil(rem/h_max - 1e-9)) cells
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

EPS0 = 8.8541878128e-12      # vacuum permittivity, F/m (CODATA 2018)
MICRON = 1e-6                 # metres per coordinate unit


@dataclass
class Layout:
    name: str
    boxes: list               # [(lo(3), hi(3), cond)]
    n_conductors: int
    rule: tuple
    eps_r: float = 3.9
    length_unit_m: float = MICRON
    meta: dict = field(default_factory=dict)

    def arrays(self):
        lo = np.array([b[0] for b in self.boxes], dtype=np.float64).reshape(-1, 3)
        hi = np.array([b[1] for b in self.boxes], dtype=np.float64).reshape(-1, 3)
        cond = np.array([b[2] for b in self.boxes], dtype=np.int32)
        return lo, hi, cond


def two_plates(gap: float = 0.2, h: float = 0.1, eps_r: float = 3.9) -> Layout:
    """Two 1 x 1 x 0.1 um boxes stacked face to face ``gap`` apart (480 panels at h=0.1)."""
    t = 0.1
    boxes = [((0.0, 0.0, 0.0), (1.0, 1.0, t), 0),
             ((0.0, 0.0, t + gap), (1.0, 1.0, 2 * t + gap), 1)]
    return Layout("two_plates", boxes, 2, ("uniform", h), eps_r)


def crossing_bus(eps_r: float = 3.9, rule=("graded", 0.01, 1.2, 0.03)) -> Layout:
    """Two metal layers x 5 wires (0.1 x 0.1 x 2 um, pitch 0.2 um, layer gap 0.1 um),
    layer 1 along x, layer 2 along y; 10 conductors, about 21k panels with the
    default edge-graded rule."""
    boxes = []
    for k in range(5):
        boxes.append(((0.0, 0.5 + 0.2 * k, 0.0), (2.0, 0.6 + 0.2 * k, 0.1), k))
    for k in range(5):
        boxes.append(((0.5 + 0.2 * k, 0.0, 0.2), (0.6 + 0.2 * k, 2.0, 0.3), 5 + k))
    return Layout("crossing_bus", boxes, 10, rule, eps_r)


def three_layer_bus(n_per_layer: int = 16, length: float = 10.0, h: float = 0.0646,
                    eps_r: float = 3.9) -> Layout:
    """3 layers x 16 wires, 0.1 x 0.1 x 10 um, pitch 0.2 um, layers 0.1 um apart,
    directions x, y, x, each layer centred on (5, 5); 59,904 panels at h=0.0646."""
    boxes = []
    c = 0
    half = 0.5 * length
    y0 = half - 0.2 * n_per_layer / 2 + 0.05
    for layer in range(3):
        z0 = 0.2 * layer
        for i in range(n_per_layer):
            a = y0 + 0.2 * i
            if layer % 2 == 0:   # along x
                boxes.append(((0.0, a, z0), (length, a + 0.1, z0 + 0.1), c))
            else:                # along y
                boxes.append(((a, 0.0, z0), (a + 0.1, length, z0 + 0.1), c))
            c += 1
    return Layout("three_layer_bus", boxes, c, ("uniform", h), eps_r)


def crossing_bars_in_box(rule=("graded", 0.25, 1.5, 4.0), eps_r: float = 1.0) -> Layout:
    """The paper's single-dielectric experiment (section 5): bars 4x1x1 um at
    (-2,-0.5,1)-(2,0.5,2) and (-0.5,-2,3)-(0.5,2,4) inside a grounded box
    (-20,-20,0)-(20,20,10).  The permittivity is not given there; 1 is used."""
    boxes = [((-2.0, -0.5, 1.0), (2.0, 0.5, 2.0), 0),
             ((-0.5, -2.0, 3.0), (0.5, 2.0, 4.0), 1),
             ((-20.0, -20.0, 0.0), (20.0, 20.0, 10.0), -1)]
    return Layout("crossing_bars_in_box", boxes, 2, rule, eps_r)


def unit_cube(h: float = 0.25, eps_r: float = 1.0) -> Layout:
    return Layout("unit_cube", [((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 0)], 1, ("uniform", h), eps_r)


def parallel_plates(w: float, d: float, t: float, h: float, eps_r: float = 1.0) -> Layout:
    """Two w x w plates of thickness t with face-to-face gap d."""
    boxes = [((0.0, 0.0, 0.0), (w, w, t), 0), ((0.0, 0.0, t + d), (w, w, 2 * t + d), 1)]
    return Layout("parallel_plates", boxes, 2, ("uniform", h), eps_r)


def _count_uniform(boxes, h):
    n = 0
    for lo, hi, _ in boxes:
        c = [max(1, math.ceil((hi[k] - lo[k]) / h - 1e-9)) for k in range(3)]
        n += 2 * (c[0] * c[1] + c[1] * c[2] + c[0] * c[2])
    return n


def random_manhattan(rng: np.random.Generator, n_target: float | None = None,
                     n_min: int = 500, n_max: int = 20000, eps_r: float = 3.9) -> Layout:
    """One random multi-layer Manhattan layout (serving stream job).

    Layers L ~ U{1,2,3}, directions x, y, x, layer k at z in [0.2k, 0.2k+0.1];
    wires W ~ U{2..16} dealt round-robin to layers; width ~ U[0.05,0.2],
    thickness 0.1, length ~ U[1,10], start offset ~ U[0,1], in-layer spacing
    ~ U[0.05,0.2].  Uniform panel size chosen so that the panel count is within
    10 % of a log-uniform target in [n_min, n_max]."""
    n_layers = int(rng.integers(1, 4))
    n_wires = int(rng.integers(2, 17))
    per_layer = [[] for _ in range(n_layers)]
    for w in range(n_wires):
        per_layer[w % n_layers].append(w)
    boxes = []
    for layer in range(n_layers):
        z0 = 0.2 * layer
        pos = 0.0
        for idx, w in enumerate(per_layer[layer]):
            width = float(rng.uniform(0.05, 0.2))
            length = float(rng.uniform(1.0, 10.0))
            start = float(rng.uniform(0.0, 1.0))
            if idx > 0:
                pos += float(rng.uniform(0.05, 0.2))
            if layer % 2 == 0:
                boxes.append(((start, pos, z0), (start + length, pos + width, z0 + 0.1), w))
            else:
                boxes.append(((pos, start, z0), (pos + width, start + length, z0 + 0.1), w))
            pos += width
    if n_target is None:
        n_target = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
    area = 0.0
    for lo, hi, _ in boxes:
        d = [hi[k] - lo[k] for k in range(3)]
        area += 2 * (d[0] * d[1] + d[1] * d[2] + d[0] * d[2])
    h = math.sqrt(area / n_target)
    lo_h, hi_h = h * 1e-3, max(h, 20.0)
    for _ in range(200):
        n = _count_uniform(boxes, h)
        if n_min <= n <= n_max and abs(n - n_target) <= 0.1 * n_target:
            break
        if n > n_target:
            lo_h = h
        else:
            hi_h = h
        h = 0.5 * (lo_h + hi_h)
    return Layout("manhattan", boxes, n_wires, ("uniform", h), eps_r,
                  meta={"n_target": n_target})


def serving_stream(n_jobs: int = 256, seed: int = 20220322, rate_hz: float = 50.0,
                   n_min: int = 500, n_max: int = 20000):
    """Seeded job stream: list of (arrival_time_s, Layout).  Job k draws its layout
    from SeedSequence(seed).spawn(n_jobs)[k]; arrivals are Poisson at rate_hz."""
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(n_jobs + 1)
    gaps = np.random.default_rng(children[-1]).exponential(1.0 / rate_hz, size=n_jobs)
    t = np.cumsum(gaps) - gaps[0]
    jobs = []
    for k in range(n_jobs):
        rng = np.random.default_rng(children[k])
        jobs.append((float(t[k]), random_manhattan(rng, n_min=n_min, n_max=n_max)))
    return jobs


def random_small_layout(seed: int, n_boxes: int = 3, h: float = 0.25) -> Layout:
    """A few random disjoint boxes, for property tests at small N."""
    rng = np.random.default_rng(seed)
    boxes = []
    tries = 0
    while len(boxes) < n_boxes and tries < 1000:
        tries += 1
        lo = rng.uniform(0.0, 3.0, size=3)
        size = rng.uniform(0.3, 1.2, size=3)
        hi = lo + size
        ok = True
        for blo, bhi, _ in boxes:
            if all(lo[k] <= bhi[k] + 0.1 and blo[k] <= hi[k] + 0.1 for k in range(3)):
                ok = False
                break
        if ok:
            boxes.append((tuple(float(x) for x in lo), tuple(float(x) for x in hi), len(boxes)))
    return Layout(f"random{seed}", boxes, len(boxes), ("uniform", h), 1.0)


# ---------------------------------------------------------------- several dielectrics
# Panel kinds of a multi-dielectric mesh (the numbering of gbem_panel_kind).
CONDUCTOR, DIRICHLET, NEUMANN, INTERFACE = 0, 1, 2, 3


@dataclass
class DielectricMesh:
    """Panels with their kind, net and the dielectric region on each side.

    lo, hi: (n, 3) corners (exactly one zero extent, the normal axis);
    region_plus / region_minus: region on the + / - side along that axis, -1
    where there is none (inside a conductor, outside the domain)."""
    name: str
    lo: np.ndarray
    hi: np.ndarray
    kind: np.ndarray
    conductor: np.ndarray
    region_plus: np.ndarray
    region_minus: np.ndarray
    eps_r: list
    n_conductors: int
    length_unit_m: float = MICRON

    @property
    def n_panels(self) -> int:
        return int(self.lo.shape[0])

    def args(self):
        """Positional arguments of the extractors: lo, hi, kind, conductor,
        region_plus, region_minus, eps_r, n_conductors, length_unit_m."""
        return (self.lo, self.hi, self.kind, self.conductor, self.region_plus, self.region_minus, self.eps_r,
                self.n_conductors, self.length_unit_m)


def _face_grid(nrm, plane, r1, r2, n1, n2):
    """n1 x n2 equal rectangles of the face {x_nrm = plane} spanning r1 along
    the first in-plane axis and r2 along the second (axes in increasing order)."""
    t1, t2 = [k for k in range(3) if k != nrm]
    out = []
    for i in range(n1):
        for j in range(n2):
            lo = [0.0] * 3
            hi = [0.0] * 3
            lo[nrm] = hi[nrm] = plane
            lo[t1] = r1[0] + (r1[1] - r1[0]) * i / n1
            hi[t1] = r1[0] + (r1[1] - r1[0]) * (i + 1) / n1
            lo[t2] = r2[0] + (r2[1] - r2[0]) * j / n2
            hi[t2] = r2[0] + (r2[1] - r2[0]) * (j + 1) / n2
            out.append((lo, hi))
    return out


def _cells(length, h):
    return max(1, int(math.ceil(length / h - 1e-9)))


class _PanelList:
    def __init__(self):
        self.rows = []

    def face(self, nrm, plane, r1, r2, h, kind, cond, rp, rm):
        for lo, hi in _face_grid(nrm, plane, r1, r2, _cells(r1[1] - r1[0], h), _cells(r2[1] - r2[0], h)):
            self.rows.append((lo, hi, kind, cond, rp, rm))

    def box_surface(self, lo, hi, h, kind, cond, region, outside):
        """The six faces of a box; `region` lies outside it when `outside`
        (a conductor in a dielectric) and inside it otherwise (the domain)."""
        for nrm in range(3):
            t1, t2 = [k for k in range(3) if k != nrm]
            r1, r2 = (lo[t1], hi[t1]), (lo[t2], hi[t2])
            # the face at lo[nrm] has the box interior on its + side
            inner_plus = (-1, region) if outside else (region, -1)
            self.face(nrm, lo[nrm], r1, r2, h, kind, cond, *inner_plus)
            self.face(nrm, hi[nrm], r1, r2, h, kind, cond, *inner_plus[::-1])

    def mesh(self, name, eps_r, n_conductors, length_unit_m=MICRON):
        cols = list(zip(*self.rows))
        return DielectricMesh(name, np.array(cols[0], float), np.array(cols[1], float),
                              np.array(cols[2], np.int32), np.array(cols[3], np.int32),
                              np.array(cols[4], np.int32), np.array(cols[5], np.int32), list(eps_r), n_conductors,
                              length_unit_m)


def two_slab_capacitor(L=1.0, d1=0.3, d2=0.7, n_xy=4, n_z=2, eps_r=(4.0, 1.0)) -> DielectricMesh:
    """Plates z = 0 (net 1) and z = d1 + d2 (net 0) of side L, region 0 in
    0 < z < d1, region 1 above, the interface at z = d1, Neumann side walls
    (no fringing field: the exact capacitance per unit permittivity is
    L^2 / (d1 / eps_0 + d2 / eps_1))."""
    H = d1 + d2
    pl = _PanelList()
    for lo, hi in _face_grid(2, 0.0, (0, L), (0, L), n_xy, n_xy):
        pl.rows.append((lo, hi, CONDUCTOR, 1, 0, -1))
    for lo, hi in _face_grid(2, H, (0, L), (0, L), n_xy, n_xy):
        pl.rows.append((lo, hi, CONDUCTOR, 0, -1, 1))
    for lo, hi in _face_grid(2, d1, (0, L), (0, L), n_xy, n_xy):
        pl.rows.append((lo, hi, INTERFACE, -1, 1, 0))
    for z0, z1, reg in ((0.0, d1, 0), (d1, H, 1)):
        for nrm in (0, 1):
            for plane, plus in ((0.0, True), (L, False)):
                for lo, hi in _face_grid(nrm, plane, (0, L), (z0, z1), n_xy, n_z):
                    pl.rows.append((lo, hi, NEUMANN, -1, reg if plus else -1, -1 if plus else reg))
    return pl.mesh(f"two_slab_{n_xy}x{n_z}", eps_r, 2)


def layered_stack(n_wires: int = 3, h: float = 0.25, h_out: float | None = None,
                  eps_r=(3.9, 2.7, 4.2)) -> DielectricMesh:
    """Synthetic interconnect stack with several dielectrics: three layers in
    a W x W x H domain (grounded top and bottom, Neumann side walls, two
    interfaces), n_wires parallel wires along x in layer 1 and n_wires along
    y in layer 2 (2 n_wires nets, each wire inside one layer).  Conductor
    faces are split into cells of at most h, the interfaces and the domain
    boundary into cells of at most h_out (default 2 h).  Micrometres."""
    h_out = 2.0 * h if h_out is None else h_out
    W = 2.0 + 1.0 * n_wires
    z = (0.0, 1.0, 2.2, 3.6)                       # layer boundaries
    pl = _PanelList()
    wires = []
    for k in range(n_wires):                       # layer 1: along x, 0.4 wide, 0.5 thick
        y0 = 1.3 + 1.0 * k
        wires.append(((0.6, y0, 1.35), (W - 0.6, y0 + 0.4, 1.85), 1))
    for k in range(n_wires):                       # layer 2: along y
        x0 = 1.3 + 1.0 * k
        wires.append(((x0, 0.6, 2.6), (x0 + 0.4, W - 0.6, 3.1), 2))
    for c, (lo, hi, layer) in enumerate(wires):
        assert z[layer] < lo[2] and hi[2] < z[layer + 1]
        pl.box_surface(lo, hi, h, CONDUCTOR, c, layer, outside=True)
    # grounded bottom and top, interfaces between the layers
    pl.face(2, z[0], (0, W), (0, W), h_out, DIRICHLET, -1, 0, -1)
    pl.face(2, z[3], (0, W), (0, W), h_out, DIRICHLET, -1, -1, 2)
    for a in (1, 2):
        pl.face(2, z[a], (0, W), (0, W), h_out, INTERFACE, -1, a, a - 1)
    # Neumann side walls, split at the layer boundaries
    for a in range(3):
        for nrm in (0, 1):
            pl.face(nrm, 0.0, (0, W), (z[a], z[a + 1]), h_out, NEUMANN, -1, a, -1)
            pl.face(nrm, W, (0, W), (z[a], z[a + 1]), h_out, NEUMANN, -1, -1, a)
    return pl.mesh(f"layered_stack_{2 * n_wires}nets_h{h:g}", eps_r, 2 * n_wires)


def two_slab_with_block(L=1.0, d1=0.3, d2=0.7, n_xy=4, n_z=2, eps_r=(4.0, 1.0, 7.0)) -> DielectricMesh:
    """The two-slab capacitor with a third dielectric (region 2) embedded in
    the lower slab: a block over the middle half of the plates (x, y in
    [L/4, 3L/4]) from z = d1/3 up to the interface z = d1, whose top face is
    the interface between regions 1 and 2.  Every region borders both others
    (the region graph is a triangle, not a chain).  n_xy: a multiple of 4."""
    assert n_xy % 4 == 0
    H = d1 + d2
    zb = d1 / 3.0
    a0, a1 = 0.25 * L, 0.75 * L
    pl = _PanelList()
    for lo, hi in _face_grid(2, 0.0, (0, L), (0, L), n_xy, n_xy):
        pl.rows.append((lo, hi, CONDUCTOR, 1, 0, -1))
    for lo, hi in _face_grid(2, H, (0, L), (0, L), n_xy, n_xy):
        pl.rows.append((lo, hi, CONDUCTOR, 0, -1, 1))
    for lo, hi in _face_grid(2, d1, (0, L), (0, L), n_xy, n_xy):
        cx, cy = 0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1])
        below = 2 if (a0 < cx < a1 and a0 < cy < a1) else 0
        pl.rows.append((lo, hi, INTERFACE, -1, 1, below))
    nb = n_xy // 2                                   # block cells across
    nbz = max(1, n_z // 2)
    for lo, hi in _face_grid(2, zb, (a0, a1), (a0, a1), nb, nb):   # block bottom: region 0 below
        pl.rows.append((lo, hi, INTERFACE, -1, 2, 0))
    for nrm in (0, 1):
        for plane, inside_plus in ((a0, True), (a1, False)):      # block sides
            for lo, hi in _face_grid(nrm, plane, (a0, a1), (zb, d1), nb, nbz):
                pl.rows.append((lo, hi, INTERFACE, -1, 2 if inside_plus else 0, 0 if inside_plus else 2))
    for z0, z1, reg in ((0.0, d1, 0), (d1, H, 1)):
        for nrm in (0, 1):
            for plane, plus in ((0.0, True), (L, False)):
                for lo, hi in _face_grid(nrm, plane, (0, L), (z0, z1), n_xy, n_z):
                    pl.rows.append((lo, hi, NEUMANN, -1, reg if plus else -1, -1 if plus else reg))
    return pl.mesh(f"two_slab_block_{n_xy}x{n_z}", eps_r, 2)


def bars_in_grounded_box(h_bar=1.0, h_box=2.0, eps_r=1.0) -> DielectricMesh:
    """One dielectric region: the paper's two crossing bars (section 5,
    4 x 1 x 1 um at z 1-2 and 3-4) inside a grounded box of 8 x 8 x 5 um (the
    paper's enclosure is 40 x 40 x 10; smaller here so the oracle stays fast),
    bar faces split into cells of at most h_bar, box faces h_box."""
    pl = _PanelList()
    pl.box_surface((-2.0, -0.5, 1.0), (2.0, 0.5, 2.0), h_bar, CONDUCTOR, 0, 0, outside=True)
    pl.box_surface((-0.5, -2.0, 3.0), (0.5, 2.0, 4.0), h_bar, CONDUCTOR, 1, 0, outside=True)
    pl.box_surface((-4.0, -4.0, 0.0), (4.0, 4.0, 5.0), h_box, DIRICHLET, -1, 0, outside=False)
    return pl.mesh(f"bars_in_grounded_box_{h_bar:g}_{h_box:g}", [eps_r], 2)


def bars_in_grounded_box_layout(h: float = 1.0) -> Layout:
    """The same geometry as boxes for the single-dielectric mesher (the
    enclosure as a grounded box, conductor id -1)."""
    boxes = [((-2.0, -0.5, 1.0), (2.0, 0.5, 2.0), 0), ((-0.5, -2.0, 3.0), (0.5, 2.0, 4.0), 1),
             ((-4.0, -4.0, 0.0), (4.0, 4.0, 5.0), -1)]
    return Layout("bars_in_grounded_box", boxes, 2, ("uniform", h), 1.0)


@dataclass
class DielectricLayout:
    """A layered dielectric layout: conductor boxes (each inside one layer),
    a box domain cut along z at z_layer, permittivity per layer, and the kind
    of the domain's bottom, top and side faces."""
    name: str
    box_lo: list
    box_hi: list
    box_net: list
    n_conductors: int
    domain_lo: tuple
    domain_hi: tuple
    z_layer: list
    eps_r: list
    bottom_kind: int = DIRICHLET
    top_kind: int = DIRICHLET
    side_kind: int = NEUMANN
    length_unit_m: float = MICRON


def layered_stack_layout(n_wires: int = 3, eps_r=(3.9, 2.7, 4.2)) -> DielectricLayout:
    """The geometry of layered_stack as a layout (for the per-main-net meshes
    of the partition rules): grounded top and bottom, Neumann side walls."""
    W = 2.0 + 1.0 * n_wires
    lo, hi, net = [], [], []
    for k in range(n_wires):
        y0 = 1.3 + 1.0 * k
        lo.append((0.6, y0, 1.35))
        hi.append((W - 0.6, y0 + 0.4, 1.85))
        net.append(k)
    for k in range(n_wires):
        x0 = 1.3 + 1.0 * k
        lo.append((x0, 0.6, 2.6))
        hi.append((x0 + 0.4, W - 0.6, 3.1))
        net.append(n_wires + k)
    return DielectricLayout(f"layered_stack_{2 * n_wires}nets", lo, hi, net, 2 * n_wires, (0.0, 0.0, 0.0),
                            (W, W, 3.6), [0.0, 1.0, 2.2, 3.6], list(eps_r))
