"""ctypes binding of libgbem (include/gbem.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  PyTorch appears only to hand device buffers and streams to the
``*_device`` entry points.  Loading fails loudly when the library is missing;
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgbem.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOTPD, ENOCONV, EBUSY, ETIMEOUT = range(8)
F64, F32, F16, BF16 = range(4)
KERNEL_CLASSES = ["far", "near_list", "near_eval", "diag", "trsm", "syrk", "solve", "residual", "panel", "other"]
NCLS = len(KERNEL_CLASSES)   # GBEM_K_COUNT
DTYPES = {"f64": F64, "f32": F32, "f16": F16, "bf16": BF16}

EXPORTS = [
    "gbem_version", "gbem_status_str", "gbem_last_error", "gbem_default_opts", "gbem_create",
    "gbem_destroy", "gbem_extract", "gbem_extract_device", "gbem_submit", "gbem_poll", "gbem_wait",
    "gbem_job_free", "gbem_server_stats", "gbem_mesh_boxes", "gbem_mesh_buf_free", "gbem_near_list",
    "gbem_assemble", "gbem_assemble_sample", "gbem_assemble_scaled_sample", "gbem_cholesky_device",
    "gbem_cholesky_solve_device", "gbem_mesh_partition", "gbem_extract_partitioned",
    "gbem_extract_device_noalloc", "gbem_load_tuning", "gbem_set_tuning_override", "gbem_tuning_source",
    "gbem_extract_dielectric", "gbem_assemble_double_layer", "gbem_mesh_dielectric_partition",
    "gbem_dmesh_buf_free", "gbem_extract_dielectric_partitioned",
]
# gbem_panel_kind
CONDUCTOR, DIRICHLET, NEUMANN, INTERFACE = range(4)


class GbemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gbem status {status}: {msg}")
        self.status = status


class Mesh(ctypes.Structure):
    _fields_ = [("n_panels", ctypes.c_int32), ("n_conductors", ctypes.c_int32),
                ("lo", ctypes.c_void_p), ("hi", ctypes.c_void_p), ("conductor", ctypes.c_void_p),
                ("eps_r", ctypes.c_double), ("length_unit_m", ctypes.c_double), ("basis", ctypes.c_int32)]


class DMesh(ctypes.Structure):
    _fields_ = [("n_panels", ctypes.c_int32), ("n_conductors", ctypes.c_int32), ("n_regions", ctypes.c_int32),
                ("lo", ctypes.c_void_p), ("hi", ctypes.c_void_p), ("kind", ctypes.c_void_p),
                ("conductor", ctypes.c_void_p), ("region_plus", ctypes.c_void_p),
                ("region_minus", ctypes.c_void_p), ("eps_r", ctypes.c_void_p), ("length_unit_m", ctypes.c_double)]


class DLayout(ctypes.Structure):
    _fields_ = [("n_boxes", ctypes.c_int32), ("box_lo", ctypes.c_void_p), ("box_hi", ctypes.c_void_p),
                ("box_net", ctypes.c_void_p), ("n_conductors", ctypes.c_int32),
                ("domain_lo", ctypes.c_double * 3), ("domain_hi", ctypes.c_double * 3),
                ("n_layers", ctypes.c_int32), ("z_layer", ctypes.c_void_p), ("eps_r", ctypes.c_void_p),
                ("bottom_kind", ctypes.c_int32), ("top_kind", ctypes.c_int32), ("side_kind", ctypes.c_int32),
                ("length_unit_m", ctypes.c_double)]


class DMeshBuf(ctypes.Structure):
    _fields_ = [("n_panels", ctypes.c_int32), ("lo", ctypes.POINTER(ctypes.c_double)),
                ("hi", ctypes.POINTER(ctypes.c_double)), ("kind", ctypes.POINTER(ctypes.c_int32)),
                ("conductor", ctypes.POINTER(ctypes.c_int32)), ("region_plus", ctypes.POINTER(ctypes.c_int32)),
                ("region_minus", ctypes.POINTER(ctypes.c_int32))]


class Opts(ctypes.Structure):
    _fields_ = [("far_order", ctypes.c_int32), ("near_eta", ctypes.c_double),
                ("far_dtype", ctypes.c_int32), ("factor_dtype", ctypes.c_int32),
                ("refine_tol", ctypes.c_double), ("max_refine", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("graph", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("t_assemble_ms", ctypes.c_double), ("t_factor_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double),
                ("residual", ctypes.c_double), ("asym", ctypes.c_double),
                ("refine_iters", ctypes.c_int32), ("factor_used", ctypes.c_int32),
                ("n_near", ctypes.c_int64), ("n_panels", ctypes.c_int64),
                ("prof_ms", ctypes.c_double * NCLS), ("prof_launches", ctypes.c_int64 * NCLS),
                ("prof_flops", ctypes.c_double * NCLS), ("prof_bytes", ctypes.c_double * NCLS),
                ("outer_width", ctypes.c_int32), ("super_panels", ctypes.c_int32),
                ("graph_used", ctypes.c_int32), ("graph_instantiated", ctypes.c_int32)]

    def as_dict(self):
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            d[k] = list(v) if k.startswith("prof_") else v
        d["profile"] = {name: {"ms": d["prof_ms"][i], "launches": d["prof_launches"][i],
                               "flops": d["prof_flops"][i], "bytes": d["prof_bytes"][i]}
                        for i, name in enumerate(KERNEL_CLASSES) if d["prof_launches"][i]}
        for k in ("prof_ms", "prof_launches", "prof_flops", "prof_bytes"):
            del d[k]
        return d


class Tuning(ctypes.Structure):
    """Tile shapes of the factorisation (gbem_tuning)."""
    _fields_ = [("outer_width", ctypes.c_int32), ("super_panels", ctypes.c_int32)]


def load_tuning(path: str | None):
    """Replace the process-wide shape cache (None: built-in defaults)."""
    lib = load()
    _check(lib.gbem_load_tuning(path.encode() if path else None))


def set_tuning_override(outer_width: int = 0, super_panels: int = 0):
    """Force shapes for later factorisations (0: from the cache)."""
    lib = load()
    t = Tuning(outer_width, super_panels)
    _check(lib.gbem_set_tuning_override(ctypes.byref(t) if (outer_width or super_panels) else None))


def tuning_source() -> str:
    return load().gbem_tuning_source().decode()


class MeshRule(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("h", ctypes.c_double), ("h_min", ctypes.c_double),
                ("growth", ctypes.c_double), ("h_max", ctypes.c_double)]


class Partition(ctypes.Structure):
    """Partition rule of section 3.3 (gbem_partition)."""
    _fields_ = [("p1", ctypes.c_double), ("p2", ctypes.c_double), ("p3", ctypes.c_double),
                ("p5", ctypes.c_double)]


class MeshBuf(ctypes.Structure):
    _fields_ = [("n_panels", ctypes.c_int32), ("lo", ctypes.POINTER(ctypes.c_double)),
                ("hi", ctypes.POINTER(ctypes.c_double)), ("conductor", ctypes.POINTER(ctypes.c_int32))]


_LIB = None
_vp = ctypes.c_void_p


def load():
    """Load libgbem.so (built by ``python -m paper_2203_11733_amd.build``); raises if missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2203_11733_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    lib.gbem_version.restype = ctypes.c_char_p
    lib.gbem_status_str.restype = ctypes.c_char_p
    lib.gbem_status_str.argtypes = [ctypes.c_int]
    lib.gbem_last_error.restype = ctypes.c_char_p
    lib.gbem_default_opts.argtypes = [ctypes.POINTER(Opts)]
    lib.gbem_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(_vp)]
    lib.gbem_destroy.argtypes = [_vp]
    lib.gbem_extract.argtypes = [_vp, ctypes.POINTER(Mesh), ctypes.POINTER(Opts), _vp, ctypes.POINTER(Report)]
    lib.gbem_extract_device.argtypes = [_vp, ctypes.POINTER(Mesh), ctypes.POINTER(Opts), _vp, _vp,
                                        ctypes.POINTER(Report)]
    lib.gbem_extract_device_noalloc.argtypes = [_vp, ctypes.POINTER(Mesh), ctypes.POINTER(Opts), _vp, _vp,
                                                ctypes.POINTER(Report)]
    lib.gbem_load_tuning.argtypes = [ctypes.c_char_p]
    lib.gbem_set_tuning_override.argtypes = [ctypes.POINTER(Tuning)]
    lib.gbem_tuning_source.restype = ctypes.c_char_p
    lib.gbem_submit.argtypes = [_vp, ctypes.POINTER(Mesh), ctypes.POINTER(Opts), ctypes.POINTER(_vp)]
    lib.gbem_poll.argtypes = [_vp]
    lib.gbem_wait.argtypes = [_vp, ctypes.c_double, _vp, ctypes.POINTER(Report)]
    lib.gbem_job_free.argtypes = [_vp]
    lib.gbem_job_free.restype = None
    lib.gbem_server_stats.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_size_t),
                                      ctypes.POINTER(ctypes.c_size_t)]
    lib.gbem_mesh_boxes.argtypes = [_vp, _vp, _vp, ctypes.c_int32, ctypes.POINTER(MeshRule),
                                    ctypes.POINTER(MeshBuf)]
    lib.gbem_mesh_partition.argtypes = [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Partition),
                                        ctypes.POINTER(MeshBuf)]
    lib.gbem_extract_partitioned.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                             ctypes.c_double, ctypes.POINTER(Partition), ctypes.POINTER(Opts),
                                             _vp, _vp, ctypes.POINTER(Report)]
    lib.gbem_mesh_buf_free.argtypes = [ctypes.POINTER(MeshBuf)]
    lib.gbem_mesh_buf_free.restype = None
    lib.gbem_near_list.argtypes = [_vp, ctypes.POINTER(Mesh), ctypes.c_double, _vp, _vp, ctypes.c_int64,
                                   ctypes.POINTER(ctypes.c_int64)]
    lib.gbem_assemble.argtypes = [_vp, ctypes.POINTER(Mesh), ctypes.POINTER(Opts), _vp]
    lib.gbem_assemble_sample.argtypes = [_vp, ctypes.POINTER(Mesh), ctypes.POINTER(Opts), ctypes.c_int64,
                                         _vp, _vp, _vp]
    lib.gbem_assemble_scaled_sample.argtypes = [_vp, ctypes.POINTER(Mesh), ctypes.POINTER(Opts), ctypes.c_int64,
                                                _vp, _vp, _vp]
    lib.gbem_cholesky_device.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int64,
                                         ctypes.POINTER(ctypes.c_int32), _vp]
    lib.gbem_cholesky_solve_device.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int64,
                                               ctypes.c_int32, _vp, ctypes.c_int64, _vp]
    lib.gbem_extract_dielectric.argtypes = [_vp, ctypes.POINTER(DMesh), ctypes.POINTER(Opts), _vp,
                                            ctypes.POINTER(Report)]
    lib.gbem_assemble_double_layer.argtypes = [_vp, ctypes.c_int32, _vp, _vp, ctypes.c_double, _vp]
    lib.gbem_mesh_dielectric_partition.argtypes = [ctypes.POINTER(DLayout), ctypes.c_int32,
                                                   ctypes.POINTER(Partition), ctypes.POINTER(DMeshBuf)]
    lib.gbem_dmesh_buf_free.argtypes = [ctypes.POINTER(DMeshBuf)]
    lib.gbem_extract_dielectric_partitioned.argtypes = [_vp, ctypes.POINTER(DLayout), ctypes.POINTER(Partition),
                                                        ctypes.POINTER(Opts), _vp, _vp, ctypes.POINTER(Report)]
    for name in ("gbem_create", "gbem_destroy", "gbem_extract", "gbem_extract_device", "gbem_submit",
                 "gbem_poll", "gbem_wait", "gbem_server_stats", "gbem_mesh_boxes", "gbem_near_list",
                 "gbem_assemble", "gbem_assemble_sample", "gbem_assemble_scaled_sample", "gbem_cholesky_device",
                 "gbem_cholesky_solve_device", "gbem_mesh_partition", "gbem_extract_partitioned",
                 "gbem_extract_device_noalloc", "gbem_load_tuning", "gbem_set_tuning_override",
                 "gbem_extract_dielectric", "gbem_assemble_double_layer", "gbem_mesh_dielectric_partition",
                 "gbem_extract_dielectric_partitioned"):
        getattr(lib, name).restype = ctypes.c_int
    _LIB = lib
    return lib


def _check(st: int):
    if st != OK:
        lib = load()
        raise GbemError(st, lib.gbem_last_error().decode())


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def profile_mask(profile) -> int:
    """opts.profile: True = every kernel class, False/None = none, or an
    iterable of class names (KERNEL_CLASSES)."""
    if profile is True:
        return (1 << NCLS) - 1
    if not profile:
        return 0
    return sum(1 << KERNEL_CLASSES.index(c) for c in profile)


def make_opts(far_order=3, near_eta=2.0, far_dtype="f64", factor_dtype="f64", refine_tol=1e-6,
              max_refine=30, profile=False, graph=False) -> Opts:
    return Opts(far_order, near_eta, DTYPES[far_dtype] if isinstance(far_dtype, str) else far_dtype,
                DTYPES[factor_dtype] if isinstance(factor_dtype, str) else factor_dtype, refine_tol, max_refine,
                profile_mask(profile), int(bool(graph)))


def mesh_boxes(box_lo, box_hi, box_cond, rule):
    """Library mesher: returns (lo, hi, cond) numpy arrays."""
    lib = load()
    blo = np.ascontiguousarray(box_lo, dtype=np.float64).reshape(-1, 3)
    bhi = np.ascontiguousarray(box_hi, dtype=np.float64).reshape(-1, 3)
    bc = np.ascontiguousarray(box_cond, dtype=np.int32).reshape(-1)
    if rule[0] == "uniform":
        r = MeshRule(0, rule[1], 0.0, 0.0, 0.0)
    else:
        r = MeshRule(1, 0.0, rule[1], rule[2], rule[3])
    buf = MeshBuf()
    _check(lib.gbem_mesh_boxes(_ptr(blo), _ptr(bhi), _ptr(bc), blo.shape[0], ctypes.byref(r), ctypes.byref(buf)))
    try:
        n = buf.n_panels
        lo = np.ctypeslib.as_array(buf.lo, shape=(n * 3,)).reshape(n, 3).copy()
        hi = np.ctypeslib.as_array(buf.hi, shape=(n * 3,)).reshape(n, 3).copy()
        cond = np.ctypeslib.as_array(buf.conductor, shape=(n,)).copy()
    finally:
        lib.gbem_mesh_buf_free(ctypes.byref(buf))
    return lo, hi, cond


def mesh_layout(layout):
    blo, bhi, bcond = layout.arrays()
    return mesh_boxes(blo, bhi, bcond, layout.rule)


def _take_buf(lib, buf):
    try:
        n = buf.n_panels
        lo = np.ctypeslib.as_array(buf.lo, shape=(n * 3,)).reshape(n, 3).copy()
        hi = np.ctypeslib.as_array(buf.hi, shape=(n * 3,)).reshape(n, 3).copy()
        cond = np.ctypeslib.as_array(buf.conductor, shape=(n,)).copy()
    finally:
        lib.gbem_mesh_buf_free(ctypes.byref(buf))
    return lo, hi, cond


ALL_NETS = -2   # gbem.h GBEM_ALL_NETS: one mesh refined around every conductor


def mesh_partition(box_lo, box_hi, box_cond, main_net, p1, p2, p3, p5):
    """Library mesher, partition rule of section 3.3 for one main net (or
    ALL_NETS): (lo, hi, cond)."""
    lib = load()
    blo = np.ascontiguousarray(box_lo, dtype=np.float64).reshape(-1, 3)
    bhi = np.ascontiguousarray(box_hi, dtype=np.float64).reshape(-1, 3)
    bc = np.ascontiguousarray(box_cond, dtype=np.int32).reshape(-1)
    r = Partition(p1, p2, p3, p5)
    buf = MeshBuf()
    _check(lib.gbem_mesh_partition(_ptr(blo), _ptr(bhi), _ptr(bc), blo.shape[0], main_net, ctypes.byref(r),
                                   ctypes.byref(buf)))
    return _take_buf(lib, buf)


def dlayout(layout):
    """DLayout of a gbem_inputs.DielectricLayout and the arrays it points into."""
    blo = np.ascontiguousarray(layout.box_lo, dtype=np.float64).reshape(-1, 3)
    bhi = np.ascontiguousarray(layout.box_hi, dtype=np.float64).reshape(-1, 3)
    bn = np.ascontiguousarray(layout.box_net, dtype=np.int32).reshape(-1)
    z = np.ascontiguousarray(layout.z_layer, dtype=np.float64)
    eps = np.ascontiguousarray(layout.eps_r, dtype=np.float64)
    d = DLayout(blo.shape[0], blo.ctypes.data, bhi.ctypes.data, bn.ctypes.data, layout.n_conductors,
                (ctypes.c_double * 3)(*layout.domain_lo), (ctypes.c_double * 3)(*layout.domain_hi),
                eps.shape[0], z.ctypes.data, eps.ctypes.data, layout.bottom_kind, layout.top_kind,
                layout.side_kind, layout.length_unit_m)
    return d, (blo, bhi, bn, z, eps)


def mesh_dielectric_partition(layout, main_net, p1, p2, p3, p5):
    """Library mesher of a layered layout for one main net (sections 3.3 and
    4.1): (lo, hi, kind, conductor, region_plus, region_minus)."""
    lib = load()
    d, keep = dlayout(layout)
    buf = DMeshBuf()
    _check(lib.gbem_mesh_dielectric_partition(ctypes.byref(d), main_net, ctypes.byref(Partition(p1, p2, p3, p5)),
                                              ctypes.byref(buf)))
    try:
        n = buf.n_panels
        lo = np.ctypeslib.as_array(buf.lo, shape=(n * 3,)).reshape(n, 3).copy()
        hi = np.ctypeslib.as_array(buf.hi, shape=(n * 3,)).reshape(n, 3).copy()
        ints = [np.ctypeslib.as_array(getattr(buf, f), shape=(n,)).copy()
                for f in ("kind", "conductor", "region_plus", "region_minus")]
    finally:
        lib.gbem_dmesh_buf_free(ctypes.byref(buf))
    return (lo, hi, *ints)


class Context:
    """A device context: synchronous extraction, serving loop and stage calls."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.lib = load()
        h = _vp()
        _check(self.lib.gbem_create(device, hbm_budget_bytes, ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            self.lib.gbem_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _mesh(lo, hi, cond, n_cond, eps_r, lu):
        lo = np.ascontiguousarray(lo, dtype=np.float64)
        hi = np.ascontiguousarray(hi, dtype=np.float64)
        cond = np.ascontiguousarray(cond, dtype=np.int32)
        m = Mesh(cond.shape[0], n_cond, lo.ctypes.data, hi.ctypes.data, cond.ctypes.data, eps_r, lu)
        return m, (lo, hi, cond)

    def extract(self, lo, hi, cond, n_conductors, eps_r, length_unit_m, opts: Opts | None = None):
        m, keep = self._mesh(lo, hi, cond, n_conductors, eps_r, length_unit_m)
        C = np.zeros((n_conductors, n_conductors))
        rep = Report()
        o = opts or make_opts()
        _check(self.lib.gbem_extract(self.h, ctypes.byref(m), ctypes.byref(o), _ptr(C), ctypes.byref(rep)))
        return C, rep.as_dict()

    def extract_partitioned(self, box_lo, box_hi, box_cond, n_conductors, eps_r, length_unit_m,
                            p1, p2, p3, p5, opts: Opts | None = None):
        """Per-main-net meshes (section 3.3 rule), column k of C from mesh k.
        Returns (C, panels per mesh, report)."""
        blo = np.ascontiguousarray(box_lo, dtype=np.float64).reshape(-1, 3)
        bhi = np.ascontiguousarray(box_hi, dtype=np.float64).reshape(-1, 3)
        bc = np.ascontiguousarray(box_cond, dtype=np.int32).reshape(-1)
        C = np.zeros((n_conductors, n_conductors))
        panels = np.zeros(n_conductors, dtype=np.int32)
        rep = Report()
        o = opts or make_opts()
        r = Partition(p1, p2, p3, p5)
        _check(self.lib.gbem_extract_partitioned(self.h, _ptr(blo), _ptr(bhi), _ptr(bc), blo.shape[0], n_conductors,
                                                 eps_r, length_unit_m, ctypes.byref(r), ctypes.byref(o), _ptr(C),
                                                 _ptr(panels), ctypes.byref(rep)))
        return C, panels, rep.as_dict()

    def extract_layout(self, layout, opts: Opts | None = None):
        lo, hi, cond = mesh_layout(layout)
        return self.extract(lo, hi, cond, layout.n_conductors, layout.eps_r, layout.length_unit_m, opts)

    def extract_device(self, d_lo, d_hi, d_cond, n_conductors, eps_r, length_unit_m, d_C,
                       opts: Opts | None = None, stream=None):
        """Device-resident mesh and output (torch tensors on the context's device)."""
        m = Mesh(d_cond.shape[0], n_conductors, d_lo.data_ptr(), d_hi.data_ptr(), d_cond.data_ptr(), eps_r,
                 length_unit_m)
        rep = Report()
        o = opts or make_opts()
        st = stream.cuda_stream if stream is not None else None
        _check(self.lib.gbem_extract_device(self.h, ctypes.byref(m), ctypes.byref(o), ctypes.c_void_p(d_C.data_ptr()),
                                            ctypes.c_void_p(st), ctypes.byref(rep)))
        return rep.as_dict()

    def extract_device_noalloc(self, d_lo, d_hi, d_cond, n_conductors, eps_r, length_unit_m, d_C,
                               opts: Opts | None = None, stream=None):
        """As extract_device, through gbem_extract_device_noalloc (no device
        allocation during the call; intermediates in the library's static
        per-GPU scratch)."""
        m = Mesh(d_cond.shape[0], n_conductors, d_lo.data_ptr(), d_hi.data_ptr(), d_cond.data_ptr(), eps_r,
                 length_unit_m)
        rep = Report()
        o = opts or make_opts()
        st = stream.cuda_stream if stream is not None else None
        _check(self.lib.gbem_extract_device_noalloc(self.h, ctypes.byref(m), ctypes.byref(o),
                                                    ctypes.c_void_p(d_C.data_ptr()), ctypes.c_void_p(st),
                                                    ctypes.byref(rep)))
        return rep.as_dict()

    def extract_dielectric(self, lo, hi, kind, conductor, region_plus, region_minus, eps_r, n_conductors,
                           length_unit_m, opts: Opts | None = None):
        """Capacitance matrix of a multi-dielectric mesh (gbem_extract_dielectric).
        Returns (C, report)."""
        lo = np.ascontiguousarray(lo, dtype=np.float64).reshape(-1, 3)
        hi = np.ascontiguousarray(hi, dtype=np.float64).reshape(-1, 3)
        ints = [np.ascontiguousarray(a, dtype=np.int32).reshape(-1) for a in (kind, conductor, region_plus,
                                                                               region_minus)]
        eps = np.ascontiguousarray(eps_r, dtype=np.float64).reshape(-1)
        m = DMesh(lo.shape[0], n_conductors, eps.shape[0], lo.ctypes.data, hi.ctypes.data, ints[0].ctypes.data,
                  ints[1].ctypes.data, ints[2].ctypes.data, ints[3].ctypes.data, eps.ctypes.data, length_unit_m)
        C = np.zeros((n_conductors, n_conductors))
        rep = Report()
        o = opts or make_opts()
        _check(self.lib.gbem_extract_dielectric(self.h, ctypes.byref(m), ctypes.byref(o), _ptr(C), ctypes.byref(rep)))
        return C, rep.as_dict()

    def extract_dielectric_partitioned(self, layout, p1, p2, p3, p5, opts: Opts | None = None):
        """One mesh per main net of a layered layout (gbem_extract_dielectric_partitioned).
        Returns (C, panels per mesh, report)."""
        d, keep = dlayout(layout)
        m = layout.n_conductors
        C = np.zeros((m, m))
        panels = np.zeros(m, dtype=np.int32)
        rep = Report()
        o = opts or make_opts()
        _check(self.lib.gbem_extract_dielectric_partitioned(self.h, ctypes.byref(d),
                                                            ctypes.byref(Partition(p1, p2, p3, p5)),
                                                            ctypes.byref(o), _ptr(C), _ptr(panels), ctypes.byref(rep)))
        return C, panels, rep.as_dict()

    def assemble_double_layer(self, lo, hi, near_eta=2.0):
        """Q (n x n) of section 4.2 (gbem_assemble_double_layer)."""
        lo = np.ascontiguousarray(lo, dtype=np.float64).reshape(-1, 3)
        hi = np.ascontiguousarray(hi, dtype=np.float64).reshape(-1, 3)
        n = lo.shape[0]
        Q = np.zeros((n, n))
        _check(self.lib.gbem_assemble_double_layer(self.h, n, _ptr(lo), _ptr(hi), near_eta, _ptr(Q)))
        return Q

    def near_list(self, lo, hi, near_eta=2.0):
        n = np.asarray(lo).shape[0]
        m, keep = self._mesh(lo, hi, np.zeros(n, dtype=np.int32), 1, 1.0, 1.0)
        rp = np.zeros(n + 1, dtype=np.int64)
        nnz = ctypes.c_int64(0)
        _check(self.lib.gbem_near_list(self.h, ctypes.byref(m), near_eta, _ptr(rp), None, 0, ctypes.byref(nnz)))
        col = np.zeros(max(nnz.value, 1), dtype=np.int32)
        _check(self.lib.gbem_near_list(self.h, ctypes.byref(m), near_eta, _ptr(rp), _ptr(col), col.shape[0],
                                       ctypes.byref(nnz)))
        return rp, col[:nnz.value]

    def assemble(self, lo, hi, opts: Opts | None = None):
        n = np.asarray(lo).shape[0]
        m, keep = self._mesh(lo, hi, np.zeros(n, dtype=np.int32), 1, 1.0, 1.0)
        A = np.zeros((n, n))
        o = opts or make_opts()
        _check(self.lib.gbem_assemble(self.h, ctypes.byref(m), ctypes.byref(o), _ptr(A)))
        return A

    def assemble_sample(self, lo, hi, ii, jj, opts: Opts | None = None, cond=None, n_conductors=1):
        n = np.asarray(lo).shape[0]
        if cond is None:
            cond = np.zeros(n, dtype=np.int32)
        m, keep = self._mesh(lo, hi, cond, n_conductors, 1.0, 1.0)
        ii = np.ascontiguousarray(ii, dtype=np.int32)
        jj = np.ascontiguousarray(jj, dtype=np.int32)
        out = np.zeros(ii.shape[0])
        o = opts or make_opts()
        _check(self.lib.gbem_assemble_sample(self.h, ctypes.byref(m), ctypes.byref(o), ii.shape[0], _ptr(ii),
                                             _ptr(jj), _ptr(out)))
        return out

    def assemble_scaled_sample(self, lo, hi, ii, jj, opts: Opts):
        """Sampled entries F[ii, jj] (ii >= jj) of the FP32 factor input S A S."""
        n = np.asarray(lo).shape[0]
        m, keep = self._mesh(lo, hi, np.zeros(n, dtype=np.int32), 1, 1.0, 1.0)
        ii = np.ascontiguousarray(ii, dtype=np.int32)
        jj = np.ascontiguousarray(jj, dtype=np.int32)
        out = np.zeros(ii.shape[0], dtype=np.float32)
        _check(self.lib.gbem_assemble_scaled_sample(self.h, ctypes.byref(m), ctypes.byref(opts), ii.shape[0],
                                                    _ptr(ii), _ptr(jj), _ptr(out)))
        return out

    def cholesky_device(self, A, dtype="f64", stream=None):
        """In-place Cholesky of a square torch tensor (column-major view: pass A.T of a row-major tensor)."""
        n = A.shape[0]
        info = ctypes.c_int32(0)
        st = stream.cuda_stream if stream is not None else None
        lda = A.stride(1) if A.stride(0) == 1 else A.stride(0)
        _check(self.lib.gbem_cholesky_device(self.h, n, DTYPES[dtype], ctypes.c_void_p(A.data_ptr()), lda,
                                             ctypes.byref(info), ctypes.c_void_p(st)))
        return info.value

    def cholesky_solve_device(self, L, B, dtype="f64", stream=None):
        n = L.shape[0]
        st = stream.cuda_stream if stream is not None else None
        lda = L.stride(1) if L.stride(0) == 1 else L.stride(0)
        ldb = B.stride(1)
        _check(self.lib.gbem_cholesky_solve_device(self.h, n, DTYPES[dtype], ctypes.c_void_p(L.data_ptr()), lda,
                                                   B.shape[1], ctypes.c_void_p(B.data_ptr()), ldb,
                                                   ctypes.c_void_p(st)))

    # ---- serving
    def submit(self, lo, hi, cond, n_conductors, eps_r, length_unit_m, opts: Opts | None = None):
        m, keep = self._mesh(lo, hi, cond, n_conductors, eps_r, length_unit_m)
        o = opts or make_opts()
        j = _vp()
        _check(self.lib.gbem_submit(self.h, ctypes.byref(m), ctypes.byref(o), ctypes.byref(j)))
        return Job(self.lib, j, n_conductors)

    def server_stats(self):
        """jobs_done; peak_bytes: largest admitted reservation (footprints);
        peak_held_bytes: largest sum of the workers' real workspace sizes."""
        d = ctypes.c_int64(0)
        p = ctypes.c_size_t(0)
        h = ctypes.c_size_t(0)
        _check(self.lib.gbem_server_stats(self.h, ctypes.byref(d), ctypes.byref(p), ctypes.byref(h)))
        return {"jobs_done": d.value, "peak_bytes": p.value, "peak_held_bytes": h.value}


class Job:
    def __init__(self, lib, h, m):
        self.lib, self.h, self.m = lib, h, m

    def poll(self) -> int:
        return self.lib.gbem_poll(self.h)

    def wait(self, timeout_s: float = -1.0):
        C = np.zeros((self.m, self.m))
        rep = Report()
        _check(self.lib.gbem_wait(self.h, timeout_s, _ptr(C), ctypes.byref(rep)))
        return C, rep.as_dict()

    def free(self):
        if self.h:
            self.lib.gbem_job_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
