"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point include/gbem.h declares, and its mesher is bit-exact with
the oracle's."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

import gbem_inputs as gi
import oracle
from paper_2203_11733_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gbem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gbem_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    names = declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(binding.EXPORTS) == names


def test_status_strings_and_version():
    lib = binding.load()
    assert b"gfx950" in lib.gbem_version()
    for s in range(8):
        assert lib.gbem_status_str(s)
    o = binding.Opts()
    lib.gbem_default_opts(ctypes.byref(o))
    assert (o.far_order, o.near_eta, o.far_dtype, o.factor_dtype) == (3, 2.0, 0, 0)


@pytest.mark.parametrize("layout", [gi.two_plates(), gi.crossing_bus(), gi.three_layer_bus(),
                                    gi.crossing_bars_in_box(), gi.random_small_layout(3)],
                         ids=["two_plates", "crossing_bus", "three_layer_bus", "bars_in_box", "random3"])
def test_mesher_bit_exact_vs_oracle(layout):
    a = binding.mesh_layout(layout)
    b = oracle.mesh_layout(layout)
    for x, y in zip(a, b):
        assert x.dtype == y.dtype and x.shape == y.shape
        assert x.tobytes() == y.tobytes()


def test_mesher_serving_layouts_bit_exact():
    for t, lay in gi.serving_stream(n_jobs=6):
        a = binding.mesh_layout(lay)
        b = oracle.mesh_layout(lay)
        assert all(x.tobytes() == y.tobytes() for x, y in zip(a, b))
        assert 450 <= a[0].shape[0] <= 22000


def test_mesher_rejects_bad_boxes():
    with pytest.raises(binding.GbemError) as e:
        binding.mesh_boxes([[0, 0, 0], [0.5, 0, 0]], [[1, 1, 1], [2, 1, 1]], [0, 1], ("uniform", 0.5))
    assert e.value.status == binding.EINVAL
    with pytest.raises(binding.GbemError):
        binding.mesh_boxes([[0, 0, 0]], [[1, 0, 1]], [0], ("uniform", 0.5))   # flat box
    with pytest.raises(binding.GbemError):
        binding.mesh_boxes([[0, 0, 0]], [[1, 1, 1]], [0], ("uniform", -1.0))
    # touching boxes are rejected, a box strictly inside another is accepted
    with pytest.raises(binding.GbemError):
        binding.mesh_boxes([[0, 0, 0], [1, 0, 0]], [[1, 1, 1], [2, 1, 1]], [0, 1], ("uniform", 0.5))
    lo, hi, c = binding.mesh_boxes([[0, 0, 0], [-5, -5, -5]], [[1, 1, 1], [5, 5, 5]], [0, -1], ("uniform", 0.5))
    assert lo.shape[0] == 24 + 6 * 400


def test_context_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(binding.GbemError) as e:
        binding.Context(0)
    assert e.value.status == binding.EDEVICE


def _host_mesh(lo, hi, cond, m=2, basis=0):
    return binding.Mesh(cond.shape[0], m, lo.ctypes.data, hi.ctypes.data, cond.ctypes.data, 3.9, 1e-6, basis)


@pytest.mark.parametrize("eta", [0.0, -1.0, 1e-9, float("nan"), float("inf")])
def test_near_threshold_that_misses_self_pairs_is_refused(eta):
    """The near test is strict (dist^2 < eta^2 diam^2): at eta = 0 no pair, not
    even a panel with itself, would be near, and the far rule would evaluate
    1/r at r = 0.  Such thresholds are refused before any device work (the
    arguments are checked before the context, so this runs without a GPU)."""
    lib = binding.load()
    lo, hi, cond = binding.mesh_layout(gi.two_plates(h=0.5))
    mesh = _host_mesh(lo, hi, cond)
    o = binding.make_opts(3, eta)
    C = np.zeros((2, 2))
    st = lib.gbem_extract(None, ctypes.byref(mesh), ctypes.byref(o), C.ctypes.data, None)
    assert st == binding.EINVAL
    assert b"near_eta" in lib.gbem_last_error()
    rp = np.zeros(lo.shape[0] + 1, dtype=np.int64)
    nnz = ctypes.c_int64(0)
    st = lib.gbem_near_list(None, ctypes.byref(mesh), eta, rp.ctypes.data, None, 0, ctypes.byref(nnz))
    assert st == binding.EINVAL


def test_argument_checks_before_context():
    lib = binding.load()
    lo, hi, cond = binding.mesh_layout(gi.two_plates(h=0.5))
    C = np.zeros((2, 2))
    o = binding.make_opts()
    # only the piecewise constant basis exists
    mesh = _host_mesh(lo, hi, cond, basis=1)
    assert lib.gbem_extract(None, ctypes.byref(mesh), ctypes.byref(o), C.ctypes.data, None) == binding.EINVAL
    assert b"basis" in lib.gbem_last_error()
    # a valid mesh and options reach the context check
    mesh = _host_mesh(lo, hi, cond)
    assert lib.gbem_extract(None, ctypes.byref(mesh), ctypes.byref(o), C.ctypes.data, None) == binding.EINVAL
    assert b"context" in lib.gbem_last_error()
    o = binding.make_opts(0)
    assert lib.gbem_extract(None, ctypes.byref(mesh), ctypes.byref(o), C.ctypes.data, None) == binding.EINVAL
    assert b"far_order" in lib.gbem_last_error()


def test_tuning_cache_loader(tmp_path):
    """The shape cache the autotuner writes is parsed strictly: a valid file
    becomes the source, malformed ones and unsupported shapes are refused
    (the previous cache stays), NULL returns to the built-in defaults, and
    the override accepts only supported shapes."""
    lib = binding.load()
    good = tmp_path / "tune.json"
    good.write_text(json.dumps({"entries": [
        {"factor": "16bit", "npad_min": 0, "npad_max": 32768, "outer_width": 256, "super_panels": 2,
         "ms": {"256x2": 1.0, "512x4": 2.0}},
        {"factor": "f64", "npad_min": 0, "npad_max": 1 << 30, "outer_width": 512, "super_panels": 1}]}))
    binding.load_tuning(str(good))
    assert binding.tuning_source() == str(good)
    for bad in ({"nothing": []}, {"entries": [{"factor": "f16", "npad_min": 0, "npad_max": 1, "outer_width": 256}]},
                {"entries": [{"factor": "16bit", "npad_min": 0, "npad_max": 10, "outer_width": 384,
                              "super_panels": 2}]},
                {"entries": [{"factor": "16bit", "npad_min": 0, "npad_max": 10, "outer_width": 512,
                              "super_panels": 3}]},
                {"entries": [{"factor": "f64", "npad_min": 5, "npad_max": 5, "outer_width": 512}]}):
        p = tmp_path / "bad.json"
        p.write_text(json.dumps(bad))
        with pytest.raises(binding.GbemError) as e:
            binding.load_tuning(str(p))
        assert e.value.status == binding.EINVAL
        assert binding.tuning_source() == str(good)
    with pytest.raises(binding.GbemError):
        binding.load_tuning(str(tmp_path / "missing.json"))
    binding.load_tuning(None)
    assert binding.tuning_source() == "built-in defaults"
    with pytest.raises(binding.GbemError):
        binding.set_tuning_override(384, 0)
    with pytest.raises(binding.GbemError):
        binding.set_tuning_override(512, 3)
    binding.set_tuning_override(512, 4)
    binding.set_tuning_override(0, 0)


def test_committed_tuning_cache_parses():
    """The committed cache (written by the autotuner on the GPU) loads and
    covers every padded order for both factor classes."""
    path = os.path.join(ROOT, "paper_2203_11733_amd", "tune_gfx950.json")
    if not os.path.exists(path):
        pytest.skip("no tuning cache committed yet")
    cache = json.load(open(path))
    for cls in ("16bit", "f64"):
        ranges = sorted((e["npad_min"], e["npad_max"]) for e in cache["entries"] if e["factor"] == cls)
        assert ranges[0][0] == 0
        assert all(a[1] == b[0] for a, b in zip(ranges, ranges[1:]))
    binding.load_tuning(path)
    assert binding.tuning_source() == path
    binding.load_tuning(None)


def test_dielectric_mesh_checks_before_context():
    """gbem_extract_dielectric refuses inconsistent meshes before touching the
    device: a conductor panel with regions on both sides, a net without
    panels; a consistent mesh reaches the context check."""
    lib = binding.load()
    m = gi.two_slab_capacitor(n_xy=2, n_z=1)

    def call(kind=None, cond=None, rp=None, rm=None, n_cond=2):
        arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in
                (m.kind if kind is None else kind, m.conductor if cond is None else cond,
                 m.region_plus if rp is None else rp, m.region_minus if rm is None else rm)]
        lo, hi = np.ascontiguousarray(m.lo), np.ascontiguousarray(m.hi)
        eps = np.ascontiguousarray(m.eps_r, dtype=np.float64)
        d = binding.DMesh(m.n_panels, n_cond, len(m.eps_r), lo.ctypes.data, hi.ctypes.data, arrs[0].ctypes.data,
                          arrs[1].ctypes.data, arrs[2].ctypes.data, arrs[3].ctypes.data, eps.ctypes.data, 1e-6)
        C = np.zeros((n_cond, n_cond))
        st = lib.gbem_extract_dielectric(None, ctypes.byref(d), None, C.ctypes.data, None)
        return st, lib.gbem_last_error()

    rm = m.region_minus.copy()
    rm[0] = 1 - m.region_plus[0] if m.region_plus[0] >= 0 else 0
    st, msg = call(rm=rm)
    assert st == binding.EINVAL and b"panel 0" in msg
    st, msg = call(n_cond=3)
    assert st == binding.EINVAL and b"conductor 2 has no panels" in msg
    kind = m.kind.copy()
    kind[0] = 7
    st, msg = call(kind=kind)
    assert st == binding.EINVAL and b"panel 0" in msg
    st, msg = call()
    assert st == binding.EINVAL and b"context" in msg


def test_graph_option_checked_before_context():
    lib = binding.load()
    lo, hi, cond = binding.mesh_layout(gi.two_plates(h=0.5))
    mesh = _host_mesh(lo, hi, cond)
    C = np.zeros((2, 2))
    o = binding.make_opts(graph=True)
    assert o.graph == 1
    assert lib.gbem_extract(None, ctypes.byref(mesh), ctypes.byref(o), C.ctypes.data, None) == binding.EINVAL
    assert b"context" in lib.gbem_last_error()
    o.graph = 2
    assert lib.gbem_extract(None, ctypes.byref(mesh), ctypes.byref(o), C.ctypes.data, None) == binding.EINVAL
    assert b"graph must be 0 or 1" in lib.gbem_last_error()
    d = binding.Opts()
    lib.gbem_default_opts(ctypes.byref(d))
    assert d.graph == 0
