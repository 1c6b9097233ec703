"""The no-allocation extraction (gbem_extract_device_noalloc) against the
allocating one (gbem_extract_device): same kernels and launches, so the same
capacitances; two calls in a row, the second on a smaller mesh, so the second
call runs on scratch the first one left behind.  Also: the call leaves the
device's free memory unchanged, and oversize meshes and profiling requests
are refused with a clear error."""
import sys

import numpy as np
import pytest

import gbem_inputs as gi
from paper_2203_11733_amd import binding

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def jobs(gpu_lib):
    """The largest and the smallest mesh of a short seeded stream (2,944 and
    938 panels, 16 and 13 conductors)."""
    import torch
    dev = torch.device("cuda:0")
    out = []
    for _, lay in gi.serving_stream(n_jobs=8, seed=7, n_min=500, n_max=3000):
        lo, hi, cond = binding.mesh_layout(lay)
        out.append((lay, torch.tensor(lo, device=dev), torch.tensor(hi, device=dev), torch.tensor(cond, device=dev)))
    out.sort(key=lambda j: -j[3].shape[0])
    return out[0], out[-1]


MODES = {"f64": lambda: binding.make_opts(),
         "mixed": lambda: binding.make_opts(3, 2.0, "f32", "f16", 1e-8, 40)}


@pytest.mark.parametrize("mode", sorted(MODES))
def test_noalloc_matches_extract_device_twice(jobs, mode):
    import torch
    opts = MODES[mode]()
    stream = torch.cuda.current_stream()
    with binding.Context(0) as ctx:
        results = []
        for lay, d_lo, d_hi, d_cond in jobs:            # larger mesh, then the smaller one
            m = lay.n_conductors
            d_ref = torch.zeros((m, m), dtype=torch.float64, device="cuda:0")
            d_out = torch.full((m, m), float("nan"), dtype=torch.float64, device="cuda:0")
            say(f"noalloc {mode}: N={d_cond.shape[0]} M={m}: reference extract_device")
            ctx.extract_device(d_lo, d_hi, d_cond, m, lay.eps_r, lay.length_unit_m, d_ref, opts, stream)
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            say(f"noalloc {mode}: N={d_cond.shape[0]} M={m}: extract_device_noalloc")
            rep = ctx.extract_device_noalloc(d_lo, d_hi, d_cond, m, lay.eps_r, lay.length_unit_m, d_out, opts,
                                             stream)
            torch.cuda.synchronize()
            free1 = torch.cuda.mem_get_info()[0]
            C, Cref = d_out.cpu().numpy(), d_ref.cpu().numpy()
            err = rel_err(C, Cref)
            say(f"  rel err vs extract_device {err:.3e}; free memory {free0} -> {free1}; report {rep}")
            # same kernels, launches and reduction orders: equal to the FP64 path's bar and below
            assert np.all(np.isfinite(C))
            assert err <= 1e-12
            assert rep["n_panels"] == d_cond.shape[0]
            # an extraction of this size would need tens of MiB if it allocated
            assert free0 - free1 < (16 << 20)
            results.append(err)
        assert len(results) == 2


def test_noalloc_refuses_oversize_mesh(gpu_lib):
    import torch
    lay = gi.two_plates(h=0.03)
    lo, hi, cond = binding.mesh_layout(lay)
    assert lo.shape[0] > 5632                          # beyond the largest padded order of the scratch
    dev = torch.device("cuda:0")
    d_lo, d_hi, d_cond = torch.tensor(lo, device=dev), torch.tensor(hi, device=dev), torch.tensor(cond, device=dev)
    d_C = torch.zeros((2, 2), dtype=torch.float64, device=dev)
    with binding.Context(0) as ctx:
        with pytest.raises(binding.GbemError) as ei:
            ctx.extract_device_noalloc(d_lo, d_hi, d_cond, 2, lay.eps_r, lay.length_unit_m, d_C)
        say(f"oversize: {ei.value}")
        assert ei.value.status == binding.ENOMEM
        assert "MiB" in str(ei.value)
        with pytest.raises(binding.GbemError) as ei:
            ctx.extract_device_noalloc(d_lo[:300], d_hi[:300], d_cond[:300], 2, lay.eps_r, lay.length_unit_m, d_C,
                                       binding.make_opts(profile=True))
        assert ei.value.status == binding.EINVAL
