"""Autotuner of the Cholesky tile shapes (writes the library's shape cache).

For each padded-order bucket and factor class, time whole extractions of a
representative synthetic layout under every candidate shape (forced with
gbem_set_tuning_override) and keep the fastest.  The shapes are schedule
parameters only (outer panel width, outer panels per 16-bit trailing
update); they do not change what an entry of the factor is, beyond the
rounding order of the trailing sums, and every candidate's capacitances are
checked against the first candidate's before its time counts.

    python -m paper_2203_11733_amd.autotune [--out PATH] [--quick]

writes ``paper_2203_11733_amd/tune_gfx950.json`` (read by the library when
the first context is created).  Needs the GPU; about two minutes.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import gbem_inputs as gi  # noqa: E402
from paper_2203_11733_amd import binding  # noqa: E402

DEFAULT_OUT = os.path.join(HERE, "tune_gfx950.json")

# padded-order buckets [lo, hi) and a layout whose padded order falls in each
BUCKETS = [
    (0, 4096, "random Manhattan layout, ~3,000 panels", lambda: _random_layout(3000, 11)),
    (4096, 8192, "random Manhattan layout, ~6,000 panels", lambda: _random_layout(6000, 12)),
    (8192, 16384, "random Manhattan layout, ~12,000 panels", lambda: _random_layout(12000, 13)),
    (16384, 32768, "crossing bus (21,420 panels)", lambda: gi.crossing_bus()),
    (32768, 49152, "three-layer bus, 11 wires per layer (41,184 panels)", lambda: gi.three_layer_bus(n_per_layer=11)),
    (49152, 1 << 30, "three-layer bus (59,904 panels)", lambda: gi.three_layer_bus()),
]
CANDIDATES = {
    "16bit": [(256, 1), (256, 2), (256, 4), (512, 1), (512, 2), (512, 4)],
    "f64": [(256, 0), (512, 0)],
}
MODES = {
    "16bit": dict(far_dtype="f32", factor_dtype="f16", refine_tol=1e-6, max_refine=30),
    "f64": dict(far_dtype="f64", factor_dtype="f64"),
}


def _random_layout(n_target: float, seed: int):
    rng = np.random.default_rng(seed)
    for _ in range(100):
        lay = gi.random_manhattan(rng, n_target=n_target)
        n = binding.mesh_layout(lay)[0].shape[0]
        if 0.8 * n_target <= n <= 1.2 * n_target:
            return lay
    return lay


def time_extractions(ctx, dev, lay, opts, reps):
    """Median device time (ms) of `reps` extractions and the last C."""
    import torch
    lo, hi, cond = binding.mesh_layout(lay)
    m = lay.n_conductors
    d_lo, d_hi, d_cond = (torch.tensor(x, device=dev) for x in (lo, hi, cond))
    d_C = torch.zeros((m, m), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    ctx.extract_device(d_lo, d_hi, d_cond, m, lay.eps_r, lay.length_unit_m, d_C, opts, stream)   # warm
    times, rep = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = ctx.extract_device(d_lo, d_hi, d_cond, m, lay.eps_r, lay.length_unit_m, d_C, opts, stream)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(times)), d_C.cpu().numpy(), rep, lo.shape[0]


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--quick", action="store_true", help="one repetition per candidate")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("the autotuner times candidates on the GPU")
    dev = torch.device("cuda:0")
    binding.load_tuning(None)          # sweep against the built-in defaults
    entries = []
    with binding.Context(0) as ctx:
        for lo_b, hi_b, desc, make in BUCKETS:
            lay = make()
            for cls, cands in CANDIDATES.items():
                reps = 1 if args.quick else (2 if cls == "f64" or lo_b >= 32768 else 3)
                results, C_ref = {}, None
                for ow, sp in cands:
                    binding.set_tuning_override(ow, sp)
                    ms, C, rep, n = time_extractions(ctx, dev, lay, binding.make_opts(3, 2.0, **MODES[cls]), reps)
                    err = 0.0 if C_ref is None else float(np.abs(C - C_ref).max() / np.abs(C_ref).max())
                    if C_ref is None:
                        C_ref = C
                    tol = 1e-12 if cls == "f64" else 1e-6
                    ok = err <= tol and (rep["outer_width"], rep["super_panels"]) == (ow, sp if cls == "16bit" else 1)
                    results[f"{ow}x{sp}" if sp else f"{ow}"] = {"ms": ms, "C_rel_dev": err, "ok": bool(ok)}
                    print(f"autotune: {desc} N={n} {cls} outer_width={ow} super_panels={sp}: {ms:.2f} ms"
                          f" (C dev {err:.1e}{'' if ok else ', REJECTED'})", flush=True)
                binding.set_tuning_override(0, 0)
                good = {k: v for k, v in results.items() if v["ok"]}
                best = min(good, key=lambda k: good[k]["ms"])
                ow, _, sp = best.partition("x")
                entries.append({"factor": cls, "npad_min": lo_b, "npad_max": hi_b, "outer_width": int(ow),
                                "super_panels": int(sp) if sp else 1, "workload": desc, "n_panels": n,
                                "ms": {k: round(v["ms"], 3) for k, v in results.items()}})
    props = torch.cuda.get_device_properties(0)
    out = {"device": f"{props.name} ({getattr(props, 'gcnArchName', 'gfx950')})",
           "written_by": "paper_2203_11733_amd/autotune.py",
           "date": time.strftime("%Y-%m-%d"), "host": platform.node() or "unknown host",
           "entries": entries}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(f"autotune: wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
