"""Benchmark: whole capacitance extractions of the three-layer bus on one GPU.

One step = one full extraction (panel table, near list, far and near
assembly, Cholesky, solves, refinement, charge sums) of a device-resident
mesh: 3 layers x 16 wires (0.1 x 0.1 x 10 um, pitch 0.2 um), 59,904
panels, 48 conductors, the largest single-GPU workload.  Default mode: FP32
far field + FP16 trailing updates + FP64 refinement to 1e-6; the plain FP64
path is timed over the same number of steps beside it, and both capacitance
matrices are compared with the oracle's stored result for this layout.
After the timed steps the seeded 256-job serving stream is replayed in the
same mode and in FP64 (p50/p99 latency at 50 jobs/s, saturation jobs/s), and
the six-net multi-dielectric stack is extracted a few times.

Prints one JSON line.  Options: --gpus N (only 1 is supported), --steps K,
--warmup W, --mode mixed|f64, --layout three_layer_bus|crossing_bus|two_plates|small_job,
--no-f64, --no-cpu-baseline, --no-serving, --no-dielectric, --graph; other
workloads alone: --serving, --partition, --exact, --dielectric, --sweep.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MODES = {
    # FP16 factor of the Jacobi-scaled matrix (entries of L bounded by 1, so
    # FP16's range suffices and its 11-bit mantissa beats BF16's 8): one FP64
    # refinement sweep where BF16 needs two
    "mixed": dict(far_dtype="f32", factor_dtype="f16", refine_tol=1e-6, max_refine=30),
    "mixed_bf16": dict(far_dtype="f32", factor_dtype="bf16", refine_tol=1e-6, max_refine=30),
    "mixed_f32": dict(far_dtype="f32", factor_dtype="f32", refine_tol=1e-6, max_refine=30),
    "f64": dict(far_dtype="f64", factor_dtype="f64"),
}
DTYPE_LABEL = {"mixed": "f32+f16+f64", "mixed_bf16": "f32+bf16+f64", "mixed_f32": "f32+f64", "f64": "f64"}

# MI355X peaks (dense): HBM3E 8 TB/s; MFMA bf16/f16 2.5 PFLOP/s, fp32 157.3, fp64 78.6;
# vector fp32 157.3 (packed), fp64 78.6 TFLOP/s.
HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"mfma_bf16": 2500.0, "mfma_f16": 2500.0, "mfma_f32": 157.3, "mfma_f64": 78.6,
               "alu_f32": 157.3, "alu_f64": 78.6}
# source file of each kernel class (the counters of a committed PMC summary
# only apply while that file is unchanged)
CLASS_SOURCE = {"far": "far.hip", "near_list": "near.hip", "near_eval": "near_eval.hip", "diag": "chol.hip",
                "trsm": "chol.hip", "syrk": "chol.hip", "panel": "chol.hip", "solve": "solve.hip",
                "residual": "solve.hip"}


def compute_peak(cls, mode):
    """(bound kind, peak TFLOP/s) of a kernel class in a mode."""
    fac = MODES[mode]["factor_dtype"]
    far = MODES[mode]["far_dtype"]
    if cls == "far":
        return "alu", PEAK_TFLOPS["alu_" + far]
    if cls == "syrk":
        return "mfma", PEAK_TFLOPS["mfma_" + fac]
    if cls == "trsm":
        return "mfma", PEAK_TFLOPS["mfma_" + ("f64" if fac == "f64" else "f32")]
    if cls in ("diag",):
        return "alu", PEAK_TFLOPS["alu_" + ("f64" if fac == "f64" else "f32")]
    return "alu", PEAK_TFLOPS["alu_f64"]


# classes whose launches wait on flags set inside the same launch (the panel
# factorisation): their duration is set by that dependency chain
CHAIN_CLASSES = ("trsm",)


def roofline_of(profile, mode, layout_name, cls=None):
    """Roofline object of kernel class cls (default: the class with the
    largest GPU time)."""
    if cls is None:
        cls = max(profile.items(), key=lambda kv: kv[1]["ms"])[0]
    d = profile[cls]
    kind, peak_tf = compute_peak(cls, mode)
    secs = d["ms"] / 1e3
    t_compute = d["flops"] / (peak_tf * 1e12) if d["flops"] else 0.0
    t_memory = d["bytes"] / (HBM_PEAK_GBS * 1e9)
    per_launch = max(1, d["launches"])
    if t_memory >= t_compute:
        ach = d["bytes"] / secs / 1e9
        roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}
    else:
        ach = d["flops"] / secs / 1e12
        roof = {"bound": kind, "achieved": ach, "peak": peak_tf, "unit": "TFLOP/s", "frac": ach / peak_tf}
    roof.update({"kernel_class": cls, "launches": d["launches"], "avg_launch_ms": d["ms"] / per_launch,
                 "algorithmic_flops_per_launch": d["flops"] / per_launch,
                 "algorithmic_bytes_per_launch": d["bytes"] / per_launch,
                 "traffic": measured_traffic(cls, mode, layout_name, per_launch)})
    if cls in CHAIN_CLASSES:
        roof["note"] = ("the panel kernel waits on in-kernel flags for the diagonal blocks it factors: its "
                        "duration is set by that dependency chain, not by MFMA or HBM throughput")
    return roof


def measured_traffic(cls, mode, layout_name, launches):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it was
    taken on the current source of that kernel; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    rec = table.get(f"{cls}/{mode}/{layout_name}")
    if not rec:
        return None
    src = os.path.join(ROOT, "paper_2203_11733_amd", "csrc", CLASS_SOURCE.get(cls, "api.cpp"))
    with open(src, "rb") as f:
        digest = hashlib.sha1(f.read()).hexdigest()
    if digest != rec.get("source_sha1"):
        return None
    return rec.get("bytes_per_launch")


def golden_C(layout_name, p, eta):
    """The oracle's capacitance matrix for this layout, stored by
    tests/golden/make_golden.py (None if there is none for these settings)."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"{layout_name}_C.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    if g.get("far_order") != p or g.get("near_eta") != eta:
        return None
    return np.array(g["C"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def small_job():
    """A serving-size job: the seeded random Manhattan layout of about 3,000
    panels the autotuner times for its smallest order bucket."""
    import numpy as np

    import gbem_inputs as gi
    rng = np.random.default_rng(11)
    for _ in range(100):
        lay = gi.random_manhattan(rng, n_target=3000)
        if 2400 <= lay_panels(lay) <= 3600:
            return lay
    return lay


def lay_panels(lay):
    from paper_2203_11733_amd import binding
    return binding.mesh_layout(lay)[0].shape[0]


def layout_of(name):
    import gbem_inputs as gi
    return {"crossing_bus": gi.crossing_bus, "three_layer_bus": gi.three_layer_bus,
            "two_plates": gi.two_plates, "crossing_bars_in_box": gi.crossing_bars_in_box,
            "small_job": small_job}[name]()


FULL_ORACLE_MAX_N = 25000   # whole oracle extractions up to this order take ~10-30 s on 16 cores


def cpu_baseline(lo, hi, cond, layout, p, eta):
    """Time the CPU oracle on the workload (or a bounded sample of it).

    Up to FULL_ORACLE_MAX_N panels the oracle runs the whole extraction: every
    matrix entry (near pairs by the section 3.4 reductions, far pairs by
    Gauss), the LAPACK Cholesky solve and the charge sums; its capacitance
    matrix is returned beside the timing.  Larger meshes: all entries of 1 %
    of the rows (chosen at random) plus a LAPACK Cholesky solve of an
    (N/2)-order matrix, the extraction time estimated as pairs / (pairs/s of
    the sample) + 8 x the half-order solve time."""
    import numpy as np

    import oracle
    n = lo.shape[0]
    total_pairs = n * (n + 1) / 2
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    if n <= FULL_ORACLE_MAX_N:
        t0 = time.perf_counter()
        C = oracle.extract_panels(lo, hi, cond, layout.n_conductors, layout.eps_r, layout.length_unit_m, p, eta)
        t = time.perf_counter() - t0
        return {"value": total_pairs / t, "unit": "panel-pair integrals/s", "cores": threads, "kind": "oracle",
                "sample": f"the whole oracle extraction of this workload ({total_pairs:.0f} entries, LAPACK "
                          f"Cholesky solve of order {n}, charge sums): {t:.1f} s",
                "extractions_per_s": 1.0 / t}, C
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(n, max(1, n // 100), replace=False))
    ii = np.concatenate([np.full(r + 1, r, np.int32) for r in rows])
    jj = np.concatenate([np.arange(r + 1, dtype=np.int32) for r in rows])
    t0 = time.perf_counter()
    oracle.entries(lo, hi, ii, jj, p, eta)
    t_asm = time.perf_counter() - t0
    pairs_per_s = ii.shape[0] / t_asm
    h = n // 2
    sub_lo, sub_hi = lo[:h], hi[:h]
    # a well-conditioned SPD matrix of the same order as half the problem
    A = oracle.assemble(sub_lo[: min(h, 2000)], sub_hi[: min(h, 2000)], p, eta)
    M = np.eye(h) * A[0, 0]
    M[: A.shape[0], : A.shape[0]] = A
    B = np.ones((h, layout.n_conductors))
    t0 = time.perf_counter()
    oracle.solve(M, B)
    t_chol_half = time.perf_counter() - t0
    t_est = total_pairs / pairs_per_s + 8.0 * t_chol_half
    return {"value": total_pairs / t_est, "unit": "panel-pair integrals/s", "cores": threads,
            "kind": "oracle",
            "sample": f"oracle assembly of {len(rows)} random rows ({ii.shape[0]} entries, {t_asm:.1f} s) + "
                      f"LAPACK Cholesky solve of order {h} ({t_chol_half:.1f} s) scaled by 8 to order {n}; "
                      f"estimated {t_est:.1f} s per extraction",
            "extractions_per_s": 1.0 / t_est}, None


def serving(args, binding, np):
    """Replay the seeded job stream through gbem_submit/gbem_wait.

    Arrivals follow the stream's Poisson times (50 jobs/s); latency is
    submission -> completion.  A second pass submits every job at t = 0 for
    the saturation throughput."""
    import threading

    import gbem_inputs as gi
    stream = gi.serving_stream(n_jobs=args.jobs)
    meshes = [(t, lay, *binding.mesh_layout(lay)) for t, lay in stream]
    opts = binding.make_opts(args.p, args.eta, graph=args.graph, **MODES[args.mode])
    n_list = [m[2].shape[0] for m in meshes]
    log(f"serving: {len(meshes)} jobs, N from {min(n_list)} to {max(n_list)}, mode {args.mode}")
    out = {"metric": "served extractions/s + p50/p99 latency", "unit": "extractions/s", "n_gpus": 1,
           "mode": args.mode, "graph": bool(args.graph), "dtype": DTYPE_LABEL[args.mode], "data": "synthetic",
           "config": {"workload": f"serving stream: {len(meshes)} random Manhattan layouts, "
                                  f"N {min(n_list)}-{max(n_list)}, Poisson 50 jobs/s"}}
    with binding.Context(0) as ctx:
        # warm the workers
        w = [ctx.submit(m[2], m[3], m[4], m[1].n_conductors, m[1].eps_r, m[1].length_unit_m, opts) for m in meshes[:4]]
        for j in w:
            j.wait(300.0)
            j.free()
        for phase in ("poisson", "saturation"):
            submitted = []                     # (submit time, job)
            finished = {}                      # index -> completion time
            lock = threading.Lock()
            stop = threading.Event()

            def watcher():
                # observe completions as they happen (poll, not wait in order)
                while not stop.is_set() or len(finished) < len(meshes):
                    with lock:
                        pending = [(k, j) for k, (_, j) in enumerate(submitted) if k not in finished]
                    now = time.perf_counter()
                    for k, j in pending:
                        if j.poll() != binding.EBUSY:
                            finished[k] = now
                    if stop.is_set() and len(finished) == len(meshes):
                        break
                    time.sleep(0.0005)

            th = threading.Thread(target=watcher)
            th.start()
            t0 = time.perf_counter()
            for k, (t_arr, lay, lo, hi, cond) in enumerate(meshes):
                if phase == "poisson":
                    delay = t_arr - (time.perf_counter() - t0)
                    if delay > 0:
                        time.sleep(delay)
                j = ctx.submit(lo, hi, cond, lay.n_conductors, lay.eps_r, lay.length_unit_m, opts)
                with lock:
                    submitted.append((time.perf_counter(), j))
            stop.set()
            th.join(timeout=900)
            span = max(finished.values()) - t0
            lat_ms = np.array([(finished[k] - submitted[k][0]) * 1e3 for k in range(len(meshes))])
            for _, j in submitted:
                j.wait(600.0)
                j.free()
            out[phase] = {"jobs_per_s": len(meshes) / span, "p50_ms": float(np.percentile(lat_ms, 50)),
                          "p99_ms": float(np.percentile(lat_ms, 99)), "span_s": span}
            log(f"serving {phase}: {out[phase]}")
        out["server_stats"] = ctx.server_stats()
    out["value"] = out["saturation"]["jobs_per_s"]
    return out


def sweep(args, binding, np):
    """Precision sweep (p x eta x factor dtype) on one layout: time of one
    extraction and capacitance error against the FP64 path with p = 8, eta = 4
    (the FP64 path is parity-tested against the CPU oracle; the oracle itself
    is far too slow at this size).  One JSON object per configuration."""
    import torch
    lay = layout_of(args.layout)
    lo, hi, cond = binding.mesh_layout(lay)
    n, m = lo.shape[0], lay.n_conductors
    dev = torch.device("cuda:0")
    d_lo, d_hi = torch.tensor(lo, device=dev), torch.tensor(hi, device=dev)
    d_cond = torch.tensor(cond, device=dev)
    d_C = torch.zeros((m, m), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    rows = []
    with binding.Context(0) as ctx:
        def run(o):
            rep = ctx.extract_device(d_lo, d_hi, d_cond, m, lay.eps_r, lay.length_unit_m, d_C, o, stream)
            torch.cuda.synchronize()
            return d_C.cpu().numpy().copy(), rep
        log(f"sweep: {lay.name} N={n} M={m}: reference FP64 p=8 eta=4")
        Cref, rref = run(binding.make_opts(8, 4.0))
        rows.append({"p": 8, "eta": 4.0, "factor": "f64", "far": "f64", "ms": rref["t_total_ms"],
                     "C_rel_err_vs_ref": 0.0, "n_near": rref["n_near"], "reference": True})
        for p in (2, 3, 4):
            for eta in (1.0, 2.0, 4.0):
                for fac in ("f64", "f32", "f16", "bf16"):
                    far = "f64" if fac == "f64" else "f32"
                    o = binding.make_opts(p, eta, far, fac, 1e-6, 30)
                    run(o)                                   # warm (allocations, code objects)
                    t0 = time.perf_counter()
                    C, rep = run(o)
                    wall = (time.perf_counter() - t0) * 1e3
                    err = float(np.abs(C - Cref).max() / np.abs(Cref).max())
                    row = {"p": p, "eta": eta, "factor": fac, "far": far, "ms": wall,
                           "t_assemble_ms": rep["t_assemble_ms"], "t_factor_ms": rep["t_factor_ms"],
                           "t_solve_ms": rep["t_solve_ms"], "refine_iters": rep["refine_iters"],
                           "factor_used": rep["factor_used"], "n_near": rep["n_near"], "C_rel_err_vs_ref": err}
                    rows.append(row)
                    log(f"sweep: {row}")
    return {"metric": "precision sweep", "config": {"workload": f"{lay.name}: N={n}, M={m}"},
            "reference": "FP64 path, p=8, eta=4", "rows": rows}


PARTITION_SETS = {
    # section 3.3 rule (p1, p2, p3, p5); lengths in the layout's unit (um)
    # the last three land near Table 2's sizes (about 74, 183 and 594 pieces per mesh)
    "crossing_bars_in_box": [(1.0, 4.0, 1.0, 1.0), (0.5, 4.0, 0.25, 2.0), (0.1, 4.0, 1.0, 1.0),
                             (0.5, 4.0, 2.0, 0.5), (0.2, 4.0, 4.0, 0.5), (1.5, 4.0, 0.5, 4.0)],
    "crossing_bus": [(0.01, 4.0, 1.0, 0.2), (0.005, 4.0, 1.0, 0.2), (0.0025, 4.0, 1.0, 0.2), (0.001, 4.0, 1.0, 0.2)],
}
# one mesh for all conductors: the settings that give Table 2's sizes (74, 184, 588 panels)
SHARED_SETS = {"crossing_bars_in_box": [(2.0, 2.0, 2.0, 1.0), (0.75, 2.0, 1.0, 1.0), (0.375, 2.0, 0.5, 1.5)]}


def partitioned(args, binding, np):
    """Per-main-net meshes (section 3.3 partition rule, one mesh and one column
    of C per conductor) against the layout's own mesh in FP64, and for the
    paper's bars in a box against section 5, Table 2."""
    import torch
    lay = layout_of(args.layout)
    blo, bhi, bc = lay.arrays()
    m = lay.n_conductors
    ctx = binding.Context(0)
    lo, hi, cond = binding.mesh_layout(lay)
    C_ref, rep_ref = ctx.extract(lo, hi, cond, m, lay.eps_r, lay.length_unit_m, binding.make_opts(args.p, args.eta))
    t0 = time.perf_counter()
    for _ in range(2):
        ctx.extract(lo, hi, cond, m, lay.eps_r, lay.length_unit_m, binding.make_opts(args.p, args.eta))
    ref_ms = (time.perf_counter() - t0) / 2 * 1e3
    log(f"partition: {lay.name} own mesh N={lo.shape[0]} FP64 {ref_ms:.1f} ms")
    rows = []
    for prm in PARTITION_SETS.get(lay.name, PARTITION_SETS["crossing_bus"]):
        for mode in ("f64", "mixed"):
            o = binding.make_opts(args.p, args.eta, **MODES[mode])
            C, panels, rep = ctx.extract_partitioned(blo, bhi, bc, m, lay.eps_r, lay.length_unit_m, *prm, opts=o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = max(1, args.steps)
            for _ in range(reps):
                C, panels, rep = ctx.extract_partitioned(blo, bhi, bc, m, lay.eps_r, lay.length_unit_m, *prm, opts=o)
            ms = (time.perf_counter() - t0) / reps * 1e3
            row = {"p1_p2_p3_p5": list(prm), "mode": mode, "panels_per_mesh": panels.tolist(),
                   "panels_total": int(panels.sum()), "ms_per_extraction": ms,
                   "C_rel_err_vs_own_mesh_f64": float(np.abs(C - C_ref).max() / np.abs(C_ref).max()),
                   "asym": rep["asym"]}
            if lay.name == "crossing_bars_in_box":
                row["C_aF"] = np.round(C * 1e18, 2).tolist()
            rows.append(row)
            log(f"partition: {row}")
    # one mesh refined around every conductor (GBEM_ALL_NETS): all of C from
    # one system, the reading of Table 2's equal coupling columns; the rule
    # settings that land on the table's three sizes for the bars in a box
    shared = []
    for prm in SHARED_SETS.get(lay.name, []):
        slo, shi, scond = binding.mesh_partition(blo, bhi, bc, binding.ALL_NETS, *prm)
        for mode in ("f64", "mixed"):
            o = binding.make_opts(args.p, args.eta, **MODES[mode])
            ctx.extract(slo, shi, scond, m, lay.eps_r, lay.length_unit_m, o)
            t0 = time.perf_counter()
            reps = max(1, args.steps)
            for _ in range(reps):
                C, rep = ctx.extract(slo, shi, scond, m, lay.eps_r, lay.length_unit_m, o)
            ms = (time.perf_counter() - t0) / reps * 1e3
            row = {"p1_p2_p3_p5": list(prm), "mode": mode, "panels": int(slo.shape[0]), "ms_per_extraction": ms,
                   "C_rel_err_vs_own_mesh_f64": float(np.abs(C - C_ref).max() / np.abs(C_ref).max()),
                   "asym": rep["asym"], "C_aF": np.round(C * 1e18, 2).tolist()}
            shared.append(row)
            log(f"partition (shared mesh): {row}")
    out = {"metric": "partitioned extraction (per-main-net meshes)", "unit": "ms per extraction",
           "config": {"workload": f"{lay.name}: own mesh N={lo.shape[0]}, M={m}"},
           "own_mesh_f64_ms": ref_ms, "own_mesh_C": (np.round(C_ref * 1e18, 2).tolist()
                                                    if lay.name == "crossing_bars_in_box" else None),
           "rows": rows, "shared_mesh_rows": shared}
    if lay.name == "crossing_bars_in_box":
        out["paper_table2_aF"] = {"74 panels": [222, -58.6, -58.6, 178], "183 panels": [225, -58.3, -58.3, 179],
                                  "594 panels": [226, -58.7, -58.7, 179], "comparator": [230, -61, -61, 180.6]}
    ctx.close()
    return out


def exact_mode(args, binding, np):
    """Exact reference mode (every pair through the exact integral) against the
    default far-field rule and the p = 8, eta = 4 setting, FP64 throughout."""
    lay = layout_of(args.layout)
    lo, hi, cond = binding.mesh_layout(lay)
    n, m = lo.shape[0], lay.n_conductors
    ctx = binding.Context(0)
    res = {}
    for name, (p, eta) in (("exact", (3, 1e6)), ("p8_eta4", (8, 4.0)), ("p3_eta2", (3, 2.0))):
        o = binding.make_opts(p, eta)
        ctx.extract(lo, hi, cond, m, lay.eps_r, lay.length_unit_m, o)
        t0 = time.perf_counter()
        C, rep = ctx.extract(lo, hi, cond, m, lay.eps_r, lay.length_unit_m, o)
        res[name] = (C, (time.perf_counter() - t0) * 1e3, rep)
        log(f"exact: {name} {res[name][1]:.1f} ms, near pairs {rep['n_near']}")
    Ce = res["exact"][0]
    rows = [{"setting": k, "ms": v[1], "assemble_ms": v[2]["t_assemble_ms"], "near_pairs": v[2]["n_near"],
             "C_rel_dev_from_exact": float(np.abs(v[0] - Ce).max() / np.abs(Ce).max())} for k, v in res.items()]
    ctx.close()
    return {"metric": "exact reference mode", "unit": "ms per extraction (FP64)",
            "config": {"workload": f"{lay.name}: N={n}, M={m}"}, "pairs": n * (n + 1) // 2, "rows": rows}


def dielectric(args, binding, np):
    """Multi-dielectric extraction (section 4) of the synthetic six-net,
    three-layer stack: whole extractions timed between device
    synchronisations, with the library's stage split."""
    import gbem_inputs as gi
    mesh = gi.layered_stack(3, args.dl_h)
    n = mesh.n_panels
    nu = n + int((mesh.kind == gi.INTERFACE).sum())
    ctx = binding.Context(0)
    o = binding.make_opts(args.p, args.eta)
    log(f"dielectric: {mesh.name} N={n} unknowns={nu} steps={args.steps} warmup={args.warmup}")
    for _ in range(args.warmup):
        ctx.extract_dielectric(*mesh.args(), opts=o)
    times, reps = [], []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        C, rep = ctx.extract_dielectric(*mesh.args(), opts=o)
        times.append((time.perf_counter() - t0) * 1e3)
        reps.append(rep)
    # one mesh per main net by the section 3.3 / 4.1 partition rules (the
    # paper's method): every column from its own, smaller mesh
    # (a fine rule, and a coarse one whose 280-330 panels per net are of the
    # size the paper's own experiment with several dielectrics used)
    lay = gi.layered_stack_layout(3)
    partitioned = {}
    for name, rule in (() if args.dl_uniform_only else
                       (("fine", (0.04, 4.0, 0.5, 0.5)), ("coarse", (0.25, 2.0, 1.0, 0.5)))):
        ctx.extract_dielectric_partitioned(lay, *rule, opts=o)
        pt = []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            Cp, panels, prep = ctx.extract_dielectric_partitioned(lay, *rule, opts=o)
            pt.append((time.perf_counter() - t0) * 1e3)
        partitioned[name] = {"rule_p1_p2_p3_p5": list(rule), "panels_per_mesh": [int(x) for x in panels],
                             "ms_all_columns": float(np.median(pt)),
                             "C_rel_dev_from_uniform": float(np.abs(Cp - C).max() / np.abs(C).max()),
                             "C_diag_aF": [float(Cp[k, k] * 1e18) for k in range(mesh.n_conductors)]}
    ctx.close()
    ms = float(np.median(times))
    stage = {k: float(np.median([r[k] for r in reps])) for k in ("t_assemble_ms", "t_factor_ms", "t_solve_ms")}
    return {"metric": "multi-dielectric extractions per second", "value": 1e3 / ms, "unit": "extractions/s",
            "ms_per_extraction": ms, "steps": args.steps, "warmup": args.warmup, "dtype": "f64",
            "data": "synthetic", "stages_ms": stage, "residual": reps[-1]["residual"],
            "refine_iters": reps[-1]["refine_iters"], "asym": reps[-1]["asym"],
            "config": {"workload": f"{mesh.name}: N={n} panels, {nu} unknowns, M=6, 3 dielectrics",
                       "far_order": args.p, "near_eta": args.eta},
            "C_diag_aF": [float(C[k, k] * 1e18) for k in range(mesh.n_conductors)], "partitioned": partitioned}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="mixed", choices=sorted(MODES))
    ap.add_argument("--layout", default=None,
                    help="default three_layer_bus (crossing_bus for --partition and --exact)")
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--eta", type=float, default=2.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f64", action="store_true", help="do not time the plain FP64 path beside the mode")
    ap.add_argument("--serving", action="store_true",
                    help="replay the seeded serving stream (256 jobs, Poisson 50 jobs/s) instead")
    ap.add_argument("--jobs", type=int, default=256)
    ap.add_argument("--no-serving", action="store_true",
                    help="do not replay the serving stream (mixed and FP64) after the headline steps")
    ap.add_argument("--no-profile", action="store_true",
                    help="time without the library's per-launch HIP events (no roofline)")
    ap.add_argument("--sweep", action="store_true",
                    help="precision sweep p x eta x factor dtype on --layout (default three_layer_bus)")
    ap.add_argument("--partition", action="store_true",
                    help="per-main-net meshes by the section 3.3 rule on --layout (crossing_bus or "
                         "crossing_bars_in_box) against the layout's own mesh")
    ap.add_argument("--exact", action="store_true",
                    help="exact reference mode (every pair exact) on --layout vs the far-field settings")
    ap.add_argument("--graph", action="store_true",
                    help="opts.graph: replay each job's factor/solve launches as a captured hipGraph "
                         "(ignored while the library's profiling events are on: use with --no-profile)")
    ap.add_argument("--dielectric", action="store_true",
                    help="multi-dielectric extraction of the six-net three-layer stack instead")
    ap.add_argument("--no-dielectric", action="store_true",
                    help="do not time the multi-dielectric stack after the headline steps")
    ap.add_argument("--dl-uniform-only", action="store_true",
                    help="--dielectric: only the uniform mesh (no per-main-net meshes), e.g. for a kernel profile")
    ap.add_argument("--dl-h", type=float, default=0.1,
                    help="conductor panel size of the --dielectric stack (interfaces and walls 2x)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (the reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the extraction runs on a single GPU; multi-GPU runs are not supported, use --gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2203_11733_amd import binding

    if args.layout is None:
        args.layout = "crossing_bus" if (args.partition or args.exact) else "three_layer_bus"
    if args.serving:
        print(json.dumps(serving(args, binding, np)))
        return
    if args.partition:
        print(json.dumps(partitioned(args, binding, np)))
        return
    if args.exact:
        print(json.dumps(exact_mode(args, binding, np)))
        return
    if args.dielectric:
        print(json.dumps(dielectric(args, binding, np)))
        return
    if args.sweep:
        print(json.dumps(sweep(args, binding, np)))
        return

    lay = layout_of(args.layout)
    lo, hi, cond = binding.mesh_layout(lay)
    n, m = lo.shape[0], lay.n_conductors
    log(f"bench: layout={lay.name} N={n} M={m} mode={args.mode} steps={args.steps} warmup={args.warmup}")
    dev = torch.device("cuda:0")
    d_lo = torch.tensor(lo, device=dev)
    d_hi = torch.tensor(hi, device=dev)
    d_cond = torch.tensor(cond, device=dev)
    d_C = torch.zeros((m, m), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    ctx = binding.Context(0)

    def run_steps(mode_opts, steps):
        """Time `steps` whole extractions: wall clock of the run bracketed by
        device synchronisations, and each step's host-side latency."""
        lat, reps = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s0 = time.perf_counter()
            reps.append(ctx.extract_device(d_lo, d_hi, d_cond, m, lay.eps_r, lay.length_unit_m, d_C, mode_opts,
                                           stream))
            lat.append(time.perf_counter() - s0)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, np.array(lat) * 1e3, reps

    # warmup; the last warmup step times every kernel class once (untimed) to
    # find the dominant one; the timed steps record HIP events around that
    # class's launches only (events around every launch cost ~7 % here)
    opts_all = binding.make_opts(args.p, args.eta, profile=True, **MODES[args.mode])
    rep_all = None
    for w in range(max(1, args.warmup)):
        rep_all = ctx.extract_device(d_lo, d_hi, d_cond, m, lay.eps_r, lay.length_unit_m, d_C,
                                     opts_all if w == max(1, args.warmup) - 1 else
                                     binding.make_opts(args.p, args.eta, **MODES[args.mode]), stream)
    torch.cuda.synchronize()
    dominant = max(rep_all["profile"].items(), key=lambda kv: kv[1]["ms"])[0]
    # the trailing update (the throughput kernel) is timed too when the
    # panel chain is the largest class
    timed = [dominant] + (["syrk"] if dominant != "syrk" and "syrk" in rep_all["profile"] else [])
    opts = binding.make_opts(args.p, args.eta, profile=None if args.no_profile else timed, graph=args.graph,
                             **MODES[args.mode])
    log(f"bench: warmup done; dominant kernel class {dominant}")
    elapsed, lat_ms, reps = run_steps(opts, args.steps)
    C = d_C.cpu().numpy()
    log(f"bench: {args.mode} {elapsed / args.steps * 1e3:.2f} ms per step")

    # the plain FP64 path over the same number of steps (parity-tested
    # against the CPU oracle; the mixed result's error is taken against it)
    f64 = None
    C64 = None
    if args.mode != "f64" and not args.no_f64:
        o64 = binding.make_opts(args.p, args.eta)
        for _ in range(max(1, args.warmup)):
            ctx.extract_device(d_lo, d_hi, d_cond, m, lay.eps_r, lay.length_unit_m, d_C, o64, stream)
        el64, lat64, reps64 = run_steps(o64, args.steps)
        C64 = d_C.cpu().numpy().copy()
        f64 = {"value": n * (n + 1) / 2 * args.steps / el64, "ms_per_step": el64 / args.steps * 1e3,
               "extractions_per_s": args.steps / el64,
               "latency_ms": {"p50": float(np.percentile(lat64, 50)), "p99": float(np.percentile(lat64, 99))},
               "stage_ms": {k: float(np.mean([r[k] for r in reps64]))
                            for k in ("t_assemble_ms", "t_factor_ms", "t_solve_ms", "t_total_ms")}}
        log(f"bench: f64 {f64['ms_per_step']:.2f} ms per step")
    elif args.mode == "f64":
        C64 = C.copy()
    err = float(np.abs(C - C64).max() / np.abs(C64).max()) if C64 is not None else None
    pairs = n * (n + 1) / 2
    r_last = reps[-1]
    stage = {k: float(np.mean([r[k] for r in reps])) for k in ("t_assemble_ms", "t_factor_ms", "t_solve_ms",
                                                              "t_total_ms")}
    # per kernel class over the timed steps (HIP events inside the library)
    profile = {}
    for r in reps:
        for cls, d in r["profile"].items():
            acc = profile.setdefault(cls, {"ms": 0.0, "launches": 0, "flops": 0.0, "bytes": 0.0})
            for key in acc:
                acc[key] += d[key]
    out = {
        "metric": "panel-pair integrals/s (whole extraction)",
        "value": pairs * args.steps / elapsed,
        "unit": "panel-pair integrals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE_LABEL[args.mode], "data": "synthetic",
        "config": {"workload": f"{lay.name}: N={n} panels, M={m} conductors, p={args.p}, eta={args.eta}",
                   "mode": args.mode},
        "extractions_per_s": args.steps / elapsed,
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "C_rel_err_vs_f64": err,
        "refine_iters": r_last["refine_iters"], "residual": r_last["residual"],
        "factor_used": r_last["factor_used"], "graph_used": bool(r_last["graph_used"]),
        "tile_shapes": {"outer_width": r_last["outer_width"], "super_panels": r_last["super_panels"],
                        "source": os.path.relpath(binding.tuning_source(), ROOT)
                        if os.path.isabs(binding.tuning_source()) else binding.tuning_source()},
        "stage_ms": stage,
        "f64": f64,
        "kernel_ms_per_step": {c: d["ms"] / args.steps for c, d in sorted(profile.items(), key=lambda kv: -kv[1]["ms"])},
        "roofline": roofline_of(profile, args.mode, lay.name, dominant) if profile else None,
        "roofline_trailing_update": (roofline_of(profile, args.mode, lay.name, "syrk")
                                     if "syrk" in profile and dominant != "syrk" else None),
        "kernel_ms_untimed_step": {c: d["ms"] for c, d in sorted(rep_all["profile"].items(), key=lambda kv: -kv[1]["ms"])},
    }
    Cg = golden_C(lay.name, args.p, args.eta)
    if Cg is not None:
        # the oracle's whole extraction of this layout (stored; the oracle
        # needs minutes and 30 GB of host memory at this size)
        out["C_rel_err_vs_oracle"] = {args.mode: float(np.abs(C - Cg).max() / np.abs(Cg).max())}
        if C64 is not None and args.mode != "f64":
            out["C_rel_err_vs_oracle"]["f64"] = float(np.abs(C64 - Cg).max() / np.abs(Cg).max())
    # stage rates (per step, from the library's HIP events)
    nnz = r_last["n_near"]
    far_pairs = pairs - nnz
    rates = {"near_pairs": nnz, "far_pairs": far_pairs, "from": "the all-class profiled warmup step"}
    pa = rep_all["profile"]
    if "far" in pa:
        far_s = pa["far"]["ms"] / 1e3
        rates["far_pair_integrals_per_s"] = far_pairs / far_s
        rates["far_kernel_evals_per_s"] = far_pairs * args.p ** 4 / far_s
    if "near_eval" in pa:
        rates["near_pairs_per_s"] = nnz / (pa["near_eval"]["ms"] / 1e3)
    out["rates"] = rates
    if not args.no_serving:
        # the seeded 256-job serving stream in this mode and in plain FP64
        # (its own context: jobs through gbem_submit / gbem_poll)
        out["serving"] = {}
        for smode in dict.fromkeys((args.mode, "f64")):
            sargs = argparse.Namespace(**vars(args))
            sargs.mode = smode
            sv = serving(sargs, binding, np)
            out["serving"].setdefault("workload", sv["config"]["workload"])
            out["serving"][smode] = {"dtype": sv["dtype"], "poisson": sv["poisson"], "saturation": sv["saturation"]}
    if not args.no_dielectric:
        # the multi-dielectric extraction (section 4) of the six-net stack,
        # a few whole extractions in its own context
        dargs = argparse.Namespace(**vars(args))
        dargs.steps, dargs.warmup = 5, 1
        dl = dielectric(dargs, binding, np)
        out["dielectric"] = {k: dl[k] for k in ("metric", "value", "unit", "ms_per_extraction", "dtype", "stages_ms",
                                                "residual", "refine_iters", "config", "partitioned")}
    if args.copy_calibration:
        # a plain copy kernel of known size: 256 MiB read + 256 MiB written per launch
        src = torch.ones(32 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = src.numel() * 8
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle sample")
        out["cpu_baseline"], C_or = cpu_baseline(lo, hi, cond, lay, args.p, args.eta)
        if C_or is not None:
            # the whole extraction against the oracle's, at the workload's full size
            out["C_rel_err_vs_oracle"] = {args.mode: float(np.abs(C - C_or).max() / np.abs(C_or).max())}
            if C64 is not None and args.mode != "f64":
                out["C_rel_err_vs_oracle"]["f64"] = float(np.abs(C64 - C_or).max() / np.abs(C_or).max())
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
