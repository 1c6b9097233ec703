"""Write the stored expected capacitances of the full-size layouts.

Every number written here comes from the CPU FP64 oracle (``oracle/``) alone:
its own mesher, its own pair integrals (section 3.4 reductions for near pairs,
p x p Gauss for far pairs), LAPACK's Cholesky factorisation and exact charge
sums.  Nothing from the GPU library is read.

    python tests/golden/make_golden.py three_layer_bus

writes ``tests/golden/three_layer_bus_C.json`` (method mode p = 3, eta = 2:
the parity reference of the GPU path on the 59,904-panel, 48-conductor bus).
The dense FP64 matrix (28.7 GB) is factored in place, so about 30 GB of host
memory and some minutes of all host cores are needed.
"""
from __future__ import annotations

import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import gbem_inputs as gi  # noqa: E402
import oracle  # noqa: E402

LAYOUTS = {"three_layer_bus": gi.three_layer_bus}


def make(name: str, p: int = 3, eta: float = 2.0) -> dict:
    lay = LAYOUTS[name]()
    lo, hi, cond = oracle.mesh_layout(lay)
    n, m = lo.shape[0], lay.n_conductors
    t0 = time.time()
    A = oracle.assemble(lo, hi, p, eta)          # row-major, symmetric
    t1 = time.time()
    diag = np.array(np.diagonal(A))
    B = oracle.rhs(cond, m)
    # LAPACK dpotrf/dpotrs with 64-bit indices, in place (no second 28.7 GB
    # copy); factor and solve are timed together
    X = oracle.solve_inplace(A, B)
    t2 = time.time()
    C = oracle.charges(X, cond, m, lay.eps_r, lay.length_unit_m)
    t3 = time.time()
    del A
    return {
        "layout": name,
        "written_by": "tests/golden/make_golden.py (oracle only)",
        "n_panels": int(n),
        "n_conductors": int(m),
        "far_order": p,
        "near_eta": eta,
        "eps_r": lay.eps_r,
        "length_unit_m": lay.length_unit_m,
        "C": C.tolist(),
        "diag_A_first": diag[:8].tolist(),
        "X_col_sums": X.sum(axis=0).tolist(),
        "oracle_seconds": {"assemble": t1 - t0, "cholesky_and_solve": t2 - t1, "charges": t3 - t2},
        "host": {"cpus": os.cpu_count(), "machine": platform.machine()},
    }


def main(argv):
    names = argv[1:] or list(LAYOUTS)
    for name in names:
        res = make(name)
        out = os.path.join(HERE, f"{name}_C.json")
        with open(out, "w") as f:
            json.dump(res, f, indent=1)
        print(f"wrote {out}: N={res['n_panels']} M={res['n_conductors']} {res['oracle_seconds']}")


if __name__ == "__main__":
    main(sys.argv)
