"""Compile libgbem.so (HIP for gfx950) in-tree: paper_2203_11733_amd/libgbem.so."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "libgbem.so")
BUILD = os.path.join(PKG, "_build")
ARCH = os.environ.get("GBEM_OFFLOAD_ARCH", "gfx950")

# per-file flags: the near/far test and the mesher must be bit-exact, so no
# FMA contraction there.
SOURCES = {
    "api.cpp": [],
    "mesh.cpp": ["-ffp-contract=off"],
    "panels.hip": [],
    "near.hip": ["-ffp-contract=off"],
    "near_eval.hip": [],
    "far.hip": [],
    "chol.hip": [],
    "refine.hip": [],
    "solve.hip": [],
    "dielectric.hip": [],
    "tune.cpp": [],
}


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str, extra: list[str]) -> str:
    obj = os.path.join(BUILD, src + ".o")
    cmd = [hipcc(), "-c", "-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", INC, "-I", CSRC, "-Wall", "-Wno-unused-function", "-Werror=return-type",
           *extra, "-o", obj, os.path.join(CSRC, src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(lambda kv: _compile(*kv), SOURCES.items()))
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lpthread", "-ldl"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    # a kernel whose host launch stub the compiler dropped links fine and
    # fails only when the library is loaded: refuse it here
    nm = subprocess.run(["nm", "-D", "--undefined-only", tmp], capture_output=True, text=True)
    missing = [ln.split()[-1] for ln in nm.stdout.splitlines() if "gbem" in ln]
    if nm.returncode == 0 and missing:
        os.remove(tmp)
        raise RuntimeError("libgbem.so has undefined symbols of its own: " + ", ".join(missing[:5]))
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
