"""Build libst.so (the HIP/C-ABI library) for gfx950 with hipcc.

Usage: python -m paper_2508_07476_amd.csrc.build [--jobs N]
Objects go to <repo>/_build/, the shared library to paper_2508_07476_amd/libst.so.
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libst.so")
# (source, extra defines, object name); the strided instantiations are split into
# groups so that the largest radii compile in parallel
STRIDED_GROUPS = 8
UNITS = ([("st_api.hip", [], "st_api"), ("st_batch.hip", [], "st_batch"), ("st_noalloc.hip", [], "st_noalloc"), ("st_surrogate.hip", [], "st_surrogate"),
          ("k_surrogate.hip", [], "k_surrogate"), ("k_surrogate_train.hip", [], "k_surrogate_train"), ("k_sg_fallback.hip", [], "k_sg_fallback"), ("k_batch.hip", [], "k_batch"), ("k_strided.hip", [], "k_strided"),
          ("k_xpass.hip", [], "k_xpass"), ("k_xgrad.hip", [], "k_xgrad"),
          ("k_xfinala.hip", [], "k_xfinala"), ("k_xfinalb.hip", [], "k_xfinalb"),
          ("k_angles.hip", [], "k_angles"), ("k_gradf.hip", [], "k_gradf")] +
         [("k_strided_inst.hip", [f"-DST_STRIDED_GROUP={g}"], f"k_strided_g{g}")
          for g in range(STRIDED_GROUPS)])
# most expensive first, so they do not finish last
COST = {"k_strided_g7": 9, "k_strided_g6": 8, "k_strided_g5": 7, "k_strided_g4": 6, "k_strided_g3": 5}
ARCH = "gfx950"

CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++20", "-fPIC", "-Wall", "-Wno-unused-result",
    # packed FP32 VALU instructions stay disabled: float code compiles to scalar FP32 ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(unit):
    src, defs, name = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [hipcc(), *CFLAGS, *defs, "-c", os.path.join(HERE, src), "-o", obj]
    t = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, time.time() - t, r.stderr


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(UNITS), os.cpu_count() or 4, 16)
    order = sorted(UNITS, key=lambda u: -COST.get(u[2], 0))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_compile, order))
    objs = [o for o, _, _ in results]
    if verbose:
        for (o, dt, err) in results:
            print(f"  {os.path.basename(o)}: {dt:.1f}s", file=sys.stderr)
            if err.strip():
                print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args()
    t = time.time()
    lib = build(a.jobs, a.verbose)
    print(f"built {lib} in {time.time() - t:.1f}s")


if __name__ == "__main__":
    main()
