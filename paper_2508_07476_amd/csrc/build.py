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
SOURCES = ["st_api.hip", "k_strided.hip", "k_strided_u16.hip", "k_strided_f32d.hip", "k_strided_f32a.hip",
           "k_strided_f32b.hip", "k_xpass.hip", "k_xgrad.hip", "k_xfinala.hip", "k_xfinalb.hip", "k_angles.hip"]
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


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *CFLAGS, "-c", os.path.join(HERE, src), "-o", obj]
    t = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, time.time() - t, r.stderr


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4, 16)
    # the largest translation units first, so they do not finish last
    order = sorted(SOURCES, key=lambda f: -os.path.getsize(os.path.join(HERE, f)))
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
