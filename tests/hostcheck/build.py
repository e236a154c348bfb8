"""Builds the host-code check (see hostcheck.h): the library's host
translation units and the stand-ins, compiled for the host only with
AddressSanitizer and UBSan, linked without the HIP runtime.

    python tests/hostcheck/build.py [out_dir]   -> <out_dir>/hostcheck (default _build/hostcheck)
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2508_07476_amd", "csrc")
LIB_UNITS = ["st_api.hip", "st_batch.hip", "st_surrogate.hip", "st_noalloc.hip"]
OWN_UNITS = ["hip_stub.cpp", "stub_kernels.cpp", "driver.cpp"]
# sanitizers apply to host code only (each -fsanitize= right after -Xarch_host)
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def tool(name):
    for cand in (os.path.join("/opt/rocm/bin", name), os.path.join("/opt/rocm/llvm/bin", name), shutil.which(name) or ""):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError(f"{name} not found")


def _compile(src, obj):
    cmd = [tool("hipcc"), "-x", "hip", "--offload-host-only", "-O1", "-g", "-std=c++20", "-fPIC",
           *SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", HERE, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{r.stderr}")
    return obj


def build(out_dir=None) -> str:
    out_dir = out_dir or os.path.join(ROOT, "_build", "hostcheck")
    os.makedirs(out_dir, exist_ok=True)
    srcs = [os.path.join(CSRC, u) for u in LIB_UNITS] + [os.path.join(HERE, u) for u in OWN_UNITS]
    objs = [os.path.join(out_dir, os.path.splitext(os.path.basename(s))[0] + ".o") for s in srcs]
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        list(ex.map(_compile, srcs, objs))
    # host-only objects still name the device-code blobs of their units: give them empty stand-ins
    names = set()
    for o in objs:
        r = subprocess.run([tool("nm"), "-u", o], capture_output=True, text=True, check=True)
        names |= set(re.findall(r"\b(__hip_fatbin_\w+)", r.stdout))
    blobs = os.path.join(out_dir, "fatbin_blobs.c")
    with open(blobs, "w") as fh:
        fh.write("".join(f"const char {n}[16] = {{0}};\n" for n in sorted(names)))
    blob_obj = os.path.join(out_dir, "fatbin_blobs.o")
    subprocess.run([tool("clang"), "-c", blobs, "-o", blob_obj], check=True, capture_output=True)
    exe = os.path.join(out_dir, "hostcheck")
    cmd = [tool("clang++"), "-fsanitize=address,undefined", *objs, blob_obj, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stderr}")
    return exe


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else None))
