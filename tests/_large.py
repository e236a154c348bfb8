"""Shared driver for the 2048 x 1024 x 1024 two-annuli workload (test code only).

Runs the HIP path once on the whole uint16 volume (2^31 voxels: every output
plane beyond the first lies past 2^31 elements, so 64-bit indexing is
exercised) and compares sampled sub-blocks with the FP64 oracle run on the
same padded crops (halo = R_sigma + R_rho makes each crop's interior exact).
"""

from __future__ import annotations

import sys
import time

import numpy as np
import torch

import oracle
import paper_2508_07476_amd as st
from phantom import helix

from _oracle_worker import oracle_block
from _parity import compare

SIGMA, RHO = 2.0, 6.0
SHAPE = (2048, 1024, 1024)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_full(device="cuda:0"):
    spec = helix.spec_two_annuli_u16(shape=SHAPE)
    t = time.time()
    ph = helix.generate(spec, device=device)
    torch.cuda.synchronize()
    log(f"phantom {SHAPE} generated in {time.time() - t:.1f} s")
    t = time.time()
    res = st.st_compute(ph["volume"], SIGMA, RHO, axis_center=ph["center"], axis_direction=ph["direction"],
                        outputs=("e3", "fa", "ha", "ia", "flags"))
    torch.cuda.synchronize()
    log(f"st_compute on {np.prod(SHAPE)} voxels: {time.time() - t:.2f} s (first call, includes setup)")
    return spec, ph, res


def crop_for(ph, origin, B):
    """Host copy of the block at ``origin`` padded by R_sigma + R_rho (clipped at the faces)."""
    halo = oracle.radius(SIGMA) + oracle.radius(RHO)
    lo = [max(0, c - halo) for c in origin]
    hi = [min(SHAPE[i], origin[i] + B + halo) for i in range(3)]
    return ph["volume"][lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]].cpu().numpy(), lo


def gpu_block(res, origin, B):
    gs = tuple(slice(origin[i], origin[i] + B) for i in range(3))
    return {k: (v[(slice(None),) + gs] if v.dim() == 4 else v[gs]).cpu().numpy() for k, v in res.items()}


def compare_block(ph, res, origin, B, ob=None):
    if ob is None:
        crop, lo = crop_for(ph, origin, B)
        ob = oracle_block(crop, lo, origin, B, SIGMA, RHO, ph["center"], ph["direction"])
    gb = gpu_block(res, origin, B)
    return compare(gb, ob, (B, B, B), ph["center"], ph["direction"], origin=origin), ob


def time_full(ph, res, reps=3):
    """Average time of ``reps`` further whole-volume runs into the same outputs and
    workspace (inputs resident), with the per-pass split from the library's
    event profiler."""
    vol = ph["volume"]
    torch.cuda.empty_cache()  # the first call's library-sized workspace is no longer needed
    ws = torch.empty(st.st_workspace_bytes(tuple(vol.shape)), dtype=torch.uint8, device=vol.device)
    run = lambda: st.st_compute(vol, SIGMA, RHO, axis_center=ph["center"], axis_direction=ph["direction"],
                                outputs=tuple(res.keys()), out=res, workspace=ws)
    run()
    torch.cuda.synchronize()
    st.profile_reset()
    st.profile_enable(True)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        run()
    t1.record()
    torch.cuda.synchronize()
    st.profile_enable(False)
    kern = st.profile_read()
    ms = t0.elapsed_time(t1) / reps
    del ws
    return ms, {k: v[0] / v[1] for k, v in kern.items()}


def block_origins(count, B, seed=2):
    """Sub-blocks spread over the three noise bands (z thirds) and both annuli,
    plus one against the far z face (z = nz - B) inside the outer annulus,
    which takes the reflection at that face and the largest output indices."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = SHAPE
    c = (ny - 1) / 2.0
    out = []
    for i in range(count - 1):
        band = i % 3
        z = int(band * nz / 3 + rng.integers(0, nz // 3 - B))
        r = [192.0, 400.0][i % 2] + rng.uniform(-40, 40)  # inside the inner / outer annulus
        th = rng.uniform(0, 2 * np.pi)
        y = int(np.clip(c + r * np.sin(th) - B / 2, 0, ny - B))
        x = int(np.clip(c + r * np.cos(th) - B / 2, 0, nx - B))
        out.append((z, y, x))
    th = np.pi / 4  # on the outer annulus' mid-radius, in the high-y, high-x quadrant
    out.append((nz - B, int(c + 400.0 * np.sin(th) - B / 2), int(c + 400.0 * np.cos(th) - B / 2)))
    return out
