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


def compare_block(ph, res, origin, B):
    halo = oracle.radius(SIGMA) + oracle.radius(RHO)
    lo = [max(0, c - halo) for c in origin]
    hi = [min(SHAPE[i], origin[i] + B + halo) for i in range(3)]
    crop = ph["volume"][lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]].cpu().numpy()
    o = oracle.compute(crop, None, SIGMA, RHO, axis_center=ph["center"], axis_direction=ph["direction"],
                       origin=tuple(lo))
    s = tuple(slice(origin[i] - lo[i], origin[i] - lo[i] + B) for i in range(3))
    ob = {k: (v[(slice(None),) + s] if v.ndim == 4 else v[s]) for k, v in o.items() if v is not None}
    gs = tuple(slice(origin[i], origin[i] + B) for i in range(3))
    gb = {k: (v[(slice(None),) + gs] if v.dim() == 4 else v[gs]).cpu().numpy() for k, v in res.items()}
    return compare(gb, ob, (B, B, B), ph["center"], ph["direction"], origin=origin), ob


def block_origins(count, B, seed=2):
    """Sub-blocks spread over the three noise bands (z thirds) and both annuli, plus the last corner."""
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
    out.append((nz - B, ny - B, nx - B))
    return out
