"""Whole-volume comparison of the 512^3 uint16 workload (annulus mask, sigma
1.5, rho 4) with the FP64 oracle: every voxel of the volume.

The HIP path runs once on the whole volume; the oracle runs on 32 boxes of
64 (z) x 128 (y) x 512 (x) voxels, each padded by R_sigma + R_rho = 22 and
clipped at the volume's faces (which makes every box's values those of the
whole volume), in worker processes over the host cores (at most 16).  Writes
a Markdown table of the maximum errors per gap/trace bin and the flag
mismatches, and exits non-zero if any tolerance is exceeded.  Not collected by
pytest; run on a GPU machine:

    python tests/report_whole_512.py [out.md]
"""

import multiprocessing
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import numpy as np  # noqa: E402
import torch  # noqa: E402

import oracle  # noqa: E402
import paper_2508_07476_amd as st  # noqa: E402
from phantom import helix  # noqa: E402

from _oracle_worker import compare_region  # noqa: E402
from _parity import ANGLE_TOL, E3_TOL, FA_TOL  # noqa: E402

SHAPE = (512, 512, 512)
SIGMA, RHO = 1.5, 4.0
OUTS = ("e3", "fa", "ha", "ia", "flags")
BOX = (64, 128, 512)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main(out_path):
    ph = helix.generate(helix.spec_headline_u16(shape=SHAPE), device="cuda:0")
    res = st.st_compute(ph["volume"], SIGMA, RHO, mask=ph["mask"], axis_center=ph["center"],
                        axis_direction=ph["direction"], outputs=OUTS)
    torch.cuda.synchronize()
    log("st_compute done on", SHAPE)
    vol = ph["volume"].cpu().numpy()
    msk = ph["mask"].cpu().numpy()
    halo = oracle.radius(SIGMA) + oracle.radius(RHO)
    try:
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        workers = max(1, min(16, os.cpu_count() or 1))
    pool = ProcessPoolExecutor(max_workers=workers, mp_context=multiprocessing.get_context("spawn"))
    futs = []
    t0 = time.time()
    for z in range(0, SHAPE[0], BOX[0]):
        for y in range(0, SHAPE[1], BOX[1]):
            x = 0
            org = (z, y, x)
            lo = [max(0, org[d] - halo) for d in range(3)]
            hi = [min(SHAPE[d], org[d] + BOX[d] + halo) for d in range(3)]
            sl = tuple(slice(lo[d], hi[d]) for d in range(3))
            cut = tuple((org[d] - lo[d], org[d] - lo[d] + BOX[d]) for d in range(3))
            gs = tuple(slice(org[d], org[d] + BOX[d]) for d in range(3))
            gpu = {k: (v[(slice(None),) + gs] if v.dim() == 4 else v[gs]).cpu().numpy() for k, v in res.items()}
            futs.append((org, pool.submit(compare_region, vol[sl], msk[sl], tuple(lo), cut, gpu, SIGMA, RHO,
                                          ph["center"], ph["direction"])))
    keys = ("e3_max", "fa_max", "ha_max", "ia_max")
    tot = {k: 0.0 for k in keys}
    counts = {"n": 0, "n_checked": 0, "n_ha": 0, "n_ia": 0, "flag_deg_mismatch": 0, "flag_other_mismatch": 0}
    bins_err = {}
    bins_n = {}
    for org, f in futs:
        s = f.result()
        for k in keys:
            tot[k] = max(tot[k], s.get(k, 0.0))
        for k in counts:
            counts[k] += s.get(k, 0)
        for b, (n, e) in s["e3_bins"].items():
            bins_err[b] = max(bins_err.get(b, 0.0), e)
            bins_n[b] = bins_n.get(b, 0) + n
        log(org, {k: s.get(k) for k in keys + ("n_checked",)})
    pool.shutdown()
    wall = time.time() - t0
    ok = (tot["e3_max"] <= E3_TOL and tot["fa_max"] <= FA_TOL and tot["ha_max"] <= ANGLE_TOL and
          tot["ia_max"] <= ANGLE_TOL and counts["flag_deg_mismatch"] == 0 and counts["flag_other_mismatch"] == 0
          and counts["n"] == int(np.prod(SHAPE)))
    lines = [
        "# Whole-volume parity: 512^3 uint16 phantom + annulus mask, sigma 1.5, rho 4",
        "",
        "Command: `python tests/report_whole_512.py <out.md>` (HIP path on the whole volume; FP64 oracle on "
        f"32 boxes of {BOX[0]}x{BOX[1]}x{BOX[2]} padded by {halo}, {workers} worker processes, {wall:.0f} s).",
        "",
        f"Voxels compared: {counts['n']} (every voxel); checked (inside the mask, oracle gap/trace >= 1e-3): "
        f"{counts['n_checked']}; HA checked {counts['n_ha']}, IA checked {counts['n_ia']}.",
        "",
        "| gap/trace | voxels | max e3 error (rad) |",
        "|---|---|---|",
    ]
    for b in bins_err:
        lines.append(f"| {b} | {bins_n[b]} | {bins_err[b]:.2e} |")
    lines += [
        "",
        f"Maxima over every checked voxel: e3 {tot['e3_max']:.2e} rad (tol {E3_TOL:g}), FA {tot['fa_max']:.2e} "
        f"(tol {FA_TOL:g}), HA {tot['ha_max']:.2e} rad, IA {tot['ia_max']:.2e} rad (tol {ANGLE_TOL:g}).",
        f"Flag mismatches: degeneracy bit (outside the 2 % band) {counts['flag_deg_mismatch']}, mask / on-axis bits "
        f"{counts['flag_other_mismatch']}.",
        "",
        f"Result: {'PASS' if ok else 'FAIL'}",
    ]
    text = "\n".join(lines) + "\n"
    if out_path:
        with open(out_path, "w") as fh:
            fh.write(text)
    print(text)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main(sys.argv[1] if len(sys.argv) > 1 else None))
