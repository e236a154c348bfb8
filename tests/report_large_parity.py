"""Stratified error report for the 2048 x 1024 x 1024 two-annuli workload.

Runs the HIP path on the whole uint16 volume (sigma 2, rho 6), then the FP64
oracle on 16 sampled 128^3 sub-blocks (each padded by R_sigma + R_rho), and
writes a Markdown table of maximum errors per gap/trace bin.  Not collected by
pytest; run on a GPU machine:

    python tests/report_large_parity.py [out.md]
"""

import multiprocessing
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle  # noqa: E402
from _large import (SHAPE, SIGMA, RHO, block_origins, compare_block, crop_for, log, run_full,  # noqa: E402
                    time_full)
from _oracle_worker import oracle_block  # noqa: E402
from _parity import wrap_pi, angle_between  # noqa: E402

BINS = ((1e-3, 1e-2), (1e-2, 1e-1), (1e-1, np.inf))


def main(out_path, workers=8):
    spec, ph, res = run_full()
    ms, per_pass = time_full(ph, res)
    nvox = int(np.prod(SHAPE))
    log(f"whole volume: {ms:.1f} ms per run, {nvox / ms / 1e6:.2f} Gvoxels/s; passes {per_pass}")
    B = 128
    origins = block_origins(16, B)
    pool = ProcessPoolExecutor(max_workers=workers, mp_context=multiprocessing.get_context("spawn"))
    futs = []
    for org in origins:
        crop, lo = crop_for(ph, org, B)
        futs.append(pool.submit(oracle_block, crop, lo, org, B, SIGMA, RHO, ph["center"], ph["direction"]))
    acc = {b: {"n": 0, "e3": 0.0, "fa": 0.0, "ha": 0.0, "ia": 0.0} for b in BINS}
    n_deg = n_all = 0
    t0 = time.time()
    for k, org in enumerate(origins):
        stats, ob = compare_block(ph, res, org, B, ob=futs[k].result())
        gs = tuple(slice(org[i], org[i] + B) for i in range(3))
        g = {kk: (v[(slice(None),) + gs] if v.dim() == 4 else v[gs]).cpu().numpy() for kk, v in res.items()}
        gap = ob["gap"]
        e_r, e_t, a, r = oracle.cylindrical_frame((B, B, B), ph["center"], ph["direction"], org)
        f_r = (ob["e3"] * e_r).sum(0); f_t = (ob["e3"] * e_t).sum(0); f_a = (ob["e3"] * a.reshape(3, 1, 1, 1)).sum(0)
        for lo, hi in BINS:
            m = (gap >= lo) & (gap < hi)
            if not m.any():
                continue
            d = acc[(lo, hi)]
            d["n"] += int(m.sum())
            d["e3"] = max(d["e3"], float(angle_between(g["e3"][:, m], ob["e3"][:, m]).max()))
            d["fa"] = max(d["fa"], float(np.abs(g["fa"][m] - ob["fa"][m]).max()))
            mh = m & (r >= 1) & (np.hypot(f_t, f_a) >= 0.1)
            mi = m & (r >= 1) & (np.hypot(f_t, f_r) >= 0.1)
            if mh.any():
                d["ha"] = max(d["ha"], float(wrap_pi(g["ha"][mh] - ob["ha"][mh]).max()))
            if mi.any():
                d["ia"] = max(d["ia"], float(wrap_pi(g["ia"][mi] - ob["ia"][mi]).max()))
        n_deg += int((gap < oracle.DEGENERATE_GAP).sum())
        n_all += gap.size
        log(f"block {k + 1}/16 {org}: checked {stats['n_checked']}, e3 max {stats.get('e3_max', 0):.2e} "
            f"({time.time() - t0:.0f} s)")
    pool.shutdown()
    lines = [f"# Stratified parity — {SHAPE[0]}x{SHAPE[1]}x{SHAPE[2]} uint16 two-annuli phantom, sigma {SIGMA}, rho {RHO}",
             "", "Command: `python tests/report_large_parity.py` (HIP path on the whole volume; FP64 oracle on",
             f"16 sampled {B}^3 sub-blocks padded by R_sigma + R_rho = {oracle.radius(SIGMA) + oracle.radius(RHO)}).", "",
             f"Degenerate voxels (gap/trace < 1e-3 or trace <= 0, excluded): {n_deg} of {n_all}.", "",
             f"Whole-volume throughput (inputs resident, outputs e3, FA, HA, IA, flags; mean of 3 runs): "
             f"{ms:.1f} ms, {nvox / ms / 1e6:.2f} Gvoxels/s.  Per pass (ms): "
             + ", ".join(f"{k} {v:.1f}" for k, v in per_pass.items()) + ".", "",
             "| gap/trace bin | voxels | max e3 angle (rad) | max abs FA | max abs HA (rad) | max abs IA (rad) |",
             "|---|---|---|---|---|---|"]
    for (lo, hi), d in acc.items():
        lines.append(f"| [{lo:g}, {hi:g}) | {d['n']} | {d['e3']:.2e} | {d['fa']:.2e} | {d['ha']:.2e} | {d['ia']:.2e} |")
    lines += ["", "Tolerances: e3 <= 1e-3 rad; FA, HA, IA <= 1e-4 (HA/IA where the fibre's projection on the "
              "angle's plane is >= 0.1 and r >= 1).", ""]
    text = "\n".join(lines) + "\n"
    with open(out_path, "w") as fh:
        fh.write(text)
    print(text)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "large_parity.md")
