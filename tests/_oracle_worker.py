"""CPU-only helper for running the oracle on a padded crop in a worker process
(imports numpy and the oracle only: no torch, no GPU)."""

import numpy as np

import oracle


def oracle_block(crop, lo, origin, B, sigma, rho, center, direction):
    """Oracle outputs on ``crop`` (whose [0,0,0] is global index ``lo``), cut to
    the B^3 block at global ``origin``."""
    o = oracle.compute(crop, None, sigma, rho, axis_center=center, axis_direction=direction,
                       origin=tuple(lo))
    s = tuple(slice(origin[i] - lo[i], origin[i] - lo[i] + B) for i in range(3))
    return {k: np.ascontiguousarray(v[(slice(None),) + s] if v.ndim == 4 else v[s])
            for k, v in o.items() if v is not None}


def oracle_cut(crop, mask, sigma, rho, center, direction, origin, cut):
    """Oracle outputs on ``crop`` (optional ``mask``; ``origin`` = global index
    of crop[0, 0, 0]), restricted to the index box ``cut`` = ((z0, z1), (y0, y1),
    (x0, x1)) of the crop."""
    o = oracle.compute(crop, mask, sigma, rho, axis_center=center, axis_direction=direction,
                       origin=tuple(origin))
    s = tuple(slice(a, b) for a, b in cut)
    return {k: np.ascontiguousarray(v[(slice(None),) + s] if v.ndim == 4 else v[s])
            for k, v in o.items() if v is not None}


def compare_region(crop, mask, origin, cut, gpu, sigma, rho, center, direction):
    """Runs the oracle on ``crop`` (global index ``origin`` at crop[0, 0, 0]) and
    compares the region ``cut`` of it with the GPU outputs ``gpu`` of that
    region; returns the error statistics without the per-voxel arrays."""
    from _parity import compare

    o = oracle_cut(crop, mask, sigma, rho, center, direction, origin, cut)
    shape = tuple(b - a for a, b in cut)
    gorg = tuple(origin[d] + cut[d][0] for d in range(3))
    stats = compare(gpu, o, shape, center, direction, origin=gorg)
    stats.pop("e3_err", None)
    gap = o["gap"]
    stats["gap_bins"] = {f"[{lo:g},{hi:g})": int(((gap >= lo) & (gap < hi)).sum())
                         for lo, hi in ((1e-3, 1e-2), (1e-2, 1e-1), (1e-1, np.inf))}
    return stats
