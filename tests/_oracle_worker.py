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
