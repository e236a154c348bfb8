"""The whole structure-tensor orientation path on one volume or padded block (oracle, FP64).

Order of the steps follows Figure 1 (a)-(c) and the orientation module of the
paper's Architecture section: input volume and optional mask -> structure
tensor -> eigen-decomposition (fibre = e3) -> cylindrical frame -> HA, IA, FA.

Mask reading (Figure 1(a) only calls it "optional"): the tensor is computed
from the raw, unmasked intensities; outside the mask every output is 0 and the
voxel carries only the "outside mask" flag.

Flags (uint8): bit0 degenerate (trace <= 0 or gap/trace < 1e-3), bit1 outside
mask, bit2 on the axis (r < 1e-9).
"""

from __future__ import annotations

import numpy as np

from .angles import cylindrical_frame, helix_intrusion
from .eigen import degenerate, eigen_sorted, fractional_anisotropy, gap_ratio
from .tensor import structure_tensor

FLAG_DEGENERATE = 1
FLAG_OUTSIDE_MASK = 2
FLAG_ON_AXIS = 4


def compute(volume, mask=None, sigma=1.0, rho=3.0, truncate=4.0,
            axis_center=None, axis_direction=None, origin=(0, 0, 0), keep_tensor=False):
    """Run the oracle on ``volume`` (nz, ny, nx).

    ``origin`` is the global (z, y, x) index of ``volume[0, 0, 0]`` (used only
    for the cylindrical frame, so a padded block of a larger volume yields the
    same angles as the whole volume).  Returns a dict of float64/uint8 arrays:
    e3 (3, ...), evals (3, ...), fa, ha, ia (None without an axis), flags,
    gap (gap/trace ratio) and, if ``keep_tensor``, S (6, ...).
    """
    v = np.asarray(volume, dtype=np.float64)
    S = structure_tensor(v, sigma, rho, truncate)
    evals, e3 = eigen_sorted(S)
    fa = fractional_anisotropy(evals)
    flags = np.where(degenerate(evals), FLAG_DEGENERATE, 0).astype(np.uint8)
    ha = ia = None
    if axis_center is not None:
        frame = cylindrical_frame(v.shape, axis_center, axis_direction, origin)
        ha, ia, on_axis = helix_intrusion(e3, frame)
        flags |= np.where(on_axis, FLAG_ON_AXIS, 0).astype(np.uint8)
    if mask is not None:
        out = np.asarray(mask) == 0
        e3 = np.where(out[None], 0.0, e3)
        evals = np.where(out[None], 0.0, evals)
        fa = np.where(out, 0.0, fa)
        if ha is not None:
            ha = np.where(out, 0.0, ha)
            ia = np.where(out, 0.0, ia)
        flags = np.where(out, FLAG_OUTSIDE_MASK, flags).astype(np.uint8)
    res = {"e3": e3, "evals": evals, "fa": fa, "ha": ha, "ia": ia, "flags": flags,
           "gap": gap_ratio(evals)}
    if keep_tensor:
        res["S"] = S
    return res
