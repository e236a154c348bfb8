"""Cylindrical frame and helix / intrusion angles (oracle, FP64, test infrastructure).

Figure 1(c) of the paper rotates the fibre field into a cylindrical coordinate
system about the left-ventricular axis and reads off the helix angle (HA) and
the intrusion angle (IA); the formulas are not printed.  Readings taken:

* voxel position p = (i, j, k) in (z, y, x) voxel units, axis centre c,
  axis direction a = d / |d|;
* q = p - c, q_perp = q - (q . a) a, r = |q_perp|, e_r = q_perp / r;
* e_theta = a x e_r evaluated in right-handed (x, y, z) order (the (z, y, x)
  array order is an odd permutation, so a cross product taken directly on
  (z, y, x) arrays would return -e_theta);
* with f_r = e3 . e_r, f_t = e3 . e_theta, f_a = e3 . a and sgn(0) = +1:
  HA = atan2(f_a sgn f_t, |f_t|),  IA = atan2(f_r sgn f_t, |f_t|)
  (radians, invariant under e3 -> -e3; HA > 0 for a right-handed helix);
* where r < 1e-9 the frame is undefined: HA = IA = 0 and the voxel is
  flagged "on axis".
"""

from __future__ import annotations

import numpy as np

ON_AXIS_RADIUS = 1e-9


def _cross_xyz(a, b):
    """a x b for (3, ...) vectors stored in (z, y, x) order, computed in right-handed (x, y, z)."""
    az, ay, ax = a
    bz, by, bx = b
    cx = ay * bz - az * by
    cy = az * bx - ax * bz
    cz = ax * by - ay * bx
    return np.stack([cz, cy, cx])


def cylindrical_frame(shape, center, direction, origin=(0, 0, 0)):
    """Return (e_r, e_theta, a, r) for a block of ``shape`` whose first voxel is at ``origin``.

    e_r and e_theta are (3, nz, ny, nx) in (z, y, x) component order (NaN on the
    axis); a is (3,); r is (nz, ny, nx).
    """
    nz, ny, nx = shape
    d = np.asarray(direction, dtype=np.float64)
    a = d / np.linalg.norm(d)
    zz, yy, xx = np.meshgrid(np.arange(nz, dtype=np.float64) + origin[0],
                             np.arange(ny, dtype=np.float64) + origin[1],
                             np.arange(nx, dtype=np.float64) + origin[2], indexing="ij")
    q = np.stack([zz - center[0], yy - center[1], xx - center[2]])
    qa = (q * a.reshape(3, 1, 1, 1)).sum(axis=0)
    qp = q - qa[None] * a.reshape(3, 1, 1, 1)
    r = np.sqrt((qp * qp).sum(axis=0))
    with np.errstate(invalid="ignore", divide="ignore"):
        e_r = np.where(r[None] >= ON_AXIS_RADIUS, qp / r[None], np.nan)
    e_t = _cross_xyz(np.broadcast_to(a.reshape(3, 1, 1, 1), e_r.shape), e_r)
    return e_r, e_t, a, r


def helix_intrusion(e3, frame):
    """Return (HA, IA, on_axis) for unit vectors ``e3`` (3, ...) in ``frame``."""
    e_r, e_t, a, r = frame
    e3 = np.asarray(e3, dtype=np.float64)
    f_r = (e3 * e_r).sum(axis=0)
    f_t = (e3 * e_t).sum(axis=0)
    f_a = (e3 * a.reshape((3,) + (1,) * (e3.ndim - 1))).sum(axis=0)
    sgn = np.where(f_t >= 0, 1.0, -1.0)
    on_axis = r < ON_AXIS_RADIUS
    ha = np.where(on_axis, 0.0, np.arctan2(f_a * sgn, np.abs(f_t)))
    ia = np.where(on_axis, 0.0, np.arctan2(f_r * sgn, np.abs(f_t)))
    return ha, ia, on_axis
