"""Gradient, outer product and integration steps of the structure tensor (oracle, FP64).

Follows the paper's orientation module (Architecture section: "chunked 3D
structure tensor pipeline") and Figure 1(b).  Textbook definition used, arrays
in (z, y, x) order with unit isotropic spacing:

* gradient at scale sigma:  g_z = Dz Gy Gx V,  g_y = Gz Dy Gx V,  g_x = Gz Gy Dx V
  (G = normalised Gaussian taps, D = derivative taps, each a 1-D correlation
  along one axis);
* outer product:  P_ab = g_a g_b for ab in (zz, zy, zx, yy, yx, xx);
* integration at scale rho:  S_ab = Gz Gy Gx P_ab with the Gaussian of scale rho.
"""

from __future__ import annotations

import numpy as np

from .filters import correlate_axis, taps

COMPONENTS = ("zz", "zy", "zx", "yy", "yx", "xx")


def gradients(volume, sigma: float, truncate: float = 4.0):
    """Gaussian-derivative gradient (g_z, g_y, g_x) of ``volume`` at scale ``sigma``."""
    v = np.asarray(volume, dtype=np.float64)
    w0, w1 = taps(sigma, truncate)

    def sep(wz, wy, wx):
        return correlate_axis(correlate_axis(correlate_axis(v, wx, 2), wy, 1), wz, 0)

    return sep(w1, w0, w0), sep(w0, w1, w0), sep(w0, w0, w1)


def outer_products(gz, gy, gx):
    """Six unique components of g g^T, stacked (6, ...) in COMPONENTS order."""
    return np.stack([gz * gz, gz * gy, gz * gx, gy * gy, gy * gx, gx * gx])


def integrate(P, rho: float, truncate: float = 4.0):
    """Gaussian integration of each component of ``P`` (6, nz, ny, nx) at scale ``rho``."""
    w0, _ = taps(rho, truncate)
    out = np.empty(np.shape(P), dtype=np.float64)
    for c in range(np.shape(P)[0]):
        out[c] = correlate_axis(correlate_axis(correlate_axis(P[c], w0, 2), w0, 1), w0, 0)
    return out


def structure_tensor(volume, sigma: float, rho: float, truncate: float = 4.0):
    """S (6, nz, ny, nx) float64 in COMPONENTS order."""
    return integrate(outer_products(*gradients(volume, sigma, truncate)), rho, truncate)
