"""Sampled Gaussian filters and the reflect boundary (oracle, FP64, test infrastructure).

The paper computes the structure tensor from image intensity gradients
(Statement of Need; Implementation section, which delegates the tensor to a
structure-tensor library) without writing the filters down.  Reading taken:

* sampled Gaussian of scale ``s`` truncated at ``R = floor(truncate * s + 0.5)``
  and normalised to unit sum:  ``w0(k) = exp(-k^2 / (2 s^2)) / sum_j exp(-j^2 / (2 s^2))``;
* derivative taps ``w1(k) = (k / s^2) w0(k)``, applied as *correlation*, so the
  result approximates ``+d/dn`` of the Gaussian-smoothed signal;
* half-sample symmetric reflection at every face: ``-1 -> 0``, ``n -> n-1``,
  folded with period ``2n`` when ``R >= n``.
"""

from __future__ import annotations

import math

import numpy as np


def radius(scale: float, truncate: float = 4.0) -> int:
    """Half-width of the truncated kernel: floor(truncate * scale + 0.5)."""
    return int(math.floor(truncate * scale + 0.5))


def taps(scale: float, truncate: float = 4.0):
    """Return (w0, w1), each of length 2R+1, index m <-> offset k = m - R."""
    R = radius(scale, truncate)
    k = np.arange(-R, R + 1, dtype=np.float64)
    g = np.exp(-(k * k) / (2.0 * scale * scale))
    w0 = g / g.sum()
    w1 = (k / (scale * scale)) * w0
    return w0, w1


def reflect_index(idx, n: int):
    """Map any integer index to [0, n) by half-sample symmetric reflection."""
    idx = np.asarray(idx, dtype=np.int64)
    m = np.mod(idx, 2 * n)
    return np.where(m < n, m, 2 * n - 1 - m)


def correlate_axis(f, w, axis: int):
    """out[i] = sum_{k=-R..R} w[k+R] * f[reflect(i+k)] along ``axis`` (k ascending)."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[axis]
    R = (len(w) - 1) // 2
    base = np.arange(n)
    out = np.zeros(f.shape, dtype=np.float64)
    for m, wk in enumerate(w):
        out += wk * np.take(f, reflect_index(base + (m - R), n), axis=axis)
    return out
