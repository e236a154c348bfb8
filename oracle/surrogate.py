"""Oracle of the learned orientation surrogate: a dense 3-D CNN that maps
intensities to a fibre direction, an FA estimate and a confidence per voxel.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The surrogate is not a method of the paper: it is a learned approximation of
the orientation output of the structure-tensor path (Figure 1(b)).  This
module writes its forward pass out directly, in float64, with the network's
storage rounding made explicit so that the GPU path can be compared with it
element by element:

  x0 = bf16(v * in_scale + in_offset)
  x_l = relu(b_l + sum_{c, t} W_l[:, c, t] * x_{l-1}[c, p + off(t)])   l = 1..5
        (3x3x3 correlation, index clamped at every face), rounded to bf16 for
        l < 5; the weights are rounded to bf16; the last layer stays unrounded
  h = bh + Wh x_5
  e3 = h[0:3] / |h[0:3]| with the canonical sign (largest |component|
       positive, ties to z then y); (1, 0, 0) when h[0:3] = 0
  FA = sigmoid(h[3]); confidence = sigmoid(h[4])

Weights blob (float32, in this order): in_scale, in_offset; W1 [32][1][27],
b1 [32]; W2..W5 [32][32][27], b [32] each; Wh [5][32], bh [5].  Tap
t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1).

Pinned by tests/test_oracle_surrogate.py: the 3-D correlation against
scipy.ndimage.correlate (mode "nearest"), the bf16 rounding against PyTorch's
bfloat16 conversion, hand-built weights whose output has a closed form, and
constant-volume / translation invariances.
"""

from __future__ import annotations

import numpy as np

CHANNELS = 32
LAYERS = 5
HEAD = 5


def n_weights() -> int:
    n = 2 + CHANNELS * 27 + CHANNELS
    n += (LAYERS - 1) * (CHANNELS * CHANNELS * 27 + CHANNELS)
    n += HEAD * CHANNELS + HEAD
    return n


def unpack(blob) -> dict:
    """Split a weights blob into named float64 arrays."""
    b = np.asarray(blob, dtype=np.float64).ravel()
    if b.size != n_weights():
        raise ValueError(f"weights blob has {b.size} values, expected {n_weights()}")
    out = {"in_scale": b[0], "in_offset": b[1]}
    i = 2
    for layer in range(1, LAYERS + 1):
        cin = 1 if layer == 1 else CHANNELS
        n = CHANNELS * cin * 27
        out[f"W{layer}"] = b[i:i + n].reshape(CHANNELS, cin, 27)
        i += n
        out[f"b{layer}"] = b[i:i + CHANNELS]
        i += CHANNELS
    out["Wh"] = b[i:i + HEAD * CHANNELS].reshape(HEAD, CHANNELS)
    i += HEAD * CHANNELS
    out["bh"] = b[i:i + HEAD]
    return out


def bf16(a):
    """Round float values to the nearest bfloat16 (ties to even), returned as float64.

    bfloat16 keeps the top 16 bits of an IEEE float32; the value is first
    rounded to float32 (the GPU holds it in float32 before the conversion)."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def conv3x3x3(x, w, b):
    """y[o, p] = b[o] + sum_{c, t} w[o, c, t] x[c, clamp(p + off(t))] for x (C, Z, Y, X)."""
    x = np.asarray(x, dtype=np.float64)
    cin = x.shape[0]
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1)), mode="edge")
    Z, Y, X = x.shape[1:]
    y = np.empty((w.shape[0], Z, Y, X))
    y[:] = np.asarray(b, dtype=np.float64)[:, None, None, None]
    for t in range(27):
        dz, dy, dx = t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1
        sh = xp[:, 1 + dz:1 + dz + Z, 1 + dy:1 + dy + Y, 1 + dx:1 + dx + X]
        # (O, C) x (C, Z*Y*X)
        y += (w[:, :, t] @ sh.reshape(cin, -1)).reshape(y.shape)
    return y


def canonical(v):
    """Largest-|component| entry positive, ties to the lower axis (z, then y)."""
    a = np.abs(v)
    lead = np.where((a[0] >= a[1]) & (a[0] >= a[2]), v[0], np.where(a[1] >= a[2], v[1], v[2]))
    return np.where(lead < 0, -v, v)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(volume, blob, mask=None):
    """Surrogate outputs for a (Z, Y, X) volume: e3 (3, Z, Y, X), fa, confidence
    (zeros outside a given mask)."""
    w = unpack(blob)
    v = np.asarray(volume, dtype=np.float64)
    x = bf16(v * w["in_scale"] + w["in_offset"])[None]
    for layer in range(1, LAYERS + 1):
        y = np.maximum(conv3x3x3(x, bf16(w[f"W{layer}"]), w[f"b{layer}"]), 0.0)
        x = bf16(y) if layer < LAYERS else y
    h = np.einsum("oc,czyx->ozyx", w["Wh"], x) + w["bh"][:, None, None, None]
    u = h[:3]
    n = np.sqrt((u * u).sum(0))
    e3 = np.where(n > 0, u / np.where(n > 0, n, 1.0), np.array([1.0, 0.0, 0.0])[:, None, None, None])
    e3 = canonical(e3)
    fa = sigmoid(h[3])
    conf = sigmoid(h[4])
    if mask is not None:
        out = np.asarray(mask) == 0
        e3 = np.where(out[None], 0.0, e3)
        fa = np.where(out, 0.0, fa)
        conf = np.where(out, 0.0, conf)
    return {"e3": e3, "fa": fa, "confidence": conf}
