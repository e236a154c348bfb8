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


# ---- training objective and its gradient -------------------------------------
#
# The surrogate is trained on patches of phantoms labelled by the structure-
# tensor path.  Per voxel, with u = h[0:3] / |h[0:3]|, label direction t, label
# FA f and loss weight w (1 where the loss applies, else 0):
#   l_dir  = 1 - (u . t)^2                      (invariant under u -> -u, t -> -t)
#   l_fa   = (sigmoid(h[3]) - f)^2
#   l_conf = softplus(h[4]) - c h[4],  c = [angle(u, t) < CONF_DEG]  (c is a target, not differentiated)
#   L = sum_v w (l_dir + l_fa + conf_weight l_conf) / sum_v w   (W_CONF by default)
# Training rounds every stored activation to bf16, x_5 included (inference
# keeps x_5 in float32), and the backward pass rounds each stored gradient
# dL/d(pre-activation) to bf16; the weights enter both passes rounded to bf16
# and are updated in float32.  Gradients are accumulated unnormalised and
# divided by sum_v w at the end.

CONF_DEG = 2.0
W_CONF = 0.1


def conv3x3x3_backward(g, x, w):
    """Gradients of y = conv3x3x3(x, w, b) (indices clamped at every face) for an
    upstream gradient g (O, Z, Y, X): returns (dx, dw, db).  A clamped tap
    passes its gradient to the face voxel it read."""
    x = np.asarray(x, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    cin, (Z, Y, X) = x.shape[0], x.shape[1:]
    o = g.shape[0]
    dx = np.zeros_like(x)
    dw = np.zeros((o, cin, 27))
    g2 = g.reshape(o, -1)
    for t in range(27):
        dz, dy, ddx = t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1
        iz = np.clip(np.arange(Z) + dz, 0, Z - 1)
        iy = np.clip(np.arange(Y) + dy, 0, Y - 1)
        ix = np.clip(np.arange(X) + ddx, 0, X - 1)
        sh = x[:, iz][:, :, iy][:, :, :, ix]
        dw[:, :, t] = g2 @ sh.reshape(cin, -1).T
        contrib = (w[:, :, t].T @ g2).reshape(cin, Z, Y, X)
        np.add.at(dx, (slice(None), iz[:, None, None], iy[None, :, None], ix[None, None, :]), contrib)
    return dx, dw, g2.sum(axis=1)


def train_loss_grad(blob, patches, target_e3, target_fa, weight, round_bf16=True, conf_weight=W_CONF):
    """Training objective (see above) over patches (B, P, P, P) of raw
    intensities, with label directions target_e3 (B, 3, P, P, P), label FA
    (B, P, P, P) and loss weights (B, P, P, P).  Each patch is its own volume.
    Returns the losses, sum_v w, the number of weighted voxels within
    CONF_DEG, and the gradient of L in the blob layout (zero for in_scale and
    in_offset, which are not trained)."""
    w = unpack(blob)
    r = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    names = [f"W{l}" for l in range(1, LAYERS + 1)] + [f"b{l}" for l in range(1, LAYERS + 1)] + ["Wh", "bh"]
    grad = {k: np.zeros_like(w[k]) for k in names}
    tot = {"dir": 0.0, "fa": 0.0, "conf": 0.0, "wsum": 0.0, "within": 0.0}
    wr = {l: r(w[f"W{l}"]) for l in range(1, LAYERS + 1)}
    for b in range(patches.shape[0]):
        v = np.asarray(patches[b], dtype=np.float64)
        xs = [r(v * w["in_scale"] + w["in_offset"])[None]]
        for layer in range(1, LAYERS + 1):
            xs.append(r(np.maximum(conv3x3x3(xs[-1], wr[layer], w[f"b{layer}"]), 0.0)))
        x5 = xs[-1]
        h = np.einsum("oc,czyx->ozyx", w["Wh"], x5) + w["bh"][:, None, None, None]
        wt = np.asarray(weight[b], dtype=np.float64)
        t = np.asarray(target_e3[b], dtype=np.float64)
        nrm = np.sqrt((h[:3] ** 2).sum(0))
        safe = np.where(nrm > 0, nrm, 1.0)
        u = h[:3] / safe
        dot = (u * t).sum(0)
        l_dir = 1.0 - dot * dot
        s3 = sigmoid(h[3])
        l_fa = (s3 - target_fa[b]) ** 2
        cross = np.sqrt(((np.cross(u, t, axis=0)) ** 2).sum(0))
        ang = np.degrees(np.arctan2(cross, np.abs(dot)))
        c = (ang < CONF_DEG).astype(np.float64)
        l_conf = np.logaddexp(0.0, h[4]) - c * h[4]
        tot["dir"] += float((wt * l_dir).sum())
        tot["fa"] += float((wt * l_fa).sum())
        tot["conf"] += float((wt * l_conf).sum())
        tot["wsum"] += float(wt.sum())
        tot["within"] += float((wt * c).sum())
        dh = np.empty_like(h)
        dh[:3] = wt * (-2.0 * dot) * (t - dot * u) / safe
        dh[3] = wt * 2.0 * (s3 - target_fa[b]) * s3 * (1.0 - s3)
        dh[4] = wt * conf_weight * (sigmoid(h[4]) - c)
        grad["Wh"] += np.einsum("ozyx,czyx->oc", dh, x5)
        grad["bh"] += dh.sum(axis=(1, 2, 3))
        g = r(np.einsum("oc,ozyx->czyx", w["Wh"], dh) * (x5 > 0))
        for layer in range(LAYERS, 0, -1):
            dx, dw, db = conv3x3x3_backward(g, xs[layer - 1], wr[layer])
            grad[f"W{layer}"] += dw
            grad[f"b{layer}"] += db
            if layer > 1:
                g = r(dx * (xs[layer - 1] > 0))
    ws = max(tot["wsum"], 1e-300)
    flat = [np.zeros(2)]
    for layer in range(1, LAYERS + 1):
        flat += [grad[f"W{layer}"].ravel() / ws, grad[f"b{layer}"] / ws]
    flat += [grad["Wh"].ravel() / ws, grad["bh"] / ws]
    return {"loss_dir": tot["dir"] / ws, "loss_fa": tot["fa"] / ws, "loss_conf": tot["conf"] / ws,
            "loss": (tot["dir"] + tot["fa"] + conf_weight * tot["conf"]) / ws, "wsum": tot["wsum"],
            "within": tot["within"], "grad": np.concatenate(flat)}
