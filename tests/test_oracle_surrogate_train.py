"""Pins of the surrogate's training objective and its gradient in the oracle
(CPU): the adjoint identities of the clamped 3-D correlation, central finite
differences of the objective in every layer, the direction term's sign
invariance, and a constant network whose losses and gradient have closed
forms."""

import numpy as np
import pytest

from oracle import surrogate as S


def _blob(rng, scale=0.08):
    b = rng.normal(scale=scale, size=S.n_weights())
    b[0], b[1] = 1.0 / 1000.0, -0.5
    return b


def _batch(rng, B=1, P=12, margin=5):
    pt = rng.uniform(0, 1000, size=(B, P, P, P))
    t = rng.normal(size=(B, 3, P, P, P))
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    fa = rng.uniform(0.1, 0.9, size=(B, P, P, P))
    wt = np.zeros((B, P, P, P))
    wt[:, margin:P - margin, margin:P - margin, margin:P - margin] = 1.0
    return pt, t, fa, wt


def test_conv_backward_is_the_adjoint_of_the_clamped_correlation():
    # y = conv(x, w, 0) is linear in x and in w: <g, y> = <dx, x> = <dw, w>
    rng = np.random.default_rng(3)
    x = rng.normal(size=(3, 5, 6, 4))
    w = rng.normal(size=(2, 3, 27))
    g = rng.normal(size=(2, 5, 6, 4))
    y = S.conv3x3x3(x, w, np.zeros(2))
    dx, dw, db = S.conv3x3x3_backward(g, x, w)
    ref = float((g * y).sum())
    assert abs(float((dx * x).sum()) - ref) <= 1e-10 * abs(ref)
    assert abs(float((dw * w).sum()) - ref) <= 1e-10 * abs(ref)
    np.testing.assert_allclose(db, g.sum(axis=(1, 2, 3)), rtol=1e-13)
    # the face voxels receive the gradient of the taps clamped onto them
    g1 = np.zeros((1, 1, 1, 3))
    g1[0, 0, 0, 0] = 1.0
    x1 = np.zeros((1, 1, 1, 3))
    w1 = np.zeros((1, 1, 27))
    w1[0, 0, :] = 1.0  # every tap reads a clamped neighbour of voxel 0 or itself
    dx1, _, _ = S.conv3x3x3_backward(g1, x1, w1)
    assert dx1[0, 0, 0, 0] == 18.0 and dx1[0, 0, 0, 1] == 9.0 and dx1[0, 0, 0, 2] == 0.0


def test_gradient_matches_central_differences_in_every_layer():
    rng = np.random.default_rng(11)
    blob = _blob(rng)
    pt, t, fa, wt = _batch(rng)
    o = S.train_loss_grad(blob, pt, t, fa, wt, round_bf16=False)
    # a few coordinates of every weight group: W1..W5, b1..b5, Wh, bh
    off = [2, 2 + 864, 2 + 864 + 32]
    for _ in range(3):
        off.append(off[-1] + 32 * 32 * 27)
        off.append(off[-1] + 32)
    idx = []
    for a in range(len(off)):
        lo = off[a]
        hi = off[a + 1] if a + 1 < len(off) else S.n_weights()
        idx += list(rng.integers(lo, hi, size=2))
    idx += [S.n_weights() - 5 * 32 - 5 + 3, S.n_weights() - 1, S.n_weights() - 3]
    eps = 1e-6
    for i in idx:
        bp, bm = blob.copy(), blob.copy()
        bp[i] += eps
        bm[i] -= eps
        fd = (S.train_loss_grad(bp, pt, t, fa, wt, round_bf16=False)["loss"] -
              S.train_loss_grad(bm, pt, t, fa, wt, round_bf16=False)["loss"]) / (2 * eps)
        assert abs(fd - o["grad"][i]) <= 2e-5 * max(1e-3, abs(fd)), (i, fd, o["grad"][i])
    assert o["grad"][0] == 0 and o["grad"][1] == 0


def test_direction_loss_is_sign_invariant():
    rng = np.random.default_rng(5)
    blob = _blob(rng)
    pt, t, fa, wt = _batch(rng)
    a = S.train_loss_grad(blob, pt, t, fa, wt)
    b = S.train_loss_grad(blob, pt, -t, fa, wt)
    assert a["loss"] == pytest.approx(b["loss"], rel=1e-12)
    np.testing.assert_allclose(a["grad"], b["grad"], rtol=1e-10, atol=1e-14)


def test_constant_network_closed_form():
    # all convolution weights zero: x5 = relu(b5), h = Wh relu(b5) + bh = bh;
    # with bh[0:3] = the (uniform) label direction and sigmoid(bh[3]) = label FA,
    # l_dir = l_fa = 0, the angle is 0 (c = 1), l_conf = log(1 + exp(-bh[4])),
    # and the only non-zero gradient entries are those of h[4]
    P = 12
    blob = np.zeros(S.n_weights())
    blob[0], blob[1] = 1e-3, 0.0
    n = S.n_weights()
    t_dir = np.array([0.48, 0.6, 0.64])
    fa_val = 0.3
    bh = np.array([*t_dir, np.log(fa_val / (1 - fa_val)), 1.5])
    blob[n - 5:] = bh
    pt = np.zeros((1, P, P, P))
    t = np.broadcast_to(t_dir[None, :, None, None, None], (1, 3, P, P, P)).copy()
    fa = np.full((1, P, P, P), fa_val)
    wt = np.zeros((1, P, P, P))
    wt[:, 5:7, 5:7, 5:7] = 1.0
    o = S.train_loss_grad(blob, pt, t, fa, wt, round_bf16=False)
    assert o["loss_dir"] == pytest.approx(0.0, abs=1e-15)
    assert o["loss_fa"] == pytest.approx(0.0, abs=1e-15)
    assert o["loss_conf"] == pytest.approx(np.log1p(np.exp(-1.5)), rel=1e-12)
    assert o["within"] == 8.0 and o["wsum"] == 8.0
    g = o["grad"]
    assert g[n - 1] == pytest.approx(S.W_CONF * (1 / (1 + np.exp(-1.5)) - 1.0), rel=1e-12)
    # x5 = relu(b5) = 0, so the head weights and every earlier layer get nothing;
    # the FA entry is zero up to the rounding of sigmoid(logit(0.3))
    assert np.abs(g[:n - 1]).max() <= 1e-15
    # the confidence term's weight scales its gradient and its share of L only
    o3 = S.train_loss_grad(blob, pt, t, fa, wt, round_bf16=False, conf_weight=0.7)
    assert o3["grad"][n - 1] == pytest.approx(0.7 * (1 / (1 + np.exp(-1.5)) - 1.0), rel=1e-12)
    assert o3["loss"] == pytest.approx(0.7 * np.log1p(np.exp(-1.5)), rel=1e-12)
    assert o3["loss_conf"] == o["loss_conf"]


def test_confidence_weight_splits_the_gradient_linearly():
    # the gradient is linear in the confidence term's weight: the part of every
    # parameter's gradient that comes from l_conf scales with it, the rest stays
    rng = np.random.default_rng(9)
    blob = _blob(rng)
    pt, t, fa, wt = _batch(rng, B=1, P=12)
    g = {cw: S.train_loss_grad(blob, pt, t, fa, wt, round_bf16=False, conf_weight=cw)["grad"]
         for cw in (0.0, 0.1, 1.0)}
    np.testing.assert_allclose(g[1.0] - g[0.0], 10.0 * (g[0.1] - g[0.0]), rtol=1e-9, atol=1e-14)
    assert np.abs(g[1.0] - g[0.0]).max() > 0
