"""Pins of the surrogate oracle (CPU): the 3-D correlation against SciPy, the
bfloat16 rounding against PyTorch, hand-built weights with a closed-form output,
and invariances."""

import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

from oracle import surrogate as S


def test_weight_count_and_unpack_layout():
    n = S.n_weights()
    assert n == 2 + 32 * 27 + 32 + 4 * (32 * 32 * 27 + 32) + 5 * 32 + 5
    blob = np.arange(n, dtype=np.float64)
    w = S.unpack(blob)
    assert w["in_scale"] == 0 and w["in_offset"] == 1
    assert w["W1"].shape == (32, 1, 27) and w["W1"][0, 0, 0] == 2 and w["b1"][0] == 2 + 864
    assert w["W2"][0, 0, 0] == 2 + 864 + 32
    assert w["bh"][-1] == n - 1
    with pytest.raises(ValueError):
        S.unpack(blob[:-1])


def test_conv_matches_scipy_correlate_nearest():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(3, 7, 6, 9))
    w = rng.normal(size=(2, 3, 27))
    b = rng.normal(size=2)
    y = S.conv3x3x3(x, w, b)
    for o in range(2):
        ref = np.full(x.shape[1:], b[o])
        for c in range(3):
            ref += ndi.correlate(x[c], w[o, c].reshape(3, 3, 3), mode="nearest")
        np.testing.assert_allclose(y[o], ref, rtol=1e-12, atol=1e-12)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    a = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.uniform(-6, 6, size=5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 65504.0, 3.4e38]])
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(S.bf16(a), ref)


def _identity_blob(scale=1.0 / 1000.0, offset=0.0, head=(1.0, 0.0, 0.0, 1.0, -1.0)):
    """Weights under which channel 0 carries x0 = bf16(v*scale+offset) through every layer
    (centre tap 1, positive inputs survive ReLU) and the head reads it."""
    w = np.zeros(S.n_weights())
    w[0], w[1] = scale, offset
    i = 2
    for layer in range(1, 6):
        cin = 1 if layer == 1 else 32
        W = np.zeros((32, cin, 27))
        W[0, 0, 13] = 1.0  # centre tap
        w[i:i + W.size] = W.ravel()
        i += W.size + 32
    Wh = np.zeros((5, 32))
    Wh[:, 0] = head
    w[i:i + 160] = Wh.ravel()
    return w


def test_identity_network_has_closed_form_outputs():
    rng = np.random.default_rng(2)
    v = rng.integers(1, 60000, size=(5, 6, 7)).astype(np.float64)
    out = S.forward(v, _identity_blob())
    x0 = S.bf16(v / 1000.0)
    np.testing.assert_array_equal(out["e3"][0], 1.0)          # h = (x0, 0, 0): +z
    np.testing.assert_array_equal(out["e3"][1:], 0.0)
    np.testing.assert_allclose(out["fa"], 1.0 / (1.0 + np.exp(-x0)), rtol=1e-15)
    np.testing.assert_allclose(out["confidence"], 1.0 / (1.0 + np.exp(x0)), rtol=1e-15)


def test_negative_head_vector_takes_canonical_sign_and_zero_vector_is_z():
    v = np.full((3, 3, 3), 500.0)
    out = S.forward(v, _identity_blob(head=(-1.0, 0.5, 0.0, 0.0, 0.0)))
    e = np.array([-1.0, 0.5, 0.0]) / np.sqrt(1.25)
    np.testing.assert_allclose(out["e3"][:, 1, 1, 1], -e, rtol=1e-15)
    out0 = S.forward(v, _identity_blob(head=(0.0, 0.0, 0.0, 0.0, 0.0)))
    np.testing.assert_array_equal(out0["e3"][:, 0, 0, 0], [1.0, 0.0, 0.0])


def test_constant_volume_gives_constant_outputs_and_translation_equivariance():
    rng = np.random.default_rng(3)
    blob = rng.normal(size=S.n_weights()) * 0.05
    blob[0], blob[1] = 1e-3, -0.5
    c = S.forward(np.full((6, 5, 4), 1234.0), blob)
    for k in ("fa", "confidence"):
        assert np.ptp(c[k]) == 0.0
    v = rng.uniform(0, 2000, size=(14, 12, 13))
    a = S.forward(v, blob)
    b = S.forward(np.roll(v, 2, axis=2), blob)
    # away from the faces (receptive radius 5) a shifted input shifts the output
    np.testing.assert_array_equal(a["e3"][:, 5:-5, 5:-5, 5:6], b["e3"][:, 5:-5, 5:-5, 7:8])


def test_mask_zeroes_outputs():
    v = np.full((3, 3, 3), 100.0)
    m = np.ones((3, 3, 3), np.uint8)
    m[1, 1, 1] = 0
    out = S.forward(v, _identity_blob(), mask=m)
    assert out["fa"][1, 1, 1] == 0 and out["confidence"][1, 1, 1] == 0
    assert np.all(out["e3"][:, 1, 1, 1] == 0) and out["fa"][0, 0, 0] > 0
