"""The training script's exported weights blob follows the layout the oracle
(and the C ABI) define: PyTorch's replicate-padded Conv3d layers, evaluated in
float64, equal the oracle's 3x3x3 correlation on the unpacked blob (CPU)."""

import numpy as np
import torch

from oracle import surrogate as S
from paper_2508_07476_amd import surrogate_train as T


def test_export_layout_matches_oracle_layers():
    torch.manual_seed(0)
    model = T.build_model(torch).double()
    blob = T.export_blob(model.float())
    assert blob.size == S.n_weights() and blob.dtype == np.float32
    w = S.unpack(blob)
    assert w["in_scale"] == np.float32(T.IN_SCALE) and w["in_offset"] == T.IN_OFFSET
    convs = [m for m in model if isinstance(m, torch.nn.Conv3d)]
    rng = np.random.default_rng(1)
    x = rng.normal(size=(1, 6, 7, 8))
    for layer in range(1, 6):
        c = convs[layer - 1]
        c32 = torch.nn.Conv3d(c.in_channels, 32, 3, padding=1, padding_mode="replicate").double()
        c32.weight.data = torch.from_numpy(w[f"W{layer}"].reshape(32, c.in_channels, 3, 3, 3).copy())
        c32.bias.data = torch.from_numpy(w[f"b{layer}"].copy())
        ref = c32(torch.from_numpy(x)[None])[0].detach().numpy()
        got = S.conv3x3x3(x, w[f"W{layer}"], w[f"b{layer}"])
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
        x = np.maximum(got, 0.0)
    h = convs[5]
    np.testing.assert_array_equal(w["Wh"], h.weight.detach().float().numpy().reshape(5, 32))
