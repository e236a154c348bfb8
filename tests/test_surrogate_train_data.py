"""Host logic of the surrogate's trainer (CPU): the initial blob follows the
layout the oracle and the C ABI define, patch origins hold the weighted
voxels they claim (brute-force count), and the gathered stacks are the
pool's slices with the receptive-radius margin zeroed."""

import numpy as np
import torch

from oracle import surrogate as S
from paper_2508_07476_amd import surrogate_train as T


def test_initial_blob_layout():
    blob = T.init_blob(np.random.default_rng(0))
    assert blob.size == S.n_weights() and blob.dtype == np.float32
    w = S.unpack(blob)
    assert w["in_scale"] == np.float32(T.IN_SCALE) and w["in_offset"] == T.IN_OFFSET
    for layer in range(1, 6):
        cin = 1 if layer == 1 else 32
        assert w[f"W{layer}"].size == 32 * cin * 27
        assert abs(np.std(w[f"W{layer}"]) / np.sqrt(2.0 / (27 * cin)) - 1.0) < 0.15  # He-normal
        assert not np.any(w[f"b{layer}"])
    assert w["Wh"].shape == (5, 32) and not np.any(w["bh"])


def _pool(seed=0, n=3, S_=48):
    g = torch.Generator().manual_seed(seed)
    good = (torch.rand((n, S_, S_, S_), generator=g) < 0.7).to(torch.uint8)
    good[:, :, :, :6] = 0
    return {"vol": torch.randint(-30000, 30000, (n, S_, S_, S_), dtype=torch.int16, generator=g),
            "e3": torch.randn((3, n, S_, S_, S_), generator=g), "fa": torch.rand((n, S_, S_, S_), generator=g),
            "good": good}


def test_patch_origins_count_their_weight():
    pool, P, M = _pool(), 32, T.MARGIN
    o = T.patch_origins(torch, pool, 40, P, 6000, seed=1)
    assert o.shape == (40, 4)
    g = pool["good"]
    for v, z, y, x in o:
        assert int(g[v, z + M:z + P - M, y + M:y + P - M, x + M:x + P - M].sum()) >= 6000
    # one weighted 20^3 block: only origins whose interior [o + 5, o + 27) covers
    # it, o in 13..15 per axis, hold all 8000 voxels
    pool["good"].zero_()
    pool["good"][1, 20:40, 20:40, 20:40] = 1
    o = T.patch_origins(torch, pool, 30, P, 8000, seed=3)
    assert set(o[:, 0].tolist()) == {1}
    assert o[:, 1:].min() >= 13 and o[:, 1:].max() <= 15
    assert len({tuple(r) for r in o[:, 1:].tolist()}) > 5


def test_gather_slices_and_margin():
    pool, P, M = _pool(3), 32, T.MARGIN
    origins = np.array([[0, 1, 2, 3], [2, 16, 0, 16], [1, 8, 8, 8]])
    vol, e3, fa, w = T.Gatherer(torch, pool, P, 3, "cpu")(origins)
    assert vol.dtype == torch.uint16 and vol.shape == (3 * P, P, P)
    for b, (v, z, y, x) in enumerate(origins):
        sl = (slice(z, z + P), slice(y, y + P), slice(x, x + P))
        assert torch.equal(vol[b * P:(b + 1) * P].view(torch.int16), pool["vol"][(v,) + sl])
        assert torch.equal(e3[:, b * P:(b + 1) * P], pool["e3"][(slice(None), v) + sl])
        assert torch.equal(fa[b * P:(b + 1) * P], pool["fa"][(v,) + sl])
        want = pool["good"][(v,) + sl].clone()
        for d in range(3):
            idx = [slice(None)] * 3
            idx[d] = slice(0, M)
            want[tuple(idx)] = 0
            idx[d] = slice(P - M, P)
            want[tuple(idx)] = 0
        assert torch.equal(w[b * P:(b + 1) * P], want)
