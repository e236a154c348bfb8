"""Per-tile fallback of st_surrogate_infer on the GPU (MI355X only), through the
C ABI.

The mask holds two small boxes of a 96 x 160 x 208 phantom (one inside, one
on three of the volume's faces), so only the tiles that meet them can be
flagged and the crops are much cheaper than the whole volume: the call must
take the crop path (st_surrogate_fallback_info mode 1).  A crop's faces lie
beyond the structure-tensor path's reach or on the volume's faces, so every
voxel that falls back equals st_compute on the whole volume bit for bit (HA
and IA too: the phantom's axis centre is a multiple of 1/2); every other voxel
keeps the surrogate's outputs, bit for bit.  Cases: the fused gradient
(grouped batch), a sigma whose radius needs the three-pass gradient (chains
batch), a threshold that flags nothing, and an unmasked volume with
min_confidence 1 (the whole-volume path).
"""

import sys

import numpy as np
import pytest
import torch

import paper_2508_07476_amd as st
from paper_2508_07476_amd import surrogate_train as T
from phantom import helix

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SHAPE = (96, 160, 208)
OUTS = ("e3", "fa", "ha", "ia")


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def scene():
    spec = helix.PhantomSpec(shape=SHAPE, annuli=(helix.Annulus(30.0, 75.0, 60.0, -50.0),), period=5.0,
                             noise=(0.08,), dtype="u16", seed=21, with_mask=True)
    ph = helix.generate(spec, device=DEV)
    mask = torch.zeros(SHAPE, dtype=torch.uint8, device=DEV)
    mask[40:62, 100:124, 30:70] = 1           # inside
    mask[0:14, 0:20, SHAPE[2] - 18:] = 1       # on the z = 0, y = 0 and last-x faces
    blob = torch.from_numpy(T.init_blob(np.random.default_rng(5))).to(DEV)
    return ph["volume"], mask, blob, ph["center"], ph["direction"]


def _run(vol, mask, blob, center, direction, sigma, rho, thr):
    kw = dict(mask=mask, axis_center=center, axis_direction=direction)
    pure = st.st_surrogate_infer(vol, blob, 0.0, sigma, rho, outputs=OUTS + ("confidence",), **kw)
    mixed = st.st_surrogate_infer(vol, blob, thr, sigma, rho, outputs=OUTS + ("confidence",), **kw)
    info = st.st_surrogate_fallback_info()
    plain = st.st_compute(vol, sigma, rho, outputs=OUTS, **kw)
    torch.cuda.synchronize()
    return pure, mixed, plain, info


def _expect(pure, mixed, plain, mask, thr):
    inside = torch.ones(SHAPE, dtype=torch.bool, device=DEV) if mask is None else mask != 0
    low = inside & (pure["confidence"] < thr)
    keep = ~low
    for k in OUTS:
        lo, kp = (low, keep) if k != "e3" else (low.expand(3, -1, -1, -1), keep.expand(3, -1, -1, -1))
        assert torch.equal(mixed[k][lo], plain[k][lo]), k
        assert torch.equal(mixed[k][kp], pure[k][kp]), k
    assert torch.equal(mixed["confidence"], pure["confidence"])
    return int(low.sum()), int(inside.sum())


@pytest.mark.parametrize("sigma,rho", [(1.5, 4.0), (2.6, 3.0)])
def test_crops_match_the_whole_volume_path(scene, sigma, rho):
    vol, mask, blob, center, direction = scene
    _log(f"case: tile fallback sigma {sigma} rho {rho}")
    pure = st.st_surrogate_infer(vol, blob, 0.0, sigma, rho, mask=mask, outputs=("confidence",))
    thr = float(torch.quantile(pure["confidence"][mask != 0].float(), 0.5))
    pure, mixed, plain, info = _run(vol, mask, blob, center, direction, sigma, rho, thr)
    nlow, nin = _expect(pure, mixed, plain, mask, thr)
    _log(f"  {info}, {nlow} of {nin} masked voxels fell back")
    assert info["mode"] == 1 and info["tiles"] >= 2, info
    assert 0 < info["voxels"] < vol.numel(), info
    assert 0 < nlow < nin


def test_nothing_flagged_keeps_the_surrogate(scene):
    vol, mask, blob, center, direction = scene
    _log("case: tile fallback, threshold below every confidence")
    pure = st.st_surrogate_infer(vol, blob, 0.0, mask=mask, outputs=("confidence",))
    thr = float(pure["confidence"][mask != 0].min()) * 0.5
    if not thr > 0.0:
        pytest.skip("a masked confidence is exactly 0")
    pure, mixed, plain, info = _run(vol, mask, blob, center, direction, 1.5, 4.0, thr)
    assert info["mode"] == 0, info
    assert _expect(pure, mixed, plain, mask, thr)[0] == 0


def test_every_voxel_takes_the_whole_volume_path(scene):
    vol, _, blob, center, direction = scene
    _log("case: tile fallback, no mask, min_confidence 1")
    pure, mixed, plain, info = _run(vol, None, blob, center, direction, 1.5, 4.0, 1.0)
    nlow, nin = _expect(pure, mixed, plain, None, 1.0)
    _log(f"  {info}, {nlow} of {nin} voxels fell back")
    assert info["mode"] == 2 and info["voxels"] == vol.numel(), info


def test_streamed_whole_volume_fallback_matches(scene, monkeypatch):
    """A whole-volume fallback streamed in z slabs through small activation
    buffers (forced with ST_SURROGATE_SLAB_BYTES: 24-plane buffers, about 40
    planes of the path per slab, 16 of them its own at sigma 1, rho 2) gives
    st_compute's outputs bit for bit."""
    vol, _, blob, center, direction = scene
    monkeypatch.setenv("ST_SURROGATE_SLAB_BYTES", str(2 * 24 * SHAPE[1] * SHAPE[2] * 64))
    _log("case: streamed whole-volume fallback, sigma 1, rho 2")
    pure, mixed, plain, info = _run(vol, None, blob, center, direction, 1.0, 2.0, 1.0)
    nlow, nin = _expect(pure, mixed, plain, None, 1.0)
    _log(f"  {info}, {nlow} of {nin} voxels fell back")
    assert info["mode"] == 2 and nlow > nin // 2, info
