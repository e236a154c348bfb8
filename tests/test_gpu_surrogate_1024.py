"""The learned surrogate at its full size (MI355X only): st_surrogate_infer on
the 1024^3 uint16 surrogate volume with the shipped weights, min_confidence
0.9, sigma 1, rho 2 (the scales of the weights' training labels).

- Every voxel inside the mask whose confidence is below 0.9 must equal
  st_compute on the whole volume bit for bit (e3, FA, HA, IA): the fallback
  runs the structure-tensor path on crops whose faces lie beyond its reach.
- Every other voxel keeps the surrogate's outputs; on three sampled 16^3
  blocks (one on the z = 0 face, one mid-volume, one on the last plane across
  the outer wall) those match the FP64 oracle forward pass, evaluated on the
  block with the network's 5 voxels of context (clipped at the volume's faces,
  where both sides clamp), to the tolerance of the small-volume surrogate
  tests.
"""

import os
import sys

import numpy as np
import pytest
import torch

import paper_2508_07476_amd as st
from oracle import surrogate as S
from phantom import helix

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
N = 1024
SIGMA, RHO, THR = 1.0, 2.0, 0.9
CTX = 5  # receptive radius of the network
E3_MAX, SCALAR_MAX = 5e-2, 1e-2  # as the small-volume surrogate tests' per-voxel bounds
WEIGHTS = os.path.join(os.path.dirname(st.__file__), "surrogate_weights.npy")
BLOCKS = [(0, 504, 806), (500, 200, 504), (N - 16, 504, 944)]  # (z, y, x) origins of 16^3 blocks


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _angle(a, b):
    c = np.cross(a, b, axis=0)
    return np.arctan2(np.linalg.norm(c, axis=0), np.abs((a * b).sum(0)))


@pytest.fixture(scope="module")
def run():
    _log("case: surrogate 1024^3, min_confidence 0.9")
    ph = helix.generate(helix.spec_surrogate_u16(shape=(N, N, N)), device=DEV)
    vol, mask = ph["volume"], ph["mask"]
    blob = np.load(WEIGHTS, allow_pickle=False).astype(np.float32)
    kw = dict(mask=mask, axis_center=ph["center"], axis_direction=ph["direction"])
    outs = ("e3", "fa", "ha", "ia")
    got = st.st_surrogate_infer(vol, torch.from_numpy(blob).to(DEV), THR, SIGMA, RHO,
                                outputs=outs + ("confidence",), **kw)
    info = st.st_surrogate_fallback_info()
    torch.cuda.synchronize()
    _log("  fallback:", info)
    return ph, vol, mask, blob, kw, got, info


def test_fallen_back_voxels_equal_the_plain_path(run):
    ph, vol, mask, blob, kw, got, info = run
    low = (mask != 0) & (got["confidence"] < THR)
    nlow, nin = int(low.sum()), int((mask != 0).sum())
    _log(f"  {nlow} of {nin} masked voxels fell back ({nlow / nin:.3f})")
    assert info["mode"] in (1, 2) and nlow > 0
    plain = st.st_compute(vol, SIGMA, RHO, outputs=("e3", "fa", "ha", "ia"), **kw)
    torch.cuda.synchronize()
    for k in ("fa", "ha", "ia"):
        assert not bool(((got[k] != plain[k]) & low).any()), k
    for c in range(3):
        assert not bool(((got["e3"][c] != plain["e3"][c]) & low).any()), ("e3", c)
    del plain
    torch.cuda.empty_cache()


@pytest.mark.parametrize("origin", BLOCKS)
def test_surrogate_voxels_match_the_oracle(run, origin):
    ph, vol, mask, blob, kw, got, info = run
    z, y, x = origin
    lo = [max(0, c - CTX) for c in origin]
    hi = [min(N, c + 16 + CTX) for c in origin]
    crop = vol[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]].cpu().numpy()
    o = S.forward(crop.astype(np.float64), blob.astype(np.float64), None)
    sl = (slice(z - lo[0], z - lo[0] + 16), slice(y - lo[1], y - lo[1] + 16), slice(x - lo[2], x - lo[2] + 16))
    blk = (slice(z, z + 16), slice(y, y + 16), slice(x, x + 16))
    m = mask[blk].cpu().numpy() != 0
    conf = got["confidence"][blk].cpu().numpy()
    keep = m & ~(conf < THR)
    g_e3 = got["e3"][(slice(None),) + blk].cpu().numpy().astype(np.float64)
    g_fa = got["fa"][blk].cpu().numpy().astype(np.float64)
    o_e3, o_fa, o_cf = o["e3"][(slice(None),) + sl], o["fa"][sl], o["confidence"][sl]
    dc = np.abs(conf.astype(np.float64) - o_cf)[m]
    _log(f"  block {origin}: {int(m.sum())} masked, {int(keep.sum())} kept; conf max diff "
         f"{dc.max() if dc.size else 0:.2e}")
    assert m.sum() > 0
    if dc.size:
        assert dc.max() <= SCALAR_MAX
    if keep.any():
        ea = _angle(g_e3[:, keep], o_e3[:, keep])
        fa = np.abs(g_fa - o_fa)[keep]
        _log(f"    e3 max {ea.max():.2e} rad, fa max {fa.max():.2e}")
        assert ea.max() <= E3_MAX and fa.max() <= SCALAR_MAX
