"""The method's special inputs on the HIP path (MI355X only), each checked on
what the mathematics fixes and, where the answer is unique, against the oracle.

- A constant volume: the tensor is zero up to rounding, every voxel degenerate.
- A ramp along x: S is rank one (only S_xx survives), so FA = 1, lambda2 =
  lambda3 = 0 and e3 is any unit vector normal to x: the unique parts are
  compared (FA, lambda1, e3 . x = 0, the degeneracy flag), not e3 itself.
- sin(a z) + sin(b y): the gradient has no x component, so e3 = x exactly.
- Voxels lying exactly on the axis (straight and tilted): the on-axis flag,
  HA = IA = 0, bit for bit with the oracle.
- An all-zero mask: every output zero, every voxel flagged outside.
- Scaling the volume by 2^10 scales every intermediate by a power of two,
  which binary floating point does exactly (no overflow or underflow here):
  e3, FA, HA, IA and the flags are bitwise unchanged and the eigenvalues scale.
"""

import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2508_07476_amd as st
from phantom import helix

from _parity import angle_between, assert_parity, compare, summary

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
ALL = ("e3", "evals", "fa", "ha", "ia", "flags")


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _gpu(vol_cpu, sigma, rho, mask_cpu=None, center=None, direction=None, outputs=ALL):
    if center is None:
        outputs = tuple(k for k in outputs if k not in ("ha", "ia"))
    g = st.st_compute(vol_cpu.to(DEV), sigma, rho, mask=None if mask_cpu is None else mask_cpu.to(DEV),
                      axis_center=center, axis_direction=direction, outputs=outputs)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in g.items()}


def test_constant_volume_is_degenerate_everywhere():
    _log("case: constant u16 volume (12, 20, 70) sigma=1 rho=2")
    vol = torch.full((12, 20, 70), 1234, dtype=torch.int32).to(torch.uint16)
    center, direction = (5.5, 9.5, 34.5), (1.0, 0.0, 0.0)
    g = _gpu(vol, 1.0, 2.0, center=center, direction=direction)
    o = oracle.compute(vol.numpy(), None, 1.0, 2.0, axis_center=center, axis_direction=direction)
    assert np.all(o["flags"] & oracle.FLAG_DEGENERATE)  # the oracle agrees with the rule
    assert np.all(g["flags"] & st.ST_FLAG_DEGENERATE)
    assert np.all((g["flags"] & ~np.uint8(st.ST_FLAG_DEGENERATE)) == 0)
    # whatever rounding leaves is a valid unit vector, an FA in [0, 1] and angles in range
    assert np.abs(np.linalg.norm(g["e3"].astype(np.float64), axis=0) - 1).max() < 1e-5
    assert g["fa"].min() >= 0 and g["fa"].max() <= 1
    assert np.abs(g["ha"]).max() <= np.pi / 2 + 1e-6 and np.abs(g["ia"]).max() <= np.pi / 2 + 1e-6
    # the tensor vanishes against the input scale
    assert np.abs(g["evals"]).max() <= 1e-12 * 1234.0 ** 2


def test_ramp_is_rank_one():
    _log("case: f32 ramp 100 + 7x, (12, 20, 90) sigma=1 rho=2")
    x = torch.arange(90, dtype=torch.float64)
    vol = (100 + 7 * x).expand(12, 20, 90).to(torch.float32).contiguous()
    g = _gpu(vol, 1.0, 2.0)
    o = oracle.compute(vol.numpy(), None, 1.0, 2.0)
    h = oracle.radius(1.0) + oracle.radius(2.0)
    inner = (slice(None), slice(None), slice(h, 90 - h))  # x faces bend the ramp by reflection
    l1_o = o["evals"][0][inner]
    # the oracle: rank one, FA 1, e3 normal to x
    assert np.abs(o["evals"][1:][(slice(None),) + inner]).max() <= 1e-9 * l1_o.max()
    assert np.abs(o["fa"][inner] - 1).max() < 1e-9
    assert np.abs(o["e3"][2][inner]).max() < 1e-9
    # the HIP path: the same unique parts
    assert np.all(g["flags"][inner] & st.ST_FLAG_DEGENERATE)
    assert np.abs(g["fa"][inner] - 1).max() < 1e-4
    assert np.abs(g["e3"][2][inner]).max() < 1e-3
    assert np.abs(np.linalg.norm(g["e3"][(slice(None),) + inner].astype(np.float64), axis=0) - 1).max() < 1e-5
    assert np.abs(g["evals"][0][inner] / l1_o - 1).max() < 1e-5
    assert np.abs(g["evals"][1:][(slice(None),) + inner]).max() <= 1e-6 * l1_o.max()


def test_two_axis_texture_has_fibre_along_x():
    _log("case: f32 sin(0.7 z) + sin(0.45 y), (30, 40, 70) sigma=1 rho=2, tilted axis")
    z = torch.arange(30, dtype=torch.float64)[:, None, None]
    y = torch.arange(40, dtype=torch.float64)[None, :, None]
    vol = (torch.sin(0.7 * z) + torch.sin(0.45 * y)).expand(30, 40, 70).to(torch.float32).contiguous()
    center, direction = (14.3, 19.6, 35.2), (1.0, 0.2, -0.3)
    g = _gpu(vol, 1.0, 2.0, center=center, direction=direction)
    o = oracle.compute(vol.numpy(), None, 1.0, 2.0, axis_center=center, axis_direction=direction)
    stats = compare(g, o, vol.shape, center, direction)
    _log(summary(stats))
    assert stats["n_checked"] > 0.5 * stats["n"]
    assert_parity(stats, "sin z + sin y")
    sel = o["gap"] >= oracle.DEGENERATE_GAP
    xhat = np.zeros((3,) + vol.shape)
    xhat[2] = 1.0
    assert angle_between(o["e3"][:, sel], xhat[:, sel]).max() < 1e-9  # the oracle finds x
    assert angle_between(g["e3"][:, sel].astype(np.float64), xhat[:, sel]).max() < 1e-5
    assert np.all(g["e3"][2][sel] > 0)  # canonical sign: the largest component positive


@pytest.mark.parametrize("direction", [(1.0, 0.0, 0.0), (1.0, 1.0, 0.0)])
def test_voxels_on_the_axis(direction):
    _log(f"case: 64^3 f32 phantom, axis through voxel centres, direction {direction}")
    spec = helix.spec_small_f32()
    vol = helix.generate(spec)["volume"]
    center = (32.0, 32.0, 32.0)
    g = _gpu(vol, 1.0, 3.0, center=center, direction=direction)
    o = oracle.compute(vol.numpy(), None, 1.0, 3.0, axis_center=center, axis_direction=direction)
    on_o = (o["flags"] & oracle.FLAG_ON_AXIS) != 0
    assert on_o.sum() >= 32  # the axis passes through voxel centres
    on_g = (g["flags"] & st.ST_FLAG_ON_AXIS) != 0
    assert np.array_equal(on_g, on_o)
    assert np.all(g["ha"][on_g] == 0) and np.all(g["ia"][on_g] == 0)
    stats = compare(g, o, vol.shape, center, direction)
    _log(summary(stats))
    assert_parity(stats, f"axis {direction}")


def test_all_zero_mask():
    _log("case: f32 random (9, 17, 66), mask all zero")
    gen = torch.Generator().manual_seed(5)
    vol = torch.rand((9, 17, 66), generator=gen).to(torch.float32)
    mask = torch.zeros((9, 17, 66), dtype=torch.uint8)
    g = _gpu(vol, 1.0, 2.0, mask, center=(4.0, 8.0, 30.0), direction=(0.0, 0.0, 1.0))
    assert np.all(g["flags"] == st.ST_FLAG_OUTSIDE_MASK)
    for k in ("e3", "fa", "ha", "ia"):
        assert np.all(g[k] == 0), k


def test_power_of_two_scaling():
    _log("case: f32 random (20, 24, 70) and the same times 1024")
    gen = torch.Generator().manual_seed(11)
    vol = torch.rand((20, 24, 70), generator=gen).to(torch.float32)
    center, direction = (9.5, 11.25, 34.5), (1.0, -0.2, 0.4)
    a = _gpu(vol, 1.0, 2.0, center=center, direction=direction)
    b = _gpu(vol * 1024, 1.0, 2.0, center=center, direction=direction)
    o = oracle.compute((vol * 1024).numpy(), None, 1.0, 2.0, axis_center=center, axis_direction=direction)
    stats = compare(b, o, vol.shape, center, direction)
    _log(summary(stats))
    assert_parity(stats, "scaled")
    for k in ("e3", "fa", "ha", "ia", "flags"):
        assert np.array_equal(a[k], b[k]), k
    scale = np.abs(a["evals"]).max(axis=0, keepdims=True).astype(np.float64)
    assert np.abs(b["evals"] / 2.0 ** 20 - a["evals"]).max() <= 1e-6 * scale.max()
