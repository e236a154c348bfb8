"""HIP path vs the FP64 oracle, element by element, on seeded inputs (MI355X only).

Covers: the 64^3 float32 helical phantom whole; ragged shapes spanning several
x tiles with partial tails, odd nx (scalar stores), sizes smaller than the
filter radius (multiple reflections), uint16 and float32 input, masks, tilted
axes and radii that run on a padded compiled radius; the 512^3 uint16 phantom
in the benchmark's launch configuration on sampled sub-blocks plus whole-volume
properties; determinism; the standalone angle entry point; the library-owned
workspace path.
"""

import sys
import zlib

import numpy as np
import pytest
import torch

import oracle
import paper_2508_07476_amd as st
from phantom import helix

from _parity import assert_parity, compare, summary

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
ALL = ("e3", "evals", "fa", "ha", "ia", "flags")


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _np(res):
    return {k: v.cpu().numpy() for k, v in res.items()}


def _run_both(vol_cpu, sigma, rho, mask_cpu=None, center=None, direction=None, outputs=ALL):
    vol = vol_cpu.to(DEV)
    mask = None if mask_cpu is None else mask_cpu.to(DEV)
    if center is None:
        outputs = tuple(k for k in outputs if k not in ("ha", "ia"))
    g = st.st_compute(vol, sigma, rho, mask=mask, axis_center=center, axis_direction=direction,
                      outputs=outputs)
    torch.cuda.synchronize()
    o = oracle.compute(vol_cpu.numpy(), None if mask_cpu is None else mask_cpu.numpy(), sigma, rho,
                       axis_center=center, axis_direction=direction)
    return _np(g), o


def test_small_helical_phantom_whole_volume():
    _log("case: 64^3 f32 phantom sigma=1 rho=3")
    spec = helix.spec_small_f32()
    ph = helix.generate(spec)
    g, o = _run_both(ph["volume"], 1.0, 3.0, center=ph["center"], direction=ph["direction"])
    stats = compare(g, o, spec.shape, ph["center"], ph["direction"])
    _log(summary(stats))
    assert stats["n_checked"] > 0.9 * stats["n"]
    assert_parity(stats, "64^3 phantom")


CASES = [
    # shape, dtype, sigma, rho, mask, axis direction
    ((37, 45, 300), "u16", 1.0, 2.0, True, (1.0, 0.3, -0.2)),
    ((20, 33, 517), "f32", 1.5, 2.3, False, (0.0, 0.0, 1.0)),   # R_rho 9 -> compiled radius 10
    ((64, 20, 61), "f32", 0.9, 5.1, True, (1.0, 0.0, 0.0)),    # R_rho 20, nx odd
    ((5, 3, 7), "f32", 1.0, 2.0, False, (1.0, 1.0, 1.0)),      # every size below the radii
    ((1, 1, 1), "u16", 1.0, 1.0, False, None),
    ((9, 70, 2), "u16", 2.0, 3.0, True, (0.0, 1.0, 0.0)),
    ((130, 12, 9), "f32", 1.2, 6.0, False, (1.0, 0.5, 0.0)),   # long z axis (several chunks), R 24
    ((26, 44, 90), "u16", 2.6, 3.0, True, (1.0, -0.4, 0.3)),   # sigma radius 10: three-pass gradient
    ((70, 9, 131), "f32", 2.0, 2.0, False, (0.0, 1.0, 1.0)),   # sigma radius 8: largest fused gradient
    ((40, 36, 200), "f32", 3.6, 7.9, True, (1.0, 0.2, 0.1)),   # sigma radius 14, rho radius 32 (largest)
    ((72, 30, 129), "u16", 4.0, 7.0, False, (0.0, 1.0, 0.0)),  # sigma radius 16 (largest), rho radius 28
]


@pytest.mark.parametrize("shape,dtype,sigma,rho,use_mask,direction", CASES)
def test_ragged_random_volumes(shape, dtype, sigma, rho, use_mask, direction):
    _log(f"case: shape={shape} dtype={dtype} sigma={sigma} rho={rho} mask={use_mask} dir={direction}")
    gen = torch.Generator().manual_seed(zlib.crc32(repr((shape, dtype)).encode()))
    base = torch.rand(shape, generator=gen, dtype=torch.float64)
    # smooth-ish random texture plus noise so tensors are mostly non-degenerate
    vol = (base * 60000).round().to(torch.int32).to(torch.uint16) if dtype == "u16" else base.to(torch.float32)
    mask = (torch.rand(shape, generator=gen) > 0.25).to(torch.uint8) if use_mask else None
    center = None if direction is None else tuple((n - 1) / 2 + 0.25 for n in shape)
    g, o = _run_both(vol, sigma, rho, mask, center, direction)
    stats = compare(g, o, shape, center, direction, mask=None if mask is None else mask.numpy())
    _log(summary(stats))
    assert_parity(stats, str(shape))
    if mask is not None:
        out = mask.numpy() == 0
        assert np.all(g["flags"][out] == st.ST_FLAG_OUTSIDE_MASK)
        assert np.all(g["e3"][:, out] == 0) and np.all(g["fa"][out] == 0)


@pytest.fixture(scope="module")
def headline():
    _log("case: 512^3 u16 phantom + mask, sigma=1.5 rho=4 (benchmark configuration)")
    spec = helix.spec_headline_u16()
    ph = helix.generate(spec, device=DEV)
    res = st.st_compute(ph["volume"], 1.5, 4.0, mask=ph["mask"], axis_center=ph["center"],
                        axis_direction=ph["direction"], outputs=("e3", "fa", "ha", "ia", "flags"))
    torch.cuda.synchronize()
    return spec, ph, res


def test_headline_sampled_blocks(headline):
    spec, ph, res = headline
    halo = oracle.radius(1.5) + oracle.radius(4.0)
    n = spec.shape[0]
    rng = np.random.default_rng(1)
    B = 32
    # blocks in the wall, at the inner and outer boundary, and at volume faces
    origins = [(0, 224, 40), (n - B, 240, 400), (240, 48, 240), (100, 256 - 16, 256 + 90),
               (300, 256 + 200, 240), (n - B, n - B, n - B), (0, 0, 0)]
    origins += [tuple(int(v) for v in rng.integers(0, n - B, size=3)) for _ in range(1)]
    vol = ph["volume"]
    for org in origins:
        lo = [max(0, c - halo) for c in org]
        hi = [min(n, c + B + halo) for c in org]
        crop = vol[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]].cpu().numpy()
        mcrop = ph["mask"][lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]].cpu().numpy()
        o = oracle.compute(crop, mcrop, 1.5, 4.0, axis_center=ph["center"], axis_direction=ph["direction"],
                           origin=tuple(lo))
        s = tuple(slice(org[i] - lo[i], org[i] - lo[i] + B) for i in range(3))
        ob = {k: (v[(slice(None),) + s] if v.ndim == 4 else v[s]) for k, v in o.items() if v is not None}
        gs = tuple(slice(org[i], org[i] + B) for i in range(3))
        gb = {k: (v[(slice(None),) + gs] if v.dim() == 4 else v[gs]).cpu().numpy() for k, v in res.items()}
        stats = compare(gb, ob, (B, B, B), ph["center"], ph["direction"], mask=mcrop[s], origin=org)
        _log(org, summary(stats))
        assert_parity(stats, f"block {org}")


def test_headline_whole_volume_properties(headline):
    spec, ph, res = headline
    mask = ph["mask"].bool()
    flags = res["flags"]
    assert torch.equal((flags & st.ST_FLAG_OUTSIDE_MASK) != 0, ~mask)
    e3n = torch.linalg.vector_norm(res["e3"], dim=0)
    assert float((e3n[mask] - 1).abs().max()) < 1e-5
    assert float(e3n[~mask].abs().max()) == 0.0
    fa = res["fa"]
    assert float(fa.min()) >= 0.0 and float(fa.max()) <= 1.0
    lim = np.pi / 2 + 1e-6
    assert float(res["ha"].abs().max()) <= lim and float(res["ia"].abs().max()) <= lim
    # the fibre field follows the phantom: median |HA - alpha(r)| in the wall interior
    r = helix.cylindrical_radius(spec).to(DEV)[0]
    truth = helix.helix_angle(spec, r.cpu()).to(DEV)
    wall = (r >= 110) & (r <= 210)
    err = (res["ha"][200:312][:, wall].double() - truth[wall][None]).abs()
    med = float(torch.quantile(err.flatten()[:: 97].float(), 0.5))
    _log("median |HA - alpha| (deg):", np.degrees(med))
    assert np.degrees(med) < 3.0


def test_deterministic_bitwise():
    spec = helix.spec_small_f32()
    vol = helix.generate(spec)["volume"].to(DEV)
    a = st.st_compute(vol, 1.0, 3.0, axis_center=(31.5, 31.5, 31.5), axis_direction=(1, 0, 0), outputs=ALL)
    b = st.st_compute(vol, 1.0, 3.0, axis_center=(31.5, 31.5, 31.5), axis_direction=(1, 0, 0), outputs=ALL)
    torch.cuda.synchronize()
    for k in ALL:
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("sigma,rho", [(2.0, 6.0), (1.5, 4.0)])
def test_deterministic_bitwise_fused_gradient_and_final_pass(sigma, rho):
    """Race smoke test of the LDS-staged passes at the radii whose tiles keep
    several blocks per CU: the fused gradient's one barrier per plane over two
    alternating plane buffers (radius 8 with 4-row tiles, radius 6 with 8-row
    tiles) and the final pass's float64 rows staged in two halves (radius 24,
    16).  Three runs on a 96 x 192 x 520 volume (rows past one 256-output
    segment, a ragged last tile) must agree bit for bit."""
    _log(f"case: determinism sigma={sigma} rho={rho}")
    ph = helix.generate(helix.PhantomSpec(shape=(96, 192, 520), annuli=(helix.Annulus(30.0, 90.0),), period=4.0,
                                          noise=(0.05,), dtype="u16", seed=9, with_mask=True), device=DEV)
    kw = dict(mask=ph["mask"], axis_center=ph["center"], axis_direction=ph["direction"], outputs=ALL)
    runs = [st.st_compute(ph["volume"], sigma, rho, **kw) for _ in range(3)]
    torch.cuda.synchronize()
    for r in runs[1:]:
        for k in ALL:
            assert torch.equal(runs[0][k], r[k]), k


def test_standalone_angles_match_oracle_frame():
    spec = helix.spec_small_f32()
    ph = helix.generate(spec)
    vol = ph["volume"].to(DEV)
    res = st.st_compute(vol, 1.0, 3.0, axis_center=ph["center"], axis_direction=ph["direction"],
                        outputs=("e3", "ha", "ia", "flags"))
    c2, d2 = (30.0, 33.0, 29.5), (1.0, 0.2, -0.1)
    mask = (torch.arange(64 ** 3, device=DEV).view(64, 64, 64) % 7 != 0).to(torch.uint8)
    ang = st.st_angles(res["e3"], c2, d2, mask=mask, outputs=("ha", "ia", "flags"))
    same = st.st_angles(res["e3"], ph["center"], ph["direction"], outputs=("ha", "ia"))
    torch.cuda.synchronize()
    e3 = res["e3"].cpu().numpy().astype(np.float64)
    frame = oracle.cylindrical_frame((64, 64, 64), c2, d2)
    ha, ia, on = oracle.helix_intrusion(e3 / np.linalg.norm(e3, axis=0), frame)
    m = mask.cpu().numpy() != 0
    assert np.abs(ang["ha"].cpu().numpy() - ha)[m].max() < 2e-6
    assert np.abs(ang["ia"].cpu().numpy() - ia)[m].max() < 2e-6
    assert np.all(ang["ha"].cpu().numpy()[~m] == 0)
    assert np.all(ang["flags"].cpu().numpy()[~m] == st.ST_FLAG_OUTSIDE_MASK)
    # same axis as st_compute: only the float32 rounding of e3 separates the two
    assert float((same["ha"] - res["ha"]).abs().max()) < 2e-6
    assert float((same["ia"] - res["ia"]).abs().max()) < 2e-6


def test_library_owned_workspace_matches_caller_workspace():
    import ctypes
    lib = st.load_library()
    vol = helix.generate(helix.spec_small_f32())["volume"].to(DEV)
    ref = st.st_compute(vol, 1.0, 3.0, outputs=("e3", "fa"))
    e3 = torch.empty_like(ref["e3"])
    fa = torch.empty_like(ref["fa"])
    stream = torch.cuda.current_stream().cuda_stream
    code = lib.st_compute(vol.data_ptr(), st.ST_DTYPE_F32, None, 64, 64, 64, 1.0, 3.0, 4.0, None, None,
                          e3.data_ptr(), None, fa.data_ptr(), None, None, None, None, 0, stream)
    assert code == 0, lib.st_last_error()
    torch.cuda.synchronize()
    assert torch.equal(e3, ref["e3"]) and torch.equal(fa, ref["fa"])
    del ctypes
