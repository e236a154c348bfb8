"""st_compute_noalloc (the entry point that allocates nothing) against st_compute
through the C ABI on the GPU: two calls in a row, the second on a smaller
volume, each bitwise equal to st_compute on the same inputs (the same kernels
and workspace layout; the library's scratch keeps the first call's contents
when the second runs).  A volume beyond the scratch is rejected on the host
with its outputs untouched.  MI355X only."""

import sys

import pytest
import torch

import paper_2508_07476_amd as st

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
OUTS = ("e3", "evals", "fa", "ha", "ia", "flags")


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _case(shape, seed, dtype, sigma, rho, with_mask):
    g = torch.Generator().manual_seed(seed)
    if dtype == "u16":
        vol = torch.randint(0, 65536, shape, generator=g, dtype=torch.int32).to(torch.uint16)
    else:
        vol = torch.rand(shape, generator=g, dtype=torch.float64).to(torch.float32)
    mask = (torch.rand(shape, generator=g) < 0.8).to(torch.uint8).to(DEV) if with_mask else None
    center = tuple((s - 1) / 2.0 + 0.3 for s in shape)
    return vol.to(DEV), mask, sigma, rho, center, (1.0, 0.15, -0.2)


def _both(vol, mask, sigma, rho, center, direction):
    kw = dict(mask=mask, axis_center=center, axis_direction=direction, outputs=OUTS)
    ref = st.st_compute(vol, sigma, rho, **kw)
    got = st.st_compute_noalloc(vol, sigma, rho, **kw)
    torch.cuda.synchronize()
    return ref, got


def test_noalloc_matches_st_compute_on_two_calls_the_second_smaller():
    cases = [((70, 81, 100), 11, "f32", 1.0, 3.0, True),   # 12 planes of 70*81*128 floats
             ((40, 33, 50), 12, "u16", 1.5, 2.0, False)]   # smaller: stale scratch from the first call
    for shape, seed, dt, sigma, rho, with_mask in cases:
        _log("case: st_compute_noalloc", shape, dt, f"sigma {sigma} rho {rho} mask {with_mask}")
        ref, got = _both(*_case(shape, seed, dt, sigma, rho, with_mask))
        for k in OUTS:
            assert torch.equal(ref[k], got[k]), (shape, k)


def test_noalloc_rejects_a_volume_beyond_the_scratch():
    shape = (160, 160, 160)  # 12 planes of 160^3 floats: 196 MB > 128 MiB
    assert st.st_workspace_bytes(shape) > st.ST_NOALLOC_SCRATCH_BYTES
    vol = torch.zeros(shape, dtype=torch.float32, device=DEV)
    fa = torch.full(shape, 7.0, dtype=torch.float32, device=DEV)
    _log("case: st_compute_noalloc rejects", shape)
    with pytest.raises(st.StError) as ei:
        st.st_compute_noalloc(vol, 1.0, 2.0, outputs=("fa",), out={"fa": fa})
    assert ei.value.code == st.ST_ERR_UNSUPPORTED
    assert "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((fa == 7.0).all())
