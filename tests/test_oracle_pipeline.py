"""Pins for the oracle's whole path (CPU only): the analytic helical phantom,
invariances of the method, halo exactness of padded blocks, and the mask rule."""

import math

import numpy as np
import pytest
import torch

import oracle
from phantom import helix

SPEC = helix.spec_small_f32()


@pytest.fixture(scope="module")
def small():
    ph = helix.generate(SPEC)
    V = ph["volume"].numpy()
    res = oracle.compute(V, sigma=1.0, rho=3.0, axis_center=ph["center"], axis_direction=ph["direction"])
    return V, ph, res


def test_phantom_helix_angle_is_recovered(small):
    V, ph, res = small
    r = helix.cylindrical_radius(SPEC).numpy()[0]
    truth = helix.helix_angle(SPEC, torch.from_numpy(r)).numpy()
    zeta = np.arange(64) - ph["center"][0]
    wall = (r >= 15) & (r <= 25)
    sel = wall[None, :, :] & (np.abs(zeta)[:, None, None] < 16)
    err = np.degrees(np.abs(res["ha"] - truth[None])[sel])
    assert np.median(err) <= 3.0, np.median(err)
    assert np.percentile(err, 90) <= 6.0, np.percentile(err, 90)
    ia = np.degrees(np.abs(res["ia"][sel]))
    assert np.median(ia) <= 3.0
    # a wrong handedness of e_theta would give HA ~ -alpha: errors of order 2*alpha
    assert np.median(np.degrees(np.abs(res["ha"] + truth[None])[sel])) > 20.0


def test_affine_intensity_invariance(small):
    V, ph, res = small
    res2 = oracle.compute(3.7 * V.astype(np.float64) + 100.0, sigma=1.0, rho=3.0,
                          axis_center=ph["center"], axis_direction=ph["direction"])
    # adding a constant perturbs the (mathematically zero) gradient of the empty region
    # by rounding only: compare where the tensor carries signal
    tr = res["evals"].sum(axis=0)
    ok = (res["gap"] >= 1e-2) & (tr > 1e-8 * tr.max())
    assert ok.mean() > 0.4
    np.testing.assert_allclose(res2["fa"][ok], res["fa"][ok], atol=1e-10)
    d = np.abs(res2["e3"] - res["e3"]).max(axis=0)
    assert d[ok].max() < 1e-9
    np.testing.assert_allclose(res2["ha"][ok], res["ha"][ok], atol=1e-9)
    np.testing.assert_allclose(res2["ia"][ok], res["ia"][ok], atol=1e-9)
    np.testing.assert_allclose(res2["evals"][:, ok], 3.7 ** 2 * res["evals"][:, ok], rtol=1e-9)


def test_u16_and_f32_copies_agree():
    rng = np.random.default_rng(0)
    q = rng.integers(0, 65536, size=(10, 11, 12)).astype(np.uint16)
    a = oracle.compute(q, sigma=1.0, rho=1.5)
    b = oracle.compute(q.astype(np.float32), sigma=1.0, rho=1.5)
    for k in ("e3", "evals", "fa", "flags"):
        np.testing.assert_array_equal(a[k], b[k])


@pytest.mark.parametrize("lo,hi", [(16, 32), (0, 16), (32, 48)])
def test_padded_block_interior_is_exact(lo, hi):
    rng = np.random.default_rng(9)
    V = rng.random((48, 48, 48))
    sigma, rho = 1.0, 2.0
    halo = oracle.radius(sigma) + oracle.radius(rho)
    c = (20.5, 23.5, 22.5)
    whole = oracle.compute(V, sigma=sigma, rho=rho, axis_center=c, axis_direction=(1, 0.2, 0))
    a, b = max(0, lo - halo), min(48, hi + halo)
    blk = oracle.compute(V[a:b, a:b, a:b], sigma=sigma, rho=rho, axis_center=c,
                         axis_direction=(1, 0.2, 0), origin=(a, a, a))
    s = slice(lo - a, hi - a)
    for k in ("e3", "evals"):
        np.testing.assert_array_equal(blk[k][:, s, s, s], whole[k][:, lo:hi, lo:hi, lo:hi])
    for k in ("fa", "ha", "ia", "flags"):
        np.testing.assert_array_equal(blk[k][s, s, s], whole[k][lo:hi, lo:hi, lo:hi])


def test_mask_gates_outputs_only():
    rng = np.random.default_rng(1)
    V = rng.random((12, 13, 14))
    mask = (rng.random(V.shape) > 0.3).astype(np.uint8)
    kw = dict(sigma=1.0, rho=1.5, axis_center=(5.5, 6.5, 6.0), axis_direction=(1, 0, 0))
    plain = oracle.compute(V, **kw)
    masked = oracle.compute(V, mask=mask, **kw)
    inside = mask != 0
    for k in ("fa", "ha", "ia", "flags"):
        np.testing.assert_array_equal(masked[k][inside], plain[k][inside])
        if k != "flags":
            assert np.all(masked[k][~inside] == 0.0)
    assert np.all(masked["flags"][~inside] == oracle.FLAG_OUTSIDE_MASK)
    np.testing.assert_array_equal(masked["e3"][:, inside], plain["e3"][:, inside])
    assert np.all(masked["e3"][:, ~inside] == 0.0)
    assert math.isclose(float(inside.mean()), 0.7, abs_tol=0.05)
