"""Pins for the oracle's filter, gradient and integration steps (CPU only).

Each check is independent of the separable code it tests: a brute-force 3-D
correlation with its own boundary table, SciPy's Gaussian filters, and closed
forms of the Gaussian-derivative filter on constants, ramps and parabolas.
"""

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle


def _symmetric_table(n, R):
    """Index table for positions -R .. n-1+R built by NumPy's symmetric padding."""
    return np.pad(np.arange(n), R, mode="symmetric")


def _brute_correlate3d(V, wz, wy, wx):
    """Direct 3-D correlation with the full kernel wz (x) wy (x) wx (no separability)."""
    nz, ny, nx = V.shape
    Rz, Ry, Rx = (len(wz) - 1) // 2, (len(wy) - 1) // 2, (len(wx) - 1) // 2
    K = wz[:, None, None] * wy[None, :, None] * wx[None, None, :]
    Ez, Ey, Ex = _symmetric_table(nz, Rz), _symmetric_table(ny, Ry), _symmetric_table(nx, Rx)
    ext = V[np.ix_(Ez, Ey, Ex)]
    out = np.empty(V.shape)
    for i in range(nz):
        for j in range(ny):
            for k in range(nx):
                out[i, j, k] = (K * ext[i:i + 2 * Rz + 1, j:j + 2 * Ry + 1, k:k + 2 * Rx + 1]).sum()
    return out


def test_radius_rule():
    assert oracle.radius(1.0) == 4 and oracle.radius(1.5) == 6 and oracle.radius(2.0) == 8
    assert oracle.radius(3.0) == 12 and oracle.radius(4.0) == 16 and oracle.radius(6.0) == 24
    assert oracle.radius(1.0, truncate=3.0) == 3


def test_reflect_index_matches_symmetric_padding():
    for n in (1, 2, 3, 5, 8):
        for R in (0, 1, 4, 7, 16):
            table = _symmetric_table(n, R)
            got = oracle.reflect_index(np.arange(-R, n + R), n)
            np.testing.assert_array_equal(got, table)


def test_taps_match_scipy_impulse_response():
    for s in (1.0, 1.5, 2.0, 3.0):
        w0, w1 = oracle.taps(s)
        R = len(w0) // 2
        delta = np.zeros(4 * R + 1)
        delta[2 * R] = 1.0
        h0 = ndi.gaussian_filter1d(delta, s, order=0, mode="constant", truncate=4.0)[R:3 * R + 1]
        h1 = ndi.gaussian_filter1d(delta, s, order=1, mode="constant", truncate=4.0)[R:3 * R + 1]
        # the response to a centred impulse is the correlation taps read backwards
        np.testing.assert_allclose(w0, h0[::-1], rtol=0, atol=1e-16)
        np.testing.assert_allclose(w1, h1[::-1], rtol=0, atol=1e-16)


@pytest.mark.parametrize("shape,sigma,rho", [((3, 5, 7), 1.0, 1.0), ((6, 4, 5), 0.8, 1.2)])
def test_separable_equals_brute_force_3d(shape, sigma, rho):
    rng = np.random.default_rng(11)
    V = rng.standard_normal(shape)
    w0s, w1s = oracle.taps(sigma)
    gz_b = _brute_correlate3d(V, w1s, w0s, w0s)
    gy_b = _brute_correlate3d(V, w0s, w1s, w0s)
    gx_b = _brute_correlate3d(V, w0s, w0s, w1s)
    gz, gy, gx = oracle.gradients(V, sigma)
    for a, b in ((gz, gz_b), (gy, gy_b), (gx, gx_b)):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * np.abs(b).max())
    w0r, _ = oracle.taps(rho)
    P_b = np.stack([gz_b * gz_b, gz_b * gy_b, gz_b * gx_b, gy_b * gy_b, gy_b * gx_b, gx_b * gx_b])
    S_b = np.stack([_brute_correlate3d(P_b[c], w0r, w0r, w0r) for c in range(6)])
    S = oracle.structure_tensor(V, sigma, rho)
    np.testing.assert_allclose(S, S_b, rtol=0, atol=1e-12 * np.abs(S_b).max())


@pytest.mark.parametrize("sigma,rho", [(1.0, 3.0), (1.5, 4.0), (2.0, 2.5)])
def test_matches_scipy_gaussian_filter(sigma, rho):
    rng = np.random.default_rng(5)
    V = rng.random((20, 18, 22))
    gz, gy, gx = oracle.gradients(V, sigma)
    ref = [ndi.gaussian_filter(V, sigma, order=o, mode="reflect", truncate=4.0)
           for o in ((1, 0, 0), (0, 1, 0), (0, 0, 1))]
    for g, r in zip((gz, gy, gx), ref):
        np.testing.assert_allclose(g, r, rtol=0, atol=1e-14 * np.abs(r).max())
    P = [ref[a] * ref[b] for a, b in ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))]
    S_ref = np.stack([ndi.gaussian_filter(p, rho, mode="reflect", truncate=4.0) for p in P])
    S = oracle.structure_tensor(V, sigma, rho)
    np.testing.assert_allclose(S, S_ref, rtol=0, atol=1e-13 * np.abs(S_ref).max())


def test_constant_volume_has_zero_gradient_and_tensor():
    V = np.full((9, 10, 11), 1234.5)
    for g in oracle.gradients(V, 1.5):
        assert np.abs(g).max() <= 1e-12 * 1234.5
    assert np.abs(oracle.structure_tensor(V, 1.5, 2.0)).max() <= 1e-20


@pytest.mark.parametrize("sigma", [1.0, 1.5, 2.0])
def test_ramp_and_parabola_closed_forms(sigma):
    R = oracle.radius(sigma)
    n = 2 * R + 12
    z = np.arange(n, dtype=np.float64)
    ramp = np.broadcast_to(z[:, None, None], (n, 5, 6)).copy()
    gz, gy, gx = oracle.gradients(ramp, sigma)
    inner = slice(R, n - R)
    slope = gz[inner]
    # the continuous Gaussian derivative of a unit ramp is exactly 1; the sampled,
    # truncated filter is within 1e-3 of it and positive (the filter estimates +d/dz)
    assert np.all(np.abs(slope - 1.0) < 1e-3)
    assert np.ptp(slope) < 1e-13
    assert np.abs(gy).max() < 1e-12 and np.abs(gx).max() < 1e-12
    # parabola z^2: derivative filter is linear, odd moments vanish -> 2 z * slope
    para = np.broadcast_to((z * z)[:, None, None], (n, 5, 6)).copy()
    pz, _, _ = oracle.gradients(para, sigma)
    expect = 2.0 * z[inner, None, None] * slope.mean()
    np.testing.assert_allclose(pz[inner], np.broadcast_to(expect, pz[inner].shape), rtol=1e-12, atol=1e-10)
