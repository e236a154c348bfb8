"""Pins for the oracle's eigen-decomposition, FA and degeneracy steps (CPU only).

Checks come from linear algebra (trace, determinant, residual, orthonormality),
an independent cyclic Jacobi solver, hand-derived FA values and an exact
special case of the whole tensor: a volume constant along one axis has that
axis as an exact null direction of every gradient, hence of S.
"""

import math

import numpy as np
import pytest

import oracle


def _rand_spd(rng, n, gaps=None):
    Q, _ = np.linalg.qr(rng.standard_normal((n, 3, 3)))
    lam = rng.random((n, 3)) * 10.0 + 0.01
    if gaps is not None:
        lam[:, 1] = lam[:, 2] * (1.0 + gaps)
    return np.einsum("nij,nj,nkj->nik", Q, lam, Q)


def _six(M):
    return np.stack([M[..., 0, 0], M[..., 0, 1], M[..., 0, 2], M[..., 1, 1], M[..., 1, 2], M[..., 2, 2]])


def test_eigen_invariants_on_random_spd():
    rng = np.random.default_rng(3)
    M = _rand_spd(rng, 500)
    evals, e3 = oracle.eigen_sorted(_six(M))
    assert np.all(evals[0] >= evals[1]) and np.all(evals[1] >= evals[2])
    np.testing.assert_allclose(evals.sum(axis=0), np.trace(M, axis1=1, axis2=2), rtol=1e-13)
    np.testing.assert_allclose(evals.prod(axis=0), np.linalg.det(M), rtol=1e-11)
    np.testing.assert_allclose((e3 * e3).sum(axis=0), 1.0, rtol=1e-14)
    resid = np.einsum("nij,jn->in", M, e3) - evals[2] * e3
    norm = np.linalg.norm(M, axis=(1, 2))
    assert np.all(np.linalg.norm(resid, axis=0) <= 1e-12 * norm)


def test_jacobi_agrees_with_lapack():
    rng = np.random.default_rng(4)
    M = np.concatenate([_rand_spd(rng, 100), _rand_spd(rng, 50, gaps=1e-2), _rand_spd(rng, 50, gaps=1e-5)])
    evals, e3 = oracle.eigen_sorted(_six(M))
    for n in range(M.shape[0]):
        w, V = oracle.jacobi_eigen(M[n])
        np.testing.assert_allclose(w, evals[:, n], rtol=1e-12, atol=1e-12 * abs(w).max())
        # eigenvectors are orthonormal
        np.testing.assert_allclose(V.T @ V, np.eye(3), atol=1e-13)
        gap = (w[1] - w[2]) / w.sum()
        v = oracle.canonical_sign(V[:, 2])
        # e3 agrees to ~eps/gap
        ang = math.atan2(np.linalg.norm(np.cross(v, e3[:, n])), abs(v @ e3[:, n]))
        assert ang <= 1e-13 / gap + 1e-14


def test_canonical_sign_rule():
    v = np.array([[-0.8, 0.1, 0.5], [0.6, -0.9, 0.5], [0.0, 0.4, -0.7071]]).T
    got = oracle.canonical_sign(v)
    np.testing.assert_array_equal(got[:, 0], [0.8, -0.1, -0.5])   # z leads, was negative
    np.testing.assert_array_equal(got[:, 1], [-0.6, 0.9, -0.5])   # y leads, was negative
    np.testing.assert_array_equal(got[:, 2], [0.0, -0.4, 0.7071])   # x leads, was negative
    tie = np.array([[-0.5, -0.5, 0.1]]).T   # z and y tie: z decides
    np.testing.assert_array_equal(oracle.canonical_sign(tie)[:, 0], [0.5, 0.5, -0.1])


def test_fa_hand_values():
    # diag(3, 2, 1): mean 2, |lambda - mean| = sqrt(2), |lambda| = sqrt(14) -> sqrt(3/2 * 2/14) = sqrt(3/14)
    # (1, 1, 0): mean 2/3, deviations (1/3, 1/3, -2/3) -> sqrt(3/2 * (6/9) / 2) = 1/sqrt(2)
    # (1, 0, 0): deviations (2/3, -1/3, -1/3) -> sqrt(3/2 * (6/9) / 1) = 1
    # (5, 5, 5): isotropic -> 0;  (0, 0, 0): defined as 0
    lam = np.array([[3.0, 2.0, 1.0], [1.0, 1.0, 0.0], [1.0, 0.0, 0.0], [5.0, 5.0, 5.0], [0.0, 0.0, 0.0]]).T
    fa = oracle.fractional_anisotropy(lam)
    np.testing.assert_allclose(fa, [math.sqrt(3.0 / 14.0), 1.0 / math.sqrt(2.0), 1.0, 0.0, 0.0], atol=1e-15)


def test_fa_invariant_form_and_range():
    rng = np.random.default_rng(8)
    M = _rand_spd(rng, 1000)
    evals, _ = oracle.eigen_sorted(_six(M))
    fa = oracle.fractional_anisotropy(evals)
    tr = np.trace(M, axis1=1, axis2=2)
    F2 = (M * M).sum(axis=(1, 2))
    np.testing.assert_allclose(fa, np.sqrt(1.5 - tr * tr / (2.0 * F2)), atol=1e-12)
    assert np.all(fa >= 0.0) and np.all(fa <= 1.0)


def test_degeneracy_classification():
    lam = np.array([[3.0, 2.0, 1.0], [3.0, 1.0005, 1.0], [3.0, 1.0 + 6e-3, 1.0], [0.0, 0.0, 0.0], [-1.0, -1.0, -2.0]]).T
    # gaps/trace: 1/6, 5e-4/5.0005 (< 1e-3), 6e-3/5.006 (> 1e-3), trace 0, trace < 0
    np.testing.assert_array_equal(oracle.degenerate(lam), [False, True, False, True, True])


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_volume_constant_along_an_axis_has_that_axis_as_e3(axis):
    rng = np.random.default_rng(21 + axis)
    shape = [12, 13, 14]
    prof_shape = list(shape)
    prof_shape[axis] = 1
    V = np.broadcast_to(rng.random(prof_shape), shape).copy()
    res = oracle.compute(V, sigma=1.0, rho=2.0, keep_tensor=True)
    S = res["S"]
    # components involving the constant axis vanish (up to summation rounding)
    comp = {0: (0, 1, 2), 1: (1, 3, 4), 2: (2, 4, 5)}[axis]
    scale = np.abs(S).max()
    for c in comp:
        assert np.abs(S[c]).max() <= 1e-14 * scale
    ok = res["gap"] >= oracle.DEGENERATE_GAP
    assert ok.mean() > 0.5
    unit = np.zeros(3)
    unit[axis] = 1.0
    e3 = res["e3"][:, ok]
    np.testing.assert_allclose(np.abs(e3[axis]), 1.0, atol=1e-12)
    np.testing.assert_allclose(res["evals"][2][ok], 0.0, atol=1e-12 * scale)
