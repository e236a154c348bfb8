"""Per-voxel eigen-decomposition, FA and degeneracy (oracle, FP64, test infrastructure).

Figure 1(b) of the paper takes the fibre direction as the third eigenvector of
the structure tensor, the one of the smallest eigenvalue.  Readings taken:

* eigenvalues sorted lambda1 >= lambda2 >= lambda3, e3 a unit vector;
* canonical sign of e3: its largest-magnitude component is positive, ties go
  to the lowest array axis (z before y before x);
* fractional anisotropy (named in the Summary and Figure 1(c), not defined):
  the DT-MRI definition  FA = sqrt(3/2) |lambda - mean(lambda)| / |lambda|,
  0 when |lambda| = 0;
* a voxel is *degenerate* when trace <= 0 or (lambda2 - lambda3) / trace is
  below 1e-3: its fibre direction is then not determined to the tolerances
  used for comparisons.
"""

from __future__ import annotations

import math

import numpy as np

DEGENERATE_GAP = 1e-3


def _matrices(S):
    """(6, ...) components in (zz, zy, zx, yy, yx, xx) order -> (..., 3, 3)."""
    S = np.asarray(S, dtype=np.float64)
    zz, zy, zx, yy, yx, xx = S
    M = np.empty(zz.shape + (3, 3), dtype=np.float64)
    M[..., 0, 0] = zz
    M[..., 0, 1] = M[..., 1, 0] = zy
    M[..., 0, 2] = M[..., 2, 0] = zx
    M[..., 1, 1] = yy
    M[..., 1, 2] = M[..., 2, 1] = yx
    M[..., 2, 2] = xx
    return M


def canonical_sign(v):
    """Flip vectors (3, ...) so that the largest-|.| component is positive (ties: lowest axis)."""
    v = np.array(v, dtype=np.float64)
    a = np.abs(v)
    pick = np.argmax(a, axis=0)  # argmax returns the first maximum: lowest axis on ties
    lead = np.take_along_axis(v, pick[None], axis=0)[0]
    return np.where(lead < 0, -v, v)


def eigen_sorted(S):
    """Return (evals (3, ...) descending, e3 (3, ...) unit with canonical sign) via LAPACK eigh."""
    M = _matrices(S)
    w, V = np.linalg.eigh(M)          # ascending eigenvalues, eigenvectors in columns
    evals = np.moveaxis(w[..., ::-1], -1, 0)
    e3 = np.moveaxis(V[..., :, 0], -1, 0)
    return evals, canonical_sign(e3)


def jacobi_eigen(A, tol: float = 1e-15, max_sweeps: int = 50):
    """Cyclic Jacobi for one symmetric 3x3 matrix (Golub & Van Loan, cyclic-by-row Jacobi).

    Returns (evals descending, eigenvectors as columns in the same order).
    Pure Python/NumPy on a single matrix: cross-check for small samples only.
    """
    A = np.array(A, dtype=np.float64)
    n = 3
    V = np.eye(n)
    scale = max(np.linalg.norm(A), 1e-300)
    for _ in range(max_sweeps):
        off = math.sqrt(sum(A[i, j] ** 2 for i in range(n) for j in range(n) if i != j))
        if off <= tol * scale:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                if A[p, q] == 0.0:
                    continue
                # symmetric 2x2 Schur decomposition zeroing A[p, q]
                tau = (A[q, q] - A[p, p]) / (2.0 * A[p, q])
                t = (1.0 if tau >= 0 else -1.0) / (abs(tau) + math.sqrt(1.0 + tau * tau))
                c = 1.0 / math.sqrt(1.0 + t * t)
                s = t * c
                J = np.eye(n)
                J[p, p] = c
                J[q, q] = c
                J[p, q] = s
                J[q, p] = -s
                A = J.T @ A @ J
                V = V @ J
    w = np.diag(A).copy()
    order = np.argsort(-w, kind="stable")
    return w[order], V[:, order]


def fractional_anisotropy(evals):
    """FA = sqrt(3/2) * |lambda - mean| / |lambda| (0 where |lambda| = 0)."""
    lam = np.asarray(evals, dtype=np.float64)
    mean = lam.mean(axis=0)
    num = np.sqrt(((lam - mean) ** 2).sum(axis=0))
    den = np.sqrt((lam ** 2).sum(axis=0))
    with np.errstate(invalid="ignore", divide="ignore"):
        fa = np.sqrt(1.5) * num / den
    return np.where(den > 0, fa, 0.0)


def gap_ratio(evals):
    """(lambda2 - lambda3) / trace, and -inf where trace <= 0 (always counted as degenerate)."""
    lam = np.asarray(evals, dtype=np.float64)
    tr = lam.sum(axis=0)
    with np.errstate(invalid="ignore", divide="ignore"):
        g = (lam[1] - lam[2]) / tr
    return np.where(tr > 0, g, -np.inf)


def degenerate(evals, threshold: float = DEGENERATE_GAP):
    """True where trace <= 0 or (lambda2 - lambda3)/trace < threshold."""
    return gap_ratio(evals) < threshold
