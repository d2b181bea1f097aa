"""Truncated orthonormal mode frame (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. II works in an orthonormal basis R (R R^T = I) truncated to the modes that span the
space of interest, with the projector P = R^T R, and re-orthonormalises by the Cholesky
factor of a covariance, eq. (Cholrot): alpha' = lambda^-1 alpha, beta' = lambda^-1 beta.
The separable q-product modes are not independent in floating point once P is large (their
Gram matrix zeta0 loses rank numerically), so the factorisation is pivoted and truncated:

    Pi^T zeta0 Pi ~= L L^T,  L = [L11; L21] (n x k),  L11 k x k lower triangular,

choosing at each step the mode with the largest remaining diagonal and stopping once it
falls below tol times the largest diagonal of zeta0 (the textbook diagonally pivoted,
outer-product Cholesky).  The k kept modes (the first k of the permutation) span, to
that tolerance, everything the n modes span; T = L11^-1 [I_k 0] Pi^T is an orthonormal
frame of that span under zeta0 (T zeta0 T^T = I_k exactly), eq. (Cholrot) on the kept
modes.  Every step below is the plain definition, in FP64.
"""
from __future__ import annotations

import numpy as np


def pivoted_cholesky(Z: np.ndarray, tol: float):
    """Diagonally pivoted Cholesky of the symmetric positive semi-definite Z, truncated once
    the largest remaining diagonal is <= tol * max(diag Z).

    Returns (perm [k], L [n, k]) with L's rows in the original order of Z: Z ~= L L^T,
    the residual Z - L L^T has diagonal <= tol * max(diag Z), and L[perm] is lower
    triangular with a positive diagonal."""
    Z = np.asarray(Z, dtype=np.float64)
    n = Z.shape[0]
    d = np.diag(Z).copy()
    dmax = float(d.max())
    chosen = np.zeros(n, dtype=bool)
    perm, cols = [], []
    for _ in range(n):
        rest = np.where(chosen, -np.inf, d)
        p = int(np.argmax(rest))
        if not rest[p] > tol * dmax:
            break
        L = np.array(cols).T if cols else np.zeros((n, 0))
        col = (Z[:, p] - L @ L[p, :]) / np.sqrt(d[p])
        col[chosen] = 0.0   # rows already pivoted stay on the triangle
        chosen[p] = True
        perm.append(p)
        cols.append(col)
        d = d - col * col
        d[p] = 0.0
    L = np.array(cols).T if cols else np.zeros((n, 0))
    return np.array(perm, dtype=np.int64), L


def frame_rotate(perm: np.ndarray, L: np.ndarray, x: np.ndarray) -> np.ndarray:
    """x' = L11^-1 x[perm] for rows of x [R, n] (or one vector): the coordinates in the
    truncated orthonormal frame (eq. Cholrot on the kept modes)."""
    x = np.asarray(x, dtype=np.float64)
    L11 = L[perm, :]
    xs = x[..., perm]
    return np.linalg.solve(L11, xs.T).T if x.ndim > 1 else np.linalg.solve(L11, xs)


def estimator_in_frame(perm, L, zeta, alpha, betas):
    """E_s and sigma^2 of eqs. (modalest, modalvariance) on the kept modes, with the
    covariance rotated into the frame: zeta' = L11^-1 zeta_kk L11^-T (= I_k for zeta0)."""
    a = frame_rotate(perm, L, alpha)
    b = frame_rotate(perm, L, np.atleast_2d(betas))
    L11 = L[perm, :]
    Zk = np.asarray(zeta)[np.ix_(perm, perm)]
    Zp = np.linalg.solve(L11, np.linalg.solve(L11, Zk).T).T
    y = np.linalg.solve(Zp, a)
    norm = float(a @ y)
    return b @ y / norm, 6.0 / norm
