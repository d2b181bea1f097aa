"""Low-rank ("bivector") covariance and its estimator, plain FP64 (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper, Sec. III B ("Bivector representation of covariance matrix"): in a frame
where the ideal (Gaussian, homogeneous-noise, full-sky) modal covariance is the
identity, the noise and the mask add one dominant shape vector b~, and

    zeta ~= I + b~ b~^T                                  (eq. ic_bivector)
    zeta^-1 ~= I - b~ b~^T / (1 + |b~|^2)                (eq. ic_bivectorinv)
    1 / (alpha^T zeta^-1 alpha) = (1/|alpha|^2) (1 + (alpha.b~)^2 /
        (|alpha|^2 (1 + |b~|^2) - (alpha.b~)^2))          (eq. bivecvariance)

with the lower-triangular Cholesky factor of I + b~ b~^T written out entry by
entry in the same section; rotating alpha and beta by its inverse (eq. Cholrot)
gives a frame where E = alpha'.beta' / |alpha'|^2.  The paper announces several
such vectors found by a principal component analysis.

Readings (the paper does not say how b~ is obtained from the simulations):
  * b~ is the leading eigenvector v_1 of the sample covariance
    zeta = sum_i beta_i beta_i^T / (6 N) (eq. linearterm) scaled by
    sqrt(mu_1 - 1), mu_1 its eigenvalue: the best rank-one fit of zeta - I in
    the Frobenius norm, so that I + b~ b~^T reproduces zeta along v_1 exactly;
  * the PCA generalisation keeps the k leading eigenpairs,
    zeta ~= I + sum_j b~_j b~_j^T, b~_j = sqrt(max(mu_j - 1, 0)) v_j; an
    eigenvalue at or below 1 contributes a zero vector;
  * the sign of each b~_j is fixed so that its entry of largest magnitude is
    positive (b~_j b~_j^T, which is all the estimator uses, does not depend on it);
  * sigma^2 keeps the factor 6 of eq. (modalvariance), which eq. (bivecvariance)
    leaves out.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .closed_forms import bivector_cholesky
from .modal import covariance_sample, estimator


def noise_vectors(beta_hats: np.ndarray, k: int):
    """The k leading noise vectors b~_j [k, n] and the eigenvalues mu_j [k] of the
    sample covariance of the rows of beta_hats [N, n] (readings above)."""
    zeta = covariance_sample(beta_hats)
    mu, V = np.linalg.eigh(zeta)              # ascending
    mu = mu[::-1][:k].copy()
    V = V[:, ::-1][:, :k]
    bt = np.zeros((k, zeta.shape[0]))
    for j in range(k):
        v = V[:, j]
        if v[np.argmax(np.abs(v))] < 0:
            v = -v
        bt[j] = np.sqrt(max(mu[j] - 1.0, 0.0)) * v
    return bt, mu


def lowrank_zeta(bt: np.ndarray) -> np.ndarray:
    """zeta = I + sum_j b~_j b~_j^T (eq. ic_bivector; k rows of bt)."""
    B = np.atleast_2d(np.asarray(bt, dtype=np.float64))
    return np.eye(B.shape[1]) + B.T @ B


def estimator_lowrank(bt: np.ndarray, alpha: np.ndarray, betas: np.ndarray):
    """E_s and sigma^2 of eqs. (modalest, modalvariance) with zeta = I + sum b~ b~^T,
    by a dense solve (the estimator of the general covariance)."""
    E, s2, _ = estimator(lowrank_zeta(bt), alpha, betas)
    return E, s2


def bivector_rotate(bt: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Rows of X rotated into the orthonormal frame of zeta = I + b~ b~^T:
    y = lambda~^-1 x with lambda~ the closed-form Cholesky factor of Sec. III B
    (eq. Cholrot), by a dense triangular solve."""
    L = bivector_cholesky(bt)
    X2 = np.atleast_2d(np.asarray(X, dtype=np.float64))
    return scipy.linalg.solve_triangular(L, X2.T, lower=True).T
