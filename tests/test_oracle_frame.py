"""Pins of the truncated orthonormal frame (oracle/frame.py) without the GPU.

* a full-rank, well-conditioned zeta: no truncation (k = n), L L^T = zeta, and the
  estimator in the frame equals the plain eq. (modalest) alpha^T zeta^-1 beta / alpha^T zeta^-1 alpha;
* a rank-r semi-definite zeta = A A^T: the pivoting stops at k = r, the residual diagonal
  obeys the stopping rule, T zeta T^T = I_r, and the estimator equals the pseudo-inverse
  one alpha^T zeta^+ beta / alpha^T zeta^+ alpha (an SVD, another algorithm) for alpha,
  beta in the range of zeta;
* E(beta = alpha) = 1, and E is unchanged by an orthogonal rotation of the frame;
* the ideal covariance of the separable modes is numerically singular already at l_max 32,
  P 8: the frame truncates it by the stopping rule and stays orthonormal under it.
"""
import numpy as np

import modal_inputs as mi
from oracle import closed_forms as cf
from oracle import frame as ofr
from oracle import modal as om


def _spd(n, cond, rng):
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (U * np.geomspace(1.0, 1.0 / cond, n)) @ U.T


def test_full_rank_reproduces_cholesky_and_estimator():
    rng = np.random.default_rng(1)
    n = 40
    Z = _spd(n, 1e3, rng)
    perm, L = ofr.pivoted_cholesky(Z, 0.0)
    assert len(perm) == n and sorted(perm.tolist()) == list(range(n))
    assert np.max(np.abs(L @ L.T - Z)) < 1e-13 * np.max(np.abs(Z))
    L11 = L[perm]
    assert np.allclose(L11, np.tril(L11), atol=1e-15) and np.all(np.diag(L11) > 0)
    # pivots come in decreasing order of the remaining diagonal: the first is the largest entry
    assert perm[0] == int(np.argmax(np.diag(Z)))
    alpha = rng.standard_normal(n)
    betas = rng.standard_normal((3, n))
    E, s2 = ofr.estimator_in_frame(perm, L, Z, alpha, betas)
    E_ref, s2_ref, _ = om.estimator(Z, alpha, betas)
    assert np.max(np.abs(E - E_ref)) < 1e-12 * np.max(np.abs(E_ref)) and abs(s2 / s2_ref - 1) < 1e-12


def test_rank_deficient_truncates_to_the_range():
    rng = np.random.default_rng(2)
    n, r, tol = 60, 17, 1e-12
    A = rng.standard_normal((n, r)) * np.geomspace(1.0, 1e-3, r)
    Z = A @ A.T
    perm, L = ofr.pivoted_cholesky(Z, tol)
    assert len(perm) == r
    resid = np.diag(Z - L @ L.T)
    assert np.max(resid) <= tol * np.max(np.diag(Z)) * 1.0001 + 1e-30
    assert np.max(np.abs(Z - L @ L.T)) < 1e-9 * np.max(np.abs(Z))
    # the frame is orthonormal under Z: T Z T^T = I_r, T = L11^-1 [I 0] Pi^T
    T = np.zeros((r, n))
    T[:, perm] = np.linalg.inv(L[perm])
    assert np.max(np.abs(T @ Z @ T.T - np.eye(r))) < 1e-8
    # estimator in the frame = pseudo-inverse estimator, for alpha, beta in the range of Z
    alpha = A @ rng.standard_normal(r)
    betas = (A @ rng.standard_normal((r, 4))).T
    E, s2 = ofr.estimator_in_frame(perm, L, Z, alpha, betas)
    Zp = np.linalg.pinv(Z, rcond=1e-10)
    norm = alpha @ Zp @ alpha
    assert np.max(np.abs(E - betas @ Zp @ alpha / norm)) < 1e-7 * np.max(np.abs(E))
    assert abs(s2 * norm / 6.0 - 1.0) < 1e-7
    # E(beta = alpha) = 1; an orthogonal rotation O of the frame leaves E unchanged
    E1, _ = ofr.estimator_in_frame(perm, L, Z, alpha, alpha[None])
    assert abs(E1[0] - 1.0) < 1e-12
    O, _ = np.linalg.qr(rng.standard_normal((r, r)))
    a2 = O @ ofr.frame_rotate(perm, L, alpha)
    b2 = ofr.frame_rotate(perm, L, betas) @ O.T
    E2 = b2 @ a2 / (a2 @ a2)     # zeta' = O I O^T = I in the rotated frame
    assert np.max(np.abs(E2 - E)) < 1e-10 * np.max(np.abs(E))


def test_ideal_covariance_of_separable_modes_truncates():
    """The Gram matrix of the q-product modes is numerically singular already at l_max 32,
    P 8 (condition number ~1e14): with tol 1e-10 the frame keeps fewer than n_max modes,
    the residual obeys the stopping rule, and the frame is orthonormal under zeta0 to the
    precision its conditioning allows (kept pivots >= sqrt(tol) of the largest: ~1e-6)."""
    lmax, P, tol = 32, 8, 1e-10
    q = mi.q_basis(P, lmax)
    cl = mi.cl_signal(lmax)
    Z = cf.zeta_ideal(q, (cl > 0).astype(float))
    perm, L = ofr.pivoted_cholesky(Z, tol)
    k = len(perm)
    assert 0 < k < Z.shape[0] == mi.ntriples(P)
    assert np.max(np.diag(Z - L @ L.T)) <= tol * np.max(np.diag(Z)) * 1.0001
    T = np.zeros((k, Z.shape[0]))
    T[:, perm] = np.linalg.inv(L[perm])
    assert np.max(np.abs(T @ Z @ T.T - np.eye(k))) < 1e-5
