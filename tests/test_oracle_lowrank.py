"""Pins of the low-rank covariance oracle (Sec. III B) against closed forms.

The sample covariance is made exactly I + sum_j b_j b_j^T by construction
(B = sqrt(6N) Q C with Q orthonormal columns and C C^T the target), so the
noise vectors, the estimator and the rotated frame all have known answers:
the paper's closed-form Cholesky factor, the Sherman-Morrison inverse and the
variance formula eq. (bivecvariance).
"""
from __future__ import annotations

import math

import numpy as np

from oracle import closed_forms as cf
from oracle import lowrank as olr


def _orthonormal_columns(rng, N, n):
    Q, _ = np.linalg.qr(rng.standard_normal((N, n)))
    return Q


def _sign_fixed(v):
    return v if v[np.argmax(np.abs(v))] >= 0 else -v


def test_noise_vector_rank_one_from_closed_form_cholesky():
    rng = np.random.default_rng(31)
    n, N = 56, 200
    b = rng.standard_normal(n) * 0.6
    Lt = cf.bivector_cholesky(b)                       # Lt Lt^T = I + b b^T (Sec. III B)
    B = math.sqrt(6.0 * N) * _orthonormal_columns(rng, N, n) @ Lt.T
    bt, mu = olr.noise_vectors(B, 1)
    assert abs(mu[0] - (1.0 + b @ b)) < 1e-11 * mu[0]
    assert np.max(np.abs(bt[0] - _sign_fixed(b))) < 1e-11 * np.max(np.abs(b))


def test_noise_vectors_two_orthogonal_shapes():
    rng = np.random.default_rng(32)
    n, N = 56, 160
    U = _orthonormal_columns(rng, n, 2)
    norms = np.array([3.0, 1.5])
    # symmetric square root of I + sum |b_j|^2 u_j u_j^T for orthonormal u_j
    C = np.eye(n) + sum((math.sqrt(1.0 + s * s) - 1.0) * np.outer(U[:, j], U[:, j]) for j, s in enumerate(norms))
    B = math.sqrt(6.0 * N) * _orthonormal_columns(rng, N, n) @ C
    bt, mu = olr.noise_vectors(B, 3)
    assert np.max(np.abs(mu[:2] - (1.0 + norms ** 2))) < 1e-11 * mu[0]
    assert abs(mu[2] - 1.0) < 1e-11
    for j in range(2):
        assert np.max(np.abs(bt[j] - _sign_fixed(norms[j] * U[:, j]))) < 1e-10
    # an eigenvalue equal to one gives (up to rounding) no vector
    assert np.linalg.norm(bt[2]) < 1e-6


def test_lowrank_estimator_sherman_morrison():
    rng = np.random.default_rng(33)
    n = 41
    b = rng.standard_normal(n) * 0.8
    alpha = rng.standard_normal(n)
    betas = rng.standard_normal((4, n))
    E, s2 = olr.estimator_lowrank(b[None, :], alpha, betas)
    # eq. (ic_bivectorinv) and eq. (bivecvariance), the latter times the 6 of eq. (modalvariance)
    zi = cf.bivector_inverse(b)
    assert np.max(np.abs(E - betas @ zi @ alpha / (alpha @ zi @ alpha))) < 1e-12
    assert abs(s2 - 6.0 * cf.bivector_variance(alpha, b)) < 1e-12 * s2
    # two orthogonal shapes: the inverse is the product of two Sherman-Morrison factors
    U, _ = np.linalg.qr(rng.standard_normal((n, 2)))
    b2 = np.stack([2.0 * U[:, 0], 0.7 * U[:, 1]])
    zi2 = np.eye(n) - sum(np.outer(v, v) / (1.0 + v @ v) for v in b2)
    E2, s22 = olr.estimator_lowrank(b2, alpha, betas)
    assert np.max(np.abs(E2 - betas @ zi2 @ alpha / (alpha @ zi2 @ alpha))) < 1e-12
    assert abs(s22 - 6.0 / (alpha @ zi2 @ alpha)) < 1e-12 * s22
    # no shape: the plain isotropic estimator
    E0, s20 = olr.estimator_lowrank(np.zeros((0, n)), alpha, betas)
    assert np.max(np.abs(E0 - betas @ alpha / (alpha @ alpha))) < 1e-12
    assert abs(s20 - 6.0 / (alpha @ alpha)) < 1e-12 * s20


def test_bivector_rotation_frame():
    rng = np.random.default_rng(34)
    n = 67
    b = rng.standard_normal(n) * 0.5
    alpha = rng.standard_normal(n)
    betas = rng.standard_normal((3, n))
    ap = olr.bivector_rotate(b, alpha)[0]
    bp = olr.bivector_rotate(b, betas)
    # in the rotated frame E = alpha'.beta' / |alpha'|^2 (Sec. III B) and |alpha'|^2 = alpha^T zeta^-1 alpha
    zi = cf.bivector_inverse(b)
    assert np.max(np.abs(bp @ ap / (ap @ ap) - betas @ zi @ alpha / (alpha @ zi @ alpha))) < 1e-12
    assert abs(1.0 / (ap @ ap) - cf.bivector_variance(alpha, b)) < 1e-12 / (ap @ ap)
    # the rotation whitens zeta: lambda~^-1 (I + b b^T) lambda~^-T = I
    W = olr.bivector_rotate(b, olr.bivector_rotate(b, cf.bivector_zeta(b)).T)
    assert np.max(np.abs(W - np.eye(n))) < 1e-12
