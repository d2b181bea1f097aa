"""Closed forms used to pin the oracle (and, through it, the GPU path).

* Full-sky Gaussian expectations for isotropic whitened maps with
  <a~_lm a~*_lm> = c(l):
    <M_a(x) M_b(y)> = sum_l (2l+1)/(4 pi) c(l) q_a(l) q_b(l) P_l(x.y)
  so that <M_a M_b>(x) is constant over the sky, and (Wick, the six
  cross-pairings that survive once the linear term removes the
  self-pairings, eq. linearterm)
    zeta_{abc,a'b'c'} = (1/(48 pi)) sum_{sigma in S3} int_{-1}^{1} dmu
                        prod_i Q_{a_i b_sigma(i)}(mu),
    Q_ab(mu) = sum_l (2l+1) c(l) q_a(l) q_b(l) P_l(mu).
  (The double sphere integral of a function of x.y is 8 pi^2 int dmu; with
  K = Q/(4 pi) per leg this gives Cov = (1/(8 pi)) sum_sigma int prod Q and
  zeta = Cov/6.)
* The bivector covariance of Sec. III B, zeta = I + b b^T: its
  Sherman-Morrison inverse (eq. ic_bivectorinv), its lower-triangular
  Cholesky factor written out in the same section, and the variance formula
  eq. (bivecvariance).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import numpy.polynomial.legendre as npleg

from modal_inputs import pair_list, triple_list


def legendre_table(lmax: int, mu: np.ndarray) -> np.ndarray:
    """P_l(mu) for l = 0..lmax: [lmax+1, len(mu)]."""
    return npleg.legvander(np.asarray(mu, dtype=np.float64), lmax).T


def pair_mean_fullsky(q: np.ndarray, c: np.ndarray) -> np.ndarray:
    """<M_p M_r> for every pair p <= r on the full sky: sum_l (2l+1)/(4 pi) c q_p q_r."""
    lmax = c.size - 1
    wl = (2.0 * np.arange(lmax + 1) + 1.0) / (4.0 * math.pi) * c
    return np.array([np.sum(wl * q[p] * q[r]) for p, r in pair_list(q.shape[0])])


def zeta_ideal(q: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Full-sky modal covariance zeta_{nn'} for the separable basis (see module doc)."""
    lmax = c.size - 1
    P = q.shape[0]
    nodes, wts = npleg.leggauss(2 * lmax + 2)      # exact for degree <= 4 lmax + 3
    Pl = legendre_table(lmax, nodes)                # [L, nodes]
    wl = (2.0 * np.arange(lmax + 1) + 1.0) * c
    Q = np.einsum("l,al,bl,lk->abk", wl, q, q, Pl)  # [P, P, nodes]
    T = triple_list(P)
    n = len(T)
    Z = np.zeros((n, n))
    perms = list(itertools.permutations(range(3)))
    for i, a in enumerate(T):
        for j in range(i, n):
            b = T[j]
            s = 0.0
            for sg in perms:
                s += np.sum(wts * Q[a[0], b[sg[0]]] * Q[a[1], b[sg[1]]] * Q[a[2], b[sg[2]]])
            Z[i, j] = Z[j, i] = s / (48.0 * math.pi)
    return Z


def bivector_zeta(bt: np.ndarray) -> np.ndarray:
    bt = np.asarray(bt, dtype=np.float64)
    return np.eye(bt.size) + np.outer(bt, bt)


def bivector_inverse(bt: np.ndarray) -> np.ndarray:
    """Sherman-Morrison: (I + b b^T)^-1 = I - b b^T / (1 + |b|^2)."""
    bt = np.asarray(bt, dtype=np.float64)
    return np.eye(bt.size) - np.outer(bt, bt) / (1.0 + bt @ bt)


def bivector_cholesky(bt: np.ndarray) -> np.ndarray:
    """Lower-triangular L with L L^T = I + b b^T, entry by entry:
    L_nn  = sqrt(1 + S_n) / sqrt(1 + S_{n-1}),
    L_nk  = b_n b_k / (sqrt(1 + S_{k-1}) sqrt(1 + S_k))  for k < n,
    with S_n = sum_{i <= n} b_i^2 (S_0 = 0)."""
    bt = np.asarray(bt, dtype=np.float64)
    n = bt.size
    S = np.concatenate([[0.0], np.cumsum(bt * bt)])   # S[k] = sum_{i<k} b_i^2 (0-based)
    L = np.zeros((n, n))
    for i in range(n):
        L[i, i] = math.sqrt(1.0 + S[i + 1]) / math.sqrt(1.0 + S[i])
        for k in range(i):
            L[i, k] = bt[i] * bt[k] / (math.sqrt(1.0 + S[k]) * math.sqrt(1.0 + S[k + 1]))
    return L


def bivector_variance(alpha: np.ndarray, bt: np.ndarray) -> float:
    """1 / (alpha^T zeta^-1 alpha) for zeta = I + b b^T, in the paper's form
    (1/|a|^2) (1 + (a.b)^2 / (|a|^2 (1 + |b|^2) - (a.b)^2))."""
    a2 = float(alpha @ alpha)
    ab = float(alpha @ bt)
    b2 = float(bt @ bt)
    return (1.0 / a2) * (1.0 + ab * ab / (a2 * (1.0 + b2) - ab * ab))
