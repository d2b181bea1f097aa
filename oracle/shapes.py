"""Theory mode coefficients alpha_n of a separable bispectrum (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

eq. (abispect) with v_l = 1 and the separable modes Q_prs = q_p(l1) q_r(l2) q_s(l3):

    alpha_prs = sum_{l1 l2 l3} h^2_{l1 l2 l3} bbar_{l1 l2 l3} / sqrt(C_l1 C_l2 C_l3)
                q_p(l1) q_r(l2) q_s(l3),
    h_{l1 l2 l3} = sqrt((2l1+1)(2l2+1)(2l3+1) / (4 pi)) (l1 l2 l3; 0 0 0),

for a reduced bispectrum given as a sum of separable terms
b = sum_t X_t(l1) Y_t(l2) Z_t(l3); bbar is its symmetrisation over the six
orderings of (l1, l2, l3), the part a triple-product estimator sees.  Terms with
C_l = 0 are dropped (the whitening 1/sqrt(C_l) is zero there, as for the data).
Evaluated here as the plain triple sum with the exact Racah 3j symbols, so only
for small l_max.

``ideal_covariance`` (the Gram matrix of the separable modes under the weight
h^2 c c c, i.e. the full-sky covariance of whitened Gaussian skies with
<|a~_lm|^2> = c_l) is the same sum as the definition of zeta in eq. (cbispect)
with a diagonal covariance, written out the same way; ``closed_forms.zeta_ideal``
is its 1-D integral form.
"""
from __future__ import annotations

import itertools

import numpy as np

from modal_inputs import triple_list
from .wigner import h_geom


def _h2_table(lmax: int) -> np.ndarray:
    """h^2_{l1 l2 l3} for all l_i <= lmax (zero off the triangle or for odd l1+l2+l3)."""
    L = lmax + 1
    H = np.zeros((L, L, L))
    for l1 in range(L):
        for l2 in range(l1, L):
            for l3 in range(l2, L):
                if l3 > l1 + l2 or (l1 + l2 + l3) % 2:
                    continue
                v = h_geom(l1, l2, l3) ** 2
                for a, b, c in set(itertools.permutations((l1, l2, l3))):
                    H[a, b, c] = v
    return H


def _inv_sqrt(cl: np.ndarray) -> np.ndarray:
    cl = np.asarray(cl, dtype=np.float64)
    out = np.zeros_like(cl)
    out[cl > 0] = 1.0 / np.sqrt(cl[cl > 0])
    return out


def alpha_separable(terms: np.ndarray, cl: np.ndarray, q: np.ndarray) -> np.ndarray:
    """alpha_n [n_max] for terms [T][3][lmax+1] (X_t, Y_t, Z_t), filter spectrum cl, basis q [P][lmax+1]."""
    terms = np.asarray(terms, dtype=np.float64)
    lmax = cl.size - 1
    H = _h2_table(lmax)
    b = np.zeros((lmax + 1,) * 3)
    for X, Y, Z in terms:
        b += np.einsum("i,j,k->ijk", X, Y, Z)
    bbar = sum(np.transpose(b, p) for p in itertools.permutations(range(3))) / 6.0
    s = _inv_sqrt(cl)
    W = H * bbar * np.einsum("i,j,k->ijk", s, s, s)
    return np.array([np.einsum("ijk,i,j,k->", W, q[p], q[r], q[t]) for p, r, t in triple_list(q.shape[0])])


def ideal_covariance(q: np.ndarray, c: np.ndarray) -> np.ndarray:
    """zeta_nn' = (1/6) sum_{l1 l2 l3} h^2 c_l1 c_l2 c_l3 sum_{sigma in S3} Q_n(l) Q_n'(sigma l):
    <beta beta^T> / 6 for whitened isotropic Gaussian skies (the six cross pairings of
    Wick's theorem; the linear term removes the self pairings), by the triple sum."""
    lmax = c.size - 1
    H = _h2_table(lmax) * np.einsum("i,j,k->ijk", c, c, c)
    T = triple_list(q.shape[0])
    Qn = [np.einsum("i,j,k->ijk", q[p], q[r], q[t]) for p, r, t in T]
    Qs = [sum(np.transpose(Qm, p) for p in itertools.permutations(range(3))) for Qm in Qn]
    n = len(T)
    Z = np.zeros((n, n))
    for i in range(n):
        HQ = H * Qn[i]
        for j in range(i, n):
            Z[i, j] = Z[j, i] = np.sum(HQ * Qs[j]) / 6.0
    return Z
