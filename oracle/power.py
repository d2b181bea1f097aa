"""Modal power-spectrum estimator, plain FP64 (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. IV (other polyspectra): for the power spectrum the building blocks are
A = delta (C~_l - C_l) / sqrt(C C), B = (a a* - <a a*>) / sqrt(C C) and
C = <a a*> <a a*> / sqrt(C C C C), with isotropic basis functions
delta_{l1 l2} delta_{m1 m2} R_{n l} / (v v), supplemented for cut-sky effects.

Readings:
  * pair sums, p <= r: the two-index separable basis q_p(l1) q_r(l2) times the
    two-point Gaunt factor int w Y_l1m1 Y_l2m2 (w the pixel weight including the
    mask), so that in pixel space
        beta_pr = sum_x w(x) (M_p(x) M_r(x) - <M_p M_r>(x)),
    the quadratic analogue of eq. (bbispect) (three legs -> two, "3 C a" -> the mean
    pair product); on the full sky the Gaunt factor is delta_{l1 l2} delta_{m1,-m2} and
    beta_pr = sum_lm q_p(l) q_r(l) (|a~_lm|^2 - <|a~_lm|^2>);
  * the estimator's modes are the paper's isotropic R_n(l) (one index): the pairs
    (0, n), R_n(l) = q_0(l) q_n(l) (= q_n(l) for a basis with q_0 = 1), n < P.  On the
    full sky the products q_p q_r of the other pairs lie in the span of fewer functions
    (polynomials of degree <= 2P - 2 for a polynomial basis), so all pairs together have
    a singular covariance;
  * alpha_n = sum_l (2l + 1) q_0 q_n (C~_l - C_l) / C_l (full-sky expectation of beta for
    a sky with spectrum C~ analysed with the filter C);
  * zeta = <beta beta^T> / 2 (two cross pairings, as 6 = 3! for three legs), so
    sigma^2 = 2 / alpha^T zeta^-1 alpha; on the full sky for whitened spectra c_l,
    zeta_nn' = sum_l (2l + 1) c_l^2 q_0^2 q_n q_n'.
"""
from __future__ import annotations

import numpy as np

from modal_inputs import pair_list
from .modal import pair_products


def power_beta(M: np.ndarray, w: np.ndarray, V: np.ndarray | None = None) -> np.ndarray:
    """beta_pr = sum_x w (M_p M_r - V_pr) for the maps M [P, ...]; V [npairs, ...] or None."""
    A = pair_products(M)                                   # [npairs, npix]
    if V is not None:
        A = A - V.reshape(A.shape[0], -1)
    return A @ np.asarray(w, dtype=np.float64).reshape(-1)


def power_beta_harmonic(alm_w: np.ndarray, q: np.ndarray, lmax: int) -> np.ndarray:
    """Full-sky beta_pr = sum_lm q_p(l) q_r(l) |a~_lm|^2 (m < 0 counted through m > 0)."""
    from modal_inputs import lm_arrays
    l, m = lm_arrays(lmax)
    s = np.zeros(lmax + 1)
    np.add.at(s, l, np.where(m == 0, 1.0, 2.0) * np.abs(alm_w) ** 2)
    return np.array([np.sum(q[p] * q[r] * s) for p, r in pair_list(q.shape[0])])


def power_pair_mean(q: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Full-sky <beta_pr> = sum_l (2l + 1) c_l q_p q_r for whitened spectra c_l, every pair."""
    wl = (2.0 * np.arange(c.size) + 1.0) * c
    return np.array([np.sum(wl * q[p] * q[r]) for p, r in pair_list(q.shape[0])])


def power_alpha(dcl: np.ndarray, cl: np.ndarray, q: np.ndarray) -> np.ndarray:
    """alpha_n = sum_l (2l + 1) q_0 q_n (C~_l - C_l) / C_l for n < P, terms with C_l = 0 dropped."""
    lmax = cl.size - 1
    wl = np.zeros(lmax + 1)
    ok = cl > 0
    wl[ok] = (2.0 * np.arange(lmax + 1)[ok] + 1.0) * dcl[ok] / cl[ok]
    return np.array([np.sum(wl * q[0] * q[n]) for n in range(q.shape[0])])


def power_ideal_covariance(q: np.ndarray, c: np.ndarray) -> np.ndarray:
    """zeta_nn' = sum_l (2l + 1) c_l^2 R_n(l) R_n'(l), R_n = q_0 q_n."""
    lmax = c.size - 1
    R = q[0][None, :] * q                                              # [P, L]
    return (R * ((2.0 * np.arange(lmax + 1) + 1.0) * c * c)) @ R.T


def power_estimator(zeta: np.ndarray, alpha: np.ndarray, betas: np.ndarray):
    """E_s = alpha^T zeta^-1 beta_s / alpha^T zeta^-1 alpha, sigma^2 = 2 / alpha^T zeta^-1 alpha."""
    y = np.linalg.solve(zeta, alpha)
    norm = float(alpha @ y)
    return np.atleast_2d(betas) @ y / norm, 2.0 / norm
