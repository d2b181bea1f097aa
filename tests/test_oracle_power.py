"""Pins of the modal power-spectrum oracle (Sec. IV).

* pixel form = harmonic form on a grid exact for the product (Parseval);
* <beta> = alpha, Cov(beta) = 2 zeta and Var(E) = sigma^2 over Gaussian skies
  (statistical, 4 standard errors), <E> = the amplitude of a spectral deviation.
"""
from __future__ import annotations

import math

import numpy as np

import modal_inputs as mi
from oracle import grid as og
from oracle import modal as om
from oracle import power as opw

Z_MAX = 4.0


def test_pixel_form_equals_harmonic_form():
    lmax, P = 12, 5
    g = og.Grid(16, 32)                      # exact for degree 2 lmax products
    cl = mi.cl_signal(lmax)
    q = mi.q_basis(P, lmax)
    a = mi.gaussian_alm(cl, lmax, mi.rng_for(90, 1))
    M = om.filtered_maps(a, cl, q, g)
    b_pix = opw.power_beta(M, g.w)
    b_harm = opw.power_beta_harmonic(om.whiten(a, cl, lmax), q, lmax)
    assert np.max(np.abs(b_pix - b_harm)) < 1e-12 * np.max(np.abs(b_harm))


def _harmonic_skies(N, lmax, cl_true, cl_filter, q, first):
    out = np.empty((N, mi.npairs(q.shape[0])))
    for i in range(N):
        a = mi.gaussian_alm(cl_true, lmax, mi.rng_for(91, first + i))
        out[i] = opw.power_beta_harmonic(om.whiten(a, cl_filter, lmax), q, lmax)
    return out


def test_mean_covariance_and_estimator_statistics():
    lmax, P, N = 24, 4, 4000
    cl = mi.cl_signal(lmax)
    q = mi.q_basis(P, lmax)
    c1 = (cl > 0).astype(float)
    mean_fid = opw.power_pair_mean(q, c1)          # <beta> for C~ = C: sum (2l+1) q q
    # Gaussian skies with the fiducial spectrum: zero mean after subtraction; on the
    # estimator's modes (the pairs (0, n), the first P) Cov = 2 zeta
    Ball = _harmonic_skies(N, lmax, cl, cl, q, 0) - mean_fid
    se = Ball.std(0, ddof=1) / math.sqrt(N)
    assert np.max(np.abs(Ball.mean(0)) / se) < Z_MAX
    B = Ball[:, :P]
    assert np.max(np.abs(opw.power_alpha(cl, cl, q) - mean_fid[:P])) < 1e-12 * np.max(mean_fid)
    Z = opw.power_ideal_covariance(q, c1)
    C = np.cov(B.T)
    # sample covariance entries scatter by about sqrt((S_ii S_jj + S_ij^2) / N)
    sd = np.sqrt((np.outer(np.diag(2 * Z), np.diag(2 * Z)) + (2 * Z) ** 2) / N)
    assert np.max(np.abs(C - 2 * Z) / sd) < 5.0
    # a deviation C~ = C (1 + eps g_l): <E> = eps with alpha for dcl = C g
    gl = 0.5 * mi.q_basis(3, lmax)[2]
    alpha = opw.power_alpha(cl * gl, cl, q)
    E0, s2 = opw.power_estimator(Z, alpha, B)
    assert abs(E0.mean()) < Z_MAX * math.sqrt(s2 / N)
    assert abs(E0.var(ddof=1) / s2 - 1.0) < Z_MAX * math.sqrt(2.0 / (N - 1))
    eps = 0.05
    B1 = (_harmonic_skies(N, lmax, cl * (1.0 + eps * gl), cl, q, 0) - mean_fid)[:, :P]
    E1, _ = opw.power_estimator(Z, alpha, B1)
    assert abs(E1.mean() - eps) < Z_MAX * math.sqrt(s2 / N) * 1.2
