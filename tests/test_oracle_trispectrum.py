"""Pins of the trispectrum oracle (Sec. IV).

* closed form: for M = Y_10, int M^4 = 9/(20 pi); with a constant pair mean v the
  six pairs and three pairings give 9/(20 pi) - 6 v + 12 pi v^2;
* quadrature: the grid sum on two different exact grids agrees;
* Wick: over Gaussian skies with the exact pair means, <tau> = 0 (4 standard errors);
* the rearrangement used by the GPU: tau = (1/3) sum over the three pairings of
  K_(ab),(cd), K = sum_x w (M_a M_b - 3 V_ab)(M_c M_d - 3 V_cd) - 6 sum_x w V_ab V_cd.
"""
from __future__ import annotations

import math

import numpy as np

import modal_inputs as mi
from oracle import closed_forms as cf
from oracle import grid as og
from oracle import modal as om
from oracle import trispectrum as otr


def _y10_case(v0):
    lmax = 2
    g = og.Grid(8, 16)                        # exact for degree 4 lmax
    cl = np.array([0.0, 1.0, 1.0])
    a = np.zeros(mi.nalm(lmax), dtype=np.complex128)
    a[mi.alm_index(1, 0, lmax)] = 1.0
    M = om.filtered_maps(a, cl, np.ones((1, lmax + 1)), g)     # [1, nt, nphi] = Y_10
    V = np.full((1,) + M.shape[1:], v0)
    return otr.tau(M, g.w, V)[0]


def test_closed_form_y10():
    assert abs(_y10_case(0.0) - 9.0 / (20.0 * math.pi)) < 1e-13
    v0 = 0.37
    assert abs(_y10_case(v0) - (9.0 / (20.0 * math.pi) - 6.0 * v0 + 12.0 * math.pi * v0 * v0)) < 1e-12


def test_exact_grids_agree():
    lmax, P = 6, 3
    cl = mi.cl_signal(lmax)
    q = mi.q_basis(P, lmax)
    a = mi.gaussian_alm(cl, lmax, mi.rng_for(97, 1))
    t1 = otr.tau(om.filtered_maps(a, cl, q, og.Grid(14, 28)), og.Grid(14, 28).w)
    t2 = otr.tau(om.filtered_maps(a, cl, q, og.Grid(20, 40)), og.Grid(20, 40).w)
    assert np.max(np.abs(t1 - t2)) < 1e-12 * np.max(np.abs(t1))


def test_gaussian_mean_vanishes():
    lmax, P, N = 8, 3, 600
    g = og.Grid(18, 36)
    cl = mi.cl_signal(lmax)
    q = mi.q_basis(P, lmax)
    Vc = cf.pair_mean_fullsky(q, (cl > 0).astype(float))
    V = np.repeat(Vc[:, None], g.npix, axis=1).reshape(-1, g.ntheta, g.nphi)
    T = np.array([otr.tau(om.filtered_maps(mi.gaussian_alm(cl, lmax, mi.rng_for(98, i)), cl, q, g), g.w, V)
                  for i in range(N)])
    z = T.mean(0) / (T.std(0, ddof=1) / math.sqrt(N))
    assert np.max(np.abs(z)) < 4.0
    # the unsubtracted quartic sums do not vanish: the pins above see the coefficients
    T0 = np.array([otr.tau(om.filtered_maps(mi.gaussian_alm(cl, lmax, mi.rng_for(98, i)), cl, q, g), g.w)
                   for i in range(50)])
    assert np.max(np.abs(T0.mean(0)) / (T0.std(0, ddof=1) / math.sqrt(50))) > 10.0


def test_pairing_rearrangement():
    lmax, P = 8, 4
    g = og.Grid(18, 36)
    cl = mi.cl_signal(lmax)
    q = mi.q_basis(P, lmax)
    rng = np.random.default_rng(99)
    M = om.filtered_maps(mi.gaussian_alm(cl, lmax, mi.rng_for(99, 0)), cl, q, g).reshape(P, -1)
    pairs = mi.pair_list(P)
    V = rng.standard_normal((len(pairs), M.shape[1])) * 0.1
    pid = {pr: k for k, pr in enumerate(pairs)}
    A = np.array([M[a] * M[b] - 3.0 * V[k] for k, (a, b) in enumerate(pairs)])
    K = (A * g.w.reshape(-1)) @ A.T - 6.0 * (V * g.w.reshape(-1)) @ V.T
    ref = otr.tau(M.reshape(P, g.ntheta, g.nphi), g.w, V.reshape(-1, g.ntheta, g.nphi))
    got = []
    for p, r, s, u in otr.quad_list(P):
        got.append((K[pid[(p, r)], pid[(s, u)]] + K[pid[(p, s)], pid[(r, u)]] + K[pid[(p, u)], pid[(r, s)]]) / 3.0)
    assert np.max(np.abs(np.array(got) - ref)) < 1e-12 * np.max(np.abs(ref))
