"""Pins of the theory mode coefficients and the ideal covariance (oracle).

Both oracle functions are triple sums over (l1, l2, l3) with the exact Racah 3j
symbols.  They are pinned against the textbook identity
    int_{-1}^{1} P_l1 P_l2 P_l3 dmu = 2 (l1 l2 l3; 0 0 0)^2,
which turns h^2 into (2l1+1)(2l2+1)(2l3+1)/(8 pi) times a Legendre triple
integral, evaluated here with numpy's Gauss-Legendre rule.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import numpy.polynomial.legendre as npleg

import modal_inputs as mi
from oracle import closed_forms as cf
from oracle import shapes as osh


def _mu_rule(lmax):
    return npleg.leggauss(2 * lmax + 2)


def test_legendre_triple_integral_identity():
    """The identity itself, on a few (l1, l2, l3), against the exact 3j symbols."""
    from oracle.wigner import wigner3j
    x, w = npleg.leggauss(20)
    P = npleg.legvander(x, 12).T
    for l1, l2, l3 in [(2, 3, 5), (4, 4, 4), (1, 6, 7), (3, 5, 6), (0, 7, 7)]:
        lhs = np.sum(w * P[l1] * P[l2] * P[l3])
        assert abs(lhs - 2.0 * wigner3j(l1, l2, l3, 0, 0, 0) ** 2) < 1e-14


def test_alpha_separable_against_mu_integral():
    lmax, P = 12, 4
    rng = np.random.default_rng(61)
    q = mi.q_basis(P, lmax)
    cl = mi.cl_signal(lmax)
    terms = rng.standard_normal((2, 3, lmax + 1))
    alpha = osh.alpha_separable(terms, cl, q)
    x, w = _mu_rule(lmax)
    Pl = npleg.legvander(x, lmax).T                            # [L, nodes]
    s = np.where(cl > 0, 1.0 / np.sqrt(np.where(cl > 0, cl, 1.0)), 0.0)
    tw = (2.0 * np.arange(lmax + 1) + 1.0) * s
    F = np.einsum("l,tfl,al,lk->tfak", tw, terms, q, Pl)       # [T, 3, P, nodes]
    ref = []
    for p, r, t in mi.triple_list(P):
        v = 0.0
        for T in range(terms.shape[0]):
            for sg in itertools.permutations(range(3)):
                v += np.sum(w * F[T, sg[0], p] * F[T, sg[1], r] * F[T, sg[2], t])
        ref.append(v / (48.0 * math.pi))
    ref = np.array(ref)
    assert np.max(np.abs(alpha - ref)) < 1e-12 * np.max(np.abs(ref))


def test_alpha_symmetrisation():
    """A term and its reordering give the same alpha (only bbar enters)."""
    lmax, P = 10, 3
    rng = np.random.default_rng(62)
    q = mi.q_basis(P, lmax)
    cl = mi.cl_signal(lmax)
    X, Y, Z = rng.standard_normal((3, lmax + 1))
    a1 = osh.alpha_separable(np.array([[X, Y, Z]]), cl, q)
    a2 = osh.alpha_separable(np.array([[Z, X, Y]]), cl, q)
    assert np.max(np.abs(a1 - a2)) < 1e-13 * np.max(np.abs(a1))


def test_ideal_covariance_against_mu_integral():
    lmax, P = 10, 4
    q = mi.q_basis(P, lmax)
    c = (mi.cl_signal(lmax) > 0).astype(float) * (1.0 + 0.1 * np.arange(lmax + 1))
    Z = osh.ideal_covariance(q, c)
    Zm = cf.zeta_ideal(q, c)
    assert np.max(np.abs(Z - Zm)) < 1e-12 * np.max(np.abs(Zm))
