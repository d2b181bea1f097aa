"""Statistical pins of the oracle on seeded Gaussian skies.

Thresholds are z-scores against standard errors estimated from the samples
themselves (the cubic statistics are far from Gaussian, so no Gaussian
formula is assumed).  Seeds are fixed, so the outcome is deterministic.
"""
import math

import numpy as np
import pytest

import modal_inputs as mi
from oracle import closed_forms as cf
from oracle import grid as og
from oracle import modal as om
from oracle import sims as osims

Z_MAX = 5.0


@pytest.fixture(scope="module")
def ideal_ensemble():
    """Full-sky ideal sky (signal only) on the l_max = 32 grid, P = 8, with the
    exact (closed-form) pairing expectation as linear term."""
    c = mi.CONFIGS["tiny"]
    g = og.Grid(c.ntheta, c.nphi)
    cl = mi.cl_signal(c.lmax)
    q = mi.q_basis(c.P, c.lmax)
    N = 1500
    alms = np.array([mi.gaussian_alm(cl, c.lmax, mi.rng_for(c.cfg_id, 1000 + i)) for i in range(N)])
    cmask = (cl > 0).astype(float)
    Vconst = cf.pair_mean_fullsky(q, cmask)
    V = np.repeat(Vconst[:, None], g.npix, axis=1).reshape(-1, g.ntheta, g.nphi)
    B = np.empty((N, c.nmax))
    Bh = np.empty((N, c.nmax))
    for s0 in range(0, N, 250):
        M = om.filtered_maps(alms[s0:s0 + 250], cl, q, g)
        for i in range(M.shape[0]):
            B[s0 + i] = om.beta(M[i], g.w)
            Bh[s0 + i] = B[s0 + i] - om.linear_term(M[i], g.w, V)
    Z = cf.zeta_ideal(q, cmask)
    return dict(c=c, g=g, cl=cl, q=q, alms=alms, V=V, B=B, Bh=Bh, Z=Z, Vconst=Vconst, M_last=M)


def test_p7_zero_mean(ideal_ensemble):
    Bh = ideal_ensemble["Bh"]
    z = Bh.mean(0) / (Bh.std(0, ddof=1) / math.sqrt(Bh.shape[0]))
    assert np.max(np.abs(z)) < Z_MAX


def test_p9_pair_means_converge(ideal_ensemble):
    M = ideal_ensemble["M_last"]                 # 250 maps
    V = om.pair_means(M)                         # [pairs, nt, nphi]
    Vbar = V.reshape(V.shape[0], -1).mean(1)     # sky average removes most of the MC scatter
    ref = ideal_ensemble["Vconst"]
    # per-pair standard error from the per-map sky averages
    per_map = np.array([[np.mean(M[i, p] * M[i, r]) for p, r in mi.pair_list(M.shape[1])] for i in range(M.shape[0])])
    se = per_map.std(0, ddof=1) / math.sqrt(M.shape[0])
    assert np.max(np.abs(Vbar - ref) / se) < Z_MAX


def _quad_forms(Bh, Z, k=12, seed=0):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((k, Z.shape[0]))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    x = (Bh @ U.T) ** 2 / 6.0               # per-sim estimates of u^T zeta u
    ref = np.einsum("kn,nm,km->k", U, Z, U)
    return x, ref


def test_p8_covariance_matches_closed_form(ideal_ensemble):
    Bh, Z = ideal_ensemble["Bh"], ideal_ensemble["Z"]
    x, ref = _quad_forms(Bh, Z)
    z = (x.mean(0) - ref) / (x.std(0, ddof=1) / math.sqrt(x.shape[0]))
    assert np.max(np.abs(z)) < Z_MAX
    # the sample-covariance routine itself
    Zs = om.covariance_sample(Bh)
    assert np.allclose(np.diag(Zs), (Bh ** 2).mean(0) / 6.0, rtol=1e-12)
    # without the linear term the covariance is inflated by the self-pairings
    Bx, _ = _quad_forms(ideal_ensemble["B"], Z)
    assert np.mean(Bx.mean(0) / ref) > np.mean(x.mean(0) / ref)


def test_p12_variance_normalisation(ideal_ensemble):
    Bh, Z = ideal_ensemble["Bh"], ideal_ensemble["Z"]
    rng = np.random.default_rng(4)
    for _ in range(3):
        alpha = rng.standard_normal(Z.shape[0])
        E, s2, _ = om.estimator(Z, alpha, Bh)
        e2 = E ** 2        # zero-mean estimator: Var(E) = <E^2>
        z = (e2.mean() - s2) / (e2.std(ddof=1) / math.sqrt(e2.size))
        assert abs(z) < Z_MAX


def test_p14_fisher_expectation(ideal_ensemble):
    c, g, cl, q, alms, V, Z = (ideal_ensemble[k] for k in ("c", "g", "cl", "q", "alms", "V", "Z"))
    N = 120
    vre, vim = om.dof_variance(cl, c.lmax)
    per = []
    rng = np.random.default_rng(8)
    U = rng.standard_normal((8, Z.shape[0]))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    for a in alms[:N]:
        J = om.jacobian(a, cl, q, g, V)
        F1 = ((J.real * vre) @ J.real.T + (J.imag * vim) @ J.imag.T) / 18.0
        per.append(np.einsum("kn,nm,km->k", U, F1, U))
    per = np.array(per)
    ref = np.einsum("kn,nm,km->k", U, Z, U)
    z = (per.mean(0) - ref) / (per.std(0, ddof=1) / math.sqrt(N))
    assert np.max(np.abs(z)) < Z_MAX
    # the batch routine agrees with the per-map sum
    F = om.fisher(alms[:3], cl, cl, q, g, V)
    Fm = 0.0
    for a in alms[:3]:
        J = om.jacobian(a, cl, q, g, V)
        Fm = Fm + ((J.real * vre) @ J.real.T + (J.imag * vim) @ J.imag.T) / 18.0
    assert np.allclose(F, Fm / 3, rtol=1e-12, atol=1e-14)


def test_p10_linear_term_reduces_variance_with_mask_and_noise():
    """Appendix A: without the linear term, inhomogeneous noise and a mask add
    cross terms to the variance; subtracting the MC linear term removes them."""
    base = mi.CONFIGS["tiny"]
    c = mi.Config("tiny-wmap", 9, base.lmax, base.ntheta, base.nphi, 6, 0, "wmap", "f64")
    g = osims.wmap_like_grid(c)
    cl = mi.filter_cl(c.lmax, "wmap")
    q = mi.q_basis(c.P, c.lmax)
    mc = np.array([osims.sky_sim(c, 5000 + i, g) for i in range(150)])
    V = om.pair_means(om.filtered_maps(mc, cl, q, g))
    test = np.array([osims.sky_sim(c, i, g) for i in range(150)])
    M = om.filtered_maps(test, cl, q, g)
    B = np.array([om.beta(Mi, g.w) for Mi in M])
    Bh = np.array([om.beta_hat(Mi, g.w, V) for Mi in M])
    # paired comparison on the same maps: per-map excess of sum_n beta_n^2 over
    # sum_n beta^hat_n^2 (means removed, each mode scaled by its beta spread)
    # must be significantly positive
    sd = B.std(0)
    d = np.sum(((B - B.mean(0)) / sd) ** 2 - ((Bh - Bh.mean(0)) / sd) ** 2, axis=1)
    assert d.mean() / (d.std(ddof=1) / math.sqrt(d.size)) > 4.0
    assert np.mean(Bh.var(0) / B.var(0)) < 0.97
