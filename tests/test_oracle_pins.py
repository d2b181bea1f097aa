"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the pin and the passage it follows.  They are chosen so that a
plausible slip anywhere in the oracle (a dropped m > 0 factor of 2, a wrong
Condon-Shortley sign, a transposed operand, a missing pairing in the linear
term, the wrong 6 in sigma^2, a swapped Re/Im in the gradient) fails at least
one of them.
"""
import math

import numpy as np
import pytest

import modal_inputs as mi
from oracle import closed_forms as cf
from oracle import grid as og
from oracle import legendre as ol
from oracle import modal as om
from oracle import sims as osims
from oracle import wigner as ow


def exact_grid(lmax):
    """Grid on which a triple product of l <= lmax harmonics is integrated exactly."""
    nt = (3 * lmax + 2) // 2 + 1
    return og.Grid(nt, 3 * lmax + 2)


# ---------------------------------------------------------------------------
# P1: orthonormality of Y_lm under the grid quadrature (Sec. II: R R^T = I for
# an orthonormal harmonic basis; the grid sum must reproduce it)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("lmax,nt,nphi", [(32, 48, 96), (500, 768, 1536)])
def test_p1_orthonormality_ring(lmax, nt, nphi):
    g = og.Grid(nt, nphi)
    ms = [0, 1, 2, lmax // 3, lmax - 1, lmax] if lmax > 40 else range(lmax + 1)
    for m in ms:
        lam = ol.lambda_m(m, lmax, g.x)
        gram = (lam * g.wgl) @ lam.T * 2.0 * math.pi
        # FP64 round-off of an l_max-step recurrence plus the quadrature sum
        assert np.max(np.abs(gram - np.eye(lam.shape[0]))) < 2e-14 * lmax, m


def test_p1_orthonormality_full_grid():
    lmax, g = 6, og.Grid(8, 16)
    th, ph = np.meshgrid(g.theta, g.phi, indexing="ij")
    lms = [(l, m) for l in range(lmax + 1) for m in range(-l, l + 1)]
    Y = np.array([ol.ylm(l, m, th, ph).ravel() for l, m in lms])
    gram = (Y * g.w.ravel()) @ Y.conj().T
    assert np.max(np.abs(gram - np.eye(len(lms)))) < 1e-13


# ---------------------------------------------------------------------------
# P2: low-l closed forms and an independent special-function library
# ---------------------------------------------------------------------------

def test_p2_low_l_closed_forms():
    th = np.linspace(0.05, math.pi - 0.05, 9)
    ph = np.linspace(0.0, 2 * math.pi, 9)
    assert np.allclose(ol.ylm(0, 0, th, ph), 1 / math.sqrt(4 * math.pi), atol=1e-15)
    assert np.allclose(ol.ylm(1, 0, th, ph), math.sqrt(3 / (4 * math.pi)) * np.cos(th), atol=1e-15)
    assert np.allclose(ol.ylm(1, 1, th, ph), -math.sqrt(3 / (8 * math.pi)) * np.sin(th) * np.exp(1j * ph), atol=1e-15)
    assert np.allclose(ol.ylm(2, -1, th, ph), math.sqrt(15 / (8 * math.pi)) * np.sin(th) * np.cos(th) * np.exp(-1j * ph), atol=1e-15)


def test_p2_against_scipy():
    sp = pytest.importorskip("scipy.special")
    th = np.array([0.1, 0.7, 1.3, 2.0, 3.0])
    ph = np.array([0.3, 1.1, 2.5, 4.0, 5.9])
    for l in [0, 1, 5, 17, 64, 200]:
        for m in sorted({0, min(1, l), l // 2, l}):
            ref = sp.sph_harm_y(l, m, th, ph)
            got = ol.ylm(l, m, th, ph)
            assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref))), (l, m)


# ---------------------------------------------------------------------------
# P3: high-l recurrence with log-scaled seeds (Unsoeld's theorem and parity)
# ---------------------------------------------------------------------------

def test_p3_unsold_lmax2000():
    lmax = 2000
    x = np.cos(np.array([1e-3, 0.01, 0.3, 1.0, 1.5707]))
    acc = np.zeros((lmax + 1, x.size))
    for m in range(lmax + 1):
        lam = ol.lambda_m(m, lmax, x)
        acc[m:] += (1.0 if m == 0 else 2.0) * lam * lam
    l = np.arange(lmax + 1)
    target = ((2 * l + 1) / (4 * math.pi))[:, None]
    assert np.max(np.abs(acc / target - 1.0)) < 1e-11


def test_p3_parity():
    lmax = 300
    x = np.array([0.9, 0.31, 0.02])
    for m in [0, 1, 7, 150, 300]:
        a = ol.lambda_m(m, lmax, x)
        b = ol.lambda_m(m, lmax, -x)
        sgn = np.array([(-1) ** (l + m) for l in range(m, lmax + 1)])[:, None]
        assert np.max(np.abs(b - sgn * a)) < 1e-12


# ---------------------------------------------------------------------------
# P4: Gaunt integral on an exact grid vs the Wigner-3j closed form (Sec. II)
# ---------------------------------------------------------------------------

def test_p4_gaunt_vs_3j():
    lmax = 8
    g = exact_grid(lmax)
    th, ph = np.meshgrid(g.theta, g.phi, indexing="ij")
    rng = np.random.default_rng(5)
    cache = {}

    def Y(l, m):
        if (l, m) not in cache:
            cache[(l, m)] = ol.ylm(l, m, th, ph)
        return cache[(l, m)]
    checked = 0
    for _ in range(300):
        l1, l2, l3 = rng.integers(0, lmax + 1, 3)
        m1 = int(rng.integers(-l1, l1 + 1))
        m2 = int(rng.integers(-l2, l2 + 1))
        m3 = -m1 - m2
        if abs(m3) > l3:
            continue
        num = np.sum(g.w * Y(l1, m1) * Y(l2, m2) * Y(l3, m3))
        ref = ow.gaunt(int(l1), int(l2), int(l3), m1, m2, m3)
        assert abs(num - ref) < 1e-13, (l1, l2, l3, m1, m2, m3)
        checked += 1
    assert checked > 100


def test_p4_3j_known_values():
    # (1 1 0; 0 0 0) = -1/sqrt(3); (1 1 2; 0 0 0) = sqrt(2/15); (2 2 2; 0 0 0) = -sqrt(2/35)
    assert abs(ow.wigner3j(1, 1, 0, 0, 0, 0) + 1 / math.sqrt(3)) < 1e-15
    assert abs(ow.wigner3j(1, 1, 2, 0, 0, 0) - math.sqrt(2 / 15)) < 1e-15
    assert abs(ow.wigner3j(2, 2, 2, 0, 0, 0) + math.sqrt(2 / 35)) < 1e-15
    # orthogonality sum_{m1 m2} (j1 j2 j; m1 m2 m)^2 = 1/(2j+1)
    j1, j2, j = 3, 2, 4
    s = sum(ow.wigner3j(j1, j2, j, m1, m2, -m1 - m2) ** 2
            for m1 in range(-j1, j1 + 1) for m2 in range(-j2, j2 + 1) if m1 + m2 == 0)
    assert abs(s - 1 / 9) < 1e-14


# ---------------------------------------------------------------------------
# P5: pixel-space beta equals the brute-force Gaunt triple sum (eq. bbispect)
# ---------------------------------------------------------------------------

def _full_alm(a, lmax):
    """dict (l, m) -> a_lm for all m via a_{l,-m} = (-1)^m a_lm^*."""
    out = {}
    for l in range(lmax + 1):
        for m in range(0, l + 1):
            v = a[mi.alm_index(l, m, lmax)]
            out[(l, m)] = v
            if m:
                out[(l, -m)] = (-1) ** m * np.conj(v)
    return out


def test_p5_beta_brute_force():
    lmax, P = 5, 3
    g = exact_grid(lmax)
    cl = mi.cl_signal(lmax)
    q = mi.q_basis(P, lmax)
    a = mi.gaussian_alm(cl, lmax, mi.rng_for(99, 0))
    at = _full_alm(om.whiten(a, cl, lmax), lmax)
    M = om.filtered_maps(a, cl, q, g)
    beta = om.beta(M, g.w)
    ref = np.zeros(len(beta))
    lms = list(at.keys())
    for n, (p, r, s) in enumerate(mi.triple_list(P)):
        tot = 0.0
        for (l1, m1) in lms:
            for (l2, m2) in lms:
                m3 = -m1 - m2
                for l3 in range(abs(m3), lmax + 1):
                    gnt = ow.gaunt(l1, l2, l3, m1, m2, m3)
                    if gnt == 0.0:
                        continue
                    tot += gnt * q[p, l1] * q[r, l2] * q[s, l3] * at[(l1, m1)] * at[(l2, m2)] * at[(l3, m3)]
        ref[n] = tot.real
    assert np.max(np.abs(beta - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


# ---------------------------------------------------------------------------
# P6: Parseval for the filtered maps (orthonormal harmonic basis, Sec. II)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("cfg", ["tiny"])
def test_p6_parseval(cfg):
    c = mi.CONFIGS[cfg]
    g = og.Grid(c.ntheta, c.nphi)
    cl = mi.cl_signal(c.lmax)
    q = mi.q_basis(c.P, c.lmax)
    a = mi.gaussian_alm(cl, c.lmax, mi.rng_for(c.cfg_id, 3))
    at = om.whiten(a, cl, c.lmax)
    l, m = mi.lm_arrays(c.lmax)
    power = np.zeros(c.lmax + 1)
    np.add.at(power, l, np.where(m == 0, 1.0, 2.0) * np.abs(at) ** 2)
    M = om.filtered_maps(a, cl, q, g)
    for p, r in mi.pair_list(c.P):
        lhs = np.sum(g.w * M[p] * M[r])
        rhs = np.sum(q[p] * q[r] * power)
        assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(rhs))


def test_maps_fft_equals_explicit_sum():
    lmax, g = 7, og.Grid(10, 20)
    cl = mi.cl_signal(lmax)
    q = mi.q_basis(2, lmax)
    a = mi.gaussian_alm(cl, lmax, mi.rng_for(1, 1))
    M = om.filtered_maps(a, cl, q, g)
    at = _full_alm(om.whiten(a, cl, lmax), lmax)
    th, ph = np.meshgrid(g.theta, g.phi, indexing="ij")
    ref = np.zeros((2,) + th.shape)
    for (l, m), v in at.items():
        y = ol.ylm(l, m, th, ph)
        for p in range(2):
            ref[p] += (q[p, l] * v * y).real
    assert np.max(np.abs(M - ref)) < 1e-13


# ---------------------------------------------------------------------------
# P10: the linear term is the Monte-Carlo mean gradient contracted with a
# (eq. linearterm: the linear term removes exactly the pairings of the data
# with itself) - an exact algebraic identity for the same MC set.
# ---------------------------------------------------------------------------

def test_p10_linear_term_is_mean_gradient():
    c = mi.CONFIGS["tiny"]
    lmax, P = 12, 3
    g = og.Grid(20, 40)
    cl = mi.cl_signal(lmax)
    q = mi.q_basis(P, lmax)
    mc = [mi.gaussian_alm(cl, lmax, mi.rng_for(c.cfg_id, 100 + i)) for i in range(4)]
    Ms = om.filtered_maps(np.array(mc), cl, q, g)
    V = om.pair_means(Ms)
    a = mi.gaussian_alm(cl, lmax, mi.rng_for(c.cfg_id, 7))
    lin = om.linear_term(om.filtered_maps(a, cl, q, g), g.w, V)
    # <grad beta>(a^(i)) . a averaged over the MC maps; gradient of beta alone (V=None)
    nmax = mi.ntriples(P)
    l, m = mi.lm_arrays(lmax)
    acc = np.zeros(nmax)
    for ai in mc:
        J = om.vjp(ai, cl, q, g, None, np.eye(nmax))          # [nmax, nalm]
        acc += J.real @ a.real + J.imag @ a.imag
    acc /= len(mc)
    assert np.max(np.abs(acc - lin)) < 1e-11 * max(1.0, np.max(np.abs(lin)))


# ---------------------------------------------------------------------------
# P11: Cholesky / inverse / estimator against the bivector closed forms (Sec. III B)
# ---------------------------------------------------------------------------

def test_p11_bivector_closed_forms():
    rng = np.random.default_rng(11)
    n = 37
    bt = rng.standard_normal(n) * 0.7
    Z = cf.bivector_zeta(bt)
    L = cf.bivector_cholesky(bt)
    assert np.max(np.abs(L @ L.T - Z)) < 1e-12
    assert np.max(np.abs(np.linalg.cholesky(Z) - L)) < 1e-12
    assert np.max(np.abs(cf.bivector_inverse(bt) @ Z - np.eye(n))) < 1e-12
    alpha = rng.standard_normal(n)
    betas = rng.standard_normal((5, n))
    E, s2, Lo = om.estimator(Z, alpha, betas)
    assert np.max(np.abs(Lo - L)) < 1e-12
    # sigma^2 = 6 / alpha^T zeta^-1 alpha; bivector formula gives 1 / alpha^T zeta^-1 alpha
    assert abs(s2 - 6.0 * cf.bivector_variance(alpha, bt)) < 1e-12 * s2
    Zi = cf.bivector_inverse(bt)
    ref = betas @ Zi @ alpha / (alpha @ Zi @ alpha)
    assert np.max(np.abs(E - ref)) < 1e-12
    # E(beta = alpha) = 1, and invariance under a change of basis T (Sec. II, Cholesky rotation)
    E1, _, _ = om.estimator(Z, alpha, alpha[None, :])
    assert abs(E1[0] - 1.0) < 1e-13
    T = np.eye(n) + 0.1 * rng.standard_normal((n, n))
    E2, s22, _ = om.estimator(T @ Z @ T.T, T @ alpha, betas @ T.T)
    assert np.max(np.abs(E2 - E)) < 1e-10 and abs(s22 - s2) < 1e-10 * s2


# ---------------------------------------------------------------------------
# P13: gradient - finite differences and Euler homogeneity
# ---------------------------------------------------------------------------

def _gradient_setup():
    lmax, P = 10, 3
    g = og.Grid(17, 32, ring_mask=np.repeat(mi.mask_rings(og.Grid(17, 32).theta)[:, None], 32, axis=1))
    cl = mi.cl_signal(lmax)
    q = mi.q_basis(P, lmax)
    mc = np.array([mi.gaussian_alm(cl, lmax, mi.rng_for(3, 200 + i)) for i in range(3)])
    V = om.pair_means(om.filtered_maps(mc, cl, q, g))
    a = mi.gaussian_alm(cl, lmax, mi.rng_for(3, 5))
    return lmax, P, g, cl, q, V, a


def test_p13_gradient_finite_difference():
    lmax, P, g, cl, q, V, a = _gradient_setup()
    rng = np.random.default_rng(13)
    cot = rng.standard_normal(mi.ntriples(P))
    grad = om.vjp(a, cl, q, g, V, cot)[0]

    def f(aa):
        return float(cot @ om.beta_hat(om.filtered_maps(aa, cl, q, g), g.w, V))
    l, m = mi.lm_arrays(lmax)
    for k in [mi.alm_index(2, 0, lmax), mi.alm_index(5, 3, lmax), mi.alm_index(10, 10, lmax), mi.alm_index(7, 1, lmax)]:
        for part in ([1.0] if m[k] == 0 else [1.0, 1j]):
            h = 1e-3 * math.sqrt(cl[l[k]])
            e = np.zeros_like(a)
            e[k] = part
            # 4-point stencil is exact for cubic polynomials in h
            d = (8 * (f(a + h * e) - f(a - h * e)) - (f(a + 2 * h * e) - f(a - 2 * h * e))) / (12 * h)
            got = grad[k].real if part == 1.0 else grad[k].imag
            assert abs(got - d) < 1e-9 * max(1.0, abs(d)), (k, part, got, d)


def test_p13_euler_homogeneity():
    lmax, P, g, cl, q, V, a = _gradient_setup()
    nmax = mi.ntriples(P)
    J = om.vjp(a, cl, q, g, V, np.eye(nmax))
    lhs = J.real @ a.real + J.imag @ a.imag
    M = om.filtered_maps(a, cl, q, g)
    rhs = 3 * om.beta(M, g.w) - om.linear_term(M, g.w, V)
    assert np.max(np.abs(lhs - rhs)) < 1e-11 * max(1.0, np.max(np.abs(rhs)))


# ---------------------------------------------------------------------------
# sims: analysis inverts synthesis on an exact grid (generator sanity)
# ---------------------------------------------------------------------------

def test_sims_analysis_inverts_synthesis():
    lmax = 20
    g = og.Grid(32, 64)
    a = mi.gaussian_alm(mi.cl_signal(lmax) + 1e-3, lmax, mi.rng_for(0, 0))
    f = osims.synth_scalar(a, lmax, g)
    b = osims.analysis(f, lmax, g)
    assert np.max(np.abs(a - b)) < 1e-13


def test_p9_pair_mean_fullsky_is_the_addition_theorem():
    """<M_p(x) M_r(x)> over isotropic skies with <|a~_lm|^2> = c_l is
    sum_l c_l q_p q_r sum_m |Y_lm(x)|^2 at every point x.  The m-sum is taken from the
    oracle's own lambda_lm recurrence (sum over -l..l = lambda_l0^2 + 2 sum_{m>0}
    lambda_lm^2), so the closed form's (2l+1)/(4 pi) is checked against the harmonics
    the maps are built from, at several colatitudes."""
    lmax, P = 24, 4
    q = mi.q_basis(P, lmax)
    c = mi.cl_signal(lmax) * (1.0 + np.arange(lmax + 1) % 3)       # any spectrum
    ref = cf.pair_mean_fullsky(q, c)
    x = np.cos(np.array([0.05, 0.7, 1.3, 1.5707963, 2.4, 3.1]))
    msum = np.zeros((lmax + 1, x.size))
    for m in range(lmax + 1):
        lam = ol.lambda_m(m, lmax, x)                                  # [lmax + 1 - m, nx]
        msum[m:] += (1.0 if m == 0 else 2.0) * lam ** 2
    for j in range(x.size):
        got = np.array([np.sum(c * q[p] * q[r] * msum[:, j]) for p, r in mi.pair_list(P)])
        assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))


def test_c12_noise_power_of_the_sim_generator():
    """The generator's pixel noise (variance sigma^2(theta) Omega_bar / dA per pixel,
    independent pixels) analysed on an unmasked grid has the harmonic power nl at every l:
    E|a_lm|^2 = sum_x var_x |d a_lm / d f_x|^2, with d a_lm / d f_x the oracle's analysis of
    a unit impulse (the same on every pixel of a ring up to a phase); the m-average
    (|a_l0|^2 + 2 sum_{m>0} |a_lm|^2) / (2l + 1) must be nl = Omega_bar <sigma^2>."""
    lmax = 20
    g = og.Grid(40, 80)
    nl = 3.7e-6
    var = osims.noise_pixel_variance(g, nl)
    E = np.zeros(mi.nalm(lmax))
    for j in range(g.x.size):
        f = np.zeros((g.x.size, g.nphi))
        f[j, 0] = 1.0
        E += g.nphi * var[j, 0] * np.abs(osims.analysis(f, lmax, g)) ** 2
    l, m = mi.lm_arrays(lmax)
    for ll in range(lmax + 1):
        per_l = (E[(l == ll) & (m == 0)].sum() + 2.0 * E[(l == ll) & (m > 0)].sum()) / (2 * ll + 1)
        assert abs(per_l / nl - 1.0) < 1e-12, (ll, per_l / nl)
    # a Monte-Carlo draw of the same noise agrees within its scatter
    rng = np.random.default_rng(3)
    acc = np.zeros(mi.nalm(lmax))
    n = 40
    for _ in range(n):
        acc += np.abs(osims.analysis(rng.standard_normal(var.shape) * np.sqrt(var), lmax, g)) ** 2
    assert abs(np.sum(acc / n) / np.sum(E) - 1.0) < 0.05


def test_centered_sample_covariance():
    """The mean-subtracted sample covariance: numpy's own unbiased covariance / 6; for
    N = 2 it is (b1 - b2)(b1 - b2)^T / 12; a common shift of all rows changes nothing; for
    rows of zero sample mean it is N / (N - 1) times the uncentered covariance."""
    rng = np.random.default_rng(11)
    B = rng.standard_normal((7, 5))
    Z = om.covariance_sample(B, centered=True)
    assert np.max(np.abs(Z - np.cov(B, rowvar=False, ddof=1) / 6.0)) < 1e-15
    d = B[0] - B[1]
    assert np.max(np.abs(om.covariance_sample(B[:2], centered=True) - np.outer(d, d) / 12.0)) < 1e-15
    shift = rng.standard_normal(5) * 10
    assert np.max(np.abs(om.covariance_sample(B + shift, centered=True) - Z)) < 1e-13
    B0 = B - B.mean(axis=0)
    assert np.max(np.abs(om.covariance_sample(B0, centered=True) * 6 / 7 - om.covariance_sample(B0))) < 1e-15


def test_leave_one_out_beta_hat():
    """beta^hat with sky i's own maps left out of the pair means equals
    ((N + 2) beta_i - N lin_i(V over all N)) / (N - 1): V^(-i) = (N V - M_p M_r) / (N - 1)
    and the three pairings of M_p M_r M_s sum to 3 beta.  For N = 2 the other sky alone
    makes the pair means."""
    lmax, nt, nphi, P = 12, 20, 40, 4
    g = og.Grid(nt, nphi)
    cl = mi.filter_cl(lmax, "wmap")
    q = mi.q_basis(P, lmax)
    alms = np.array([mi.gaussian_alm(cl, lmax, mi.rng_for(5, i)) for i in range(4)])
    Ms = om.filtered_maps(alms, cl, q, g)
    N = Ms.shape[0]
    V = om.pair_means(Ms)
    for i in range(N):
        loo = om.beta_hat_leave_one_out(Ms, g.w, i)
        b = om.beta(Ms[i], g.w)
        lin = om.linear_term(Ms[i], g.w, V)
        alt = ((N + 2) * b - N * lin) / (N - 1)
        assert np.max(np.abs(loo - alt)) < 1e-12 * np.max(np.abs(b))
    two = om.beta_hat_leave_one_out(Ms[:2], g.w, 0)
    ref = om.beta(Ms[0], g.w) - om.linear_term(Ms[0], g.w, om.pair_means(Ms[1:2]))
    assert np.max(np.abs(two - ref)) < 1e-13 * np.max(np.abs(ref))


def test_ring_chunked_beta_and_linear_term_equal_whole_grid():
    """beta and lin are pixel sums and V a per-pixel mean, so summing the definitions over
    ring groups (7 rings, a ragged last group, a masked grid) gives the whole-grid values."""
    import modal_inputs as mi
    from oracle import grid as og
    from oracle import modal as om
    lmax, nt, nphi, P = 16, 25, 50, 5
    g0 = og.Grid(nt, nphi)
    g = og.Grid(nt, nphi, ring_mask=np.repeat(mi.mask_rings(g0.theta)[:, None], nphi, 1))
    cl = mi.filter_cl(lmax, "wmap")
    q = mi.q_basis(P, lmax)
    alms = np.array([mi.gaussian_alm(cl, lmax, mi.rng_for(77, i)) for i in range(2)])
    mc = np.array([mi.gaussian_alm(cl, lmax, mi.rng_for(77, 10 + i)) for i in range(3)])
    b, lin = om.beta_and_linear_by_rings(alms, mc, cl, q, g, rings_per_chunk=7)
    M = om.filtered_maps(alms, cl, q, g)
    V = om.pair_means(om.filtered_maps(mc, cl, q, g))
    for s in range(2):
        ref_b = om.beta(M[s], g.w)
        ref_l = om.linear_term(M[s], g.w, V)
        assert np.max(np.abs(b[s] - ref_b)) < 1e-12 * np.sqrt(np.mean(ref_b ** 2))
        assert np.max(np.abs(lin[s] - ref_l)) < 1e-12 * np.sqrt(np.mean(ref_l ** 2))
    b2, none = om.beta_and_linear_by_rings(alms, None, cl, q, g, rings_per_chunk=25)
    assert none is None and np.allclose(b2, b, rtol=0, atol=1e-12 * np.abs(b).max())


def test_sims_cached_lambda_table_is_the_same_transform():
    """Synthesis and analysis with a lambda table computed once give the same numbers as the
    per-call recurrence, and the analysis inverts the synthesis on an exact grid."""
    from oracle import legendre as ol
    lmax = 16
    g = og.Grid(26, 52)
    lam = ol.lambda_table(lmax, g.x)
    a = mi.gaussian_alm(mi.cl_signal(lmax), lmax, mi.rng_for(9, 0))
    f1 = osims.synth_scalar(a, lmax, g)
    f2 = osims.synth_scalar(a, lmax, g, lam)
    assert np.max(np.abs(f1 - f2)) < 1e-14
    assert np.max(np.abs(osims.analysis(f1, lmax, g) - osims.analysis(f1, lmax, g, lam))) < 1e-14
    assert np.max(np.abs(osims.analysis(f2, lmax, g, lam) - a)) < 1e-13
