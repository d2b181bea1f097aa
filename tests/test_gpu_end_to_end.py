"""End to end on the GPU: toy non-Gaussian skies with a known separable bispectrum.

T(x) is a full-sky Gaussian field with spectrum C_l; T + f (T^2 - <T^2>) has, to
first order in f, the reduced bispectrum b = 2 f (C_l1 C_l2 + C_l2 C_l3 + C_l1 C_l3).
With alpha from modal_alpha_separable for f = 1, beta from modal_beta, and the
ideal full-sky covariance from modal_ideal_covariance, the estimator
E = alpha^T zeta^-1 beta / alpha^T zeta^-1 alpha (modal_fnl) must average to f
(eq. modalest), to f = 0 on the Gaussian skies, whose scatter must match
sigma^2 = 6 / alpha^T zeta^-1 alpha (eq. modalvariance).  Statistical bounds: 4
standard errors; the O(f^3) bias at f sigma_T ~ 0.1 is about 1 % of f.

The skies are drawn and analysed by the oracle's sky generator (synthesis,
squaring on a grid exact for the product, quadrature analysis); every estimator
step runs in the library.
"""
import math

import numpy as np
import pytest

import modal_inputs as mi
from oracle import grid as og
from oracle import sims as osims

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LMAX, P, N = 32, 8, 240


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _skies(f, first):
    cl = mi.cl_signal(LMAX)
    var = float(np.sum((2.0 * np.arange(LMAX + 1) + 1.0) * cl) / (4.0 * math.pi))
    g = og.Grid(64, 128)            # exact for T^2 Y_lm at l_max 32
    out = []
    for i in range(N):
        a = mi.gaussian_alm(cl, LMAX, mi.rng_for(77, first + i))
        if f:
            T = osims.synth_scalar(a, LMAX, g)
            a = osims.analysis(T + f * (T * T - var), LMAX, g)
        out.append(a)
    return np.array(out), var


@pytest.mark.parametrize("prec", ["f64", "bf16x3"])
def test_local_toy_estimator_recovers_f(prec):
    from paper_1105_2791_amd import ModalContext
    cl = mi.cl_signal(LMAX)
    c = ModalContext(LMAX, 64, 128, P, prec, mi.q_basis(P, LMAX), cl)
    one = np.ones(LMAX + 1)
    alpha = c.alpha_separable(np.array([[2 * cl, cl, one], [2 * cl, one, cl], [2 * one, cl, cl]]))
    zeta0 = c.ideal_covariance()
    print(f"[end to end] {prec}: Gaussian skies", flush=True)
    aG, var = _skies(0.0, 0)
    EG, s2 = c.fnl(zeta0, alpha, c.beta(aG).reshape(N, -1))
    sigma = math.sqrt(s2)
    se = sigma / math.sqrt(N)
    assert abs(EG.mean()) < 4 * se, (EG.mean(), se)
    assert abs(EG.var(ddof=1) / s2 - 1.0) < 4 * math.sqrt(2.0 / (N - 1)), (EG.var(ddof=1), s2)
    f = 8 * se                      # an 8-sigma signal in the mean of N skies
    print(f"[end to end] {prec}: non-Gaussian skies f={f:.4f} (f sigma_T = {f * math.sqrt(var):.3f})", flush=True)
    aN, _ = _skies(f, 0)            # same Gaussian seeds: the scatter of E - E_G is small
    EN, _ = c.fnl(zeta0, alpha, c.beta(aN).reshape(N, -1))
    d = EN - EG
    assert abs(EN.mean() - f) < 4 * se + 0.03 * f, (EN.mean(), f, se)
    # with shared seeds the f-response is measured far more precisely than either mean
    assert abs(d.mean() / f - 1.0) < 4 * d.std(ddof=1) / math.sqrt(N) / f + 0.03, (d.mean(), f)


LMAX_F, P_F, N_F = 500, 40, 48


def test_local_toy_frame_lmax500_recovers_f():
    """The same toy at l_max 500, P 40 (n_max 11,480 modes): the ideal covariance is too
    ill-conditioned for a full Cholesky, so the estimator runs in the truncated orthonormal
    frame (modal_frame, modal_fnl_frame).  The skies come from the oracle's generator on a
    768 x 1536 Gauss-Legendre grid, exact for T^2 Y_lm at l_max 500 (degree 1500)."""
    from paper_1105_2791_amd import ModalContext
    from oracle import legendre as ol
    import time
    cl = mi.cl_signal(LMAX_F)
    var = float(np.sum((2.0 * np.arange(LMAX_F + 1) + 1.0) * cl) / (4.0 * math.pi))
    t0 = time.perf_counter()
    g = og.Grid(768, 1536)
    lam = ol.lambda_table(LMAX_F, g.x)
    aG = np.array([mi.gaussian_alm(cl, LMAX_F, mi.rng_for(78, i)) for i in range(N_F)])
    c = ModalContext(LMAX_F, 768, 1536, P_F, "bf16x3", mi.q_basis(P_F, LMAX_F), cl)
    one = np.ones(LMAX_F + 1)
    alpha = c.alpha_separable(np.array([[2 * cl, cl, one], [2 * cl, one, cl], [2 * one, cl, cl]]))
    zeta0 = c.ideal_covariance()
    k, perm, L11 = c.frame(zeta0, 1e-10)
    print(f"[end to end] l_max 500 P 40: frame keeps {k} of {c.nmax} modes", flush=True)
    EG, s2 = c.fnl_frame(zeta0, perm, alpha, c.beta(aG))
    sigma = math.sqrt(s2)
    se = sigma / math.sqrt(N_F)
    print(f"[end to end] l_max 500: Gaussian <E> = {EG.mean():.4e}, sd {EG.std(ddof=1):.4e}, "
          f"sigma {sigma:.4e}", flush=True)
    assert abs(EG.mean()) < 4 * se, (EG.mean(), se)
    assert abs(EG.var(ddof=1) / s2 - 1.0) < 4 * math.sqrt(2.0 / (N_F - 1)), (EG.var(ddof=1), s2)
    f = 8 * se
    aN = []
    for a in aG:                    # same Gaussian seeds
        T = osims.synth_scalar(a, LMAX_F, g, lam)
        aN.append(osims.analysis(T + f * (T * T - var), LMAX_F, g, lam))
    print(f"[end to end] l_max 500: f = {f:.4e} (f sigma_T = {f * math.sqrt(var):.2e}), "
          f"skies in {time.perf_counter() - t0:.1f} s", flush=True)
    EN, _ = c.fnl_frame(zeta0, perm, alpha, c.beta(np.array(aN)))
    d = EN - EG
    print(f"[end to end] l_max 500: <E> = {EN.mean():.4e} for f = {f:.4e}; response "
          f"{d.mean() / f:.4f} +- {d.std(ddof=1) / math.sqrt(N_F) / f:.4f}", flush=True)
    assert abs(EN.mean() - f) < 4 * se + 0.03 * f, (EN.mean(), f, se)
    assert abs(d.mean() / f - 1.0) < 4 * d.std(ddof=1) / math.sqrt(N_F) / f + 0.03, (d.mean(), f)
    c.close()
