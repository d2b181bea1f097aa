"""The differentiation workload at its own shape: l_max 500, Gauss-Legendre 768 x 1536,
P = 30 modes (n_max 4,960), the WMAP-like sky recipe (a_lm of the filter spectrum
f_sky (b_l^2 C_l + N_l), the |lat| < 10 deg cut in the pixel weights).

* The FP32 adjoint (modal_beta_vjp) against central finite differences with h = 1e-4
  relative on 64 random real degrees of freedom, taken with the FP64 context of the same
  shape (whose maps and beta are pinned to the oracle at smaller shapes): beta^hat is cubic
  in a, so the central difference is exact up to h^2 (1e-8 relative).
* The Fisher covariance from the gradients of 256 simulations, then the estimator with it
  (eqs. modalest, modalvariance): zeta_F must factor in FP64, and for the same 256
  Gaussian skies (linear term from all of them, each sky's own maps left out: modal_beta_loo)
  E must average to zero within 4 standard errors and scatter with variance sigma^2
  within 4 standard errors of a variance estimate: E[J C J^T] = 18 zeta for Gaussian a_lm of
  covariance C, and the skies are drawn with exactly the C given to the Fisher call.
"""
import math

import numpy as np
import pytest

import modal_inputs as mi
from oracle import grid as og

from test_gpu_parity import log_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

LMAX, NT, NPHI, P = 500, 768, 1536, 30
CFG = mi.CONFIGS["adjoint500"]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _ctx(prec):
    from paper_1105_2791_amd import ModalContext
    g0 = og.Grid(NT, NPHI)
    mask = np.repeat(mi.mask_rings(g0.theta)[:, None], NPHI, axis=1)
    return ModalContext(LMAX, NT, NPHI, P, prec, mi.q_basis(P, LMAX), mi.filter_cl(LMAX, "wmap"), mask=mask)


def _skies(first, n):
    cl = mi.filter_cl(LMAX, "wmap")
    return np.array([mi.gaussian_alm(cl, LMAX, mi.rng_for(CFG.cfg_id, first + i)) for i in range(n)])


def _state(c, mc):
    st = c.linear_state()
    c.linear_reset(st)
    for i in range(0, len(mc), 8):
        c.linear_accumulate(st, mc[i:i + 8])
    c.linear_finalize(st)
    return st


def test_adjoint500_fp32_vjp_against_fp64_central_differences():
    print("[case] adjoint500: contexts and states", flush=True)
    c32, c64 = _ctx("f32"), _ctx("f64")
    mc = _skies(100, 16)
    st32, st64 = _state(c32, mc), _state(c64, mc)
    a = _skies(0, 1)[0]
    rng = np.random.default_rng(31)
    cot = rng.standard_normal(c32.nmax)
    print("[case] adjoint500: fp32 vjp", flush=True)
    g = c32.beta_vjp(a[None], cot[None], state=st32).cpu().numpy()[0]
    l, m = mi.lm_arrays(LMAX)
    idx = rng.choice(np.where(l >= 2)[0], 64, replace=False)
    parts = [1.0 if m[k] == 0 or rng.random() < 0.5 else 1j for k in idx]
    hs, pert = [], []
    for k, part in zip(idx, parts):
        h = 1e-4 * max(abs(a[k]), math.sqrt(mi.filter_cl(LMAX, "wmap")[l[k]] / 2))
        hs.append(h)
        for f in (1, -1):
            e = a.copy()
            e[k] += f * h * part
            pert.append(e)
    print("[case] adjoint500: fp64 central differences (128 skies)", flush=True)
    B = np.concatenate([c64.beta(np.array(pert[i:i + 16]), state=st64).cpu().numpy() @ cot
                        for i in range(0, len(pert), 16)]).reshape(64, 2)
    fd = (B[:, 0] - B[:, 1]) / (2.0 * np.array(hs))
    got = np.array([g[k].real if p == 1.0 else g[k].imag for k, p in zip(idx, parts)])
    err = float(np.max(np.abs(got - fd)) / np.sqrt(np.mean(fd ** 2)))
    log_err("adjoint500 fp32 vjp vs fp64 central differences", err)
    assert err < 1e-4
    c32.close()
    c64.close()


def test_adjoint500_fisher_from_256_sims_and_estimator():
    c = _ctx("f32")
    N = 256
    print("[case] adjoint500: 256 skies, linear-term state", flush=True)
    sk = _skies(1000, N)
    st = _state(c, sk)
    cl = mi.filter_cl(LMAX, "wmap")
    print("[case] adjoint500: Fisher covariance from 256 gradients", flush=True)
    zf = c.covariance_fisher(sk, cl, state=st)
    Z = zf.cpu().numpy()
    assert np.all(np.isfinite(Z)) and np.max(np.abs(Z - Z.T)) <= 1e-12 * np.max(np.abs(Z))
    assert np.all(np.diag(Z) > 0)
    one = np.ones(LMAX + 1)
    alpha = c.alpha_separable(np.array([[2 * cl, cl, one], [2 * cl, one, cl], [2 * one, cl, cl]]))
    print("[case] adjoint500: beta^hat (leave-one-out) and the estimator", flush=True)
    bh = torch.cat([c.beta_loo(sk[i:i + 8], st) for i in range(0, N, 8)])
    E, s2 = c.fnl(zf, alpha, bh)
    se = math.sqrt(s2 / N)
    log_err("adjoint500 estimator mean / standard error", abs(E.mean()) / se)
    log_err("adjoint500 var(E) / sigma^2 - 1", abs(E.var(ddof=1) / s2 - 1.0))
    print(f"[adjoint500] <E> = {E.mean():.3e} +- {se:.3e}, var(E)/sigma^2 = {E.var(ddof=1) / s2:.3f}", flush=True)
    assert abs(E.mean()) < 4 * se
    assert abs(E.var(ddof=1) / s2 - 1.0) < 4 * math.sqrt(2.0 / (N - 1))
    c.close()
