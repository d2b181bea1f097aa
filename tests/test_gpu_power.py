"""GPU parity of the modal power-spectrum estimator (Sec. IV) against the FP64 oracle.

beta: the maps carry the precision's synthesis error (MAP_TOL of the bispectrum
tests) and each pair sum doubles it; errors are max |diff| over the rms of the
unsubtracted pair sums (the size of the terms), so that the Monte-Carlo mean
subtraction does not inflate them.  alpha, the ideal covariance and the
estimator are FP64 sums in another order: 1e-11.  At l_max 1000 the oracle's
maps are out of reach; there the full-sky pixel sums are compared with the
harmonic form sum_lm q_p q_r |a~_lm|^2, which they equal exactly on an exact grid.
"""
import math

import numpy as np
import pytest

import modal_inputs as mi
from oracle import modal as om
from oracle import power as opw

from helpers import CASES

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {"f64": 1e-10, "f32": 2e-5, "bf16x3": 2e-4, "f16x3": 2e-5}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_ctx = {}


def ctx_case(case, prec):
    from paper_1105_2791_amd import ModalContext
    key = (case.name, prec)
    if key not in _ctx:
        print(f"[case] create {case.name} {prec}", flush=True)
        _ctx[key] = ModalContext(case.lmax, case.ntheta, case.nphi, case.P, prec, case.q, case.cl, mask=case.mask())
    return _ctx[key]


_or = {}


def oracle_case(case):
    if case.name not in _or:
        alms = case.alms(0, case.S)
        mc = case.alms(500, 4)
        M = case.maps(alms)
        V = om.pair_means(case.maps(mc))
        g = case.grid
        b0 = np.array([opw.power_beta(M[i], g.w) for i in range(case.S)])
        b1 = np.array([opw.power_beta(M[i], g.w, V) for i in range(case.S)])
        _or[case.name] = dict(alms=alms, mc=mc, b0=b0, b1=b1)
    return _or[case.name]


@pytest.mark.parametrize("name,prec", [("tiny", "f64"), ("tiny", "f32"), ("tiny", "bf16x3"), ("ragged", "f64"),
                                       ("ragged", "bf16x3"), ("ragged", "f16x3"), ("odd", "f32"), ("odd", "bf16x3")])
def test_power_beta_matches_oracle(name, prec):
    case = CASES[name]
    c = ctx_case(case, prec)
    o = oracle_case(case)
    print(f"[case] power beta {name} {prec}", flush=True)
    scale = np.sqrt(np.mean(o["b0"] ** 2))
    got0 = c.power_beta(o["alms"]).cpu().numpy()
    assert np.max(np.abs(got0 - o["b0"])) / scale < TOL[prec]
    st = c.linear_state()
    c.linear_reset(st)
    c.linear_accumulate(st, o["mc"][:3])
    c.linear_accumulate(st, o["mc"][3:])
    c.linear_finalize(st)
    got1 = c.power_beta(o["alms"], st).cpu().numpy()
    err = np.max(np.abs(got1 - o["b1"])) / scale
    print(f"[err] power beta {name} {prec}: {err:.3e}", flush=True)
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", ["bf16x3", "f32"])
def test_power_beta_metric_size_parseval(prec):
    """l_max 1000, GL 1536 x 3072, P 40 (820 pairs), full sky, 4 skies: every pair sum
    against sum_lm q_p(l) q_r(l) |a~_lm|^2."""
    from paper_1105_2791_amd import ModalContext
    lmax, P, S = 1000, 40, 4
    cl = mi.filter_cl(lmax, "wmap")
    q = mi.q_basis(P, lmax)
    print(f"[power] metric size {prec}", flush=True)
    c = ModalContext(lmax, 1536, 3072, P, prec, q, cl)
    alms = np.stack([mi.gaussian_alm(cl, lmax, mi.rng_for(93, i)) for i in range(S)])
    got = c.power_beta(alms).cpu().numpy()
    ref = np.array([opw.power_beta_harmonic(om.whiten(alms[i], cl, lmax), q, lmax) for i in range(S)])
    err = np.max(np.abs(got - ref)) / np.sqrt(np.mean(ref ** 2))
    print(f"[err] power beta metric {prec}: {err:.3e}", flush=True)
    assert err < TOL[prec]


def test_power_alpha_covariance_estimator_match_oracle():
    case = CASES["ragged"]
    c = ctx_case(case, "f64")
    rng = np.random.default_rng(95)
    dcl = case.cl * rng.standard_normal(case.lmax + 1) * 0.1
    a = c.power_alpha(dcl).cpu().numpy()
    ao = opw.power_alpha(dcl, case.cl, case.q)
    assert np.max(np.abs(a - ao)) < 1e-11 * np.max(np.abs(ao))
    cw = (case.cl > 0) * (1.0 + 0.01 * np.arange(case.lmax + 1))
    Z = c.power_ideal_covariance(cw)
    Zo = opw.power_ideal_covariance(case.q, cw)
    assert np.max(np.abs(Z.cpu().numpy() - Zo)) < 1e-11 * np.max(np.abs(Zo))
    assert a.shape == (case.P,) and Zo.shape == (case.P, case.P)
    betas = rng.standard_normal((5, c.npairs))           # the estimator uses the pairs (0, n): columns < P
    E, s2 = c.power_fnl(Z, a, betas)
    Eo, s2o = opw.power_estimator(Zo, ao, betas[:, :case.P])
    assert np.max(np.abs(E - Eo)) < 1e-9 * max(1.0, np.max(np.abs(Eo)))
    assert abs(s2 - s2o) < 1e-9 * s2o


def test_power_estimator_recovers_amplitude():
    """Gaussian skies with C~ = C (1 + eps g_l): <E> = eps and Var(E) = sigma^2 (4 standard
    errors), every step on the GPU (maps, pair sums, alpha, ideal covariance, Cholesky)."""
    case = CASES["tiny"]
    c = ctx_case(case, "f64")
    lmax, cl, N = case.lmax, case.cl, 400
    gl = 0.5 * mi.q_basis(3, lmax)[2]
    mean_fid = torch.as_tensor(opw.power_pair_mean(case.q, (cl > 0).astype(float)), device="cuda")
    assert torch.allclose(c.power_alpha(cl), mean_fid[:case.P], rtol=1e-12, atol=0)
    alpha = c.power_alpha(cl * gl)
    Z = c.power_ideal_covariance()
    out = {}
    for eps in (0.0, 0.04):
        alms = np.stack([mi.gaussian_alm(cl * (1.0 + eps * gl), lmax, mi.rng_for(96, i)) for i in range(N)])
        B = torch.cat([c.power_beta(alms[i:i + 50]) for i in range(0, N, 50)]) - mean_fid
        out[eps] = c.power_fnl(Z, alpha, B)
    E0, s2 = out[0.0]
    E1, _ = out[0.04]
    se = math.sqrt(s2 / N)
    assert abs(E0.mean()) < 4 * se
    assert abs(E0.var(ddof=1) / s2 - 1.0) < 4 * math.sqrt(2.0 / (N - 1))
    assert abs(E1.mean() - 0.04) < 4 * se * 1.1


def test_power_and_trispectrum_error_paths():
    """Host-side argument checks of the C ABI (no kernel runs): short workspace, null
    a_lm, no skies, a state that is not finalised."""
    from paper_1105_2791_amd import ModalError
    from paper_1105_2791_amd import _lib as L
    case = CASES["tiny"]
    c = ctx_case(case, "bf16x3")
    a = torch.as_tensor(case.alms(0, 1)).to("cuda", torch.complex64)
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    nq = c._lib.modal_nquad(c._h)
    for fn, width in ((c._lib.modal_power_beta, c.npairs), (c._lib.modal_trispectrum, nq)):
        out = torch.empty((1, width), dtype=torch.float64, device="cuda")
        assert fn(c._h, a.data_ptr(), 1, None, out.data_ptr(), ws.data_ptr(), 16, None) == L.ENOSPACE
        assert fn(c._h, None, 1, None, out.data_ptr(), ws.data_ptr(), 16, None) == L.EINVAL
        assert fn(c._h, a.data_ptr(), 0, None, out.data_ptr(), ws.data_ptr(), 16, None) == L.EINVAL
    st = c.linear_state()
    c.linear_reset(st)
    for call in (c.power_beta, c.trispectrum):
        with pytest.raises(ModalError) as ei:
            call(case.alms(0, 1), st)
        assert ei.value.status == L.ENOTREADY
