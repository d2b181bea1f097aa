"""The two flag variants of the linear term and the covariance, through the C ABI,
against the FP64 oracle:
  * modal_beta_loo: beta^hat of Monte-Carlo skies with each sky's own maps left out of
    the pair means (oracle: beta_hat_leave_one_out, the pair means recomputed over the
    other N - 1 skies);
  * MODAL_COV_SAMPLE_CENTERED: the mean-subtracted 1 / (6 (N - 1)) sample covariance.
Tolerances are those of the beta^hat parity tests."""
import numpy as np
import pytest

import modal_inputs as mi
from oracle import modal as om

from helpers import CASES, rel_inf
from test_gpu_parity import TOL, ctx_for, log_err, oracle_for

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("name,prec", [("tiny", "f64"), ("ragged", "f64"), ("ragged", "f32"),
                                       ("ragged", "bf16x3"), ("odd", "f16x3")])
def test_beta_loo_matches_oracle(name, prec):
    case = CASES[name]
    c = ctx_for(case, prec)
    o = oracle_for(case)
    print(f"[case] beta_loo {name} {prec}", flush=True)
    mc = o["mc"]
    st = c.linear_state()
    c.linear_reset(st)
    c.linear_accumulate(st, mc)
    c.linear_finalize(st)
    got = c.beta_loo(mc, st).cpu().numpy()
    Mmc = case.maps(mc)
    errs = []
    for i in range(mc.shape[0]):
        ref = om.beta_hat_leave_one_out(Mmc, case.grid.w, i)
        errs.append(rel_inf(got[i], ref))
    log_err(f"beta_loo {name} {prec}", max(errs))
    assert max(errs) < TOL[prec]
    # it differs from the plain beta^hat by the O(1/N) self term
    plain = c.beta(mc, state=st).cpu().numpy()
    assert rel_inf(plain[0], got[0]) > 10 * TOL[prec]


def test_beta_loo_needs_two_skies_and_a_state():
    from paper_1105_2791_amd import _lib as L
    case = CASES["tiny"]
    c = ctx_for(case, "f64")
    o = oracle_for(case)
    st = c.linear_state()
    c.linear_reset(st)
    c.linear_accumulate(st, o["mc"][:1])
    c.linear_finalize(st)
    with pytest.raises(L.ModalError) as e:
        c.beta_loo(o["mc"][:1], st)
    assert e.value.status == L.ENOTREADY
    with pytest.raises(L.ModalError) as e:
        c.beta_loo(o["mc"][:1], None)
    assert e.value.status == L.EINVAL


@pytest.mark.parametrize("N", [2, 9])
def test_centered_covariance_matches_oracle(N):
    case = CASES["ragged"]
    c = ctx_for(case, "f64")
    rng = np.random.default_rng(23)
    B = rng.standard_normal((N, c.nmax)) + 3.0 * rng.standard_normal(c.nmax)   # a nonzero mean
    print(f"[case] covariance centered N {N}", flush=True)
    got = c.covariance_sample(B, centered=True).cpu().numpy()
    ref = om.covariance_sample(B, centered=True)
    err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    log_err(f"covariance centered N {N}", err)
    assert err < 1e-13
    # the uncentered one is unchanged by the flag's presence
    got0 = c.covariance_sample(B).cpu().numpy()
    assert np.max(np.abs(got0 - om.covariance_sample(B))) < 1e-13 * np.max(np.abs(got0))


def test_centered_covariance_rejects_one_row():
    from paper_1105_2791_amd import _lib as L
    c = ctx_for(CASES["tiny"], "f64")
    with pytest.raises(L.ModalError) as e:
        c.covariance_sample(np.ones((1, c.nmax)), centered=True)
    assert e.value.status == L.EINVAL
