"""modal_beta_noalloc (the entry point for callers that cannot allocate device memory)
against modal_beta through the C ABI: two calls in a row, the second with a smaller
input, and the size limit of its fixed scratch array."""
import ctypes as C

import numpy as np
import pytest

from helpers import CASES
from test_gpu_parity import TOL, log_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _ctx(case, prec):
    from paper_1105_2791_amd import ModalContext
    return ModalContext(case.lmax, case.ntheta, case.nphi, case.P, prec, case.q, case.cl, mask=case.mask())


def _noalloc(ctx, alm, state):
    """The entry point called directly through the C ABI (ctypes)."""
    from paper_1105_2791_amd import _lib as L
    a = ctx._alm(alm)
    S = a.shape[0]
    out = torch.full((S, ctx.nmax), float("nan"), dtype=torch.float64, device=ctx.device)
    st = L.lib().modal_beta_noalloc(ctx._h, a.data_ptr(), S, None if state is None else state.data_ptr(),
                                    out.data_ptr(), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == L.OK, ctx._lib.modal_last_error(ctx._h).decode()
    return out


def _rel(got, ref):
    return max(float(np.max(np.abs(got[s] - ref[s])) / np.sqrt(np.mean(ref[s] ** 2))) for s in range(ref.shape[0]))


@pytest.mark.parametrize("prec", ["bf16x3", "f32", "f64"])
def test_noalloc_matches_beta_two_calls(prec):
    # call 1: ragged case (l_max 150, 199 x 400 rings, P 13), 3 skies, with a linear-term state
    big = CASES["ragged"]
    print(f"[case] noalloc ragged {prec} S=3", flush=True)
    c1 = _ctx(big, prec)
    alms = big.alms(0, 3)
    st = c1.linear_state()
    c1.linear_reset(st)
    c1.linear_accumulate(st, big.alms(100, 2))
    c1.linear_finalize(st)
    ref1 = c1.beta(alms, state=st).cpu().numpy()
    got1 = _noalloc(c1, alms, st).cpu().numpy()
    e1 = _rel(got1, ref1)
    log_err(f"noalloc vs beta ragged {prec} (bitwise equal: {np.array_equal(got1, ref1)})", e1)
    assert np.all(np.isfinite(got1)) and e1 <= TOL[prec]
    # call 2: a smaller input on the same GPU's scratch - the tiny case, one sky, no state
    small = CASES["tiny"]
    print(f"[case] noalloc tiny {prec} S=1", flush=True)
    c2 = _ctx(small, prec)
    a2 = small.alms(0, 1)
    ref2 = c2.beta(a2).cpu().numpy()
    got2 = _noalloc(c2, a2, None).cpu().numpy()
    e2 = _rel(got2, ref2)
    log_err(f"noalloc vs beta tiny {prec} (bitwise equal: {np.array_equal(got2, ref2)})", e2)
    assert np.all(np.isfinite(got2)) and e2 <= TOL[prec]
    # call 3: the first context again with fewer skies (the scratch keeps call 2's contents)
    got3 = _noalloc(c1, alms[:1], st).cpu().numpy()
    e3 = _rel(got3, ref1[:1])
    log_err(f"noalloc vs beta ragged {prec} S=1 after tiny", e3)
    assert e3 <= TOL[prec]
    del st
    c1.close()
    c2.close()


def test_noalloc_rejects_oversized_shapes():
    from paper_1105_2791_amd import ModalContext, _lib as L
    import modal_inputs as mi
    lmax, nt, nphi, P = 500, 768, 1536, 30
    print("[case] noalloc oversize lmax 500 P 30", flush=True)
    c = ModalContext(lmax, nt, nphi, P, "f32", mi.q_basis(P, lmax), mi.filter_cl(lmax, "wmap"))
    assert c.workspace_size(L.OP_BETA, 1) > L.NOALLOC_SCRATCH_BYTES
    alm = c._alm(mi.gaussian_alm(mi.filter_cl(lmax, "wmap"), lmax, mi.rng_for(2, 0)))
    out = torch.zeros((1, c.nmax), dtype=torch.float64, device=c.device)
    st = L.lib().modal_beta_noalloc(c._h, alm.data_ptr(), 1, None, out.data_ptr(),
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == L.ENOSPACE
    assert "fixed scratch" in c._lib.modal_last_error(c._h).decode()
    # the context still works through the caller-workspace entry point
    assert torch.isfinite(c.beta(alm)).all()
    c.close()
