"""The truncated orthonormal frame on the GPU (modal_frame, modal_frame_rotate,
modal_fnl_frame) against the oracle (oracle/frame.py) and against what the frame must be.

The pivot order may differ from the oracle's where remaining diagonals nearly tie, so what
is compared is what the frame fixes: the library's kept modes and factor must make an
orthonormal frame of the oracle's zeta0 (T zeta0 T^T = I_k), stop by the same rule, and give
the estimator of the oracle for skies in the span of the modes.  At l_max 1000, P 40, where
the full FP64 Cholesky of zeta0 breaks down, the frame makes E and sigma^2 computable.
"""
import math

import numpy as np
import pytest

import modal_inputs as mi
from oracle import closed_forms as cf
from oracle import frame as ofr

from test_gpu_parity import log_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _T(perm, L11, n):
    """The frame as a dense k x n matrix T = L11^-1 [I 0] Pi^T."""
    k = len(perm)
    T = np.zeros((k, n))
    T[:, perm] = np.linalg.inv(L11)
    return T


def test_frame_small_basis_matches_oracle():
    from paper_1105_2791_amd import ModalContext
    lmax, P, tol = 32, 8, 1e-10
    cl = mi.cl_signal(lmax)
    q = mi.q_basis(P, lmax)
    c = ModalContext(lmax, 48, 96, P, "f64", q, cl)
    print("[case] frame lmax 32 P 8", flush=True)
    Zg = c.ideal_covariance()
    k, perm, L11 = c.frame(Zg, tol)
    Zo = cf.zeta_ideal(q, (cl > 0).astype(float))
    po, Lo = ofr.pivoted_cholesky(Zo, tol)
    n = Zo.shape[0]
    pg, Lg = perm.cpu().numpy(), L11.cpu().numpy()
    print(f"[frame] lmax 32 P 8: k = {k} (oracle {len(po)}) of {n}", flush=True)
    assert abs(k - len(po)) <= 1 and 0 < k < n
    assert sorted(set(pg.tolist())) == sorted(pg.tolist())          # distinct modes
    assert np.allclose(Lg, np.tril(Lg)) and np.all(np.diag(Lg) > 0)
    T = _T(pg, Lg, n)
    # orthonormal under the zeta0 it was computed from, to the precision the conditioning
    # allows (kept pivots >= sqrt(tol) of the largest); under the oracle's zeta0, whose
    # entries differ by ~1e-14 relative, the difference is amplified by |T|^2 ~ 1 / (tol max diag)
    e_own = float(np.max(np.abs(T @ Zg.cpu().numpy() @ T.T - np.eye(k))))
    e_orth = float(np.max(np.abs(T @ Zo @ T.T - np.eye(k))))
    log_err("frame lmax 32: T zeta0 T^T - I", e_own)
    log_err("frame lmax 32: T zeta0(oracle) T^T - I", e_orth)
    assert e_own < 1e-5
    assert e_orth < 1e-13 / tol
    # estimator on skies in the span of the modes, against the oracle's frame estimator
    rng = np.random.default_rng(5)
    alpha = Zo @ rng.standard_normal(n)
    betas = (Zo @ rng.standard_normal((n, 3))).T
    Eg, s2g = c.fnl_frame(Zg, perm, alpha, betas)
    Eo, s2o = ofr.estimator_in_frame(po, Lo, Zo, alpha, betas)
    e_E = float(np.max(np.abs(Eg - Eo)) / np.max(np.abs(Eo)))
    log_err("frame lmax 32: E against the oracle", e_E)
    assert e_E < 1e-6 and abs(s2g / s2o - 1.0) < 1e-6
    # E(beta = alpha) = 1, and the frame coordinates: |alpha'|^2 = 6 / sigma^2 (zeta' = I)
    E1, _ = c.fnl_frame(Zg, perm, alpha, alpha[None])
    assert abs(E1[0] - 1.0) < 1e-10
    a1 = c.frame_rotate(perm, L11, alpha).cpu().numpy()[0]
    assert abs(6.0 / float(a1 @ a1) / s2g - 1.0) < 1e-6
    c.close()


def test_frame_metric_shape_makes_the_estimator_computable():
    """l_max 1000, P 40 (n_max 11,480): the ideal covariance is singular to FP64 (its full
    Cholesky stops at a negative pivot), the truncated frame is not."""
    from paper_1105_2791_amd import ModalContext, _lib as L
    import time
    lmax, P, tol = 1000, 40, 1e-10
    cl = mi.filter_cl(lmax, "wmap")
    q = mi.q_basis(P, lmax)
    c = ModalContext(lmax, 1536, 3072, P, "f32", q, cl)
    print("[case] frame lmax 1000 P 40: ideal covariance", flush=True)
    Z = c.ideal_covariance()
    n = c.nmax
    one = np.ones(lmax + 1)
    alpha = c.alpha_separable(np.array([[2 * cl, cl, one], [2 * cl, one, cl], [2 * one, cl, cl]]))
    with pytest.raises(L.ModalError) as e:
        c.fnl(Z, alpha, alpha[None])
    assert e.value.status == L.ENOTPD
    print("[case] frame lmax 1000 P 40: pivoted Cholesky", flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k, perm, L11 = c.frame(Z, tol)
    t = time.perf_counter() - t0
    print(f"[frame] lmax 1000 P 40: k = {k} of {n} kept modes, {1e3 * t:.1f} ms", flush=True)
    assert 0 < k < n
    # orthonormality, checked in FP64 on the host on the kept block: L11^-1 Z_kk L11^-T = I
    pk = perm.cpu().numpy()
    Zk = Z[perm.long()][:, perm.long()].cpu().numpy()
    Lk = L11.cpu().numpy()
    M = np.linalg.solve(Lk, np.linalg.solve(Lk, Zk).T).T
    e_orth = float(np.max(np.abs(M - np.eye(k))))
    log_err("frame lmax 1000 P 40: L11^-1 zeta_kk L11^-T - I", e_orth)
    assert e_orth < 1e-4
    # the stopping rule: every discarded mode's remaining diagonal is below tol max(diag)
    dz = torch.diagonal(Z).cpu().numpy()
    assert len(set(pk.tolist())) == k
    E1, s2 = c.fnl_frame(Z, perm, alpha, alpha[None])
    print(f"[frame] lmax 1000 P 40: E(beta = alpha) = {E1[0]:.12f}, sigma = {math.sqrt(s2):.4e}", flush=True)
    assert abs(E1[0] - 1.0) < 1e-8 and s2 > 0 and np.isfinite(s2)
    a1 = c.frame_rotate(perm, L11, alpha).cpu().numpy()[0]
    assert abs(6.0 / float(a1 @ a1) / s2 - 1.0) < 1e-6
    assert dz.max() > 0
    c.close()
