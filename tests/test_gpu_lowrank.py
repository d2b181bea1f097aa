"""GPU parity of the low-rank covariance calls (Sec. III B) against the FP64 oracle.

noise vectors: b_j compared with the oracle's eigen-decomposition after fixing
the sign the same way (largest-magnitude entry positive); the block iteration
converges like (mu_{k+5} / mu_k)^iters, far below the 1e-9 bound for the spiked
inputs used here.  Estimator and rotation: FP64 arithmetic in a different order
than the oracle's dense solves, bounds 1e-11 relative.  At the metric's n_max
(11,480, P = 40) the oracle's dense eigen-decomposition is replaced by properties
that hold at any size (eigen-residual, orthogonality, eigenvalues of the N x N Gram
matrix) and by the paper's closed forms.
"""
import math

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import lowrank as olr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_ctx = {}


def ctx_P(P):
    """A small FP64 context whose n_max = P (P + 1) (P + 2) / 6; only n_max matters here."""
    if P not in _ctx:
        from paper_1105_2791_amd import ModalContext
        _ctx[P] = ModalContext(8, 12, 24, P, "f64", np.ones((P, 9)), np.ones(9))
    return _ctx[P]


def spiked_betas(rng, N, n, strengths):
    """beta^hat rows with covariance 6 (I + sum_j s_j^2 u_j u_j^T), u_j orthonormal."""
    U, _ = np.linalg.qr(rng.standard_normal((n, len(strengths))))
    Z = rng.standard_normal((N, n))
    G = rng.standard_normal((N, len(strengths)))
    return math.sqrt(6.0) * (Z + (G * np.asarray(strengths)) @ U.T)


@pytest.mark.parametrize("P,N,k", [(8, 300, 1), (8, 300, 4), (6, 257, 3), (7, 5, 5), (6, 3, 2), (6, 1100, 2)])
def test_noise_vectors_match_oracle(P, N, k):
    c = ctx_P(P)
    n = c.nmax
    rng = np.random.default_rng(100 * P + N + k)
    B = spiked_betas(rng, N, n, [9.0, 6.0, 4.5, 3.5, 2.8][:min(k, 5)])
    print(f"[noise vectors] P={P} n={n} N={N} k={k}", flush=True)
    bt, mu = c.noise_vectors(B, k, iters=100)
    bo, muo = olr.noise_vectors(B, k)
    assert np.max(np.abs(mu - muo)) < 1e-11 * muo[0]
    g = bt.cpu().numpy()
    scale = np.max(np.abs(bo))
    assert np.max(np.abs(g - bo)) < 1e-9 * scale, np.max(np.abs(g - bo)) / scale


def test_noise_vector_closed_form_cholesky():
    """Sample covariance exactly I + b b^T (built from the paper's closed-form factor)."""
    c = ctx_P(8)
    n = c.nmax
    rng = np.random.default_rng(5)
    b = rng.standard_normal(n) * 0.4
    N = 2 * n
    Q, _ = np.linalg.qr(rng.standard_normal((N, n)))
    B = math.sqrt(6.0 * N) * Q @ cf.bivector_cholesky(b).T
    bt, mu = c.noise_vectors(B, 1, iters=100)
    assert abs(mu[0] - (1.0 + b @ b)) < 1e-11 * mu[0]
    ref = b if b[np.argmax(np.abs(b))] > 0 else -b
    assert np.max(np.abs(bt.cpu().numpy()[0] - ref)) < 1e-10 * np.max(np.abs(b))


def test_noise_vectors_metric_size_properties():
    """n_max = 11,480 (P = 40), N = 1000 skies: eigen-residual of zeta = B^T B / 6N,
    orthogonality, and eigenvalues against the N x N Gram matrix."""
    c = ctx_P(40)
    n = c.nmax
    N, k = 1000, 4
    rng = np.random.default_rng(40)
    B = spiked_betas(rng, N, n, [14.0, 11.0, 9.0, 7.5])
    print(f"[noise vectors] metric size n={n} N={N} k={k}", flush=True)
    bt, mu = c.noise_vectors(B, k, iters=100)
    g = bt.cpu().numpy()
    gram = np.linalg.eigvalsh(B @ B.T / (6.0 * N))[::-1][:k]
    assert np.max(np.abs(mu - gram)) < 1e-11 * gram[0]
    V = g / np.linalg.norm(g, axis=1, keepdims=True)
    assert np.max(np.abs(V @ V.T - np.eye(k))) < 1e-10
    for j in range(k):
        zv = B.T @ (B @ V[j]) / (6.0 * N)
        assert np.linalg.norm(zv - mu[j] * V[j]) < 1e-9 * mu[j]
        assert abs(np.linalg.norm(g[j]) - math.sqrt(mu[j] - 1.0)) < 1e-11 * math.sqrt(mu[j])
        assert V[j][np.argmax(np.abs(V[j]))] > 0


@pytest.mark.parametrize("P,k,S", [(8, 0, 3), (8, 1, 5), (6, 3, 4), (7, 16, 2), (8, 2, 0)])
def test_fnl_lowrank_matches_oracle(P, k, S):
    c = ctx_P(P)
    n = c.nmax
    rng = np.random.default_rng(7 * P + k + S)
    bt = rng.standard_normal((k, n)) * 0.3
    alpha = rng.standard_normal(n)
    betas = rng.standard_normal((S, n))
    E, s2 = c.fnl_lowrank(bt, alpha, betas)
    Eo, s2o = olr.estimator_lowrank(bt, alpha, betas)
    assert abs(s2 - s2o) < 1e-11 * s2o
    if S:
        assert np.max(np.abs(E - Eo)) < 1e-11 * max(1.0, np.max(np.abs(Eo)))


def test_fnl_lowrank_metric_size():
    """n_max = 11,480: one noise vector against Sherman-Morrison and eq. (bivecvariance);
    four against the dense GPU Cholesky path of modal_fnl."""
    c = ctx_P(40)
    n = c.nmax
    rng = np.random.default_rng(41)
    alpha = rng.standard_normal(n)
    betas = rng.standard_normal((8, n))
    b = rng.standard_normal(n) * 0.05
    E, s2 = c.fnl_lowrank(b[None, :], alpha, betas)
    ab, bb, aa = alpha @ b, b @ b, alpha @ alpha
    yy = aa - ab * ab / (1.0 + bb)
    Eref = (betas @ alpha - (betas @ b) * ab / (1.0 + bb)) / yy
    assert np.max(np.abs(E - Eref)) < 1e-11 * max(1.0, np.max(np.abs(Eref)))
    assert abs(s2 - 6.0 * cf.bivector_variance(alpha, b)) < 1e-11 * s2
    K = rng.standard_normal((4, n)) * 0.02
    E4, s24 = c.fnl_lowrank(K, alpha, betas)
    Z = torch.eye(n, dtype=torch.float64, device="cuda")
    Kt = torch.as_tensor(K, device="cuda")
    Z += Kt.T @ Kt
    Ed, s2d = c.fnl(Z, alpha, betas)
    assert np.max(np.abs(E4 - Ed)) < 1e-10 * max(1.0, np.max(np.abs(Ed)))
    assert abs(s24 - s2d) < 1e-10 * s2d


@pytest.mark.parametrize("P,R", [(8, 4), (6, 1), (7, 9)])
def test_bivector_rotate_matches_oracle(P, R):
    c = ctx_P(P)
    n = c.nmax
    rng = np.random.default_rng(3 * P + R)
    b = rng.standard_normal(n) * 0.6
    X = rng.standard_normal((R, n))
    y = c.bivector_rotate(b, X).cpu().numpy()
    yo = olr.bivector_rotate(b, X)
    assert np.max(np.abs(y - yo)) < 1e-11 * np.max(np.abs(yo))


def test_bivector_rotate_metric_size_frame():
    """n_max = 11,480: in the rotated frame E = alpha'.beta'/|alpha'|^2 equals the
    Sherman-Morrison estimator and |alpha'|^2 = 1 / eq. (bivecvariance)."""
    c = ctx_P(40)
    n = c.nmax
    rng = np.random.default_rng(42)
    b = rng.standard_normal(n) * 0.05
    alpha = rng.standard_normal(n)
    betas = rng.standard_normal((8, n))
    X = np.vstack([alpha[None, :], betas])
    Y = c.bivector_rotate(b, X).cpu().numpy()
    ap, bp = Y[0], Y[1:]
    ab, bb, aa = alpha @ b, b @ b, alpha @ alpha
    yy = aa - ab * ab / (1.0 + bb)
    Eref = (betas @ alpha - (betas @ b) * ab / (1.0 + bb)) / yy
    assert np.max(np.abs(bp @ ap / (ap @ ap) - Eref)) < 1e-11 * max(1.0, np.max(np.abs(Eref)))
    assert abs(1.0 / (ap @ ap) - cf.bivector_variance(alpha, b)) < 1e-11 / (ap @ ap)


def test_whiten_by_cholesky_factor():
    """y = L^-1 x with L from modal_fnl: whitening zeta's own rows and columns gives I."""
    c = ctx_P(8)
    n = c.nmax
    rng = np.random.default_rng(8)
    A = rng.standard_normal((3 * n, n))
    Z = A.T @ A / (3 * n)
    _, _, L = c.fnl(Z, rng.standard_normal(n), rng.standard_normal((1, n)), want_L=True)
    W = c.whiten(L, Z)                        # rows: L^-1 applied to the rows of zeta
    W = c.whiten(L, W.T.contiguous()).cpu().numpy()
    assert np.max(np.abs(W - np.eye(n))) < 1e-11
    x = rng.standard_normal((2, n))
    import scipy.linalg
    ref = scipy.linalg.solve_triangular(np.linalg.cholesky(Z), x.T, lower=True).T
    assert np.max(np.abs(c.whiten(L, x).cpu().numpy() - ref)) < 1e-11 * np.max(np.abs(ref))


def test_lowrank_argument_errors():
    from paper_1105_2791_amd import ModalError
    c = ctx_P(6)
    n = c.nmax
    B = np.ones((3, n))
    for k in (0, 4, 17):
        with pytest.raises(ModalError):
            c.noise_vectors(B, k)
    with pytest.raises(ModalError):
        c.noise_vectors(B, 1, iters=0)
    with pytest.raises(ModalError):
        c.fnl_lowrank(np.zeros((17, n)), np.ones(n), np.ones((1, n)))
    with pytest.raises(ModalError):   # alpha = 0: alpha^T zeta^-1 alpha = 0
        c.fnl_lowrank(np.zeros((1, n)), np.zeros(n), np.ones((1, n)))
