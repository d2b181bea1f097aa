"""Modal bispectrum estimator, plain FP64 definitions (oracle).

Notation (paper Sec. III A, with the separable isotropic basis
R_n(l1,l2,l3) = q_p(l1) q_r(l2) q_s(l3) and unit weight v_l = 1):

  whitened coefficients   a~_lm = a_lm / sqrt(C_l)          (0 where C_l = 0)
  filtered maps           M_p(x) = sum_lm q_p(l) a~_lm Y_lm(x)
  cubic mode coefficients beta_prs = sum_x w(x) M_p M_r M_s,  p <= r <= s
  linear term             lin_prs  = sum_x w(x) [V_pr M_s + V_ps M_r + V_rs M_p]
                          V_pr(x)  = < M_p M_r >(x) over Monte-Carlo Gaussian maps
  data vector             beta^hat = beta - lin                 (eq. bbispect)
  modal covariance        zeta = <beta^hat beta^hat^T> / 6       (eq. linearterm)
  estimator               E = alpha^T zeta^-1 beta / alpha^T zeta^-1 alpha   (eq. modalest)
  variance                sigma^2 = 6 / alpha^T zeta^-1 alpha    (eq. modalvariance)

beta_prs is eq. (bbispect) with the Gaunt sum carried out in pixel space: with
R_n separable, sum_{l_i m_i} G q_p q_r q_s a~ a~ a~ = int M_p M_r M_s dOmega, and
the grid sum equals the integral when the quadrature is exact for the triple
product.  The "3 C a" linear term of eq. (bispectrumest) is the sum over the
three ways of pairing two of the three legs; with the pairing expectation
estimated from Monte-Carlo maps (Sec. II: "calculated from Monte Carlo
simulations") it becomes the V-weighted sum above.

Storage conventions match the C ABI: a_lm m-major (modal_inputs.alm_index),
maps [P][ntheta][nphi], pairs (p<=r) and triples (p<=r<=s) lexicographic.
"""
from __future__ import annotations

import numpy as np

from modal_inputs import alm_index, lm_arrays, pair_list, triple_list, npairs
from .legendre import lambda_m

_CHUNK = 1 << 16   # pixels per block of the pixel sums (memory only)


# ---------------------------------------------------------------------------
# maps
# ---------------------------------------------------------------------------

def whiten(alm: np.ndarray, cl: np.ndarray, lmax: int) -> np.ndarray:
    """a~_lm = a_lm / sqrt(C_l), zero where C_l = 0 (eq. legoestimator's 1/sqrt(C))."""
    l, _ = lm_arrays(lmax)
    inv = np.zeros_like(cl)
    nz = cl > 0
    inv[nz] = 1.0 / np.sqrt(cl[nz])
    return np.asarray(alm) * inv[l]


def ring_coefficients(alm_w: np.ndarray, q: np.ndarray, lmax: int, x: np.ndarray) -> np.ndarray:
    """F_{s,p,m}(theta_j) = sum_l q_p(l) a~_{s,lm} lambda_lm(theta_j).

    alm_w: [S, nalm] whitened; returns [S, P, ntheta, lmax+1] complex."""
    alm_w = np.atleast_2d(alm_w)
    S = alm_w.shape[0]
    P = q.shape[0]
    F = np.zeros((S, P, x.size, lmax + 1), dtype=np.complex128)
    for m in range(lmax + 1):
        lam = lambda_m(m, lmax, x)                                # [L_m, ntheta]
        a = alm_w[:, alm_index(np.arange(m, lmax + 1), m, lmax)]  # [S, L_m]
        coef = q[None, :, m:] * a[:, None, :]                      # [S, P, L_m]
        F[:, :, :, m] = coef @ lam
    return F


def maps_from_ring_coefficients(F: np.ndarray, nphi: int) -> np.ndarray:
    """M(theta_j, phi_k) = sum_{m>=0} (2 - delta_m0) Re(F_m(theta_j) e^{i m phi_k}).

    Uses numpy's inverse real FFT: nphi * irfft(H) = Re H_0 + 2 Re sum_{m>=1} H_m
    e^{2 pi i m k / nphi} when H vanishes at the Nyquist index (lmax < nphi/2)."""
    lmax = F.shape[-1] - 1
    if not 2 * lmax < nphi:
        raise ValueError("need lmax < nphi/2")
    H = np.zeros(F.shape[:-1] + (nphi // 2 + 1,), dtype=np.complex128)
    H[..., :lmax + 1] = F
    return nphi * np.fft.irfft(H, n=nphi, axis=-1)


def filtered_maps(alm, cl, q, grid) -> np.ndarray:
    """M_{s,p}(x) on the grid, shape [S, P, ntheta, nphi] (or [P, ...] for 1-D alm)."""
    alm = np.asarray(alm)
    single = alm.ndim == 1
    lmax = cl.size - 1
    F = ring_coefficients(whiten(np.atleast_2d(alm), cl, lmax), q, lmax, grid.x)
    M = maps_from_ring_coefficients(F, grid.nphi)
    return M[0] if single else M


# ---------------------------------------------------------------------------
# cubic and linear modal coefficients
# ---------------------------------------------------------------------------

def _pair_index(P):
    pl = pair_list(P)
    return {pr: i for i, pr in enumerate(pl)}, pl


def pair_mode_sums(A: np.ndarray, M: np.ndarray, w: np.ndarray) -> np.ndarray:
    """sum_x w(x) A_k(x) M_t(x) for every row k of A and mode t: [K, P]."""
    A = A.reshape(A.shape[0], -1)
    M = M.reshape(M.shape[0], -1)
    w = w.reshape(-1)
    out = np.zeros((A.shape[0], M.shape[0]))
    for c0 in range(0, w.size, _CHUNK):
        sl = slice(c0, c0 + _CHUNK)
        out += (A[:, sl] * w[sl]) @ M[:, sl].T
    return out


def pair_products(M: np.ndarray) -> np.ndarray:
    """M_p(x) M_r(x) for all pairs p <= r: [npairs, npix]."""
    P = M.shape[0]
    Mf = M.reshape(P, -1)
    return np.stack([Mf[p] * Mf[r] for p, r in pair_list(P)])


def beta(M: np.ndarray, w: np.ndarray) -> np.ndarray:
    """beta_prs = sum_x w M_p M_r M_s for p <= r <= s (eq. bbispect, cubic part)."""
    P = M.shape[0]
    idx, _ = _pair_index(P)
    E = pair_mode_sums(pair_products(M), M, w)
    return np.array([E[idx[(p, r)], s] for p, r, s in triple_list(P)])


def pair_means(Ms: np.ndarray) -> np.ndarray:
    """V_pr(x) = (1/N) sum_i M^i_p(x) M^i_r(x) over Monte-Carlo maps Ms [N, P, ...]."""
    Ms = np.asarray(Ms)
    N, P = Ms.shape[0], Ms.shape[1]
    V = np.zeros((npairs(P),) + Ms.shape[2:])
    for i in range(N):
        for k, (p, r) in enumerate(pair_list(P)):
            V[k] += Ms[i, p] * Ms[i, r]
    return V / N


def linear_term(M: np.ndarray, w: np.ndarray, V: np.ndarray) -> np.ndarray:
    """lin_prs = sum_x w [V_pr M_s + V_ps M_r + V_rs M_p] (the three pairings of "3 C a")."""
    P = M.shape[0]
    idx, _ = _pair_index(P)
    L = pair_mode_sums(V, M, w)
    return np.array([L[idx[(p, r)], s] + L[idx[(p, s)], r] + L[idx[(r, s)], p]
                     for p, r, s in triple_list(P)])


def beta_hat(M, w, V=None) -> np.ndarray:
    """beta - lin (beta alone when V is None)."""
    b = beta(M, w)
    return b if V is None else b - linear_term(M, w, V)


def beta_and_linear_by_rings(alms, mc_alms, cl, q, grid, rings_per_chunk: int = 128, with_abs: bool = False):
    """beta and lin of every sky in ``alms`` [S, nalm] over the whole grid, with the pair
    means V taken from the Monte-Carlo skies ``mc_alms`` [N, nalm] (None: no linear term).

    beta_prs and lin_prs are sums over pixels (eq. bbispect and the three pairings of
    "3 C a"), and V(x) is a per-pixel mean, so both are accumulated over groups of rings
    with the definitions above applied to each group: memory stays bounded at full
    resolution (a ring group's maps, pair products and pair means only).
    with_abs: also the sums of the terms' magnitudes, sum_x w |M_p M_r M_s| and
    sum_x w (|V_pr M_s| + |V_ps M_r| + |V_rs M_p|) (w >= 0): the scale that rounding in the
    maps and in the summation is relative to (forward error of a sum).
    Returns (beta [S, nmax], lin [S, nmax] or None), plus (beta_abs, lin_abs) with_abs."""
    from .grid import RingSubset
    alms = np.atleast_2d(alms)
    P = q.shape[0]
    n = len(triple_list(P))
    b = np.zeros((alms.shape[0], n))
    lin = None if mc_alms is None else np.zeros((alms.shape[0], n))
    b_abs = np.zeros_like(b) if with_abs else None
    lin_abs = None if (mc_alms is None or not with_abs) else np.zeros_like(b)
    for j0 in range(0, grid.ntheta, rings_per_chunk):
        sub = RingSubset(grid, np.arange(j0, min(grid.ntheta, j0 + rings_per_chunk)))
        M = filtered_maps(alms, cl, q, sub)
        V = None if mc_alms is None else pair_means(filtered_maps(np.atleast_2d(mc_alms), cl, q, sub))
        for s in range(alms.shape[0]):
            b[s] += beta(M[s], sub.w)
            if with_abs:
                b_abs[s] += beta(np.abs(M[s]), sub.w)
            if V is not None:
                lin[s] += linear_term(M[s], sub.w, V)
                if with_abs:
                    lin_abs[s] += linear_term(np.abs(M[s]), sub.w, np.abs(V))
        del M, V
    return (b, lin, b_abs, lin_abs) if with_abs else (b, lin)


# ---------------------------------------------------------------------------
# covariance and estimator
# ---------------------------------------------------------------------------

def covariance_sample(beta_hats: np.ndarray, centered: bool = False) -> np.ndarray:
    """zeta = (1/(6N)) sum_i beta^hat_i beta^hat_i^T  (eq. linearterm, <beta beta^T> = 6 zeta).

    centered: the mean m = (1/N) sum_i beta^hat_i is subtracted first and the sum divided
    by 6 (N - 1) instead (the unbiased sample covariance when the mean is not known)."""
    B = np.atleast_2d(beta_hats)
    N = B.shape[0]
    if not centered:
        return B.T @ B / (6.0 * N)
    m = B.sum(axis=0) / N
    D = B - m[None, :]
    return D.T @ D / (6.0 * (N - 1))


def beta_hat_leave_one_out(Ms: np.ndarray, w: np.ndarray, i: int) -> np.ndarray:
    """beta^hat of Monte-Carlo sky i with the pair means taken over the other N - 1 skies
    of ``Ms`` [N, P, ...] (the linear term from simulations, Sec. II, without the sky's own
    maps): beta(M_i) - lin(M_i; V over j != i)."""
    Ms = np.asarray(Ms)
    others = np.concatenate([Ms[:i], Ms[i + 1:]], axis=0)
    return beta(Ms[i], w) - linear_term(Ms[i], w, pair_means(others))


def estimator(zeta: np.ndarray, alpha: np.ndarray, betas: np.ndarray):
    """E_s = alpha^T zeta^-1 beta_s / alpha^T zeta^-1 alpha and sigma^2 = 6 / alpha^T zeta^-1 alpha
    (eqs. modalest, modalvariance); also the Cholesky factor zeta = L L^T (eq. Cholrot)."""
    y = np.linalg.solve(zeta, alpha)
    norm = float(alpha @ y)
    E = np.atleast_2d(betas) @ y / norm
    return E, 6.0 / norm, np.linalg.cholesky(zeta)


# ---------------------------------------------------------------------------
# gradient (vector-Jacobian product) of beta^hat with respect to a_lm
# ---------------------------------------------------------------------------

def slot_matrix(cot: np.ndarray, P: int) -> np.ndarray:
    """K[b, u, pair]: d(sum_n c_n beta^hat_n)/dM_u = w sum_pair K[u, pair] (M_a M_b - V_ab).

    Each triple n = (p, r, s) contributes c_n to (u=p, pair rs), (u=r, pair ps),
    (u=s, pair pr): the derivative of the product M_p M_r M_s with respect to
    each of its three legs."""
    cot = np.atleast_2d(cot)
    idx, _ = _pair_index(P)
    K = np.zeros((cot.shape[0], P, npairs(P)))
    for n, (p, r, s) in enumerate(triple_list(P)):
        K[:, p, idx[(r, s)]] += cot[:, n]
        K[:, r, idx[(p, s)]] += cot[:, n]
        K[:, s, idx[(p, r)]] += cot[:, n]
    return K


def vjp(alm, cl, q, grid, V, cot) -> np.ndarray:
    """g = sum_n c_n d(beta^hat_n)/d a_lm for one map and a batch of cotangents.

    Real degrees of freedom: for m > 0, g_lm = d/dRe a_lm + i d/dIm a_lm (a_{l,-m}
    follows from reality); for m = 0, g_l0 = d/da_l0 (real).  V = None means no
    linear term.  Returns [B, nalm] complex for cot [B, nmax]."""
    lmax = cl.size - 1
    P = q.shape[0]
    M = filtered_maps(alm, cl, q, grid)                       # [P, nt, nphi]
    A = pair_products(M)                                      # [npairs, npix]
    if V is not None:
        A = A - V.reshape(A.shape)
    K = slot_matrix(cot, P)                                   # [B, P, npairs]
    B = K.shape[0]
    G = (K.reshape(B * P, -1) @ A) * grid.w.reshape(1, -1)    # dL/dM_u(x)
    G = G.reshape(B, P, grid.ntheta, grid.nphi)
    Gh = np.fft.rfft(G, axis=-1)[..., :lmax + 1]              # sum_k G e^{-i m phi_k}
    inv = np.zeros_like(cl)
    inv[cl > 0] = 1.0 / np.sqrt(cl[cl > 0])
    g = np.zeros((B, alm_index(lmax, lmax, lmax) + 1), dtype=np.complex128)
    for m in range(lmax + 1):
        lam = lambda_m(m, lmax, grid.x)                       # [L_m, nt]
        D = np.einsum("lj,buj->bul", lam, Gh[..., m])         # [B, P, L_m]
        gm = np.einsum("ul,bul->bl", q[:, m:], D)             # [B, L_m]
        gm = gm * (1.0 if m == 0 else 2.0) * inv[m:]
        if m == 0:
            gm = gm.real + 0j
        g[:, alm_index(np.arange(m, lmax + 1), m, lmax)] = gm
    return g


def jacobian(alm, cl, q, grid, V) -> np.ndarray:
    """J[n, lm] = d beta^hat_n / d a_lm in the complex packing of ``vjp``."""
    P = q.shape[0]
    nmax = len(triple_list(P))
    return vjp(alm, cl, q, grid, V, np.eye(nmax))


def dof_variance(cl_true: np.ndarray, lmax: int):
    """Variance of the real degrees of freedom of a Gaussian isotropic a_lm:
    C_l for a_l0; C_l/2 for each of Re and Im of a_lm (m > 0)."""
    l, m = lm_arrays(lmax)
    vre = np.where(m == 0, cl_true[l], 0.5 * cl_true[l])
    vim = np.where(m == 0, 0.0, 0.5 * cl_true[l])
    return vre, vim


def fisher(alms, cl, cl_true, q, grid, V) -> np.ndarray:
    """F = (1/(18 N)) sum_i J_i C J_i^T with C the (diagonal) covariance of the real dof.

    For Gaussian maps, E[J C J^T] = 18 zeta when lin is the exact pairing expectation,
    so F estimates zeta from gradients (parity of the estimator is then tested
    statistically)."""
    lmax = cl.size - 1
    vre, vim = dof_variance(cl_true, lmax)
    alms = np.atleast_2d(alms)
    F = 0.0
    for a in alms:
        J = jacobian(a, cl, q, grid, V)
        F = F + (J.real * vre) @ J.real.T + (J.imag * vim) @ J.imag.T
    return F / (18.0 * alms.shape[0])
