"""Thin torch-facing wrapper over the C ABI (include/modal.h).

PyTorch provides device memory and the stream; every step of the computation
runs in libmodal's HIP kernels.  Tensors passed in must live on the context's
GPU; they are made contiguous and of the context's dtype here (marshalling
only).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

from . import _lib as L


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


class ModalContext:
    """One (grid, lmax, P, precision) configuration on one GPU."""

    def __init__(self, lmax: int, ntheta: int, nphi: int, P: int, prec: str, q, cl, mask=None,
                 device: int | str | torch.device = 0, lambda_table: bool | None = None):
        self._lib = L.lib()
        self.device = torch.device("cuda", torch.device(device).index if not isinstance(device, int) else device)
        self.lmax, self.ntheta, self.nphi, self.P = lmax, ntheta, nphi, P
        self.prec_name = prec
        self.prec = L.PREC_NAMES[prec]
        q = np.ascontiguousarray(q, dtype=np.float64)
        cl = np.ascontiguousarray(cl, dtype=np.float64)
        if q.shape != (P, lmax + 1) or cl.shape != (lmax + 1,):
            raise ValueError("q must be [P][lmax+1] and cl [lmax+1]")
        mk = None
        if mask is not None:
            mk = np.ascontiguousarray(np.broadcast_to(np.asarray(mask, dtype=np.float64), (ntheta, nphi)))
        self._h = C.c_void_p()
        # the context's tables: one caller-owned device buffer sized by modal_ctx_bytes; the
        # split precisions keep the synthesis's lambda table when it fits (a tenth of the
        # device, half of the free memory) unless lambda_table=False (default: unless the
        # environment sets MODAL_LAMBDA_TABLE=0)
        flags = 0
        want = os.environ.get("MODAL_LAMBDA_TABLE", "1") != "0" if lambda_table is None else bool(lambda_table)
        if self.prec in (L.BF16X3, L.F16X3) and want:
            extra = (self._lib.modal_ctx_bytes(lmax, ntheta, nphi, P, self.prec, L.CTX_LAMBDA_TABLE)
                     - self._lib.modal_ctx_bytes(lmax, ntheta, nphi, P, self.prec, 0))
            free, total = torch.cuda.mem_get_info(self.device)
            if extra <= total // 10 and extra < free // 2:
                flags = L.CTX_LAMBDA_TABLE
        nbytes = self._lib.modal_ctx_bytes(lmax, ntheta, nphi, P, self.prec, flags)
        if nbytes == 0:   # rejected arguments: modal_create names the reason (before any device call)
            st = self._lib.modal_create(C.byref(self._h), lmax, ntheta, nphi, P, self.prec, flags, q.ctypes.data,
                                        cl.ctypes.data, None, None, 0)
            raise L.ModalError(st, "modal_create rejected the arguments")
        self.lambda_table = bool(flags & L.CTX_LAMBDA_TABLE)
        self._tables = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            st = self._lib.modal_create(C.byref(self._h), lmax, ntheta, nphi, P, self.prec, flags,
                                        q.ctypes.data, cl.ctypes.data, None if mk is None else mk.ctypes.data,
                                        self._tables.data_ptr(), nbytes)
        if st != L.OK:
            self._tables = None
            raise L.ModalError(st, "modal_create failed")
        self.nalm = self._lib.modal_nalm(self._h)
        self.nmax = self._lib.modal_nmax(self._h)
        self.npairs = self._lib.modal_npairs(self._h)
        self.nquad = self._lib.modal_nquad(self._h)
        self.real_dtype = torch.float64 if self.prec == L.F64 else torch.float32
        self.complex_dtype = torch.complex128 if self.prec == L.F64 else torch.complex64
        self._ws = None

    # ------------------------------------------------------------------ utils
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.modal_destroy(self._h)
            self._h = C.c_void_p()
        self._tables = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != L.OK:
            raise L.ModalError(st, self._lib.modal_last_error(self._h).decode())

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def workspace_size(self, op: int, S: int) -> int:
        n = C.c_size_t()
        self._check(self._lib.modal_workspace_size(self._h, op, S, C.byref(n)))
        return int(n.value)

    def workspace(self, op: int, S: int) -> torch.Tensor:
        need = max(256, self.workspace_size(op, S))
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def grid(self):
        x = np.empty(self.ntheta)
        w = np.empty(self.ntheta)
        self._check(self._lib.modal_grid(self._h, x.ctypes.data, w.ctypes.data))
        return x, w

    def profile(self, enable: bool = True):
        self._check(self._lib.modal_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self, reset: bool = True) -> dict:
        """Per-stage summed GPU milliseconds and launch counts since the last reset."""
        ms = np.zeros(len(L.STAGES))
        n = np.zeros(len(L.STAGES), dtype=np.int64)
        self._check(self._lib.modal_profile_read(self._h, ms.ctypes.data, n.ctypes.data, 1 if reset else 0))
        return {name: (float(ms[i]), int(n[i])) for i, name in enumerate(L.STAGES)}

    def cubic_path(self) -> dict:
        """Which contraction kernel the context uses ('valu' or 'mfma') and the
        multiply-adds it issues per pixel and map (tile padding and split products
        included)."""
        code = int(self._lib.modal_cubic_path(self._h))
        return {"path": "valu" if code == 0 else "mfma", "code": code,
                "issued_macs_per_pixel": float(self._lib.modal_cubic_issued_macs(self._h))}

    def _alm(self, alm) -> torch.Tensor:
        a = torch.as_tensor(alm)
        if a.dim() == 1:
            a = a[None]
        if a.shape[-1] != self.nalm:
            raise ValueError(f"alm last dim {a.shape[-1]} != nalm {self.nalm}")
        return a.to(device=self.device, dtype=self.complex_dtype).contiguous()

    # --------------------------------------------------------------- hot path
    def filter_maps(self, alm, out=None) -> torch.Tensor:
        a = self._alm(alm)
        S = a.shape[0]
        if out is None:
            out = torch.empty((S, self.P, self.ntheta, self.nphi), dtype=self.real_dtype, device=self.device)
        ws = self.workspace(L.OP_FILTER_MAPS, S)
        self._check(self._lib.modal_filter_maps(self._h, _ptr(a), S, _ptr(out), _ptr(ws), ws.numel(),
                                                self._stream()))
        return out

    def beta(self, alm, state=None, out=None) -> torch.Tensor:
        a = self._alm(alm)
        S = a.shape[0]
        if out is None:
            out = torch.empty((S, self.nmax), dtype=torch.float64, device=self.device)
        ws = self.workspace(L.OP_BETA, S)
        self._check(self._lib.modal_beta(self._h, _ptr(a), S, _ptr(state), _ptr(out), _ptr(ws), ws.numel(),
                                         self._stream()))
        return out

    def beta_loo(self, alm, state, out=None) -> torch.Tensor:
        """modal_beta_loo: beta^hat of skies that were accumulated into ``state``, each with
        its own maps left out of the Monte-Carlo pair means."""
        a = self._alm(alm)
        S = a.shape[0]
        if out is None:
            out = torch.empty((S, self.nmax), dtype=torch.float64, device=self.device)
        ws = self.workspace(L.OP_BETA_LOO, S)
        self._check(self._lib.modal_beta_loo(self._h, _ptr(a), S, _ptr(state), _ptr(out), _ptr(ws), ws.numel(),
                                             self._stream()))
        return out

    def beta_noalloc(self, alm, state=None, out=None) -> torch.Tensor:
        """modal_beta_noalloc: beta with the library's fixed device scratch as workspace."""
        a = self._alm(alm)
        S = a.shape[0]
        if out is None:
            out = torch.empty((S, self.nmax), dtype=torch.float64, device=self.device)
        self._check(self._lib.modal_beta_noalloc(self._h, _ptr(a), S, _ptr(state), _ptr(out), self._stream()))
        return out

    def autotune(self, alm, state=None) -> dict:
        """Pick the fastest launch configuration for modal_beta on these inputs."""
        a = self._alm(alm)
        S = a.shape[0]
        out = torch.empty((S, self.nmax), dtype=torch.float64, device=self.device)
        ws = self.workspace(L.OP_BETA, S)
        ch, rr = C.c_int(), C.c_int()
        self._check(self._lib.modal_autotune(self._h, _ptr(a), S, _ptr(state), _ptr(out), _ptr(ws), ws.numel(),
                                             self._stream(), C.byref(ch), C.byref(rr)))
        return {"chunk_px": ch.value, "fft_rings": rr.value}

    def linear_state(self) -> torch.Tensor:
        n = int(self._lib.modal_linear_state_size(self._h))
        return torch.empty(n, dtype=torch.uint8, device=self.device)

    def linear_reset(self, state):
        self._check(self._lib.modal_linear_term(self._h, L.LIN_RESET, None, 0, _ptr(state), None, None, 0,
                                                self._stream()))

    def linear_accumulate(self, state, alm):
        a = self._alm(alm)
        S = a.shape[0]
        ws = self.workspace(L.OP_LINEAR_ACCUMULATE, S)
        self._check(self._lib.modal_linear_term(self._h, L.LIN_ACCUMULATE, _ptr(a), S, _ptr(state), None,
                                                _ptr(ws), ws.numel(), self._stream()))

    def linear_finalize(self, state):
        ws = self.workspace(L.OP_LINEAR_FINALIZE, 1)
        self._check(self._lib.modal_linear_term(self._h, L.LIN_FINALIZE, None, 0, _ptr(state), None, _ptr(ws),
                                                ws.numel(), self._stream()))

    def linear_apply(self, state, alm) -> torch.Tensor:
        a = self._alm(alm)
        S = a.shape[0]
        out = torch.empty((S, self.nmax), dtype=torch.float64, device=self.device)
        ws = self.workspace(L.OP_LINEAR_APPLY, S)
        self._check(self._lib.modal_linear_term(self._h, L.LIN_APPLY, _ptr(a), S, _ptr(state), _ptr(out),
                                                _ptr(ws), ws.numel(), self._stream()))
        return out

    def pair_means(self, state) -> torch.Tensor:
        """View of a finalised state as V[pair][ntheta][nphi]."""
        n = self.npairs * self.ntheta * self.nphi
        return state.view(self.real_dtype)[:n].view(self.npairs, self.ntheta, self.nphi)

    def beta_vjp(self, alm, cot, state=None) -> torch.Tensor:
        a = self._alm(alm)
        S = a.shape[0]
        c = torch.as_tensor(cot).to(device=self.device, dtype=torch.float64).reshape(S, self.nmax).contiguous()
        g = torch.empty((S, self.nalm), dtype=self.complex_dtype, device=self.device)
        ws = self.workspace(L.OP_BETA_VJP, S)
        self._check(self._lib.modal_beta_vjp(self._h, _ptr(a), S, _ptr(state), _ptr(c), _ptr(g), _ptr(ws),
                                             ws.numel(), self._stream()))
        return g

    def covariance_sample(self, beta, centered: bool = False) -> torch.Tensor:
        """zeta from beta^hat rows: sum b b^T / (6N), or with the mean subtracted and
        1 / (6 (N - 1)) when ``centered``."""
        b = torch.as_tensor(beta).to(device=self.device, dtype=torch.float64).contiguous()
        N = b.shape[0]
        z = torch.empty((self.nmax, self.nmax), dtype=torch.float64, device=self.device)
        op, method = (L.OP_COVARIANCE_CENTERED, L.COV_SAMPLE_CENTERED) if centered else \
            (L.OP_COVARIANCE_SAMPLE, L.COV_SAMPLE)
        ws = self.workspace(op, N)
        self._check(self._lib.modal_covariance(self._h, method, _ptr(b), None, None, None, N, _ptr(z),
                                               _ptr(ws), ws.numel(), self._stream()))
        return z

    def covariance_fisher(self, alm, cvar, state=None) -> torch.Tensor:
        """zeta_F = (1/(18N)) sum_i J_i C J_i^T for the N maps alm [N][nalm]; cvar[l] is the
        variance C_l of a_lm (C_l for a_l0, C_l/2 for Re and Im of a_lm, m > 0)."""
        a = self._alm(alm)
        N = a.shape[0]
        cv = np.ascontiguousarray(cvar, dtype=np.float64)
        if cv.shape != (self.lmax + 1,):
            raise ValueError("cvar must have lmax+1 entries")
        z = torch.empty((self.nmax, self.nmax), dtype=torch.float64, device=self.device)
        ws = self.workspace(L.OP_COVARIANCE_FISHER, N)
        self._check(self._lib.modal_covariance(self._h, L.COV_FISHER, None, _ptr(a), _ptr(state), cv.ctypes.data,
                                               N, _ptr(z), _ptr(ws), ws.numel(), self._stream()))
        return z

    def fnl(self, zeta, alpha, beta, want_L: bool = False):
        z = torch.as_tensor(zeta).to(device=self.device, dtype=torch.float64).contiguous()
        al = torch.as_tensor(alpha).to(device=self.device, dtype=torch.float64).contiguous()
        b = torch.as_tensor(beta).to(device=self.device, dtype=torch.float64).reshape(-1, self.nmax).contiguous()
        S = b.shape[0]
        E = np.zeros(S)
        s2 = np.zeros(1)
        Ld = torch.empty_like(z) if want_L else None
        ws = self.workspace(L.OP_FNL, S)
        self._check(self._lib.modal_fnl(self._h, _ptr(z), _ptr(al), _ptr(b), S, E.ctypes.data, s2.ctypes.data,
                                        _ptr(Ld), _ptr(ws), ws.numel(), self._stream()))
        return (E, float(s2[0]), Ld) if want_L else (E, float(s2[0]))


    # -- truncated orthonormal frame (Sec. II, eq. Cholrot) -----------------------------

    def frame(self, zeta0, tol: float = 1e-10):
        """Pivoted, truncated Cholesky of zeta0: (k, perm [k] int32, L11 [k][k]) with the
        k kept modes perm and the lower factor L11 of zeta0 restricted to them."""
        z = torch.as_tensor(zeta0).to(device=self.device, dtype=torch.float64).contiguous()
        perm = torch.empty(self.nmax, dtype=torch.int32, device=self.device)
        L11 = torch.empty(self.nmax * self.nmax, dtype=torch.float64, device=self.device)
        k = C.c_int()
        ws = self.workspace(L.OP_FRAME, 0)
        self._check(self._lib.modal_frame(self._h, _ptr(z), float(tol), C.byref(k), _ptr(perm), _ptr(L11),
                                          _ptr(ws), ws.numel(), self._stream()))
        k = k.value
        return k, perm[:k].clone(), L11[:k * k].reshape(k, k).clone()

    def frame_rotate(self, perm, L11, x):
        """Rows x [R][nmax] -> L11^-1 x[perm] [R][k] (the coordinates in the frame)."""
        k = int(L11.shape[0])
        p = torch.zeros(self.nmax, dtype=torch.int32, device=self.device)
        p[:k] = perm
        xx = torch.as_tensor(x).to(device=self.device, dtype=torch.float64).reshape(-1, self.nmax).contiguous()
        y = torch.empty((xx.shape[0], k), dtype=torch.float64, device=self.device)
        self._check(self._lib.modal_frame_rotate(self._h, k, _ptr(p), _ptr(L11.contiguous()), _ptr(xx), xx.shape[0],
                                                 _ptr(y), self._stream()))
        return y

    def fnl_frame(self, zeta, perm, alpha, beta):
        """E [S] and sigma^2 of the estimator on the kept modes perm [k] (zeta any covariance)."""
        k = int(perm.shape[0])
        p = torch.zeros(self.nmax, dtype=torch.int32, device=self.device)
        p[:k] = perm
        z = torch.as_tensor(zeta).to(device=self.device, dtype=torch.float64).contiguous()
        al = torch.as_tensor(alpha).to(device=self.device, dtype=torch.float64).contiguous()
        b = torch.as_tensor(beta).to(device=self.device, dtype=torch.float64).reshape(-1, self.nmax).contiguous()
        S = b.shape[0]
        E = np.zeros(S)
        s2 = np.zeros(1)
        ws = self.workspace(L.OP_FNL_FRAME, S)
        self._check(self._lib.modal_fnl_frame(self._h, _ptr(z), k, _ptr(p), _ptr(al), _ptr(b), S, E.ctypes.data,
                                              s2.ctypes.data, _ptr(ws), ws.numel(), self._stream()))
        return E, float(s2[0])

    # -- low-rank covariance I + sum_j b_j b_j^T (Sec. III B) --------------------------

    def noise_vectors(self, beta, k: int = 1, iters: int = 100):
        """The k leading noise vectors b_j [k][nmax] of the sample covariance of the rows of
        beta [N][nmax] (b_j = sqrt(max(mu_j - 1, 0)) v_j) and the eigenvalues mu_j."""
        b = torch.as_tensor(beta).to(device=self.device, dtype=torch.float64).reshape(-1, self.nmax).contiguous()
        N = b.shape[0]
        bt = torch.empty((k, self.nmax), dtype=torch.float64, device=self.device)
        mu = np.zeros(k)
        ws = self.workspace(L.OP_NOISE_VECTORS, N)
        self._check(self._lib.modal_noise_vectors(self._h, _ptr(b), N, k, iters, _ptr(bt), mu.ctypes.data, _ptr(ws),
                                                  ws.numel(), self._stream()))
        return bt, mu

    def fnl_lowrank(self, bt, alpha, beta):
        """E_s and sigma^2 with zeta = I + sum_j b_j b_j^T (rows of bt, possibly none)."""
        v = torch.as_tensor(bt).to(device=self.device, dtype=torch.float64).reshape(-1, self.nmax).contiguous()
        al = torch.as_tensor(alpha).to(device=self.device, dtype=torch.float64).contiguous()
        b = torch.as_tensor(beta).to(device=self.device, dtype=torch.float64).reshape(-1, self.nmax).contiguous()
        S, k = b.shape[0], v.shape[0]
        E = np.zeros(S)
        s2 = np.zeros(1)
        ws = self.workspace(L.OP_FNL_LOWRANK, S)
        self._check(self._lib.modal_fnl_lowrank(self._h, _ptr(v) if k else None, k, _ptr(al), _ptr(b), S,
                                                E.ctypes.data, s2.ctypes.data, _ptr(ws), ws.numel(), self._stream()))
        return E, float(s2[0])

    def bivector_rotate(self, b, x) -> torch.Tensor:
        """Rows of x rotated by the inverse closed-form Cholesky factor of I + b b^T."""
        bv = torch.as_tensor(b).to(device=self.device, dtype=torch.float64).contiguous()
        xv = torch.as_tensor(x).to(device=self.device, dtype=torch.float64).reshape(-1, self.nmax).contiguous()
        y = torch.empty_like(xv)
        self._check(self._lib.modal_bivector_rotate(self._h, _ptr(bv), _ptr(xv), xv.shape[0], _ptr(y),
                                                    self._stream()))
        return y

    def alpha_separable(self, terms) -> torch.Tensor:
        """alpha_n of b = sum_t X_t(l1) Y_t(l2) Z_t(l3) (terms [T][3][lmax+1], host array)."""
        tm = np.ascontiguousarray(terms, dtype=np.float64)
        if tm.ndim != 3 or tm.shape[1:] != (3, self.lmax + 1):
            raise ValueError("terms must be [T][3][lmax+1]")
        T = tm.shape[0]
        a = torch.empty(self.nmax, dtype=torch.float64, device=self.device)
        ws = self.workspace(L.OP_ALPHA_SEPARABLE, T)
        self._check(self._lib.modal_alpha_separable(self._h, tm.ctypes.data, T, _ptr(a), _ptr(ws), ws.numel(),
                                                    self._stream()))
        return a

    def ideal_covariance(self, c=None) -> torch.Tensor:
        """zeta0 [nmax][nmax] for full-sky skies with <|a~_lm|^2> = c_l (default 1 where C_l > 0)."""
        cv = None
        if c is not None:
            cv = np.ascontiguousarray(c, dtype=np.float64)
            if cv.shape != (self.lmax + 1,):
                raise ValueError("c must have lmax+1 entries")
        z = torch.empty((self.nmax, self.nmax), dtype=torch.float64, device=self.device)
        ws = self.workspace(L.OP_IDEAL_COVARIANCE, 0)
        self._check(self._lib.modal_ideal_covariance(self._h, None if cv is None else cv.ctypes.data, _ptr(z),
                                                     _ptr(ws), ws.numel(), self._stream()))
        return z

    # -- modal trispectrum (Sec. IV) ---------------------------------------------------

    def trispectrum(self, alm, state=None, out=None) -> torch.Tensor:
        """tau [S][nquad] for quadruples p <= r <= s <= u (V from a finalised linear-term state)."""
        a = self._alm(alm)
        S = a.shape[0]
        nq = self._lib.modal_nquad(self._h)
        t = out if out is not None else torch.empty((S, nq), dtype=torch.float64, device=self.device)
        ws = self.workspace(L.OP_TRISPECTRUM, S)
        self._check(self._lib.modal_trispectrum(self._h, _ptr(a), S, _ptr(state), _ptr(t), _ptr(ws), ws.numel(),
                                                self._stream()))
        return t

    # -- modal power spectrum (Sec. IV) ------------------------------------------------

    def power_beta(self, alm, state=None, out=None) -> torch.Tensor:
        """beta_pr = sum_x w (M_p M_r - V_pr) [S][npairs] (V from a finalised linear-term state)."""
        a = self._alm(alm)
        S = a.shape[0]
        b = out if out is not None else torch.empty((S, self.npairs), dtype=torch.float64, device=self.device)
        ws = self.workspace(L.OP_POWER_BETA, S)
        self._check(self._lib.modal_power_beta(self._h, _ptr(a), S, _ptr(state), _ptr(b), _ptr(ws), ws.numel(),
                                               self._stream()))
        return b

    def power_alpha(self, dcl) -> torch.Tensor:
        """alpha_n [P] on the modes (0, n) for a spectral deviation dcl = C~_l - C_l."""
        d = np.ascontiguousarray(dcl, dtype=np.float64)
        if d.shape != (self.lmax + 1,):
            raise ValueError("dcl must have lmax+1 entries")
        a = torch.empty(self.P, dtype=torch.float64, device=self.device)
        ws = self.workspace(L.OP_POWER_ALPHA, 0)
        self._check(self._lib.modal_power_alpha(self._h, d.ctypes.data, _ptr(a), _ptr(ws), ws.numel(),
                                                self._stream()))
        return a

    def power_ideal_covariance(self, c=None) -> torch.Tensor:
        cv = None
        if c is not None:
            cv = np.ascontiguousarray(c, dtype=np.float64)
            if cv.shape != (self.lmax + 1,):
                raise ValueError("c must have lmax+1 entries")
        z = torch.empty((self.P, self.P), dtype=torch.float64, device=self.device)
        ws = self.workspace(L.OP_POWER_COVARIANCE, 0)
        self._check(self._lib.modal_power_ideal_covariance(self._h, None if cv is None else cv.ctypes.data, _ptr(z),
                                                           _ptr(ws), ws.numel(), self._stream()))
        return z

    def power_fnl(self, zeta, alpha, beta):
        """E_s and sigma^2 on the modes (0, n); beta is the [S][npairs] output of power_beta."""
        z = torch.as_tensor(zeta).to(device=self.device, dtype=torch.float64).contiguous()
        al = torch.as_tensor(alpha).to(device=self.device, dtype=torch.float64).contiguous()
        b = torch.as_tensor(beta).to(device=self.device, dtype=torch.float64).reshape(-1, self.npairs).contiguous()
        S = b.shape[0]
        E = np.zeros(S)
        s2 = np.zeros(1)
        ws = self.workspace(L.OP_POWER_FNL, S)
        self._check(self._lib.modal_power_fnl(self._h, _ptr(z), _ptr(al), _ptr(b), S, E.ctypes.data, s2.ctypes.data,
                                              _ptr(ws), ws.numel(), self._stream()))
        return E, float(s2[0])

    def whiten(self, Lfac, x) -> torch.Tensor:
        """Rows of x multiplied by L^-1 (L lower triangular, as returned by fnl(want_L=True))."""
        Lv = torch.as_tensor(Lfac).to(device=self.device, dtype=torch.float64).contiguous()
        xv = torch.as_tensor(x).to(device=self.device, dtype=torch.float64).reshape(-1, self.nmax).contiguous()
        y = torch.empty_like(xv)
        self._check(self._lib.modal_whiten(self._h, _ptr(Lv), _ptr(xv), xv.shape[0], _ptr(y), self._stream()))
        return y


class BetaGraph:
    """A captured sequence of modal_beta calls (one per context, mixed l_max allowed),
    replayed with a single graph launch.  Holds references to every tensor baked
    into the graph."""

    def __init__(self, calls):
        """calls: list of (ModalContext, alm tensor [S][nalm], state or None); calls on one
        context share its workspace."""
        self._lib = L.lib()
        n = len(calls)
        self.ctxs = [c for c, _, _ in calls]
        self.alms = [c._alm(a) for c, a, _ in calls]
        self.states = [st for _, _, st in calls]
        self.betas = [torch.empty((a.shape[0], c.nmax), dtype=torch.float64, device=c.device)
                      for (c, _, _), a in zip(calls, self.alms)]
        # the calls run one after another on one stream, so calls on the same context share
        # one workspace, sized for the largest S among them
        need = {}
        for (c, _, _), a in zip(calls, self.alms):
            need[id(c)] = max(need.get(id(c), 256), c.workspace_size(L.OP_BETA, a.shape[0]))
        shared = {k: torch.empty(v, dtype=torch.uint8, device=self.ctxs[0].device) for k, v in need.items()}
        self.ws = [shared[id(c)] for c, _, _ in calls]
        arr = lambda T, vals: (T * n)(*vals)
        ctxs = arr(C.c_void_p, [c._h.value for c in self.ctxs])
        alms = arr(C.c_void_p, [a.data_ptr() for a in self.alms])
        Ss = arr(C.c_int, [a.shape[0] for a in self.alms])
        sts = arr(C.c_void_p, [None if s is None else s.data_ptr() for s in self.states])
        bts = arr(C.c_void_p, [b.data_ptr() for b in self.betas])
        wss = arr(C.c_void_p, [w.data_ptr() for w in self.ws])
        wsb = arr(C.c_size_t, [w.numel() for w in self.ws])
        self._g = C.c_void_p()
        before = [self._lib.modal_last_error(c._h) for c in self.ctxs]
        st = self._lib.modal_beta_graph_create(n, ctxs, alms, Ss, sts, bts, wss, wsb, C.byref(self._g))
        if st != L.OK:
            # a failing call records its error on its own context
            msgs = [self._lib.modal_last_error(c._h).decode() for i, c in enumerate(self.ctxs)
                    if self._lib.modal_last_error(c._h) != before[i]]
            if not msgs:
                msgs = [m.decode() for m in (self._lib.modal_last_error(c._h) for c in self.ctxs)
                        if m.startswith(b"graph call")]
            raise L.ModalError(st, "; ".join(msgs) or "graph capture failed")

    def launch(self):
        dev = self.ctxs[0].device
        st = self._lib.modal_graph_launch(self._g, C.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
        if st != L.OK:
            raise L.ModalError(st, "graph launch failed")
        return self.betas

    def close(self):
        if getattr(self, "_g", None) is not None and self._g.value:
            self._lib.modal_graph_destroy(self._g)
            self._g = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
