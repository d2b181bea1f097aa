"""torch.autograd binding of beta^hat = beta - lin with the library's adjoint.

Forward runs modal_beta; backward runs modal_beta_vjp (maps recomputed, pair
contraction, r2c ring FFT, adjoint Legendre).  The linear-term state is held
fixed (it is a Monte-Carlo average, not a function of the input map).

Gradient convention: a_lm for m > 0 are complex with independent real and
imaginary parts (a_{l,-m} follows from reality); the returned gradient packs
dL/dRe a_lm + i dL/dIm a_lm, which is what torch expects for a real-valued
loss of a complex leaf when the loss is written in terms of Re/Im.  For m = 0
only the real part is a degree of freedom.
"""
from __future__ import annotations

import torch


class ModalBeta(torch.autograd.Function):
    @staticmethod
    def forward(ctx_, alm: torch.Tensor, mctx, state=None):
        out = mctx.beta(alm.detach(), state=state)
        ctx_.mctx = mctx
        ctx_.state = state
        ctx_.save_for_backward(alm.detach())
        return out

    @staticmethod
    def backward(ctx_, grad_out: torch.Tensor):
        (alm,) = ctx_.saved_tensors
        g = ctx_.mctx.beta_vjp(alm, grad_out.contiguous(), state=ctx_.state)
        return g.to(alm.dtype).reshape(alm.shape), None, None


def modal_beta(alm: torch.Tensor, mctx, state=None) -> torch.Tensor:
    """beta^hat[S][nmax] (float64) differentiable with respect to alm [S][nalm]."""
    if alm.dim() == 1:
        return ModalBeta.apply(alm[None], mctx, state)[0]
    return ModalBeta.apply(alm, mctx, state)
