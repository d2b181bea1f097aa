"""Gaussian sky simulations with beam, inhomogeneous noise and a Galactic cut
(oracle-side generator for test inputs).

Stand-in for the WMAP-realistic simulations of Sec. III C (KQ75 mask, WMAP
beams and noise model, which are not available): signal a_lm with
C_l b_l^2, pixel white noise of variance sigma^2(theta) Omega_bar / dA(x)
(Appendix A: noise described by a pixel-variance map, 4 pi / n_pix per pixel;
here Omega_bar = 4 pi / n_pix and dA the pixel's quadrature area), a mask that
zeroes |latitude| < 10 deg (Appendix A: the mask as infinite noise), then a
quadrature analysis back to a_lm.  Random numbers come from
``modal_inputs.rng_for``.
"""
from __future__ import annotations

import math

import numpy as np

import modal_inputs as mi
from .grid import Grid
from .legendre import lambda_m
from .modal import ring_coefficients, maps_from_ring_coefficients


def synth_scalar(alm: np.ndarray, lmax: int, grid: Grid, lam=None) -> np.ndarray:
    """f(x) = sum_lm a_lm Y_lm(x) for a real field stored as m >= 0.  lam: optional
    ``legendre.lambda_table(lmax, grid.x)`` (the same lambda_lm, computed once)."""
    if lam is None:
        F = ring_coefficients(np.atleast_2d(alm), np.ones((1, lmax + 1)), lmax, grid.x)
        return maps_from_ring_coefficients(F, grid.nphi)[0, 0]
    F = np.zeros((1, 1, grid.x.size, lmax + 1), dtype=np.complex128)
    for m in range(lmax + 1):
        a = alm[mi.alm_index(np.arange(m, lmax + 1), m, lmax)]
        F[0, 0, :, m] = (a.real @ lam[m]) + 1j * (a.imag @ lam[m])
    return maps_from_ring_coefficients(F, grid.nphi)[0, 0]


def analysis(f: np.ndarray, lmax: int, grid: Grid, lam=None) -> np.ndarray:
    """a_lm = sum_x dA(x) f(x) Y*_lm(x) with the full-sky quadrature weights.  lam: optional
    ``legendre.lambda_table(lmax, grid.x)``."""
    fh = np.fft.rfft(f, axis=-1)[:, :lmax + 1] * (2.0 * math.pi / grid.nphi)   # [nt, L]
    out = np.zeros(mi.nalm(lmax), dtype=np.complex128)
    for m in range(lmax + 1):
        lm = lambda_m(m, lmax, grid.x) if lam is None else lam[m]   # [L_m, nt]
        v = grid.wgl * fh[:, m]
        out[mi.alm_index(np.arange(m, lmax + 1), m, lmax)] = (lm @ v.real) + 1j * (lm @ v.imag)
    l, m = mi.lm_arrays(lmax)
    out[m == 0] = out[m == 0].real
    return out


def noise_pixel_variance(grid: Grid, nl: float) -> np.ndarray:
    """Variance of the white noise in each pixel, sigma^2(theta) Omega_bar / dA(x) with
    Omega_bar = 4 pi / n_pix (Appendix A: the noise as a pixel-variance map at the
    mean pixel area; dividing by the pixel's own quadrature area keeps the harmonic
    noise power at Omega_bar <sigma^2> = nl on unequal-area rings).  Shape [ntheta, nphi]."""
    sig2 = mi.noise_sigma2(grid.theta, grid.npix, nl)[:, None]
    return sig2 * (4.0 * math.pi / grid.npix) / grid.area


def wmap_like_grid(cfg: mi.Config) -> Grid:
    g0 = Grid(cfg.ntheta, cfg.nphi)
    if cfg.sky == "ideal":
        return g0
    return Grid(cfg.ntheta, cfg.nphi, ring_mask=np.repeat(mi.mask_rings(g0.theta)[:, None], cfg.nphi, axis=1))


def sky_sim(cfg: mi.Config, sim_id: int, grid: Grid, lmax: int | None = None) -> np.ndarray:
    """One simulated a_lm for configuration ``cfg`` ('ideal': isotropic signal)."""
    lmax = cfg.lmax if lmax is None else lmax
    rng = mi.rng_for(cfg.cfg_id, sim_id)
    cl = mi.cl_signal(lmax)
    if cfg.sky == "ideal":
        return mi.gaussian_alm(cl, lmax, rng)
    b = mi.beam(lmax)
    a_sig = mi.gaussian_alm(cl * b * b, lmax, rng)
    f = synth_scalar(a_sig, lmax, grid)
    var = noise_pixel_variance(grid, mi.noise_level(lmax))
    f = f + rng.standard_normal(f.shape) * np.sqrt(var)
    return analysis(f * grid.mask, lmax, grid)
