"""Gauss-Legendre ring grid (oracle).

The separable evaluation of beta_n replaces the Gaunt-weighted harmonic sum of
eq. (bbispect) by a pixel sum sum_x w(x) M_p M_r M_s.  That pixel sum equals the
integral over the sphere whenever the quadrature integrates the triple
product exactly, which a Gauss-Legendre ring grid does for
ntheta >= (3 l_max + 1)/2 and nphi >= 3 l_max + 1 (Sec. II: the Gaunt
integral as the isotropic factor of the bispectrum).

Rings are ordered north to south (cos theta descending); phi_k = 2 pi k / nphi.
"""
from __future__ import annotations

import math

import numpy as np


class Grid:
    def __init__(self, ntheta: int, nphi: int, ring_mask=None):
        x, wgl = np.polynomial.legendre.leggauss(ntheta)
        order = np.argsort(-x)
        self.ntheta = ntheta
        self.nphi = nphi
        self.x = x[order]                      # cos theta_j, descending
        self.wgl = wgl[order]                  # sum = 2
        self.theta = np.arccos(self.x)
        self.phi = 2.0 * math.pi * np.arange(nphi) / nphi
        dphi = 2.0 * math.pi / nphi
        ring_w = self.wgl * dphi               # area element of a pixel on ring j
        mask = np.ones((ntheta, nphi)) if ring_mask is None else np.broadcast_to(
            np.asarray(ring_mask, dtype=np.float64).reshape(ntheta, -1), (ntheta, nphi))
        self.mask = np.array(mask, dtype=np.float64)
        self.area = np.repeat(ring_w[:, None], nphi, axis=1)   # full-sky quadrature weights
        self.w = self.area * self.mask                          # estimator weights w(x)

    @property
    def npix(self) -> int:
        return self.ntheta * self.nphi


class RingSubset:
    """The rings ``idx`` of a grid (same nodes, same nphi, same weights): the pixel sums of
    the estimator split over rings, since sum_x = sum over ring groups of sum over their
    pixels."""

    def __init__(self, grid: Grid, idx):
        idx = np.asarray(idx, dtype=np.int64)
        self.idx = idx
        self.ntheta = int(idx.size)
        self.nphi = grid.nphi
        self.x = grid.x[idx]
        self.wgl = grid.wgl[idx]
        self.theta = grid.theta[idx]
        self.phi = grid.phi
        self.mask = grid.mask[idx]
        self.area = grid.area[idx]
        self.w = grid.w[idx]

    @property
    def npix(self) -> int:
        return self.ntheta * self.nphi
