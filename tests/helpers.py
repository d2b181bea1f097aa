"""Shared test helpers: seeded cases and the oracle's expected values."""
from __future__ import annotations

import dataclasses
import functools

import numpy as np

import modal_inputs as mi
from oracle import grid as og
from oracle import modal as om
from oracle import sims as osims


def rel_inf(got, ref) -> float:
    """max |got - ref| / rms(ref)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.sqrt(np.mean(ref * ref))
    return float(np.max(np.abs(got - ref)) / (scale if scale > 0 else 1.0))


@dataclasses.dataclass
class Case:
    name: str
    lmax: int
    ntheta: int
    nphi: int
    P: int
    S: int
    sky: str        # 'ideal' | 'wmap'
    cfg_id: int

    @functools.cached_property
    def grid(self):
        g0 = og.Grid(self.ntheta, self.nphi)
        if self.sky == "ideal":
            return g0
        return og.Grid(self.ntheta, self.nphi, ring_mask=np.repeat(mi.mask_rings(g0.theta)[:, None], self.nphi, 1))

    @functools.cached_property
    def cl(self):
        return mi.filter_cl(self.lmax, self.sky)

    @functools.cached_property
    def q(self):
        return mi.q_basis(self.P, self.lmax)

    def alms(self, first: int, count: int) -> np.ndarray:
        """Isotropic Gaussian a_lm with the filter spectrum (seeded)."""
        return np.array([mi.gaussian_alm(self.cl, self.lmax, mi.rng_for(self.cfg_id, first + i))
                         for i in range(count)])

    def mask(self):
        return None if self.sky == "ideal" else self.grid.mask

    def maps(self, alms):
        return om.filtered_maps(alms, self.cl, self.q, self.grid)


CASES = {
    # the l_max = 32 workload itself (48 x 96 grid, P = 8, full sky)
    "tiny": Case("tiny", 32, 48, 96, 8, 3, "ideal", 1),
    # odd ring count (equator ring), generic FFT radices (K = 200 = 4*2*5*5),
    # two pair blocks (91 pairs), two pixel chunks with a ragged tail, mask + beam/noise spectrum
    "ragged": Case("ragged", 150, 199, 400, 13, 3, "wmap", 21),
    # npix = 1250, not a multiple of 4: the element-wise staging paths of the float kernels
    # (half-length FFT of 25 = 5 x 5), mask + beam/noise spectrum
    "odd": Case("odd", 16, 25, 50, 5, 3, "wmap", 31),
    # nphi = 94: a prime half-length ring transform (K = 47), the radix that the l_max 2000
    # grid (nphi 6016 = 128 x 47) needs, in the generic transform kernels (c2r and r2c)
    "prime": Case("prime", 32, 48, 94, 8, 2, "wmap", 41),
    # the headline mode count, P = 40 (two 32-mode tiles in the split adjoint), and the largest
    # the split adjoint takes, P = 48 (168 eight-pair groups), on the l_max = 32 grid
    "wide": Case("wide", 32, 48, 96, 40, 2, "wmap", 51),
    "wide48": Case("wide48", 32, 48, 96, 48, 2, "wmap", 61),
    # past the split adjoint's 48 modes: the vector pair contraction takes over
    "wide50": Case("wide50", 32, 48, 96, 50, 2, "wmap", 71),
    # the largest mode count, P = 64: the contraction's cover takes 14 work items, two
    # workgroup groups of 8 waves with two waves idle
    "wide64": Case("wide64", 32, 48, 96, 64, 2, "wmap", 81),
}
