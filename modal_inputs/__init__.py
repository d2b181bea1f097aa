"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds only *input data*: index helpers, the power spectra and
basis functions that parametrise a run, and seeded Gaussian harmonic
coefficients.  It contains none of the estimator's arithmetic (no spherical
harmonic transform, no quadrature, no cubic reduction) so that the oracle and
the GPU path can both draw their inputs from it without sharing any of the
computation being checked.

Workload shapes follow the paper's WMAP-resolution setting (Sec. III C:
l_max = 500 with a beam, inhomogeneous noise and a Galactic cut) and the
metric shape used for throughput (l_max = 1000 on a 1536 x 3072 ring grid).
The paper's own data (the KQ75 mask, WMAP beams and noise maps, theory
bispectra) are not available; the synthetic sky model below stands in for
them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import numpy.polynomial.legendre as npleg

__all__ = [
    "Config", "CONFIGS", "nalm", "alm_index", "lm_arrays", "npairs", "ntriples",
    "pair_list", "triple_list", "cl_signal", "beam", "noise_level",
    "filter_cl", "q_basis", "rng_for", "gaussian_alm", "mask_rings",
    "noise_sigma2", "FSKY_BAND10",
]


# ---------------------------------------------------------------------------
# index helpers (layout contract shared with the C ABI)
# ---------------------------------------------------------------------------

def nalm(lmax: int) -> int:
    """Number of stored a_lm (0 <= m <= l <= lmax)."""
    return (lmax + 1) * (lmax + 2) // 2


def alm_index(l, m, lmax: int):
    """m-major triangular index: all l for m = 0, then all l >= 1 for m = 1, ..."""
    l = np.asarray(l)
    m = np.asarray(m)
    return m * (2 * lmax + 3 - m) // 2 + (l - m)


def lm_arrays(lmax: int):
    """(l, m) of every stored coefficient, in storage order."""
    ls, ms = [], []
    for m in range(lmax + 1):
        ls.append(np.arange(m, lmax + 1))
        ms.append(np.full(lmax + 1 - m, m))
    return np.concatenate(ls), np.concatenate(ms)


def npairs(P: int) -> int:
    return P * (P + 1) // 2


def ntriples(P: int) -> int:
    return P * (P + 1) * (P + 2) // 6


def pair_list(P: int):
    """Mode pairs (p, r) with p <= r in lexicographic order."""
    return [(p, r) for p in range(P) for r in range(p, P)]


def triple_list(P: int):
    """Mode triples (p, r, s) with p <= r <= s in lexicographic order (n index)."""
    return [(p, r, s) for p in range(P) for r in range(p, P) for s in range(r, P)]


# ---------------------------------------------------------------------------
# sky model
# ---------------------------------------------------------------------------

FSKY_BAND10 = 1.0 - math.sin(math.radians(10.0))  # sky fraction outside |lat| < 10 deg


def cl_signal(lmax: int) -> np.ndarray:
    """Toy scale-invariant signal spectrum C_l = 1/(l(l+1)) for l >= 2, zero below."""
    l = np.arange(lmax + 1, dtype=np.float64)
    cl = np.zeros(lmax + 1)
    cl[2:] = 1.0 / (l[2:] * (l[2:] + 1.0))
    return cl


def beam(lmax: int, fwhm_arcmin: float = 13.0) -> np.ndarray:
    """Gaussian beam window b_l = exp(-l(l+1) sigma_b^2 / 2)."""
    sig = math.radians(fwhm_arcmin / 60.0) / math.sqrt(8.0 * math.log(2.0))
    l = np.arange(lmax + 1, dtype=np.float64)
    return np.exp(-0.5 * l * (l + 1.0) * sig * sig)


def noise_level(lmax: int, l_eq: int = 400, fwhm_arcmin: float = 13.0) -> float:
    """White-noise power N_l chosen so that signal equals noise at l = l_eq."""
    b = beam(max(lmax, l_eq), fwhm_arcmin)
    return float(b[l_eq] ** 2 / (l_eq * (l_eq + 1.0)))


def noise_sigma2(theta: np.ndarray, npix: int, nl: float) -> np.ndarray:
    """Pixel-noise variance profile sigma^2(theta) = sigma0^2 / (1 + 4 cos^2 theta).

    sigma0 is fixed by requiring the sky-averaged white-noise power
    (4 pi / npix) <sigma^2> to equal ``nl``; <1/(1+4 mu^2)> over the sphere is
    arctan(2)/2.
    """
    sigma0_sq = nl * npix / (4.0 * math.pi) * 2.0 / math.atan(2.0)
    return sigma0_sq / (1.0 + 4.0 * np.cos(theta) ** 2)


def mask_rings(theta: np.ndarray, cut_deg: float = 10.0) -> np.ndarray:
    """Per-ring mask: 0 where |90 deg - theta| < cut_deg, else 1."""
    lat = np.abs(0.5 * math.pi - np.asarray(theta))
    return (lat >= math.radians(cut_deg)).astype(np.float64)


def filter_cl(lmax: int, sky: str) -> np.ndarray:
    """C_l used to whiten a_lm.

    'ideal': the signal spectrum itself.
    'wmap' : f_sky (b_l^2 C_l + N_l), the isotropic approximation of the
             paper's Sec. III A.
    """
    cl = cl_signal(lmax)
    if sky == "ideal":
        return cl
    if sky != "wmap":
        raise ValueError(sky)
    b = beam(lmax)
    nl = noise_level(lmax)
    out = FSKY_BAND10 * (b * b * cl + nl)
    out[:2] = 0.0
    return out


def q_basis(P: int, lmax: int) -> np.ndarray:
    """Separable 1-D mode functions q_p(l) = P_p(2 l / lmax - 1), p = 0..P-1."""
    t = 2.0 * np.arange(lmax + 1, dtype=np.float64) / lmax - 1.0
    out = np.empty((P, lmax + 1))
    for p in range(P):
        c = np.zeros(p + 1)
        c[p] = 1.0
        out[p] = npleg.legval(t, c)
    return out


# ---------------------------------------------------------------------------
# seeded random numbers
# ---------------------------------------------------------------------------

def rng_for(cfg_id: int, sim_id: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(cfg_id), int(sim_id)])))


def gaussian_alm(cl: np.ndarray, lmax: int, rng: np.random.Generator) -> np.ndarray:
    """Isotropic Gaussian a_lm with <|a_lm|^2> = C_l (real a_l0 of variance C_l,
    Re and Im of variance C_l / 2 for m > 0), stored m-major."""
    l, m = lm_arrays(lmax)
    sd = np.sqrt(cl[l])
    re = rng.standard_normal(l.size)
    im = rng.standard_normal(l.size)
    a = np.where(m == 0, re * sd, re * sd / math.sqrt(2.0)) + 1j * np.where(m == 0, 0.0, im * sd / math.sqrt(2.0))
    return a.astype(np.complex128)


# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    cfg_id: int
    lmax: int
    ntheta: int
    nphi: int
    P: int
    sims: int
    sky: str          # 'ideal' (full sky, signal only) or 'wmap' (beam+noise+mask)
    prec: str         # arithmetic of the GPU path for this workload

    @property
    def npix(self) -> int:
        return self.ntheta * self.nphi

    @property
    def nmax(self) -> int:
        return ntriples(self.P)

    @property
    def npairs(self) -> int:
        return npairs(self.P)


CONFIGS = {
    "tiny": Config("tiny", 1, 32, 48, 96, 8, 1, "ideal", "f64"),
    "wmap500": Config("wmap500", 2, 500, 768, 1536, 30, 100, "wmap", "f32"),
    "adjoint500": Config("adjoint500", 3, 500, 768, 1536, 30, 256, "wmap", "f32"),
    "precision1024": Config("precision1024", 4, 1024, 1536, 3072, 40, 200, "wmap", "bf16x3"),
    "metric1000": Config("metric1000", 6, 1000, 1536, 3072, 40, 32, "wmap", "bf16x3"),
    "mixed500": Config("mixed500", 5, 500, 768, 1536, 50, 512, "wmap", "bf16x3"),
    "mixed1000": Config("mixed1000", 5, 1000, 1536, 3072, 50, 512, "wmap", "bf16x3"),
    "mixed2000": Config("mixed2000", 5, 2000, 3008, 6016, 50, 512, "wmap", "bf16x3"),
}
