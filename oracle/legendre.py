"""Normalised associated Legendre functions lambda_lm(cos theta) (oracle).

Y_lm(theta, phi) = lambda_lm(cos theta) e^{i m phi} with the Condon-Shortley
phase, so that the reality condition a_{l,-m} = (-1)^m a_lm^* matches the
signal covariance convention of Appendix A, and Y_lm is orthonormal on the
sphere (the orthonormal harmonic basis behind the Gaunt integral of Sec. II).

Textbook construction, FP64, per fixed m:
  lambda_mm     = (-1)^m sqrt((2m+1)/(4 pi) prod_{k=1..m} (2k-1)/(2k)) sin^m theta
  lambda_{m+1,m} = sqrt(2m+3) x lambda_mm
  lambda_lm     = a_lm (x lambda_{l-1,m} - b_lm lambda_{l-2,m}),
      a_lm = sqrt((4l^2-1)/(l^2-m^2)),  b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)).
The seed is carried as a logarithm and the recurrence on a scaled value with a
separate log-scale, so that l_max = 2000 never underflows before the value is
significant; values below the FP64 range come out as 0.
"""
from __future__ import annotations

import math

import numpy as np

_RESCALE = 1e100
_LOG_RESCALE = math.log(_RESCALE)


def log_seed_prefactor(m: int) -> float:
    """log sqrt((2m+1)/(4 pi) prod_{k=1..m} (2k-1)/(2k))."""
    k = np.arange(1, m + 1, dtype=np.float64)
    s = float(np.sum(np.log((2.0 * k - 1.0) / (2.0 * k)))) if m > 0 else 0.0
    return 0.5 * (math.log((2.0 * m + 1.0) / (4.0 * math.pi)) + s)


def lambda_m(m: int, lmax: int, x) -> np.ndarray:
    """lambda_lm(x) for l = m..lmax at the points x; shape [lmax-m+1, len(x)]."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    out = np.zeros((lmax - m + 1, x.size))
    sin_t = np.sqrt(np.maximum(0.0, (1.0 - x) * (1.0 + x)))
    with np.errstate(divide="ignore"):
        logscale = log_seed_prefactor(m) + (m * np.log(sin_t) if m > 0 else np.zeros_like(x))
    sign = -1.0 if (m % 2) else 1.0
    # s_prev2 = scaled lambda_{l-2}, s_prev = scaled lambda_{l-1}
    s_prev = np.full(x.size, sign)
    s_prev2 = np.zeros(x.size)

    def emit(idx, s):
        with np.errstate(divide="ignore", over="ignore", under="ignore"):
            mag = np.where(s != 0.0, np.exp(logscale + np.log(np.abs(s) + (s == 0.0))), 0.0)
        out[idx] = np.sign(s) * mag

    emit(0, s_prev)
    for l in range(m + 1, lmax + 1):
        if l == m + 1:
            s = math.sqrt(2.0 * m + 3.0) * x * s_prev
        else:
            a = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
            b = math.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
            s = a * (x * s_prev - b * s_prev2)
        s_prev2, s_prev = s_prev, s
        big = np.abs(s_prev) > _RESCALE
        if np.any(big):
            s_prev = np.where(big, s_prev / _RESCALE, s_prev)
            s_prev2 = np.where(big, s_prev2 / _RESCALE, s_prev2)
            logscale = np.where(big, logscale + _LOG_RESCALE, logscale)
        emit(l - m, s_prev)
    return out


def lambda_all(lmax: int, x) -> np.ndarray:
    """All lambda_lm(x) in m-major storage order; shape [nalm, len(x)]."""
    return np.concatenate([lambda_m(m, lmax, x) for m in range(lmax + 1)], axis=0)


def ylm(l: int, m: int, theta, phi) -> np.ndarray:
    """Complex Y_lm for any integer m (negative m through Y_{l,-m} = (-1)^m Y_lm^*)."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    am = abs(m)
    lam = lambda_m(am, l, np.cos(theta).ravel())[l - am].reshape(theta.shape)
    y = lam * np.exp(1j * am * phi)
    if m < 0:
        y = ((-1) ** am) * np.conj(y)
    return y


def lambda_table(lmax: int, x):
    """[lambda_m(m, lmax, x) for m = 0..lmax]: every lambda_lm on the points x, computed once
    (for repeated transforms on one grid)."""
    return [lambda_m(m, lmax, x) for m in range(lmax + 1)]
