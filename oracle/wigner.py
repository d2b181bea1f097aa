"""Wigner 3j symbols (Racah closed form) and the Gaunt integral (oracle, pins only).

The Gaunt integral G^{l1 l2 l3}_{m1 m2 m3} = int Y_l1m1 Y_l2m2 Y_l3m3 dOmega is the
isotropic factor of the bispectrum (Sec. II); in closed form it is
  sqrt((2l1+1)(2l2+1)(2l3+1)/(4 pi)) (l1 l2 l3; 0 0 0)(l1 l2 l3; m1 m2 m3),
and h_{l1l2l3} = sqrt((2l1+1)(2l2+1)(2l3+1)/(4 pi)) (l1 l2 l3; 0 0 0) is the
geometric factor of Sec. III A.  The 3j symbol is evaluated with Racah's
single-sum formula in exact integer arithmetic.
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache


def _f(n: int) -> int:
    return math.factorial(n)


@lru_cache(maxsize=None)
def wigner3j(j1: int, j2: int, j3: int, m1: int, m2: int, m3: int) -> float:
    if m1 + m2 + m3 != 0:
        return 0.0
    if j3 < abs(j1 - j2) or j3 > j1 + j2:
        return 0.0
    if abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
        return 0.0
    # triangle coefficient (exact)
    tri = Fraction(_f(j1 + j2 - j3) * _f(j1 - j2 + j3) * _f(-j1 + j2 + j3), _f(j1 + j2 + j3 + 1))
    pref = tri * _f(j1 + m1) * _f(j1 - m1) * _f(j2 + m2) * _f(j2 - m2) * _f(j3 + m3) * _f(j3 - m3)
    kmin = max(0, j2 - j3 - m1, j1 - j3 + m2)
    kmax = min(j1 + j2 - j3, j1 - m1, j2 + m2)
    s = Fraction(0)
    for k in range(kmin, kmax + 1):
        den = (_f(k) * _f(j3 - j2 + k + m1) * _f(j3 - j1 + k - m2) * _f(j1 + j2 - j3 - k)
               * _f(j1 - k - m1) * _f(j2 - k + m2))
        s += Fraction((-1) ** k, den)
    sign = -1 if ((j1 - j2 - m3) % 2) else 1
    # value = sign * sqrt(pref) * s ; evaluate sqrt in float at the end
    return sign * math.sqrt(float(pref)) * float(s)


def gaunt(l1: int, l2: int, l3: int, m1: int, m2: int, m3: int) -> float:
    return (math.sqrt((2 * l1 + 1) * (2 * l2 + 1) * (2 * l3 + 1) / (4.0 * math.pi))
            * wigner3j(l1, l2, l3, 0, 0, 0) * wigner3j(l1, l2, l3, m1, m2, m3))


def h_geom(l1: int, l2: int, l3: int) -> float:
    return math.sqrt((2 * l1 + 1) * (2 * l2 + 1) * (2 * l3 + 1) / (4.0 * math.pi)) * wigner3j(l1, l2, l3, 0, 0, 0)
