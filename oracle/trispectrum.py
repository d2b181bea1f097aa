"""Modal trispectrum estimator, plain FP64 (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. IV (other polyspectra): the diagonal-free trispectrum estimator is built from
B = (a a a a - 6 C a a + 3 C C) / sqrt(C C C C) with the isotropic basis
G^{l1 l2 l3 l4}_{m1 m2 m3 m4} R_n / (v v v v), G the integral of four spherical
harmonics.  With v_l = 1 and separable modes R_n = q_p q_r q_s q_u (p <= r <= s <= u),
the sum over (l_i, m_i) with the quartic Gaunt factor is the sky integral of four
filtered maps, so on a grid exact for the product

    tau_prsu = sum_x w(x) [ M_p M_r M_s M_u
                            - sum over the 6 pairs {a,b} of V_ab M_c M_d
                            + sum over the 3 pairings {a,b}{c,d} of V_ab V_cd ],

V_ab(x) = <M_a M_b>(x) the Monte-Carlo pair means ("6 C a a" and "3 C C" are the
pairings of the four legs, as "3 C a" is for three).  Modes are ordered
lexicographically over p <= r <= s <= u.
"""
from __future__ import annotations

import itertools

import numpy as np


def quad_list(P: int):
    return [(p, r, s, u) for p in range(P) for r in range(p, P) for s in range(r, P) for u in range(s, P)]


def _pair_index(P: int):
    idx = {}
    k = 0
    for a in range(P):
        for b in range(a, P):
            idx[(a, b)] = k
            k += 1
    return idx


def tau(M: np.ndarray, w: np.ndarray, V: np.ndarray | None = None) -> np.ndarray:
    """tau_n for the maps M [P, ...], weights w, pair means V [npairs, ...] or None."""
    P = M.shape[0]
    Mf = M.reshape(P, -1)
    wf = np.asarray(w, dtype=np.float64).reshape(-1)
    pid = _pair_index(P)
    Vf = None if V is None else V.reshape(V.shape[0], -1)

    def v(a, b):
        return Vf[pid[(min(a, b), max(a, b))]]

    out = []
    for q in quad_list(P):
        t = Mf[q[0]] * Mf[q[1]] * Mf[q[2]] * Mf[q[3]]
        if Vf is not None:
            for i, j in itertools.combinations(range(4), 2):          # the 6 pairs
                k, l = [m for m in range(4) if m not in (i, j)]
                t = t - v(q[i], q[j]) * Mf[q[k]] * Mf[q[l]]
            for (i, j), (k, l) in (((0, 1), (2, 3)), ((0, 2), (1, 3)), ((0, 3), (1, 2))):   # the 3 pairings
                t = t + v(q[i], q[j]) * v(q[k], q[l])
        out.append(np.dot(wf, t))
    return np.array(out)
