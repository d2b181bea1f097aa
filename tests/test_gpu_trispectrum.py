"""GPU parity of the modal trispectrum (Sec. IV) against the FP64 oracle.

Errors are max |diff| over the rms of the unsubtracted quartic sums (the size of
the terms).  FP64 contexts: 1e-10.  Float contexts run the split-bf16 matrix-core
update: the maps carry their synthesis error (MAP_TOL of the bispectrum tests,
3e-5 for bf16x3) on each of four legs, the operands 2^-17 each; bound 5e-4 for
bf16x3 and 2e-4 for the split-fp16 maps.  FP32 contexts have no trispectrum update
and must say so (EUNSUPPORTED).  At l_max 1000 the oracle's maps
are out of reach: there sampled modes are checked against FP64 sums of the
library's own maps and pair means (which the map and linear-term tests check).
"""
import math

import numpy as np
import pytest

import modal_inputs as mi
from oracle import modal as om
from oracle import trispectrum as otr

from helpers import CASES

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {"f64": 1e-10, "bf16x3": 5e-4, "f16x3": 2e-4}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_ctx = {}
_or = {}


def ctx_case(case, prec):
    from paper_1105_2791_amd import ModalContext
    key = (case.name, prec)
    if key not in _ctx:
        print(f"[case] create {case.name} {prec}", flush=True)
        _ctx[key] = ModalContext(case.lmax, case.ntheta, case.nphi, case.P, prec, case.q, case.cl, mask=case.mask())
    return _ctx[key]


def oracle_case(case, S=3):
    if case.name not in _or:
        alms = case.alms(0, S)
        mc = case.alms(500, 4)
        M = case.maps(alms)
        V = om.pair_means(case.maps(mc))
        g = case.grid
        t0 = np.array([otr.tau(M[i], g.w) for i in range(S)])
        t1 = np.array([otr.tau(M[i], g.w, V) for i in range(S)])
        _or[case.name] = dict(alms=alms, mc=mc, t0=t0, t1=t1)
    return _or[case.name]


@pytest.mark.parametrize("name,prec", [("tiny", "f64"), ("tiny", "bf16x3"), ("tiny", "f16x3"), ("ragged", "f64"),
                                       ("ragged", "bf16x3"), ("ragged", "f16x3"), ("odd", "bf16x3"),
                                       ("odd", "f16x3")])
def test_trispectrum_matches_oracle(name, prec):
    case = CASES[name]
    c = ctx_case(case, prec)
    o = oracle_case(case)
    print(f"[case] trispectrum {name} {prec}", flush=True)
    scale = np.sqrt(np.mean(o["t0"] ** 2))
    got0 = c.trispectrum(o["alms"]).cpu().numpy()
    e0 = np.max(np.abs(got0 - o["t0"])) / scale
    st = c.linear_state()
    c.linear_reset(st)
    c.linear_accumulate(st, o["mc"][:3])
    c.linear_accumulate(st, o["mc"][3:])
    c.linear_finalize(st)
    got1 = c.trispectrum(o["alms"], st).cpu().numpy()
    e1 = np.max(np.abs(got1 - o["t1"])) / scale
    print(f"[err] trispectrum {name} {prec}: no state {e0:.3e}, with state {e1:.3e}", flush=True)
    assert e0 < TOL[prec] and e1 < TOL[prec]


def test_trispectrum_f32_is_unsupported():
    """An FP32 context must not silently run a split-precision update."""
    from paper_1105_2791_amd import _lib as L
    case = CASES["tiny"]
    c = ctx_case(case, "f32")
    with pytest.raises(L.ModalError) as e:
        c.trispectrum(case.alms(0, 1))
    assert e.value.status == L.EUNSUPPORTED and "FP32" in str(e.value)


def test_trispectrum_metric_size_sampled():
    """l_max 1000, GL 1536 x 3072, P 40 (123,410 modes), bf16x3, 2 skies with a 4-sky
    Monte-Carlo state: 24 sampled modes against FP64 sums of the library's maps and V."""
    from paper_1105_2791_amd import ModalContext
    lmax, P, S = 1000, 40, 2
    cl = mi.filter_cl(lmax, "wmap")
    q = mi.q_basis(P, lmax)
    c = ModalContext(lmax, 1536, 3072, P, "bf16x3", q, cl)
    alms = np.stack([mi.gaussian_alm(cl, lmax, mi.rng_for(94, i)) for i in range(S)])
    mc = np.stack([mi.gaussian_alm(cl, lmax, mi.rng_for(94, 100 + i)) for i in range(4)])
    st = c.linear_state()
    c.linear_reset(st)
    c.linear_accumulate(st, mc)
    c.linear_finalize(st)
    print("[trispectrum] metric size", flush=True)
    tau = c.trispectrum(alms, st).cpu().numpy()
    maps = c.filter_maps(alms)
    V = c.pair_means(st)
    x, w = c.grid()
    wpix = np.repeat(w * 2.0 * math.pi / c.nphi, c.nphi)
    quads = otr.quad_list(P)
    pidx = {pr: k for k, pr in enumerate(mi.pair_list(P))}
    rng = np.random.default_rng(95)
    picks = [0, len(quads) - 1] + list(rng.integers(0, len(quads), 22))
    worst = 0.0
    for s in range(S):
        Ms = {}
        for n in picks:
            qd = quads[n]
            for p in qd:
                if p not in Ms:
                    Ms[p] = maps[s, p].reshape(-1).double().cpu().numpy()
            Vp = {}
            for i in range(4):
                for j in range(i + 1, 4):
                    a, b = sorted((qd[i], qd[j]))
                    Vp[(i, j)] = V[pidx[(a, b)]].reshape(-1).double().cpu().numpy()
            m = [Ms[p] for p in qd]
            t = m[0] * m[1] * m[2] * m[3]
            for (i, j) in Vp:
                k, l = [u for u in range(4) if u not in (i, j)]
                t = t - Vp[(i, j)] * m[k] * m[l]
            t = t + Vp[(0, 1)] * Vp[(2, 3)] + Vp[(0, 2)] * Vp[(1, 3)] + Vp[(0, 3)] * Vp[(1, 2)]
            ref = np.dot(wpix, t)
            size = np.dot(wpix, np.abs(m[0] * m[1] * m[2] * m[3]))
            worst = max(worst, abs(tau[s, n] - ref) / size)
    print(f"[err] trispectrum metric: worst |diff| / sum|w M M M M| = {worst:.3e}", flush=True)
    assert worst < 1e-4
