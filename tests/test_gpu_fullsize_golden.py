"""Element-by-element parity at the full resolution of the throughput workload (l_max 1000)
and of the precision study (l_max 1024), Gauss-Legendre 1536 x 3072 rings, P = 40 modes
(n_max = 11,480), and of the WMAP-size estimator workload (l_max 500, 768 x 1536 rings,
P = 30, n_max = 4,960), against the FP64 oracle.

The expected beta, linear term and beta^hat of two full-spectrum skies (WMAP-like filter
spectrum with a 13' beam and white noise, the |lat| < 10 deg cut in the pixel weights,
the linear term's pair means from four further skies) were written by
tests/golden/make_fullsize_golden.py, which calls only ``oracle`` (ring-chunked FP64
pixel sums), with the sums of the terms' magnitudes, sum_x w |M_p M_r M_s| and
sum_x w (|V_pr M_s| + |V_ps M_r| + |V_rs M_p|).  Every precision runs the kernels and launch
configuration of the benchmark.  Three errors per result are printed ([err] lines):
  * l2:     ||diff||_2 / ||ref||_2;
  * scaled: max_n |diff_n| / sum_x |terms_n| - the forward error of a sum of products,
            in the unit that rounding in the maps and the summation is relative to;
  * max/rms: max_n |diff_n| / rms(ref), which full-spectrum skies inflate: their per-pixel
            terms are about 10^4 times larger than rms(beta), so map rounding of 1e-12 (FP64)
            or 1e-6 (FP32) shows as 1e-8 or 1e-4 on the worst-conditioned modes.
The scaled error is bounded: 1e-10 in FP64 and 1e-5 in FP32 (the stated tolerances of the
hot path, relative to the size of the terms the sums add), loose bounds for the split
precisions, whose errors are reported, not pinned.  The l2 error carries the average
cancellation factor on top (sum |terms| / |beta| is about 400 at l_max 1000: 3e-13 scaled
shows as 1.2e-10 in l2 in FP64).
"""
import os

import numpy as np
import pytest

import modal_inputs as mi
from oracle import grid as og

from test_gpu_parity import log_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
# bounds on max_n |diff_n| / sum_x |terms_n|
TOL = {"f64": 1e-10, "f32": 1e-5, "f16x3": 1e-4, "bf16x3": 1e-3}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_mask = {}


def _golden(name):
    d = np.load(os.path.join(HERE, "golden", f"fullsize_{name}.npz"))
    return {k: d[k] for k in d.files}


def _errs(got, ref, scale):
    e_inf = max(float(np.max(np.abs(got[s] - ref[s])) / np.sqrt(np.mean(ref[s] ** 2))) for s in range(ref.shape[0]))
    e_2 = max(float(np.linalg.norm(got[s] - ref[s]) / np.linalg.norm(ref[s])) for s in range(ref.shape[0]))
    e_sc = float(np.max(np.abs(got - ref) / scale))
    return e_inf, e_2, e_sc


@pytest.mark.parametrize("name", ["metric1000", "precision1024", "wmap500"])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16x3", "bf16x3"])
def test_fullsize_golden(name, prec):
    from paper_1105_2791_amd import ModalContext
    g = _golden(name)
    lmax, nt, nphi, P, cfg_id = int(g["lmax"]), int(g["ntheta"]), int(g["nphi"]), int(g["P"]), int(g["cfg_id"])
    if nt not in _mask:
        g0 = og.Grid(nt, nphi)
        _mask[nt] = np.repeat(mi.mask_rings(g0.theta)[:, None], nphi, axis=1)
    cl = mi.filter_cl(lmax, "wmap")
    q = mi.q_basis(P, lmax)
    alms = np.array([mi.gaussian_alm(cl, lmax, mi.rng_for(cfg_id, int(i))) for i in g["sky_ids"]])
    mc = np.array([mi.gaussian_alm(cl, lmax, mi.rng_for(cfg_id, int(i))) for i in g["mc_ids"]])
    print(f"[case] fullsize golden {name} lmax={lmax} {prec}: create", flush=True)
    c = ModalContext(lmax, nt, nphi, P, prec, q, cl, mask=_mask[nt])
    print(f"[case] fullsize golden {name} {prec}: beta", flush=True)
    beta = c.beta(alms).cpu().numpy()
    print(f"[case] fullsize golden {name} {prec}: linear state", flush=True)
    st = c.linear_state()
    c.linear_reset(st)
    c.linear_accumulate(st, mc)
    c.linear_finalize(st)
    lin = c.linear_apply(st, alms).cpu().numpy()
    bh = c.beta(alms, state=st).cpu().numpy()
    del st
    c.close()
    torch.cuda.empty_cache()
    worst = 0.0
    scales = {"beta": g["beta_abs"], "lin": g["lin_abs"], "beta_hat": g["beta_abs"] + g["lin_abs"]}
    for what, got, ref in (("beta", beta, g["beta"]), ("lin", lin, g["lin"]), ("beta_hat", bh, g["beta_hat"])):
        e_inf, e_2, e_sc = _errs(got, ref, scales[what])
        log_err(f"fullsize golden {name} {what} {prec} max/rms", e_inf)
        log_err(f"fullsize golden {name} {what} {prec} l2", e_2)
        log_err(f"fullsize golden {name} {what} {prec} scaled", e_sc)
        assert np.all(np.isfinite(got))
        worst = max(worst, e_sc)
    assert worst < TOL[prec], worst


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_lmax2000_maps_sampled_pixels(prec):
    """The l_max 2000 context of the mixed-resolution batch (3008 x 6016 rings, P = 50): its
    ring transform has length 6016 = 128 x 47, so the prime radix 47 runs at full size.
    Maps of one full-spectrum sky against the oracle's synthesis at 4 rings x 64 pixels
    (tests/golden/make_lmax2000_maps_golden.py), max |diff| / rms per mode."""
    from paper_1105_2791_amd import ModalContext
    from test_gpu_parity import MAP_TOL
    d = np.load(os.path.join(HERE, "golden", "maps_lmax2000_P50.npz"))
    lmax, nt, nphi, P = int(d["lmax"]), int(d["ntheta"]), int(d["nphi"]), int(d["P"])
    cl = mi.filter_cl(lmax, "wmap")
    alm = mi.gaussian_alm(cl, lmax, mi.rng_for(int(d["cfg_id"]), int(d["sky_id"])))
    print(f"[case] lmax2000 maps {prec}: create", flush=True)
    c = ModalContext(lmax, nt, nphi, P, prec, mi.q_basis(P, lmax), cl)
    print(f"[case] lmax2000 maps {prec}: synthesis", flush=True)
    maps = c.filter_maps(alm[None])[0]                       # [P][nt][nphi]
    rings = torch.as_tensor(d["rings"], device=maps.device)
    pix = torch.as_tensor(d["pixels"], device=maps.device)
    got = maps[:, rings][:, :, pix].double().cpu().numpy()
    del maps
    c.close()
    torch.cuda.empty_cache()
    ref = d["maps"]
    err = max(float(np.max(np.abs(got[p] - ref[p])) / np.sqrt(np.mean(ref[p] ** 2))) for p in range(P))
    log_err(f"lmax2000 maps sampled {prec}", err)
    assert np.all(np.isfinite(got)) and err < MAP_TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_lmax2000_vjp_directional(prec):
    """The adjoint at l_max 2000 (its real-to-complex ring transform of length 6016 = 128 x 47
    at full size, P = 50).  The cubic beta(a) is a homogeneous cubic form, so for any
    direction d the polarisation identity
        D beta(a) . d = [beta(a + d) - beta(a - d) - 2 beta(d)] / 2 = B1
    holds exactly; with the cotangent cot = B1 the gradient's inner product
    sum_lm Re(conj(g_lm) d_lm) (g = d/dRe a + i d/dIm a) must equal |B1|^2.  A wrong
    transform gives an error of order one; rounding gives the relative error logged
    (measured 4e-8 in FP32, 4e-6 in bf16x3; bounds 1e-6 and 1e-4).  Full-spectrum skies
    (WMAP-like filter, P = 50), no oracle call."""
    from paper_1105_2791_amd import ModalContext
    lmax, nt, nphi, P = 2000, 3008, 6016, 50
    cl = mi.filter_cl(lmax, "wmap")
    a = mi.gaussian_alm(cl, lmax, mi.rng_for(20, 0))
    d = mi.gaussian_alm(cl, lmax, mi.rng_for(20, 1))
    print(f"[case] lmax2000 vjp directional {prec}: create", flush=True)
    c = ModalContext(lmax, nt, nphi, P, prec, mi.q_basis(P, lmax), cl)
    print(f"[case] lmax2000 vjp directional {prec}: forward", flush=True)
    b = c.beta(np.stack([a + d, a - d, d])).cpu().numpy()
    B1 = (b[0] - b[1] - 2.0 * b[2]) / 2.0
    print(f"[case] lmax2000 vjp directional {prec}: vjp", flush=True)
    g = c.beta_vjp(a[None], B1[None]).cpu().numpy()[0]
    c.close()
    torch.cuda.empty_cache()
    lhs = float(np.sum(g.real * d.real + g.imag * d.imag))
    rhs = float(B1 @ B1)
    err = abs(lhs - rhs) / rhs
    log_err(f"lmax2000 vjp directional {prec}", err)
    assert np.all(np.isfinite(g)) and err < {"f32": 1e-6, "bf16x3": 1e-4}[prec], (lhs, rhs)
