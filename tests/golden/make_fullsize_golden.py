#!/usr/bin/env python3
"""Write the oracle's beta, linear term and beta^hat for full-spectrum skies at the
workload shapes: l_max 1000 and l_max 1024 on the Gauss-Legendre 1536 x 3072 grid with
P = 40 modes (n_max = 11,480), and l_max 500 on 768 x 1536 with P = 30 (n_max = 4,960),
for the GPU parity test at those shapes.

Calls only ``oracle`` (FP64, ring-chunked pixel sums) and ``modal_inputs`` (seeded
inputs).  The sky recipe is the benchmark's: isotropic Gaussian a_lm drawn with the
WMAP-like filter spectrum f_sky (b_l^2 C_l + N_l) (13 arcmin beam, white noise equal
to the signal at l = 400), whitened by that spectrum, the |lat| < 10 deg cut in the
pixel weights, and the linear term's pair means from four further Monte-Carlo skies
of the same recipe.  It also writes the sums of the terms' magnitudes (the scale of
rounding errors in a sum, for the condition-scaled error of the test).

Usage: python tests/golden/make_fullsize_golden.py [metric1000|precision1024|wmap500 ...]
Writes tests/golden/fullsize_<name>.npz (0.2-0.9 MB each); takes minutes per shape.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import modal_inputs as mi  # noqa: E402
from oracle import grid as og  # noqa: E402
from oracle import modal as om  # noqa: E402

# test skies and Monte-Carlo skies (sim ids under each shape's cfg_id)
SKY_IDS = (500, 501)
MC_IDS = (600, 601, 602, 603)
RINGS_PER_CHUNK = 96


def golden_path(name: str) -> str:
    return os.path.join(HERE, f"fullsize_{name}.npz")


def make(name: str) -> str:
    cfg = mi.CONFIGS[name]
    lmax, nt, nphi, P = cfg.lmax, cfg.ntheta, cfg.nphi, cfg.P
    g0 = og.Grid(nt, nphi)
    grid = og.Grid(nt, nphi, ring_mask=np.repeat(mi.mask_rings(g0.theta)[:, None], nphi, axis=1))
    cl = mi.filter_cl(lmax, "wmap")
    q = mi.q_basis(P, lmax)
    alms = np.array([mi.gaussian_alm(cl, lmax, mi.rng_for(cfg.cfg_id, i)) for i in SKY_IDS])
    mc = np.array([mi.gaussian_alm(cl, lmax, mi.rng_for(cfg.cfg_id, i)) for i in MC_IDS])
    t0 = time.time()
    beta, lin, beta_abs, lin_abs = om.beta_and_linear_by_rings(alms, mc, cl, q, grid, RINGS_PER_CHUNK, with_abs=True)
    out = golden_path(name)
    np.savez_compressed(out, beta=beta, lin=lin, beta_hat=beta - lin, beta_abs=beta_abs, lin_abs=lin_abs,
                        lmax=lmax, ntheta=nt, nphi=nphi, P=P,
                        cfg_id=cfg.cfg_id, sky_ids=np.array(SKY_IDS), mc_ids=np.array(MC_IDS))
    print(f"{name}: lmax={lmax} grid={nt}x{nphi} P={P}: {time.time() - t0:.0f} s -> {out}", flush=True)
    return out


if __name__ == "__main__":
    for n in (sys.argv[1:] or ["metric1000", "precision1024", "wmap500"]):
        make(n)
