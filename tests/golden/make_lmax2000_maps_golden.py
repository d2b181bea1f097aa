#!/usr/bin/env python3
"""Write the oracle's filtered maps of one full-spectrum sky at sampled pixels of the
l_max 2000 grid of the mixed-resolution batch (Gauss-Legendre 3008 x 6016 rings, P = 50
modes), for the GPU parity test of that context: its ring transform has length 6016 =
128 x 47, so its half-length complex transform runs the prime radix 47.

Calls only ``oracle`` (FP64 synthesis of the sampled rings: the log-scaled recurrence and
numpy's inverse FFT) and ``modal_inputs`` (seeded inputs).  Sky: isotropic Gaussian a_lm
with the WMAP-like filter spectrum f_sky (b_l^2 C_l + N_l), whitened by it.

Usage: python tests/golden/make_lmax2000_maps_golden.py
Writes tests/golden/maps_lmax2000_P50.npz (about 0.1 MB); takes a minute or two.
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

NAME = "mixed2000"
SKY_ID = 700
RINGS = (0, 1001, 1503, 3007)   # north pole ring, mid-latitude, equator band, south pole ring
NPX = 64                        # sampled pixels per ring


def main() -> str:
    cfg = mi.CONFIGS[NAME]
    lmax, nt, nphi, P = cfg.lmax, cfg.ntheta, cfg.nphi, cfg.P
    grid = og.Grid(nt, nphi)
    cl = mi.filter_cl(lmax, "wmap")
    q = mi.q_basis(P, lmax)
    alm = mi.gaussian_alm(cl, lmax, mi.rng_for(cfg.cfg_id, SKY_ID))
    rng = np.random.default_rng(2000)
    pix = np.sort(np.unique(np.concatenate([np.arange(0, nphi, nphi // (NPX // 2)),
                                            rng.integers(0, nphi, NPX)])))[:NPX]
    t0 = time.time()
    sub = og.RingSubset(grid, np.array(RINGS))
    M = om.filtered_maps(alm, cl, q, sub)              # [P][rings][nphi]
    out = os.path.join(HERE, "maps_lmax2000_P50.npz")
    np.savez_compressed(out, maps=M[:, :, pix], rings=np.array(RINGS), pixels=pix, lmax=lmax, ntheta=nt, nphi=nphi,
                        P=P, cfg_id=cfg.cfg_id, sky_id=SKY_ID)
    print(f"{NAME}: lmax={lmax} grid={nt}x{nphi} P={P}, {len(RINGS)} rings x {len(pix)} pixels: "
          f"{time.time() - t0:.0f} s -> {out}", flush=True)
    return out


if __name__ == "__main__":
    main()
