#!/usr/bin/env python3
"""Throughput of the modal bispectrum hot path on one MI355X.

One step = filtered maps (Legendre synthesis + ring FFT) and beta^hat = beta - lin
(cubic pair x mode reduction with the Monte-Carlo linear term fused in, FP64
split-K reduction and symmetrisation) for one batch of S synthetic skies at the
metric shape: l_max = 1000, Gauss-Legendre 1536 x 3072 rings, P = 40 separable
modes (n_max = 11480), beam/noise spectrum and a |lat| < 10 deg cut.  The
linear-term state (Monte-Carlo <M_p M_r> planes) is built before timing.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sim maps/sec (filter+β_n) @lmax=1000,P=40: split-bf16 vs plain FP32; % MFMA peak"

PEAK = {  # MI355X published dense peaks
    "bf16": 2.5e15, "f16": 2.5e15, "f32_mfma": 157.3e12, "f64_vec": 78.6e12, "hbm": 8.0e12,
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(lmax, P, S, first, cfg_id=6):
    import numpy as np
    import modal_inputs as mi
    cl = mi.filter_cl(lmax, "wmap")
    alms = np.stack([mi.gaussian_alm(cl, lmax, mi.rng_for(cfg_id, first + i)) for i in range(S)])
    return alms


def cpu_baseline(lmax, ntheta, nphi, P, rings, V_sims=2, cfg_id=6):
    """FP64 oracle timed on host cores for one sky on a subset of rings (maps, beta, linear term)."""
    import numpy as np
    import modal_inputs as mi
    from oracle import grid as og
    from oracle import modal as om
    g_full = og.Grid(ntheta, nphi)
    idx = np.linspace(0, ntheta - 1, rings).round().astype(int)
    mask = mi.mask_rings(g_full.theta[idx])

    class Sub:  # the sampled rings as a grid
        pass
    sub = Sub()
    sub.x = g_full.x[idx]
    sub.nphi = nphi
    sub.ntheta = rings
    sub.w = (g_full.wgl[idx] * 2 * math.pi / nphi * mask)[:, None] * np.ones((1, nphi))
    cl = mi.filter_cl(lmax, "wmap")
    q = mi.q_basis(P, lmax)
    mc = make_inputs(lmax, P, V_sims, 10_000, cfg_id)
    V = om.pair_means(om.filtered_maps(mc, cl, q, sub))
    a = make_inputs(lmax, P, 1, 20_000, cfg_id)[0]
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()
    t0 = time.perf_counter()
    M = om.filtered_maps(a, cl, q, sub)
    bh = om.beta_hat(M, sub.w, V)
    t = time.perf_counter() - t0
    assert np.all(np.isfinite(bh))
    frac = rings / ntheta
    return {"value": frac / t, "unit": "maps/s", "cores": int(threads), "kind": "oracle",
            "sample": f"one sky, {rings} of {ntheta} rings (every ~{ntheta // rings}th), maps+beta+linear term, "
                      f"{t:.1f} s, scaled by {ntheta}/{rings}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=8, help="skies per step (S)")
    ap.add_argument("--prec", default="auto", choices=["auto", "bf16x3", "f32", "f64"])
    ap.add_argument("--lmax", type=int, default=1000)
    ap.add_argument("--ntheta", type=int, default=1536)
    ap.add_argument("--nphi", type=int, default=3072)
    ap.add_argument("--P", type=int, default=40)
    ap.add_argument("--mc", type=int, default=16, help="Monte-Carlo skies for the linear term")
    ap.add_argument("--cpu-rings", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        log("bench.py: only --gpus 1 is supported (single-GPU build)")
        sys.exit(2)

    import numpy as np
    import torch
    import modal_inputs as mi
    from paper_1105_2791_amd import ModalContext
    from paper_1105_2791_amd import _lib as L

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    lmax, nt, nphi, P, S = args.lmax, args.ntheta, args.nphi, args.P, args.batch
    prec = args.prec
    if prec == "auto":
        prec = "bf16x3"
    cl = mi.filter_cl(lmax, "wmap")
    q = mi.q_basis(P, lmax)
    # the context's own quadrature gives the ring colatitudes for the mask
    probe = ModalContext(lmax, nt, nphi, 1, "f32", q[:1], cl, device=0)
    x, _ = probe.grid()
    probe.close()
    mask = np.repeat(mi.mask_rings(np.arccos(x))[:, None], nphi, axis=1)
    try:
        ctx = ModalContext(lmax, nt, nphi, P, prec, q, cl, mask=mask, device=0)
    except L.ModalError as e:
        if prec != "bf16x3" or e.status != L.EUNSUPPORTED:
            raise
        log("bf16x3 unavailable, falling back to f32")
        prec = "f32"
        ctx = ModalContext(lmax, nt, nphi, P, prec, q, cl, mask=mask, device=0)
    log(f"bench: lmax={lmax} grid={nt}x{nphi} P={P} nmax={ctx.nmax} S={S} prec={prec}")

    # linear-term state from Monte-Carlo skies (not timed)
    state = ctx.linear_state()
    ctx.linear_reset(state)
    for b0 in range(0, args.mc, S):
        ctx.linear_accumulate(state, make_inputs(lmax, P, min(S, args.mc - b0), 1000 + b0))
    ctx.linear_finalize(state)
    alm = ctx._alm(make_inputs(lmax, P, S, 0))
    out = torch.empty((S, ctx.nmax), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    log("bench: state ready")

    tuned = None
    if not args.no_autotune:
        tuned = ctx.autotune(alm, state)
        log(f"bench: autotuned {tuned}")
    for _ in range(args.warmup):
        ctx.beta(alm, state=state, out=out)
    torch.cuda.synchronize()
    ctx.profile_read(reset=True)
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ctx.beta(alm, state=state, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile(False)
    stages = ctx.profile_read(reset=True)
    elapsed = t1 - t0
    assert torch.isfinite(out).all().item()
    value = S * args.steps / elapsed
    ms_step = 1e3 * elapsed / args.steps
    log(f"bench: {value:.2f} maps/s, {ms_step:.2f} ms/step; stages: " +
        ", ".join(f"{k}={v[0] / max(1, v[1]):.3f}ms x{v[1]}" for k, v in stages.items() if v[1]))

    # roofline of the dominant kernel (the cubic contraction), timed on the library's stream
    cub_ms, cub_n = stages["cubic"]
    cub_avg = cub_ms / max(1, cub_n)
    npix = nt * nphi
    flops = 2.0 * ctx.npairs * P * npix * S          # pair x mode contraction, one pass
    if prec == "bf16x3":
        bound, peak, unit = "mfma", PEAK["bf16"], "TFLOP/s"
    elif prec == "f32":
        bound, peak, unit = "mfma", PEAK["f32_mfma"], "TFLOP/s"
    else:
        bound, peak, unit = "alu", PEAK["f64_vec"], "TFLOP/s"
    kinfo = ctx.cubic_path()
    if kinfo["path"] == "valu":   # FP64-accumulating vector-ALU contraction
        bound, peak = "alu", PEAK["f64_vec"]
    achieved = flops / (cub_avg * 1e-3)
    roof = {"bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": unit,
            "frac": achieved / peak, "traffic": None, "kernel": "cubic pair x mode contraction",
            "avg_ms": cub_avg, "flop_per_launch": flops}
    if prec == "bf16x3":
        roof["mfma_issued_frac"] = 3.0 * achieved * kinfo.get("pad", 1.0) / peak

    cpu = None
    if not args.no_cpu_baseline:
        try:
            cpu = cpu_baseline(lmax, nt, nphi, P, args.cpu_rings)
        except Exception as e:  # the baseline is reported, never the target
            log(f"cpu baseline failed: {e!r}")

    line = {
        "metric": METRIC, "value": value, "unit": "maps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"bf16x3": "bf16", "f32": "f32", "f64": "f64"}[prec],
        "precision": {"bf16x3": "split bf16 hi+lo (3 MFMA products), fp32 accumulate, fp64 reduce",
                      "f32": "fp32 maps and products, fp64 accumulate",
                      "f64": "fp64"}[prec],
        "data": "synthetic",
        "config": {"workload": f"metric1000: lmax={lmax} GL {nt}x{nphi} P={P} nmax={ctx.nmax}, "
                               f"beam+noise spectrum, |lat|<10deg cut, MC linear term ({args.mc} skies)",
                   "batch": S, "prec": prec, "tuned": tuned},
        "stages_ms": {k: v[0] / max(1, v[1]) for k, v in stages.items() if v[1]},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
