#!/usr/bin/env python3
"""Throughput of the modal bispectrum hot path on one MI355X.

One step = filtered maps (Legendre synthesis + ring FFT) and beta^hat = beta - lin
(cubic pair x mode contraction, the Monte-Carlo linear term from the harmonic
transforms of the pair means, FP64 split-K reduction and symmetrisation) for one batch of S synthetic
skies at l_max = 1000, Gauss-Legendre 1536 x 3072 rings, P = 40 separable modes
(n_max = 11480), beam/noise spectrum and a |lat| < 10 deg cut.  The linear-term
state (Monte-Carlo <M_p M_r> planes) is built before timing.  The headline path
(split bf16 by default) is followed by a shorter run of the plain-FP32 path on the
same GPU.

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


def _host_info():
    """nproc (CPUs this process may run on) and the CPU model of the host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"nproc": nproc, "cpu_model": model}


def _host_threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([d.get("num_threads", 1) for d in threadpool_info()] + [1]))
    except Exception:
        return os.cpu_count()


def _ring_sample(lmax, ntheta, nphi, P, rings, V_sims, cfg_id):
    """The oracle's inputs on a subset of rings of the workload grid: the sampled rings as
    a grid, one sky's a_lm, the Monte-Carlo pair means on those rings."""
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
    return sub, cl, q, V, a


def cpu_baseline(lmax, ntheta, nphi, P, rings, V_sims=2, cfg_id=6, op="beta", one_thread_rings=0):
    """FP64 oracle timed on host cores for one sky on a subset of rings: maps, then beta
    and the linear term (op "beta"), the pair sums (op "power") or the quartic sums
    (op "trispectrum")."""
    import numpy as np
    from oracle import modal as om
    from oracle import power as opw
    from oracle import trispectrum as otr
    sub, cl, q, V, a = _ring_sample(lmax, ntheta, nphi, P, rings, V_sims, cfg_id)
    reduce_, what = {"beta": (om.beta_hat, "beta+linear term"), "power": (opw.power_beta, "pair sums"),
                     "trispectrum": (otr.tau, "quartic sums")}[op]
    t0 = time.perf_counter()
    M = om.filtered_maps(a, cl, q, sub)
    out = reduce_(M, sub.w, V)
    t = time.perf_counter() - t0
    assert np.all(np.isfinite(out))
    frac = rings / ntheta
    res = {"value": frac / t, "unit": "maps/s", "cores": _host_threads(), "kind": "oracle",
           "sample": f"one sky, {rings} of {ntheta} rings (every ~{ntheta // rings}th), maps+{what}, "
                     f"{t:.1f} s, scaled by {ntheta}/{rings}", "host": _host_info()}
    if one_thread_rings:
        # the same oracle on one thread (BLAS limited to one), on fewer rings
        from threadpoolctl import threadpool_limits
        sub1, cl1, q1, V1, a1 = _ring_sample(lmax, ntheta, nphi, P, one_thread_rings, V_sims, cfg_id)
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            out1 = reduce_(om.filtered_maps(a1, cl1, q1, sub1), sub1.w, V1)
            t1 = time.perf_counter() - t0
        assert np.all(np.isfinite(out1))
        res["one_thread"] = {"value": one_thread_rings / ntheta / t1, "unit": "maps/s", "cores": 1,
                             "sample": f"one sky, {one_thread_rings} of {ntheta} rings, {t1:.1f} s, "
                                       f"scaled by {ntheta}/{one_thread_rings}"}
    return res


def _baseline(args, f):
    """A workload's oracle baseline, or None when switched off or when it fails (it is
    reported, never the target)."""
    if args.no_cpu_baseline:
        return None
    try:
        return f()
    except Exception as e:
        log(f"cpu baseline failed: {e!r}")
        return None


def cpu_baseline_lowrank(B, k):
    """The oracle's noise vectors (sample covariance, its eigendecomposition) for the same
    N x n_max rows, timed whole on host cores."""
    from oracle import lowrank as olr
    t0 = time.perf_counter()
    olr.noise_vectors(B, k)
    t = time.perf_counter() - t0
    return {"value": 1e3 * t, "unit": "ms", "cores": _host_threads(), "kind": "oracle",
            "sample": f"the whole call: {B.shape[0]} x {B.shape[1]} rows, k = {k}, {t:.1f} s"}


def cpu_baseline_shapes(lmax, P, P_sample=16):
    """The oracle's full-sky ideal covariance (mu integral, one entry at a time) for the
    first P_sample modes of the basis at the same l_max, scaled by the entry count of n_max(P)."""
    import numpy as np
    import modal_inputs as mi
    from oracle import closed_forms as cf
    cl = mi.filter_cl(lmax, "wmap")
    q = mi.q_basis(P_sample, lmax)
    c = (cl > 0).astype(float)
    t0 = time.perf_counter()
    Z = cf.zeta_ideal(q, c)
    t = time.perf_counter() - t0
    assert np.all(np.isfinite(Z))
    n_s = Z.shape[0]
    n = P * (P + 1) * (P + 2) // 6
    scale = (n * (n + 1) / 2) / (n_s * (n_s + 1) / 2)
    return {"value": 1e3 * t * scale, "unit": "ms", "cores": _host_threads(), "kind": "oracle",
            "sample": f"ideal covariance of the first {P_sample} modes ({n_s} x {n_s}, l_max {lmax}), {t:.1f} s, "
                      f"scaled by the entry count {n} x {n} / {n_s} x {n_s}"}


def kernel_rooflines(ctx, stages, prec, S, op="beta"):
    """Algorithmic work per launch of each timed stage and its rate against the MI355X peak."""
    lmax, nt, nphi, P = ctx.lmax, ctx.ntheta, ctx.nphi, ctx.P
    npix = nt * nphi
    split = prec in ("bf16x3", "f16x3")
    mfma_peak = PEAK["bf16"] if split else (PEAK["f32_mfma"] if prec == "f32" else PEAK["f64_vec"])
    mfma_bound = "mfma" if prec != "f64" else "alu"
    cubic_bound = mfma_bound if ctx.cubic_path()["path"] != "valu" else "alu"
    real = 8 if prec == "f64" else 4
    # name: (work per launch, unit of work, bound, peak, issued MFMA flops per launch)
    issued_cubic = 2.0 * ctx.cubic_path()["issued_macs_per_pixel"] * npix * S
    work = {
        # F[m][ring] = sum_l lambda_lm(ring) a_lm: one complex x real MAC per (l, m, ring, column)
        "legendre": (2.0 * ctx.nalm * nt * P * S, "flop", mfma_bound, mfma_peak,
                     (4 if prec == "bf16x3" else 3) * 2.0 * ctx.nalm * nt * P * S if split else None),
        # read F (complex, m <= lmax per ring) and write the real rings
        "fft": ((lmax + 1) * nt * P * S * 2 * real + npix * P * S * real, "byte", "hbm", PEAK["hbm"], None),
        # beta_prs = sum_x (M_p M_r)(x) w(x) M_s(x): one MAC per (triple p <= r <= s, pixel)
        "cubic": (2.0 * ctx.nmax * npix * S, "flop", cubic_bound,
                  mfma_peak if cubic_bound == "mfma" else PEAK["f64_vec"], issued_cubic),
        # linear term from the harmonic pair means: one pass over Z[npairs][nalm]
        "linear": (ctx.npairs * ctx.nalm * 2 * real, "byte", "hbm", PEAK["hbm"], None),
    }
    if op == "power":
        # sum_x w M_p M_r: one read of the maps and of the weights per sky
        work["cubic"] = ((P * npix + npix) * S * real, "byte", "hbm", PEAK["hbm"], None)
    if op == "trispectrum":
        # symmetric rank-npix update over the pairs: one MAC per (pair <= pair', pixel), per sky
        # and once more for the pair means; issued: 128 x 128 tiles, three split products
        R = ctx.npairs
        nt = (R + 127) // 128
        work["cubic"] = (2.0 * R * (R + 1) / 2 * npix * (S + 1), "flop", "mfma", PEAK["bf16"],
                         2.0 * 3 * nt * (nt + 1) / 2 * 128 * 128 * npix * (S + 1))
    out = {}
    for name, (units, kind, bound, peak, issue) in work.items():
        ms, n = stages.get(name, (0.0, 0))
        if not n:
            continue
        avg = ms / n
        rate = units / (avg * 1e-3)
        r = {"bound": bound, "achieved": rate / (1e12 if kind == "flop" else 1e9),
             "peak": peak / (1e12 if kind == "flop" else 1e9), "unit": "TFLOP/s" if kind == "flop" else "GB/s",
             "frac": rate / peak, "traffic": None, "avg_ms": avg, "per_launch": units, "per_launch_unit": kind}
        if issue and bound == "mfma":
            r["issued_flop_per_launch"] = issue
            r["mfma_issued_frac"] = issue / (avg * 1e-3) / peak
        out[name] = r
    return out


def run_path(args, prec, steps, warmup, make_state=True, op="beta", lambda_table=None, autotune=None):
    """Build a context at the workload shape, time `steps` beta batches (or, op="power",
    power-spectrum batches), return the figures.  lambda_table=False: the synthesis runs its
    recurrence on the fly (no precomputed lambda table)."""
    import numpy as np
    import torch
    import modal_inputs as mi
    from paper_1105_2791_amd import ModalContext

    dev = torch.device("cuda", 0)
    lmax, nt, nphi, P, S = args.lmax, args.ntheta, args.nphi, args.P, args.batch
    cl = mi.filter_cl(lmax, "wmap")
    q = mi.q_basis(P, lmax)
    # the context's own quadrature gives the ring colatitudes for the mask
    probe = ModalContext(lmax, nt, nphi, 1, "f32", q[:1], cl, device=0)
    x, _ = probe.grid()
    probe.close()
    mask = np.repeat(mi.mask_rings(np.arccos(x))[:, None], nphi, axis=1)
    ctx = ModalContext(lmax, nt, nphi, P, prec, q, cl, mask=mask, device=0, lambda_table=lambda_table)
    log(f"bench: lmax={lmax} grid={nt}x{nphi} P={P} nmax={ctx.nmax} S={S} prec={prec}")

    # linear-term state from Monte-Carlo skies (not timed)
    state = None
    if make_state:
        state = ctx.linear_state()
        ctx.linear_reset(state)
        for b0 in range(0, args.mc, S):
            ctx.linear_accumulate(state, make_inputs(lmax, P, min(S, args.mc - b0), 1000 + b0))
        ctx.linear_finalize(state)
    alm = ctx._alm(make_inputs(lmax, P, S, 0))
    ncol = {"beta": ctx.nmax, "power": ctx.npairs, "trispectrum": ctx.nquad}[op]
    out = torch.empty((S, ncol), dtype=torch.float64, device=dev)
    call = {"beta": lambda: ctx.beta(alm, state=state, out=out),
            "power": lambda: ctx.power_beta(alm, state=state, out=out),
            "trispectrum": lambda: ctx.trispectrum(alm, state=state, out=out)}[op]
    torch.cuda.synchronize()
    log(f"bench[{prec}]: state ready")

    tuned = None
    if (args.autotune if autotune is None else autotune):
        tuned = ctx.autotune(alm, state)
        log(f"bench[{prec}]: autotuned {tuned}")
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    ctx.profile_read(reset=True)
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile(False)
    stages = ctx.profile_read(reset=True)
    assert torch.isfinite(out).all().item()
    elapsed = t1 - t0
    res = {"prec": prec, "value": S * steps / elapsed, "ms_per_step": 1e3 * elapsed / steps, "tuned": tuned,
           "lambda_table": ctx.lambda_table,
           "stages_ms": {k: v[0] / max(1, v[1]) for k, v in stages.items() if v[1]},
           "kernels": kernel_rooflines(ctx, stages, prec, S, op), "nmax": ctx.nmax, "npairs": ctx.npairs,
           "ncol": ncol}
    log(f"bench[{prec}]: {res['value']:.2f} maps/s, {res['ms_per_step']:.2f} ms/step; stages: " +
        ", ".join(f"{k}={v:.3f}ms" for k, v in res["stages_ms"].items()))
    del state, alm, out
    ctx.close()
    torch.cuda.empty_cache()
    return res


KERNEL_SOURCES = {   # dominant-kernel name -> the source file its counters belong to
    "cubic": "paper_1105_2791_amd/csrc/k_cubic_split.hip",
    "legendre": "paper_1105_2791_amd/csrc/k_legendre_split.hip",
    "fft": "paper_1105_2791_amd/csrc/k_fft.hip",
    "linear": "paper_1105_2791_amd/csrc/k_lin_harm.hip",
    "pair_sums": "paper_1105_2791_amd/csrc/k_power.hip",       # power spectrum: pair sums + reduce
    "quad": "paper_1105_2791_amd/csrc/k_trispectrum.hip",      # trispectrum: copies, update, reduce
}


def measured_traffic(kernel, prec):
    """HBM bytes per launch from the committed counter record of this kernel, or None
    when there is none or the kernel source changed since the counters were taken."""
    import hashlib
    rec_path = os.path.join(ROOT, "profiles", f"{kernel}_{prec}_traffic.json")
    src = KERNEL_SOURCES.get(kernel)
    if not src or not os.path.exists(rec_path):
        return None
    with open(rec_path) as f:
        rec = json.load(f)
    with open(os.path.join(ROOT, src), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if rec.get("source_sha256") != sha:
        return None
    return rec.get("traffic_bytes_per_launch")


def copy_calibration():
    """A plain device-to-device copy of 2 GiB, three times (the counter reference)."""
    import torch
    n = 2 << 30
    a = torch.empty(n // 4, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 3
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 3,
                      "GB_per_s_read_plus_write": 2 * n / dt / 1e9}), flush=True)


def run_lowrank(args):
    """Low-rank covariance (Sec. III B) at n_max(P): noise vectors from N beta^hat vectors,
    the estimator for S skies, and the closed-form Cholesky rotation of S + 1 vectors.
    The beta^hat rows are synthetic: unit Gaussian noise plus k spikes along fixed
    orthonormal directions, scaled by sqrt(6) so that the ideal covariance is I."""
    import numpy as np
    import torch
    from paper_1105_2791_amd import ModalContext
    P, N, k, S, iters = args.P, args.lr_sims, args.lr_k, args.batch, args.lr_iters
    ctx = ModalContext(8, 12, 24, P, "f64", np.ones((P, 9)), np.ones(9))   # only n_max(P) matters here
    n = ctx.nmax
    rng = np.random.default_rng(2011)
    U, _ = np.linalg.qr(rng.standard_normal((n, k)))
    strengths = np.linspace(14.0, 7.0, k)
    B_host = math.sqrt(6.0) * (rng.standard_normal((N, n)) + (rng.standard_normal((N, k)) * strengths) @ U.T)
    B = torch.as_tensor(B_host, device="cuda")
    alpha = torch.as_tensor(rng.standard_normal(n), device="cuda")
    betas = torch.as_tensor(rng.standard_normal((S, n)), device="cuda")
    X = torch.cat([alpha[None, :], betas])
    calls = {
        "noise_vectors": lambda: ctx.noise_vectors(B, k, iters),
        "fnl_lowrank": lambda: ctx.fnl_lowrank(bt, alpha, betas),
        "bivector_rotate": lambda: ctx.bivector_rotate(bt[0], X),
    }
    bt, mu = ctx.noise_vectors(B, k, iters)
    times = {}
    for name, f in calls.items():
        for _ in range(args.warmup):
            f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            f()
        e1.record()
        torch.cuda.synchronize()
        times[name] = e0.elapsed_time(e1) / args.steps
    gram_flop = float(N) * (N + 1) / 2 * n * 2          # lower triangle of B B^T
    t = times["noise_vectors"] * 1e-3
    line = {
        "metric": "low-rank covariance (noise vectors from N beta^hat + estimator), ms per call", "unit": "ms",
        "value": times["noise_vectors"] + times["fnl_lowrank"], "higher_is_better": False, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"n_max={n} (P={P}), N={N} beta^hat vectors, k={k} noise vectors, "
                               f"{iters} block iterations, S={S} skies", "N": N, "k": k, "S": S, "iters": iters},
        "ms": times, "mu": [float(m) for m in mu],
        # the Gram matrix's flops over the whole call (its one-workgroup steps are latency)
        "roofline": {"bound": "alu", "kernel": "noise_vectors (whole call, Gram flops)", "per_launch": gram_flop,
                     "per_launch_unit": "flop", "achieved": gram_flop / t / 1e12, "peak": PEAK["f64_vec"] / 1e12,
                     "unit": "TFLOP/s", "frac": gram_flop / t / PEAK["f64_vec"], "traffic": None},
        "cpu_baseline": _baseline(args, lambda: cpu_baseline_lowrank(B_host, k)),
    }
    print(json.dumps(line), flush=True)


def run_power(args):
    """Modal power-spectrum batches (Sec. IV): maps + sum_x w (M_p M_r - V_pr) for S skies."""
    res = run_path(args, args.prec, args.steps, args.warmup, make_state=not args.no_linear, op="power")
    pair = dict(res["kernels"]["cubic"])
    pair["kernel"] = "pair sums (k_pair_sums + k_pair_reduce)"
    pair["traffic"] = measured_traffic("pair_sums", args.prec)
    line = {
        "metric": "modal power spectrum: sim maps/sec (filter + pair sums) @lmax=1000,P=40", "unit": "maps/s",
        "value": res["value"], "ms_per_step": res["ms_per_step"], "higher_is_better": True, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "scaling": "weak", "vs_baseline": None,
        "dtype": {"bf16x3": "bf16", "f16x3": "f16", "f32": "f32", "f64": "f64"}[args.prec], "data": "synthetic",
        "config": {"workload": f"lmax={args.lmax} GL {args.ntheta}x{args.nphi} P={args.P} npairs={res['npairs']}, "
                               f"beam+noise spectrum, |lat|<10deg cut, MC pair means ({args.mc} skies)",
                   "batch": args.batch, "prec": args.prec},
        "stages_ms": res["stages_ms"], "roofline": pair, "kernels": res["kernels"],
        "cpu_baseline": _baseline(args, lambda: cpu_baseline(args.lmax, args.ntheta, args.nphi, args.P,
                                                             args.cpu_rings, op="power")),
    }
    print(json.dumps(line), flush=True)


def run_trispectrum(args):
    """Modal trispectrum batches (Sec. IV): maps + the pairs x pairs update + gather for S skies."""
    res = run_path(args, args.prec, args.steps, args.warmup, make_state=not args.no_linear, op="trispectrum")
    k = dict(res["kernels"]["cubic"])
    k["kernel"] = "pairs x pairs update (k_quad_vtile + k_quad_syrk + k_quad_reduce)"
    k["traffic"] = measured_traffic("quad", args.prec)
    line = {
        "metric": "modal trispectrum: sim maps/sec (filter + quartic reduction) @lmax=1000,P=40", "unit": "maps/s",
        "value": res["value"], "ms_per_step": res["ms_per_step"], "higher_is_better": True, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "scaling": "weak", "vs_baseline": None,
        "dtype": {"bf16x3": "bf16", "f16x3": "f16", "f32": "f32", "f64": "f64"}[args.prec], "data": "synthetic",
        "config": {"workload": f"lmax={args.lmax} GL {args.ntheta}x{args.nphi} P={args.P} npairs={res['npairs']} "
                               f"modes={res['ncol']}, beam+noise spectrum, |lat|<10deg cut, MC pair means "
                               f"({args.mc} skies)", "batch": args.batch, "prec": args.prec},
        "stages_ms": res["stages_ms"], "roofline": k, "kernels": res["kernels"],
        # few rings: the oracle's quartic sums loop over the 123,410 modes
        "cpu_baseline": _baseline(args, lambda: cpu_baseline(args.lmax, args.ntheta, args.nphi, args.P,
                                                             max(1, args.cpu_rings // 32), op="trispectrum")),
    }
    print(json.dumps(line), flush=True)


def run_shapes(args):
    """Theory side at the workload shape: alpha_n of a three-term separable shape and the
    ideal covariance zeta0 (n_max x n_max) of the separable modes."""
    import numpy as np
    import torch
    import modal_inputs as mi
    from paper_1105_2791_amd import ModalContext
    lmax, P = args.lmax, args.P
    cl = mi.filter_cl(lmax, "wmap")
    ctx = ModalContext(lmax, args.ntheta, args.nphi, P, "f32", mi.q_basis(P, lmax), cl)
    one = np.ones(lmax + 1)
    terms = np.array([[2 * cl, cl, one], [2 * cl, one, cl], [2 * one, cl, cl]])
    times = {}
    for name, f in (("alpha_separable", lambda: ctx.alpha_separable(terms)), ("ideal_covariance", ctx.ideal_covariance)):
        for _ in range(args.warmup):
            f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            f()
        torch.cuda.synchronize()
        times[name] = 1e3 * (time.perf_counter() - t0) / args.steps
    nmu = (3 * lmax + 2) // 2
    n = ctx.nmax
    # the 3 x 3 permanent expanded along its third row, its 2 x 2 permanents shared
    # across the rows of a group: 1 mul + 2 fma, then the weighted fma, per (pair of modes, node)
    flop = n * (n + 1) / 2 * nmu * 7.0
    t = times["ideal_covariance"] * 1e-3
    line = {
        "metric": "theory side: alpha_n (3 separable terms) and ideal covariance, ms per call", "unit": "ms",
        "value": times["ideal_covariance"], "higher_is_better": False, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"lmax={lmax} P={P} nmax={n}, {nmu} Gauss-Legendre nodes in mu"},
        "ms": times,
        "roofline": {"bound": "alu", "kernel": "ideal_covariance (k_ideal_cov dominant)", "per_launch": flop,
                     "per_launch_unit": "flop", "achieved": flop / t / 1e12, "peak": PEAK["f64_vec"] / 1e12,
                     "unit": "TFLOP/s", "frac": flop / t / PEAK["f64_vec"], "traffic": None},
        # the ideal covariance only: the oracle's alpha is a triple sum over an l_max^3 table
        "cpu_baseline": _baseline(args, lambda: cpu_baseline_shapes(lmax, P)),
    }
    print(json.dumps(line), flush=True)


def _time_ms(f, steps, warmup):
    import torch
    for _ in range(warmup):
        f()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        f()
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / steps


def _roof(flop, ms, bound, peak):
    rate = flop / (ms * 1e-3)
    return {"bound": bound, "per_launch": flop, "per_launch_unit": "flop", "achieved": rate / 1e12,
            "peak": peak / 1e12, "unit": "TFLOP/s", "frac": rate / peak, "traffic": None}


def run_estimator(args):
    """The estimator and gradient rows, each timed whole (host clock around synchronised
    calls): the adjoint (VJP) of beta^hat for S skies at the workload shape, the sample
    covariance of N = 200 beta^hat rows and the FP64 Cholesky estimator at n_max(P), the
    Fisher covariance at l_max 500, GL 768 x 1536, P 30 in FP32, and the replay of one graph
    holding beta calls of two contexts (l_max 500 and the workload's) against eager calls."""
    import numpy as np
    import torch
    import modal_inputs as mi
    from paper_1105_2791_amd import ModalContext
    from paper_1105_2791_amd.api import BetaGraph
    lmax, nt, nphi, P, S, prec = args.lmax, args.ntheta, args.nphi, args.P, args.batch, args.prec
    split = prec in ("bf16x3", "f16x3")
    mpeak = PEAK["bf16"] if split else (PEAK["f32_mfma"] if prec == "f32" else PEAK["f64_vec"])
    rng = np.random.default_rng(2012)
    items = {}
    cl = mi.filter_cl(lmax, "wmap")
    ctx = ModalContext(lmax, nt, nphi, P, prec, mi.q_basis(P, lmax), cl)
    n = ctx.nmax
    st = ctx.linear_state()
    ctx.linear_reset(st)
    ctx.linear_accumulate(st, make_inputs(lmax, P, S, 1000))
    ctx.linear_finalize(st)
    alm = ctx._alm(make_inputs(lmax, P, S, 0))
    cot = torch.as_tensor(rng.standard_normal((S, n)), device="cuda")
    log("estimator: vjp")
    t = _time_ms(lambda: ctx.beta_vjp(alm, cot, st), args.steps, 1)
    # adjoint Legendre (the synthesis transposed) + the cotangent contraction over the
    # triples (the cubic's count); the r2c FFT is HBM work on top
    flop = 2.0 * ctx.nalm * nt * P * S + 2.0 * n * nt * nphi * S
    # stage times of one more call from the library's own events
    ctx.profile_read(reset=True)
    ctx.profile(True)
    ctx.beta_vjp(alm, cot, st)
    torch.cuda.synchronize()
    ctx.profile(False)
    vst = {k: v[0] for k, v in ctx.profile_read(reset=True).items() if v[1] > 0}
    items["vjp"] = {"row": "A9", "shape": f"lmax={lmax} GL {nt}x{nphi} P={P} S={S} {prec}, with the linear-term state",
                    "ms": t, "gradients_per_s": S / (t * 1e-3), "stages_ms": vst,
                    "roofline": _roof(flop, t, "mfma", mpeak)}
    N = 200
    B = torch.as_tensor(rng.standard_normal((N, n)), device="cuda")
    log("estimator: sample covariance")
    t = _time_ms(lambda: ctx.covariance_sample(B), args.steps, 1)
    items["covariance_sample"] = {"row": "A7", "shape": f"N={N} rows of n_max={n}", "ms": t,
                                  "roofline": _roof(float(N) * n * (n + 1), t, "alu", PEAK["f64_vec"])}
    Z = ctx.covariance_sample(B) + torch.eye(n, dtype=torch.float64, device="cuda")
    alpha = torch.as_tensor(rng.standard_normal(n), device="cuda")
    betas = torch.as_tensor(rng.standard_normal((S, n)), device="cuda")
    log("estimator: Cholesky estimator")
    t = _time_ms(lambda: ctx.fnl(Z, alpha, betas), max(1, args.steps // 2), 1)
    items["fnl"] = {"row": "A8", "shape": f"n_max={n}, S={S} (zeta = sample covariance + I)", "ms": t,
                    "roofline": _roof(2.0 * n ** 3 / 3.0 + 2.0 * (S + 1) * n * n, t, "alu", PEAK["f64_vec"])}
    del Z, B
    # graph replay: one graph with the beta calls of two contexts against eager calls
    l2, nt2, nphi2 = 500, 768, 1536
    cl2 = mi.filter_cl(l2, "wmap")
    c2 = ModalContext(l2, nt2, nphi2, P, prec, mi.q_basis(P, l2), cl2)
    a2 = c2._alm(make_inputs(l2, P, S, 0))
    g = BetaGraph([(c2, a2, None), (ctx, alm, None)])
    o1 = torch.empty((S, c2.nmax), dtype=torch.float64, device="cuda")
    o2 = torch.empty((S, n), dtype=torch.float64, device="cuda")
    log("estimator: graph replay")
    tg = _time_ms(g.launch, args.steps, 1)
    te = _time_ms(lambda: (c2.beta(a2, out=o1), ctx.beta(alm, out=o2)), args.steps, 1)
    items["graph"] = {"row": "A11", "shape": f"beta of S={S} at lmax 500 (GL 768x1536) and lmax {lmax}, P={P}, {prec}",
                      "graph_ms": tg, "eager_ms": te}
    g.close()
    c2.close()
    ctx.close()
    # Fisher covariance at the l_max 500, P 30 FP32 shape (every pair adjoint per sky)
    lf, Pf, Nf = 500, 30, 2
    clf = mi.filter_cl(lf, "wmap")
    cf_ = ModalContext(lf, 768, 1536, Pf, "f32", mi.q_basis(Pf, lf), clf)
    stf = cf_.linear_state()
    cf_.linear_reset(stf)
    cf_.linear_accumulate(stf, make_inputs(lf, Pf, 4, 1000))
    cf_.linear_finalize(stf)
    af = cf_._alm(make_inputs(lf, Pf, Nf, 0))
    log("estimator: Fisher covariance")
    t = _time_ms(lambda: cf_.covariance_fisher(af, clf, stf), 1, 1)
    items["fisher"] = {"row": "A10", "shape": f"lmax={lf} GL 768x1536 P={Pf} (nmax={cf_.nmax}, {cf_.npairs} pair adjoints "
                                              f"per sky) f32, N={Nf} skies", "ms": t, "ms_per_sky": t / Nf}
    cf_.close()
    line = {
        "metric": "estimator and gradient rows: adjoint, covariance, Cholesky estimator, Fisher, graph replay",
        "unit": "ms", "value": items["vjp"]["ms"], "higher_is_better": False, "n_gpus": 1, "steps": args.steps,
        "dtype": {"bf16x3": "bf16", "f16x3": "f16", "f32": "f32", "f64": "f64"}[prec], "data": "synthetic",
        "config": {"workload": f"lmax={lmax} GL {nt}x{nphi} P={P} n_max={n} S={S} (value: the VJP of S skies)"},
        "items": items,
    }
    print(json.dumps(line), flush=True)


def run_batch(args):
    """Mixed-resolution Monte-Carlo batch on one GPU: 512 skies, sky i at l_max
    [500, 1000, 2000][i mod 3] on Gauss-Legendre 768 x 1536, 1536 x 3072 and 3008 x 6016 rings,
    P = 50 separable modes (n_max = 22,100), split bf16, beta of every sky.  Each context is
    autotuned first; the calls (S skies each) are captured into one HIP graph and replayed."""
    import numpy as np
    import torch
    import modal_inputs as mi
    from paper_1105_2791_amd import ModalContext
    from paper_1105_2791_amd.api import BetaGraph
    P, S, nsims, prec = args.batch_P, args.batch, args.batch_sims, args.prec
    shapes = [(500, 768, 1536), (1000, 1536, 3072), (2000, 3008, 6016)]
    ctxs, tuned = [], []
    for lmax, nt, nphi in shapes:
        cl = mi.filter_cl(lmax, "wmap")
        probe = ModalContext(lmax, nt, nphi, 1, "f32", mi.q_basis(1, lmax), cl)
        x, _ = probe.grid()
        probe.close()
        mask = np.repeat(mi.mask_rings(np.arccos(x))[:, None], nphi, axis=1)
        c = ModalContext(lmax, nt, nphi, P, prec, mi.q_basis(P, lmax), cl, mask=mask)
        log(f"batch: context lmax={lmax} grid={nt}x{nphi} P={P} nmax={c.nmax} lambda_table={c.lambda_table}")
        a = c._alm(make_inputs(lmax, P, S, 0, cfg_id=5))
        tuned.append(c.autotune(a))
        ctxs.append(c)
    # sky i -> context i mod 3; consecutive skies of a context form calls of S skies
    per = [len(range(k, nsims, 3)) for k in range(3)]
    calls = []
    for k, c in enumerate(ctxs):
        lmax = shapes[k][0]
        for b0 in range(0, per[k], S):
            n = min(S, per[k] - b0)
            calls.append((c, make_inputs(lmax, P, n, 3 * b0 + k, cfg_id=5), None))
    log(f"batch: {len(calls)} calls, skies per l_max {per}; capturing")
    g = BetaGraph(calls)
    for _ in range(args.warmup):
        g.launch()
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        g.launch()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    outs = g.betas
    assert all(torch.isfinite(o).all().item() for o in outs)
    # per-context eager time of one call of S skies (stage split)
    per_ctx = {}
    for k, c in enumerate(ctxs):
        a = c._alm(make_inputs(shapes[k][0], P, S, 0, cfg_id=5))
        out = torch.empty((S, c.nmax), dtype=torch.float64, device="cuda")
        c.beta(a, out=out)
        c.profile_read(reset=True)
        c.profile(True)
        c.beta(a, out=out)
        torch.cuda.synchronize()
        c.profile(False)
        st = {kk: v[0] for kk, v in c.profile_read(reset=True).items() if v[1]}
        per_ctx[f"lmax{shapes[k][0]}"] = {"grid": f"{shapes[k][1]}x{shapes[k][2]}", "ms_per_call": sum(st.values()),
                                          "stages_ms": st, "tuned": tuned[k]}
    g.close()
    for c in ctxs:
        c.close()
    line = {
        "metric": "mixed-resolution Monte-Carlo batch: sims/sec (filter + beta_n), graph replay", "unit": "sims/s",
        "value": nsims / t, "ms_per_batch": 1e3 * t, "higher_is_better": True, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "dtype": {"bf16x3": "bf16", "f16x3": "f16", "f32": "f32", "f64": "f64"}[prec],
        "data": "synthetic",
        "config": {"workload": f"{nsims} skies, l_max 500/1000/2000 (sky i -> [500,1000,2000][i mod 3]) on GL "
                               f"768x1536 / 1536x3072 / 3008x6016, P={P} (n_max={ctxs[0].nmax}), beam+noise "
                               f"spectrum, |lat|<10deg cut, {len(calls)} calls of up to {S} skies in one HIP graph",
                   "skies_per_lmax": per, "batch": S},
        "per_context": per_ctx,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=8, help="skies per step (S)")
    ap.add_argument("--prec", default="bf16x3", choices=["bf16x3", "f16x3", "f32", "f64"])
    ap.add_argument("--lmax", type=int, default=1000)
    ap.add_argument("--ntheta", type=int, default=1536)
    ap.add_argument("--nphi", type=int, default=3072)
    ap.add_argument("--P", type=int, default=40)
    ap.add_argument("--mc", type=int, default=16, help="Monte-Carlo skies for the linear term")
    ap.add_argument("--cpu-rings", type=int, default=64)
    ap.add_argument("--cpu-rings-1t", type=int, default=8, help="rings of the one-thread oracle run (0: skip)")
    ap.add_argument("--compare-steps", type=int, default=3, help="timed steps of the plain-FP32 comparison (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action=argparse.BooleanOptionalAction, default=True,
                    help="run the launch-shape autotuner before timing the headline path (default on)")
    ap.add_argument("--otf-steps", type=int, default=3,
                    help="timed steps of the headline path with the recurrence on the fly (no lambda table; 0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of a known size (HBM counter calibration)")
    ap.add_argument("--no-linear", action="store_true", help="beta without the linear term (diagnostic)")
    ap.add_argument("--workload", default="beta",
                    choices=["beta", "lowrank", "power", "shapes", "trispectrum", "estimator", "batch"],
                    help="beta: the hot path (default); lowrank: the low-rank covariance calls; "
                         "power: the modal power spectrum; shapes: alpha_n and the ideal covariance; "
                         "trispectrum: the modal trispectrum; estimator: adjoint, covariance, Cholesky "
                         "estimator, Fisher and graph replay; batch: 512 skies of mixed l_max 500/1000/2000 "
                         "at P 50 in one graph")
    ap.add_argument("--batch-sims", type=int, default=512, help="batch: Monte-Carlo skies")
    ap.add_argument("--batch-P", type=int, default=50, help="batch: separable modes")
    ap.add_argument("--lr-sims", type=int, default=1000, help="lowrank: beta^hat vectors N")
    ap.add_argument("--lr-k", type=int, default=4, help="lowrank: noise vectors k")
    ap.add_argument("--lr-iters", type=int, default=100, help="lowrank: block iterations")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        log("bench.py: only --gpus 1 is supported (single-GPU build)")
        sys.exit(2)

    import torch
    torch.cuda.set_device(torch.device("cuda", 0))
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "lowrank":
        run_lowrank(args)
        return
    if args.workload == "power":
        run_power(args)
        return
    if args.workload == "shapes":
        run_shapes(args)
        return
    if args.workload == "trispectrum":
        run_trispectrum(args)
        return
    if args.workload == "estimator":
        run_estimator(args)
        return
    if args.workload == "batch":
        run_batch(args)
        return
    prec = args.prec
    head = run_path(args, prec, args.steps, args.warmup, make_state=not args.no_linear)
    fp32 = None
    if args.compare_steps > 0 and prec != "f32":
        fp32 = run_path(args, "f32", args.compare_steps, 1, make_state=not args.no_linear, autotune=False)
    otf = None
    if args.otf_steps > 0 and prec in ("bf16x3", "f16x3"):
        otf = run_path(args, prec, args.otf_steps, 1, make_state=not args.no_linear, lambda_table=False,
                       autotune=False)

    for k, v in head["kernels"].items():
        v["traffic"] = measured_traffic(k, prec)
    # the dominant kernel's roofline (by time per step)
    dom = max(head["kernels"].items(), key=lambda kv: kv[1]["avg_ms"])
    roof = dict(dom[1])
    roof["kernel"] = dom[0]
    roof["traffic"] = measured_traffic(dom[0], prec)

    cpu = None
    if not args.no_cpu_baseline:
        try:
            cpu = cpu_baseline(args.lmax, args.ntheta, args.nphi, args.P, args.cpu_rings,
                               one_thread_rings=args.cpu_rings_1t)
        except Exception as e:  # the baseline is reported, never the target
            log(f"cpu baseline failed: {e!r}")

    line = {
        "metric": METRIC, "value": head["value"], "unit": "maps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"bf16x3": "bf16", "f16x3": "f16", "f32": "f32", "f64": "f64"}[prec],
        "precision": {"bf16x3": "split bf16 hi+lo on the matrix cores, fp32 accumulate, fp64 reduce",
                      "f16x3": "split fp16 hi+lo (scaled) on the matrix cores, fp32 accumulate, fp64 reduce",
                      "f32": "fp32 maps and matrix-core products, compensated fp32 accumulate, fp64 reduce",
                      "f64": "fp64"}[prec],
        "data": "synthetic",
        "config": {"workload": f"lmax={args.lmax} GL {args.ntheta}x{args.nphi} P={args.P} nmax={head['nmax']}, "
                               f"beam+noise spectrum, |lat|<10deg cut, "
                               + ("no linear term" if args.no_linear else f"MC linear term ({args.mc} skies)"),
                   "batch": args.batch, "prec": prec, "tuned": head["tuned"]},
        "stages_ms": head["stages_ms"],
        "roofline": roof,
        "kernels": head["kernels"],
        "fp32_compare": None if fp32 is None else {
            "value": fp32["value"], "ms_per_step": fp32["ms_per_step"], "steps": args.compare_steps,
            "stages_ms": fp32["stages_ms"], "speedup": head["value"] / fp32["value"],
            # the FP32 contraction against the FP32 matrix-core peak (157.3 TF), algorithmic
            # and issued (every pair x all modes, padded tiles)
            "cubic_roofline": {k: fp32["kernels"]["cubic"].get(k) for k in
                               ("achieved", "peak", "unit", "frac", "mfma_issued_frac", "avg_ms")}},
        "recurrence_on_the_fly": None if otf is None else {
            "value": otf["value"], "ms_per_step": otf["ms_per_step"], "steps": args.otf_steps,
            "stages_ms": otf["stages_ms"], "lambda_table": otf["lambda_table"],
            "note": "same path with the synthesis's recurrence computed on the fly (no precomputed lambda table)"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
