#!/usr/bin/env python3
"""Benchmark: one full Yukawa-FMM evaluation on one MI355X.

Workload (the paper-shaped FMM throughput set): 2^20 iid uniform points in the
unit square with N(0,1) charges, plus an outer circle (centre (0.5,0.5),
radius 0.5) and five circular holes of radius 0.06, 4096 nodes per curve, with
N(0,1) dipole strengths; alpha = 0.05; expansion order chosen for 1e-10
relative error.  One step = one evaluation of V[q] + DL[d] at every point
(sources = targets), FP64, with the tree already built (points are static
across time steps; the build time is reported separately).

The JSON line carries:
  value        Mpts/s = (N_D + N_Gamma) / t_pass
  config       workload, p, leaf size, relative error over 1000 sampled targets
               against FP64 direct sums on the GPU, and over 100 of them against
               the CPU oracle
  roofline     the dominant kernel (M2L on the FP64 matrix cores) against its
               peak, from HIP events recorded around its launches; the config's
               `rooflines` add the cached near field (HBM) and the near field
               evaluated on the fly (FP64 vector units)
  cpu_baseline the CPU oracle's direct sums at the sampled targets
  time_step    s/time-step of the backward-Euler heat step on the 1024^2 grid,
               plain FP64 vs FP64 and mixed precision with the learned guess

Opt-in modes that print their own JSON object instead: --heat-only (the
time-step comparison alone) and --large-steps K (the same comparison over K
steps of the large adaptive set, about 2^24 cells; the tree takes seconds).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Yukawa-FMM Mpts/s at stated rel err; s/time-step plain FP64 vs mixed+learned"
PEAK_FP64_VALU_TF = 78.6      # MI355X FP64 vector peak (256 CU x 2.4 GHz x 128 flop/clk)
PEAK_FP32_MFMA_TF = 157.3     # MI355X dense matrix-core peaks
PEAK_FP64_MFMA_TF = 78.6
PEAK_HBM_GBS = 8000.0


LOG_FLOPS = 40   # FP64 logarithm: 9 for the reciprocal with two Newton steps, 31 for the
                 # reduction, the degree-10 atanh series and the exponent recombination


def near_flops(info):
    """Algorithmic FP64 flops of the near field (the leaf kernel).

    Per charge pair: separation and r^2 (5), t = r^2/(4 alpha^2) (1), the two
    Horner series of length n (4(n-1)), -1/2 ln(t) A(t) + B(t) (3), q K0 + acc (2),
    plus the logarithm counted at the cost of its evaluation (LOG_FLOPS, an FMA
    being 2 flops), as N-body codes count a reciprocal square root.  Per dipole
    pair: the same geometry (6), the K1(z)/z series (4(n-1) + 6), (x-y).dn (3),
    scale and accumulate (3), plus the logarithm."""
    n = info.near_terms
    fq = 12 + 4 * (n - 1) + LOG_FLOPS
    fd = 18 + 4 * (n - 1) + LOG_FLOPS
    return info.pairs_charge * fq + info.pairs_dipole * fd


def rooflines(info, st, steps, fp32):
    """Per-kernel rooflines from the serialised per-stage event times.

    Near field (cached): algorithmic bytes = the interaction values read once
    per pass, 8 bytes per stored charge value and 16 per dipole pair in FP64
    (half in FP32), plus the 8-byte entries of the incoming slots the kernel
    writes; with the symmetric layout a charge value stands for two pairs
    (stored once per pair of neighbouring leaves).  Source strengths and
    outputs add under 3% and are not counted.
    M2L: 2 P^2 flops per non-empty V-list translation (padding not credited),
    against the dense matrix-core peak of the arithmetic type."""
    out = {}
    leaf_ms, leaf_calls = st["leaf"]
    if leaf_calls:
        t = leaf_ms / leaf_calls
        vb = 4 if fp32 else 8
        nbytes = info.near_charge_values * vb + info.pairs_dipole * 2 * vb + info.near_incoming * 8
        ach = nbytes / (t * 1e-3) / 1e9
        kname = ("k_near_apply_sym (cached near field, P2P; charge blocks stored once per leaf pair)"
                 if info.near_sym else "k_near_apply (cached near field, P2P)")
        out["near"] = {"kernel": kname, "bound": "hbm", "achieved": ach,
                       "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS,
                       "traffic": None if fp32 else measured_traffic("k_near_apply"), "avg_launch_ms": t,
                       "launches_per_pass": leaf_calls / steps, "algorithmic_bytes": nbytes}
    m2l_ms, m2l_calls = st["m2l"]
    if m2l_calls:
        t = m2l_ms / m2l_calls
        peak = PEAK_FP32_MFMA_TF if fp32 else PEAK_FP64_MFMA_TF
        ach = m2l_flops(info) / (t * 1e-3) / 1e12
        out["m2l"] = {"kernel": ("k_tile_gemm (M2L, all levels, FP32)" if fp32 else
                                 "k_m2l_persist (M2L, all levels, one resident round)"),
                      "bound": "mfma", "achieved": ach,
                      "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                      "traffic": None if fp32 else measured_traffic("k_m2l_persist"), "avg_launch_ms": t,
                      "launches_per_pass": m2l_calls / steps, "algorithmic_flops": m2l_flops(info)}
    # the upward and downward chain: 10 P flops per point for P2M and L2P
    # (the expansion's P terms, about ten operations each), 2 P^2 per
    # child-parent translation for M2M and L2L (one dense P x P product);
    # FP64 in both precision modes (P2M, M2M, L2P) or in FP64 mode (L2L),
    # against the FP64 peak; per pass (all launches of the stage)
    P = info.P
    chain = {"p2m": ("P2M (k_p2m_half + k_p2m_quad, or cached rows on small trees)", 10.0 * P * info.p2m_points),
             "m2m": ("M2M (k_tile_gemm on large levels, k_small_gemv on small ones)",
                     2.0 * P * P * info.m2m_children),
             "l2l": ("L2L (k_tile_gemm on large levels, k_small_gemv on small ones)",
                     2.0 * P * P * info.l2l_children),
             "l2p": ("k_l2p (L2P, writes the outputs)", 10.0 * P * info.l2p_points)}
    for key, (kname, flops) in chain.items():
        ms, calls = st[key]
        if not calls or flops <= 0:
            continue
        t_pass = ms / steps
        ach = flops / (t_pass * 1e-3) / 1e12
        out[key] = {"kernel": kname, "bound": "alu", "achieved": ach, "peak": PEAK_FP64_MFMA_TF,
                    "unit": "TFLOP/s", "frac": ach / PEAK_FP64_MFMA_TF, "traffic": None,
                    "ms_per_pass": t_pass, "launches_per_pass": calls / steps, "algorithmic_flops": flops}
    return out


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "hbm_traffic_fmm_pass_c1_fp64.md")
    src = os.path.join(ROOT, "paper_1007_5335_amd", "csrc", "fmm_kernels.hip")
    try:
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()
        for ln in open(prof):
            f = ln.split()
            if len(f) == 4 and f[0] == "traffic" and f[1] == kernel:
                kv = dict(x.split("=", 1) for x in f[2:])
                if kv.get("source_sha256") == h:
                    return float(kv["bytes_per_launch"])
    except OSError:
        pass
    return None


def m2l_flops(info):
    """Algorithmic flops of M2L: 2 P^2 per non-empty V-list translation (no padding)."""
    return 2.0 * info.P * info.P * info.m2l_translations


def run_fmm_bench(args, yk, torch, W, fp32=None, lite=False):
    """Times the FMM pass; lite skips the overlapped and on-the-fly variants."""
    if fp32 is None:
        fp32 = args.fp32
    cfg = W.config_c1(n_vol=args.n_vol, n_nodes=args.n_nodes, alpha=args.alpha, seed=1)
    b = cfg["bnd"]
    n_pts = cfg["vol"].shape[0] + b.n
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    vol, q, dip = d(cfg["vol"]), d(cfg["q"]), d(cfg["dip"])
    bd = yk.Boundary.from_workload(b)
    out_v = torch.empty(vol.shape[0], dtype=torch.float64, device="cuda")
    out_b = torch.empty(b.n, dtype=torch.float64, device="cuda")
    prec = yk.YK_PREC_FP32 if fp32 else yk.YK_PREC_FP64
    opt = yk.yk_default_options()
    opt.fmm_tol, opt.p, opt.leaf_size, opt.precision = args.tol, args.p, args.leaf, prec
    ctx = yk.yk_create(opt)
    try:
        torch.cuda.synchronize()
        yk.yk_timing_enable(ctx, True)
        t0 = time.perf_counter()
        yk.yk_fmm_potential(ctx, vol, q, bd, dip, args.alpha, out_v, out_b)   # builds the tree
        torch.cuda.synchronize()
        first_ms = (time.perf_counter() - t0) * 1e3
        near_build_ms = yk.yk_timing_read(ctx, reset=True)["near_build"][0]
        yk.yk_timing_enable(ctx, False)
        info = yk.yk_plan_info_get(ctx, 0)
        for _ in range(args.warmup):
            yk.yk_fmm_potential(ctx, vol, q, bd, dip, args.alpha, out_v, out_b)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            yk.yk_fmm_potential(ctx, vol, q, bd, dip, args.alpha, out_v, out_b)
        e1.record()
        torch.cuda.synchronize()
        total_ms = e0.elapsed_time(e1)
        # per-stage kernel times: once as run (near field overlapping the far
        # field on a second stream), once serialised for per-kernel rooflines
        stages_overlap, stages = {}, {}
        for serial, dst in ((False, stages_overlap), (True, stages)) if not lite else ((True, stages),):
            opt.debug_flags = 2 if serial else 0
            yk.yk_set_options(ctx, opt)
            yk.yk_timing_enable(ctx, True)
            yk.yk_timing_read(ctx, reset=True)
            for _ in range(args.steps):
                yk.yk_fmm_potential(ctx, vol, q, bd, dip, args.alpha, out_v, out_b)
            dst.update(yk.yk_timing_read(ctx, reset=True))
            yk.yk_timing_enable(ctx, False)
        # the near field evaluated on the fly (no cached values), serialised
        stages_otf = {"leaf": (0.0, 0)}
        if not lite:
            opt.debug_flags, opt.near_cache_mb = 2, 0
            yk.yk_set_options(ctx, opt)
            yk.yk_timing_enable(ctx, True)
            yk.yk_timing_read(ctx, reset=True)
            for _ in range(args.steps):
                yk.yk_fmm_potential(ctx, vol, q, bd, dip, args.alpha, out_v, out_b)
            stages_otf = yk.yk_timing_read(ctx, reset=True)
            yk.yk_timing_enable(ctx, False)
        opt.debug_flags, opt.near_cache_mb = 0, yk.yk_default_options().near_cache_mb
        yk.yk_set_options(ctx, opt)
        info = yk.yk_plan_info_get(ctx, 0)
        ov = out_v.cpu().numpy()
        ob = out_b.cpu().numpy()
    finally:
        yk.yk_destroy(ctx)
    # the cached near field with both orders of every pair stored (the layout
    # is chosen when a plan first meets a target set: a context of its own)
    stages_full, info_full = {"leaf": (0.0, 0)}, None
    if not lite:
        opt_f = yk.yk_default_options()
        opt_f.fmm_tol, opt_f.p, opt_f.leaf_size, opt_f.precision = args.tol, args.p, args.leaf, prec
        opt_f.debug_flags = 2 | 16
        ctx = yk.yk_create(opt_f)
        try:
            for _ in range(1 + args.warmup):
                yk.yk_fmm_potential(ctx, vol, q, bd, dip, args.alpha, out_v, out_b)
            yk.yk_timing_enable(ctx, True)
            yk.yk_timing_read(ctx, reset=True)
            for _ in range(args.steps):
                yk.yk_fmm_potential(ctx, vol, q, bd, dip, args.alpha, out_v, out_b)
            stages_full = yk.yk_timing_read(ctx, reset=True)
            info_full = yk.yk_plan_info_get(ctx, 0)
        finally:
            yk.yk_destroy(ctx)
    ms = total_ms / args.steps
    res = dict(cfg=cfg, n_pts=n_pts, ms=ms, first_ms=first_ms, info=info, stages=stages,
               stages_overlap=stages_overlap, near_build_ms=near_build_ms, stages_otf=stages_otf,
               stages_full=stages_full, info_full=info_full, out=np.concatenate([ov, ob]))
    return res


def direct_check(args, res, yk, torch):
    """Relative error over sampled targets against FP64 direct sums on the GPU."""
    cfg = res["cfg"]
    b = cfg["bnd"]
    all_xy = np.concatenate([cfg["vol"], b.xy])
    idx = np.sort(np.random.default_rng(12345).choice(res["n_pts"], size=args.samples, replace=False))
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    tgt = d(all_xy[idx])
    ctx = yk.yk_create(direct=1)
    try:
        v = torch.empty(len(idx), dtype=torch.float64, device="cuda")
        dl = torch.empty(len(idx), dtype=torch.float64, device="cuda")
        yk.yk_volume_potential(ctx, d(cfg["vol"]), d(cfg["q"]), tgt, cfg["alpha"], v)
        # the layer call weighs sigma by w_j = (2 pi / N_k) |y'|; pass sigma = d / w
        w = b.weights()
        yk.yk_double_layer_apply(ctx, yk.Boundary.from_workload(b), d(cfg["dip"] / w), tgt,
                                 cfg["alpha"], dl)
        ref = (v + dl).cpu().numpy()
    finally:
        yk.yk_destroy(ctx)
    got = res["out"][idx]
    return (float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
            float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))), idx, ref)


def oracle_baseline(args, res, idx):
    """The CPU oracle's direct sums on a bounded sample of the same targets."""
    import oracle
    oracle.build(force=False)
    cfg = res["cfg"]
    b = cfg["bnd"]
    n_vol = cfg["vol"].shape[0]
    sub = idx[: args.cpu_samples]
    tgt = np.concatenate([cfg["vol"], b.xy])[sub]
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    ref = oracle.volume_sum(cfg["vol"], cfg["q"], cfg["alpha"], tgt_xy=tgt) + \
        oracle.dl_sum(b.xy, b.normal, cfg["dip"], cfg["alpha"], tgt)
    t_cpu = time.perf_counter() - t0
    got = res["out"][sub]
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    n_src = n_vol + b.n
    cpu = {"value": len(sub) / t_cpu / 1e6, "unit": "Mpts/s", "cores": threads, "kind": "oracle",
           "sample": f"{len(sub)} sampled targets x all {n_vol} charges + {b.n} dipoles, direct FP64 "
                     f"sums in {t_cpu:.2f} s; each sampled point is one full O(N) sum",
           "pairs_per_s": len(sub) * n_src / t_cpu,
           "full_pass_s_extrapolated": t_cpu * n_src / len(sub)}
    # the same sums on one core (a tenth of the sample)
    sub1 = sub[: max(1, len(sub) // 10)]
    tgt1 = np.concatenate([cfg["vol"], b.xy])[sub1]
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.volume_sum(cfg["vol"], cfg["q"], cfg["alpha"], tgt_xy=tgt1)
        oracle.dl_sum(b.xy, b.normal, cfg["dip"], cfg["alpha"], tgt1)
        t1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(threads)
    cpu["one_core"] = {"value": len(sub1) / t1 / 1e6, "unit": "Mpts/s", "cores": 1,
                       "pairs_per_s": len(sub1) * n_src / t1, "sample": f"{len(sub1)} of the sampled targets"}
    if not args.no_cpu_steps:
        cpu["oracle_steps"] = oracle_step_timings(oracle)
        try:
            cpu["c4_direct"] = oracle_c4_rate(oracle)
        except (MemoryError, RuntimeError, ValueError) as e:   # reported, not fatal
            cpu["c4_direct"] = {"error": repr(e)}
    return err, cpu


def oracle_c4_rate(oracle):
    """Direct-sum throughput of the oracle on the large clustered set: one
    sampled target against all its charges and dipoles (the set's generation
    is not timed).  The oracle hands targets to its threads in chunks of 16,
    so one target runs on one core."""
    import workloads as W
    c = W.config_c4()
    b = c["bnd"]
    rng = np.random.default_rng(4)
    n_vol = c["vol"].shape[0]
    nt = 1
    tgt = c["vol"][rng.integers(0, n_vol, nt)]
    q = rng.uniform(0.5, 1.5, n_vol) * c["vol_w"]
    dip = rng.standard_normal(b.n) * 1e-3
    t0 = time.perf_counter()
    oracle.volume_sum(c["vol"], q, c["alpha"], tgt_xy=tgt)
    oracle.dl_sum(b.xy, b.normal, dip, c["alpha"], tgt)
    t = time.perf_counter() - t0
    n_src = n_vol + b.n
    return {"targets": nt, "cores": 1, "sources": int(n_src), "s": t, "pairs_per_s": nt * n_src / t,
            "full_pass_s_extrapolated_one_core": t * n_src / nt}


def oracle_step_timings(oracle):
    """Whole backward-Euler steps of the oracle (direct sums, dense matrix of
    the boundary system and its LU, all host cores) at the C0 size and at a
    reduced time-stepping set, and the dense LU timed at the reduced set's
    boundary size and extrapolated (n^3) to the full set's."""
    import scipy.linalg as sla
    import workloads as W
    out = {}
    c0 = W.config_c0()
    b = c0["bnd"]
    t0 = time.perf_counter()
    oracle.heat_step(b.xy, b.normal, b.weights(), b.curvature, c0["vol"], c0["vol_w"], c0["B"],
                     c0["f_next"], c0["dt"], grid_h=c0["h"], offsets=b.offset)
    out["c0_step_s"] = time.perf_counter() - t0
    out["c0_size"] = f"{c0['vol'].shape[0]} volume points, {b.n} nodes"
    c3 = W.config_c3(m=128, n_holes=10, n_nodes=256, dt=1e-3, seed=3)
    b = c3["bnd"]
    B = np.where(c3["region"] < 0, c3["u0"], c3["consts"][np.maximum(c3["region"], 0)])
    t0 = time.perf_counter()
    A = oracle.dl_matrix(b.xy, b.normal, b.weights(), b.curvature, c3["alpha"])
    t_mat = time.perf_counter() - t0
    t0 = time.perf_counter()
    lu = sla.lu_factor(A)
    t_lu = time.perf_counter() - t0
    del A, lu
    t0 = time.perf_counter()
    oracle.heat_step(b.xy, b.normal, b.weights(), b.curvature, c3["vol"], c3["vol_w"], B, c3["f_bnd"],
                     c3["dt"], grid_h=c3["h"], offsets=b.offset)
    out["reduced_c3_step_s"] = time.perf_counter() - t0
    out["reduced_c3_size"] = f"{c3['vol'].shape[0]} volume points, {b.n} nodes"
    n_full = 8192 + 10 * 2048
    out["dense_lu"] = {"n": int(b.n), "matrix_s": t_mat, "lu_s": t_lu, "n_full": n_full,
                       "matrix_s_extrapolated": t_mat * (n_full / b.n) ** 2,
                       "lu_s_extrapolated": t_lu * (n_full / b.n) ** 3,
                       "note": "measured at n, extrapolated to the full boundary (n^2 matrix, n^3 LU)"}
    return out


def heat_step_bench(args, yk, torch, W):
    """s/time-step of the backward-Euler step on the time-stepping geometry:
    plain FP64 with the previous-step guess against mixed precision with the
    learned warm start (trained on the first half of the steps), averaged over
    the second half; every step is solved to the same GMRES tolerance."""
    cfg = W.config_c3(m=args.heat_m, n_holes=10, n_nodes=2048, dt=1e-3, seed=3)
    b = cfg["bnd"]
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    vol, w = d(cfg["vol"]), d(cfg["vol_w"])
    region = torch.as_tensor(cfg["region"], dtype=torch.int32, device="cuda")
    f = d(cfg["f_bnd"])
    bd = yk.Boundary.from_workload(b)
    n_steps, half = args.heat_steps, args.heat_steps // 2
    runs = (("fp64", yk.YK_PREC_FP64, False), ("fp64_learned", yk.YK_PREC_FP64, True),
            ("mixed_learned", yk.YK_PREC_MIXED, True))
    out, finals = {}, {}
    for name, prec, learned in runs:
        ctx = yk.yk_create(fmm_tol=1e-10, leaf_size=args.leaf, precision=prec)
        ws = None
        try:
            if learned:
                ws = yk.yk_ws_create(ctx, bd)
                yk.yk_set_warm_start(ctx, ws)
            u = d(cfg["u0"])
            B = torch.empty_like(u)
            un = torch.empty_like(u)
            sig = torch.zeros(b.n, dtype=torch.float64, device="cuda")
            times, iters, res0, used, train_s, phases = [], [], [], [], None, []
            for step in range(1, n_steps + 1):
                if ws is not None and step == half + 1:
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    yk.yk_ws_train(ws)
                    train_s = time.perf_counter() - t0
                yk.yk_rhs_backward_euler(ctx, u, None, region, cfg["consts"], cfg["dt"], B)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = yk.yk_heat_step(ctx, bd, vol, w, B, yk.HEAT_GRID_SELF_CELL, f, cfg["dt"], 1e-10,
                                     sig, un)
                torch.cuda.synchronize()
                if step > half:
                    times.append(time.perf_counter() - t0)
                    iters.append(st.iters)
                    res0.append(st.res0)
                    used.append(st.guess_used == 2)
                    phases.append([st.ms[1], st.ms[4], st.ms[2], st.ms[3]])
                u, un = un, u
            finals[name] = u.cpu().numpy()
        finally:
            if ws is not None:
                yk.yk_ws_destroy(ws)
            yk.yk_destroy(ctx)
        out[name] = {"s_per_step": float(np.mean(times)), "gmres_iters": float(np.mean(iters)),
                     "initial_rel_residual": float(np.mean(res0)),
                     "learned_guess_used": float(np.mean(used)) if learned else None,
                     "train_s": train_s,
                     "phase_ms": dict(zip(("volume_to_nodes", "guess_selection", "density_solve",
                                           "volume_assembly"), np.mean(phases, axis=0).tolist()))}
    ref = finals.get("fp64", next(iter(finals.values())) if finals else None)
    for name in finals:
        out[name]["u_rel_diff_vs_fp64"] = float(np.max(np.abs(finals[name] - ref)) / np.max(np.abs(ref)))
    if "fp64" in out and "mixed_learned" in out:
        out["speedup_mixed_learned_vs_fp64"] = out["fp64"]["s_per_step"] / out["mixed_learned"]["s_per_step"]
    out["workload"] = (f"{n_steps} backward-Euler steps, dt=1e-3, alpha=sqrt(dt), {args.heat_m}^2 cell grid "
                       f"in the unit square, outer circle ({b.curves[0].n} nodes) + 10 random ellipses x "
                       f"2048 nodes, GMRES tol 1e-10; network trained on steps 1-{half}, timing and "
                       f"iterations averaged over steps {half + 1}-{n_steps}")
    return out


def box_code_bench(args, yk, torch, W):
    """The box code (cubic fits on 4x4-cell leaves, near-field integral tables,
    polynomial multipoles through the FMM) on the time-stepping grid: the
    volume potential alone, and the time step of the uniform-grid entry with
    the box code against the same entry with the lattice rule (FP64, the
    previous-step guess).  B is a seeded mixture of eight Gaussians."""
    cfg = W.config_c3(m=args.heat_m, n_holes=10, n_nodes=2048, dt=1e-3, seed=3)
    m, b, alpha = args.heat_m, cfg["bnd"], cfg["alpha"]
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    # the grid entry needs two cells between the curves and the grid's edge:
    # the square [-1/32, 1 + 1/32]^2 around the time-stepping geometry
    gb, vol = W.grid_box(-1.0 / 32, 1.0 + 1.0 / 32, m)
    grid = yk.make_grid(*gb)
    rng = np.random.default_rng(7)
    mu, sg = rng.uniform(0.2, 0.8, (8, 2)), rng.uniform(0.03, 0.15, 8)
    Bh = sum(np.exp(-((vol[:, 0] - mu[k, 0]) ** 2 + (vol[:, 1] - mu[k, 1]) ** 2) / (2 * sg[k] ** 2))
             for k in range(8))
    B, V = d(Bh), torch.empty(m * m, dtype=torch.float64, device="cuda")
    out = {}
    ctx = yk.yk_create(fmm_tol=1e-10, leaf_size=args.leaf)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        yk.yk_box_potential(ctx, grid, B, alpha, V)          # tables and the leaf tree
        torch.cuda.synchronize()
        first = (time.perf_counter() - t0) * 1e3
        for _ in range(args.warmup):
            yk.yk_box_potential(ctx, grid, B, alpha, V)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            yk.yk_box_potential(ctx, grid, B, alpha, V)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        yk.yk_timing_enable(ctx, True)
        yk.yk_timing_read(ctx, reset=True)
        for _ in range(args.steps):
            yk.yk_box_potential(ctx, grid, B, alpha, V)
        stg = {k: v[0] / args.steps for k, v in yk.yk_timing_read(ctx, reset=True).items() if v[1]}
        yk.yk_timing_enable(ctx, False)
    finally:
        yk.yk_destroy(ctx)
    nleaf = (m // 4) ** 2
    roofs = {}
    # algorithmic bytes per leaf: k_box_leaf reads the leaf's 10 coefficients
    # and its local expansion (64 doubles) and writes its 16 cells; the fit
    # reads 16 cells and writes 10 coefficients; the P2M reads 10 and writes 64
    for key, kern, per_leaf in (("leaf", "k_box_leaf (near tables + local expansion at the 16 cells)",
                                 (10 + 64 + 16) * 8),
                                ("p2m", "k_box_p2m (polynomial multipoles)", (10 + 64) * 8)):
        t = stg.get(key)
        if t:
            nbytes = nleaf * per_leaf
            ach = nbytes / (t * 1e-3) / 1e9
            roofs[key] = {"kernel": kern, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                          "frac": ach / PEAK_HBM_GBS, "traffic": None, "ms_per_call": t,
                          "algorithmic_bytes": nbytes}
    out["potential"] = {"ms": ms, "first_call_ms": first, "mcells_per_s": m * m / (ms * 1e-3) / 1e6,
                        "leaves": nleaf, "stage_ms": stg, "rooflines": roofs}
    # the same density on adaptive leaves (levels 6-10, refined towards a circle)
    lv, lx, ly = W.graded_leaves(centre=(0.5, 0.5), radius=0.3, lo=6, hi=10)
    cells = W.leaf_cell_centres(lv, lx, ly)
    Ba = d(sum(np.exp(-((cells[:, 0] - mu[k, 0]) ** 2 + (cells[:, 1] - mu[k, 1]) ** 2) / (2 * sg[k] ** 2))
               for k in range(8)))
    Va = torch.empty_like(Ba)
    ctx = yk.yk_create(fmm_tol=1e-10)
    try:
        root = (0.0, 0.0, 1.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        yk.yk_box_potential_adaptive(ctx, root, lv, lx, ly, Ba, alpha, Va)   # tables and the tree
        torch.cuda.synchronize()
        first_a = (time.perf_counter() - t0) * 1e3
        for _ in range(args.warmup):
            yk.yk_box_potential_adaptive(ctx, root, lv, lx, ly, Ba, alpha, Va)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            yk.yk_box_potential_adaptive(ctx, root, lv, lx, ly, Ba, alpha, Va)
        e1.record()
        torch.cuda.synchronize()
        ms_a = e0.elapsed_time(e1) / args.steps
        yk.yk_timing_enable(ctx, True)
        yk.yk_timing_read(ctx, reset=True)
        for _ in range(args.steps):
            yk.yk_box_potential_adaptive(ctx, root, lv, lx, ly, Ba, alpha, Va)
        stg_a = {k: v[0] / args.steps for k, v in yk.yk_timing_read(ctx, reset=True).items() if v[1]}
        yk.yk_timing_enable(ctx, False)
    finally:
        yk.yk_destroy(ctx)
    out["adaptive_potential"] = {"ms": ms_a, "first_call_ms": first_a, "leaves": int(lv.size),
                                 "cells": int(cells.shape[0]), "levels": [int(lv.min()), int(lv.max())],
                                 "mcells_per_s": cells.shape[0] / (ms_a * 1e-3) / 1e6, "stage_ms": stg_a}
    bdy = yk.Boundary.from_workload(b)
    f = d(cfg["f_bnd"])
    reg_h = b.region(vol)
    region = torch.as_tensor(reg_h, dtype=torch.int32, device="cuda")
    finals = {}
    for name, flags in (("lattice", 0), ("box_code", yk.HEAT_BOX_CODE)):
        ctx = yk.yk_create(fmm_tol=1e-10, leaf_size=args.leaf)
        try:
            u = torch.zeros(m * m, dtype=torch.float64, device="cuda")
            Bs, un = torch.empty_like(u), torch.empty_like(u)
            sig = torch.zeros(b.n, dtype=torch.float64, device="cuda")
            times, iters, first = [], [], None
            n_steps = max(4, args.heat_steps // 5)
            for step in range(1, n_steps + 1):
                yk.yk_rhs_backward_euler(ctx, u, None, region, cfg["consts"], cfg["dt"], Bs)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = yk.yk_heat_step_grid(ctx, bdy, grid, Bs, flags, f, cfg["dt"], 1e-10, sig, un)
                torch.cuda.synchronize()
                dt_s = time.perf_counter() - t0
                if step == 1:
                    first = dt_s
                else:
                    times.append(dt_s)
                    iters.append(st.iters)
                u, un = un, u
            finals[name] = u.cpu().numpy()
        finally:
            yk.yk_destroy(ctx)
        out[name + "_grid_step"] = {"s_per_step": float(np.mean(times)), "first_step_s": first,
                                    "gmres_iters": float(np.mean(iters)), "steps": n_steps}
    inside = reg_h < 0
    out["box_vs_lattice_max_diff_inside"] = float(np.max(np.abs(finals["box_code"] - finals["lattice"])[inside]))
    out["workload"] = (f"{m}^2 cell grid of [-1/32, 1+1/32]^2, alpha=sqrt(1e-3); potential of a mixture of 8 "
                       f"Gaussians ({nleaf} leaves of 4x4 cells), and of the same density on {lv.size} adaptive "
                       f"leaves of levels 6-10 of the unit square refined towards the circle of radius 0.3 about "
                       f"its centre; backward-Euler grid steps (dt=1e-3, u=0 at "
                       f"t=0) on the time-stepping geometry (outer circle + 10 ellipses x 2048 nodes), GMRES "
                       f"tol 1e-10, averages over steps 2-{max(4, args.heat_steps // 5)}")
    return out


def large_step_bench(args, yk, torch, W):
    """s/time-step on the large adaptive set (about 2^24 cells of an adaptive
    quadtree refined where a mixture of eight Gaussians is dense, weights the
    cell areas plus each cell's own integral, 20 holes x 8192 nodes,
    alpha = 1e-3, dt = alpha^2, u = c_k on hole k, u = 0 at t = 0): plain FP64 with the
    previous-step guess, FP64 and mixed precision with the learned warm start
    (trained on the first half of the steps); averages over the second half.
    Opt-in (--large-steps): the tree takes seconds to build per context."""
    c = W.config_c4()
    b, volh = c["bnd"], c["vol"]
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    region = torch.as_tensor(b.region(volh), dtype=torch.int32, device="cuda")
    inside = torch.as_tensor(b.region(volh) < 0, device="cuda")
    f = d(np.repeat(c["consts"], np.diff(b.offset)))
    vol, w = d(volh), d(c["vol_w"])
    bd = yk.Boundary.from_workload(b)
    n_steps, half = args.large_steps, args.large_steps // 2
    out, finals = {}, {}
    # one FMM pass over every point (volume charges a positive density times
    # the cell areas, unit-scale dipoles), tree already built
    tree = {"auto": yk.YK_TREE_AUTO, "uniform": yk.YK_TREE_UNIFORM, "adaptive": yk.YK_TREE_ADAPTIVE}[args.tree]
    ctx = yk.yk_create(fmm_tol=1e-10, tree=tree, leaf_size=args.large_leaf)
    try:
        rng = np.random.default_rng(5)
        q = d(rng.uniform(0.5, 1.5, volh.shape[0]) * c["vol_w"])
        dip = d(rng.standard_normal(b.n) * 1e-3)
        ov = torch.empty(volh.shape[0], dtype=torch.float64, device="cuda")
        ob = torch.empty(b.n, dtype=torch.float64, device="cuda")
        ms = []
        for k in range(4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            yk.yk_fmm_potential(ctx, vol, q, bd, dip, c["alpha"], ov, ob)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
        info = yk.yk_plan_info_get(ctx, 0)
        npts = volh.shape[0] + b.n
        out["pass"] = {"first_call_ms": ms[0], "ms": float(np.mean(ms[1:])),
                       "mpts_per_s": npts / (float(np.mean(ms[1:])) * 1e-3) / 1e6, "n_points": npts,
                       "p": info.p, "leaf_level": info.leaf_level, "n_leaves": info.n_leaves,
                       "tree": "adaptive" if info.tree == yk.YK_TREE_ADAPTIVE else "uniform",
                       "n_boxes": info.n_boxes, "w_entries": info.n_wlist,
                       "x_boxes": info.n_xboxes,
                       "tree_build_ms": info.build_ms, "near_symmetric": bool(info.near_sym),
                       "near_charge_values": info.near_charge_values, "pairs": info.pairs_charge + info.pairs_dipole}
        print(f"large set pass: {out['pass']['ms']:.1f} ms", file=sys.stderr, flush=True)
    finally:
        yk.yk_destroy(ctx)
    runs = (("fp64", yk.YK_PREC_FP64, False), ("fp64_learned", yk.YK_PREC_FP64, True),
            ("mixed_learned", yk.YK_PREC_MIXED, True))
    runs = tuple(r for r in runs if r[0] in args.large_runs.split(","))
    for name, prec, learned in runs:
        ctx = yk.yk_create(fmm_tol=1e-10, precision=prec, tree=tree, leaf_size=args.large_leaf)
        ws = None
        try:
            if learned:
                ws = yk.yk_ws_create(ctx, bd)
                yk.yk_set_warm_start(ctx, ws)
            u = torch.zeros(volh.shape[0], dtype=torch.float64, device="cuda")
            B, un = torch.empty_like(u), torch.empty_like(u)
            sig = torch.zeros(b.n, dtype=torch.float64, device="cuda")
            times, iters, res0, used, train_s, first, phases, umax = [], [], [], [], None, None, [], []
            for step in range(1, n_steps + 1):
                if ws is not None and step == half + 1:
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    yk.yk_ws_train(ws)
                    train_s = time.perf_counter() - t0
                yk.yk_rhs_backward_euler(ctx, u, None, region, c["consts"], c["dt"], B)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = yk.yk_heat_step(ctx, bd, vol, w, B, yk.HEAT_GRID_SELF_CELL, f, c["dt"], 1e-10, sig, un)
                torch.cuda.synchronize()
                dt_s = time.perf_counter() - t0
                if step == 1:
                    first = dt_s
                print(f"large set {name} step {step}: {dt_s * 1e3:.1f} ms, {st.iters} iterations", file=sys.stderr,
                      flush=True)
                if step > half:
                    times.append(dt_s)
                    iters.append(st.iters)
                    res0.append(st.res0)
                    used.append(st.guess_used == 2)
                    phases.append([st.ms[1], st.ms[4], st.ms[2], st.ms[3]])
                umax.append(float(un[inside].abs().max()))   # inside the domain (maximum principle)
                u, un = un, u
            finals[name] = u.cpu().numpy()
        finally:
            if ws is not None:
                yk.yk_ws_destroy(ws)
            yk.yk_destroy(ctx)
        out[name] = {"s_per_step": float(np.mean(times)), "gmres_iters": float(np.mean(iters)),
                     "initial_rel_residual": float(np.mean(res0)),
                     "learned_guess_used": float(np.mean(used)) if learned else None, "train_s": train_s,
                     "first_step_s": first,
                     "phase_ms": dict(zip(("volume_to_nodes", "guess_selection", "density_solve",
                                           "volume_assembly"), np.mean(phases, axis=0).tolist())),
                     "u_max_abs_per_step": umax}
    ref = finals.get("fp64", next(iter(finals.values())) if finals else None)
    for name in finals:
        out[name]["u_rel_diff_vs_fp64"] = float(np.max(np.abs(finals[name] - ref)) / np.max(np.abs(ref)))
        out[name]["u_rel_l2_vs_fp64"] = float(np.linalg.norm(finals[name] - ref) / np.linalg.norm(ref))
    if "fp64" in out and "mixed_learned" in out:
        out["speedup_mixed_learned_vs_fp64"] = out["fp64"]["s_per_step"] / out["mixed_learned"]["s_per_step"]
    out["workload"] = (f"{n_steps} backward-Euler steps on the large adaptive set ({args.tree} quad-tree): "
                       f"{volh.shape[0]} adaptive cells "
                       f"(refined by a mixture of 8 Gaussians), outer circle + 20 circular holes x 8192 nodes, "
                       f"alpha=1e-3, dt=alpha^2, "
                       f"GMRES tol 1e-10; network trained on steps 1-{half}, timing and iterations averaged over "
                       f"steps {half + 1}-{n_steps}; the first step includes the tree builds")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-vol", type=int, default=1 << 20)
    ap.add_argument("--n-nodes", type=int, default=4096)
    ap.add_argument("--alpha", type=float, default=0.05)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--p", type=int, default=0)
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--samples", type=int, default=1000)
    ap.add_argument("--cpu-samples", type=int, default=100)
    ap.add_argument("--fp32", action="store_true")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle check (profiling runs)")
    ap.add_argument("--no-cpu-steps", action="store_true", help="skip the oracle's whole-step timings")
    ap.add_argument("--heat-steps", type=int, default=100)
    ap.add_argument("--heat-m", type=int, default=1024)
    ap.add_argument("--no-heat", action="store_true")
    ap.add_argument("--no-box", action="store_true", help="skip the box-code measurements")
    ap.add_argument("--box-only", action="store_true",
                    help="only the box-code measurements (profiling runs); prints their JSON object")
    ap.add_argument("--no-fp32-pass", action="store_true", help="skip the FP32 pass of the same workload")
    ap.add_argument("--heat-only", action="store_true",
                    help="only the time-stepping comparison (profiling runs); prints its JSON object")
    ap.add_argument("--large-steps", type=int, default=0,
                    help="only the time-stepping comparison on the large adaptive set, this many steps; "
                         "prints its JSON object")
    ap.add_argument("--tree", choices=("auto", "uniform", "adaptive"), default="auto",
                    help="quad-tree of the large-set runs (--large-steps; auto: adaptive for the "
                         "clustered volume set, uniform for the boundary)")
    ap.add_argument("--large-leaf", type=int, default=64, help="leaf size of the large-set runs")
    ap.add_argument("--large-runs", default="fp64,fp64_learned,mixed_learned",
                    help="which of the large-set step runs to time (comma-separated)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the FMM runs on a single MI355X "
              "(its multi-GPU decomposition is described, not implemented); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    import paper_1007_5335_amd.yk as yk
    yk.load_library()
    torch.cuda.set_device(0)

    if args.heat_only:
        print(json.dumps(heat_step_bench(args, yk, torch, W)), flush=True)
        return
    if args.box_only:
        print(json.dumps(box_code_bench(args, yk, torch, W)), flush=True)
        return
    if args.large_steps > 0:
        print(json.dumps(large_step_bench(args, yk, torch, W)), flush=True)
        return
    if args.calib_copy:
        # a fill (writes 256 MiB) and an elementwise multiply (reads 256 MiB,
        # writes 256 MiB): reference dispatches for the HBM byte counters
        xs = torch.ones(1 << 25, dtype=torch.float64, device="cuda")
        ys = torch.empty_like(xs)
        torch.mul(xs, 2.0, out=ys)
        torch.cuda.synchronize()
        del xs, ys
    res = run_fmm_bench(args, yk, torch, W)
    info, st = res["info"], res["stages"]
    value = res["n_pts"] / (res["ms"] * 1e-3) / 1e6
    roofs = rooflines(info, st, args.steps, args.fp32)
    # the on-the-fly near-field kernel (Bessel series per pair), FP64 vector units
    otf_ms, otf_calls = res["stages_otf"]["leaf"]
    if otf_calls and not args.fp32:
        t = otf_ms / otf_calls
        lf = near_flops(info)
        ach = lf / (t * 1e-3) / 1e12
        roofs["near_on_the_fly"] = {
            "kernel": "k_leaf (near field evaluated on the fly)", "bound": "alu", "achieved": ach,
            "peak": PEAK_FP64_VALU_TF, "unit": "TFLOP/s", "frac": ach / PEAK_FP64_VALU_TF,
            "traffic": measured_traffic("k_leaf"), "avg_launch_ms": t, "launches_per_pass": 0.0,
            "algorithmic_flops": lf, "log_counted_as_flops": LOG_FLOPS}
    # the cached near field with both orders of every pair stored (the layout
    # without the symmetric saving), same workload, its own context
    full_ms, full_calls = res["stages_full"]["leaf"]
    if full_calls and res["info_full"] is not None:
        fi = res["info_full"]
        t = full_ms / full_calls
        vb = 4 if args.fp32 else 8
        nbytes = fi.pairs_charge * vb + fi.pairs_dipole * 2 * vb
        ach = nbytes / (t * 1e-3) / 1e9
        roofs["near_full_layout"] = {
            "kernel": "k_near_apply (cached near field, both orders of every pair stored)", "bound": "hbm",
            "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS,
            "traffic": None, "avg_launch_ms": t, "launches_per_pass": 0.0, "algorithmic_bytes": nbytes}
    # the dominant kernel: largest time per pass
    roof = max((r for k, r in roofs.items()
                if k not in ("near_on_the_fly", "near_full_layout", "p2m", "m2m", "l2l", "l2p")),
               key=lambda r: r["avg_launch_ms"] * r["launches_per_pass"])
    m2l_rate = roofs["m2l"]["achieved"] if "m2l" in roofs else None
    err, errmax, idx, ref = direct_check(args, res, yk, torch)
    fp32_pass = None
    if not args.fp32 and not args.no_fp32_pass:
        # the same pass with FP32 sums (P2P and M2L in FP32, M2L on FP32 matrix
        # cores) at the same expansion order; its error is set by FP32 rounding
        r32 = run_fmm_bench(args, yk, torch, W, fp32=True, lite=True)
        got = r32["out"][idx]
        fp32_pass = {
            "value": r32["n_pts"] / (r32["ms"] * 1e-3) / 1e6, "unit": "Mpts/s", "ms_per_step": r32["ms"],
            "dtype": "f32", "p": r32["info"].p,
            "rel_err_l2_sampled": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
            "stage_ms_per_step": {k: v[0] / args.steps for k, v in r32["stages"].items()},
            "rooflines": rooflines(r32["info"], r32["stages"], args.steps, True)}
    err_oracle = cpu = None
    if not args.no_cpu:
        err_oracle, cpu = oracle_baseline(args, res, idx)
    heat = None if args.no_heat else heat_step_bench(args, yk, torch, W)
    box = None if args.no_box else box_code_bench(args, yk, torch, W)
    line = {
        "metric": METRIC, "value": value, "unit": "Mpts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if args.fp32 else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"FMM pass: {args.n_vol} uniform points in the unit square, N(0,1) charges; "
                         f"outer circle + 5 circular holes x {args.n_nodes} nodes, N(0,1) dipoles; "
                         f"alpha={args.alpha}"),
            "n_points": res["n_pts"], "alpha": args.alpha, "p": info.p, "leaf_level": info.leaf_level,
            "leaf_size": args.leaf, "fmm_tol": args.tol, "rel_err_l2_sampled": err,
            "rel_err_max_sampled": errmax, "rel_err_l2_vs_oracle": err_oracle,
            "tree_build_ms": info.build_ms,
            "first_call_ms": res["first_ms"],
            "stage_ms_per_step": {k: v[0] / args.steps for k, v in st.items()},
            "stage_ms_per_step_overlapped": {k: v[0] / args.steps for k, v in res["stages_overlap"].items()},
            "stage_ms_per_step_near_on_the_fly": {k: v[0] / args.steps for k, v in res["stages_otf"].items()},
            "stage_ms_per_step_near_full_layout": {k: v[0] / args.steps for k, v in res["stages_full"].items()},
            "m2l_tflops": m2l_rate, "pairs_per_step": info.pairs_charge + info.pairs_dipole,
            "near_cache_build_ms": res["near_build_ms"],
            "near_symmetric": bool(info.near_sym), "near_charge_values": info.near_charge_values,
            "near_incoming_entries": info.near_incoming,
            "rooflines": roofs,
            "m2l_translations": info.m2l_translations,
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp32_pass": fp32_pass,
        "time_step": heat,
        "box_code": box,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
