"""Benchmark of the modified-Helmholtz layer-potential hot path on one MI355X.

Workload (the starfish configuration): boundary r(theta) = 1 + 0.3 cos(5 theta)
in 256 equal-arclength panels x 16 Gauss-Legendre nodes (N = 4096); Dirichlet
data from 8 seeded point sources on radius 2; alpha in {5, 50, 500}; targets
are the 109,314 interior points of a 512 x 512 grid on [-1.4, 1.4]^2.

One step = for each alpha: GMRES solve of (1/2 I + D) mu = g to a true relative
residual of 1e-10, then the single- and double-layer potentials of mu at all
targets (fused kernel, near-field corrections included).  Plans (near lists
and correction weights) are built once before timing, as the paper
precomputes them; their build time is reported separately.

value = far-field kernel evaluations per second of the whole step: M N for
each target evaluation and N (N - 1) / 2 for each GMRES operator application
(the FP64 on-surface operator evaluates each unordered pair once and uses it
for both of its terms); pair_terms_per_s counts the N^2 terms of each
application instead.  Prints one JSON line.
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

METRIC = "GPair-evals/s (SLP+DLP) and GMRES time-to-1e-10, mixed/batched/warm vs FP64"
FP64_PEAK_TFLOPS = 78.6        # MI355X vector FP64 (published)
# FP64 operations per (target, source) pair of the fused SLP+DLP far-field
# kernel, per alpha, from the hardware counters of the built kernel
# (SQ_INSTS_VALU_{FMA,MUL,ADD,TRANS}_F64 x 64 lanes / pairs, FMA = 2; lanes
# masked off in divergent code are counted, but the kernel classifies whole
# waves against each panel, so few are):
# profiles/far_eval_fp64_starfish4096_grid512_valu_f64.txt.  The pairs take
# the fitted piece of their z, K0 and K1 each from a fit of its own: at
# alpha = 500 nearly all z > 100 (degree 6 each; the counters read 31.2 v_fma
# (x2), 13.1 v_mul, 3.0 v_add, 2.0 v_rsq = 80.5 per pair), at alpha = 5 z of
# 2..14 (degrees 7-12, the z <= 2 series for the nearest); e^{-z} by a table
# of 2^(-j/64) and a 6-term polynomial.
FLOP_PER_PAIR_FP64 = {5.0: 101.8, 50.0: 83.4, 500.0: 80.5}
# VALU instructions per pair (all types, same counters), and the issue rate
# they are bound by: 256 CUs x 2.4 GHz, one 64-lane VALU instruction per CU
# per clock
VALU_PER_PAIR_FP64 = {5.0: 73.0, 50.0: 61.1, 500.0: 59.1}
VALU_ISSUE_PER_S = 256 * 2.4e9 * 64
# the gradient kernel (grad S and grad D of the same densities) evaluates K0
# and K1(z)/r per pair as the fused evaluation does (the fine piece of the
# plan's (wave, panel) class table; alpha carried by the staged densities),
# then 1/r^2, (x-y).d, (alpha K0 + 2 K1/r)/r^2 and the four accumulations:
# FLOP per pair from the FP64 VALU counters of each alpha (2 FMA + MUL + ADD +
# TRANS; at alpha = 500 36.3 v_fma, 17.1 v_mul, 4.0 v_add, 2.0 v_rsq),
# profiles/far_grad_fp64_starfish4096_grid512_valu_f64.txt
FLOP_PER_PAIR_GRAD = {5.0: 116.8, 50.0: 98.5, 500.0: 95.6}
# modified-Stokes double layer (2x2 stresslet per pair): K0 and K1(z)/r from
# the class table's fine piece, alpha K1/r, 1/r^2, the closed forms of
# alpha^2 T1, alpha^4 T2, alpha^2 T3 (App. B) and the contraction D_ij w mu_j
# into two accumulators (z <= 2: the fitted smooth parts with log z): counted
# per alpha (at alpha = 500 45.3 v_fma, 34.1 v_mul, 6.0 v_add, 2.0 v_rsq)
FLOP_PER_PAIR_STOKES = {5.0: 158.7, 50.0: 135.8, 500.0: 132.7}
# target gradient of the stresslet double layer (velocity gradient, 4 outputs):
# the same K0, K1(z)/r, 1/r^2 and A_k, B_k = A_k'(r)/r from K0 and A_k, and the
# contraction d_l D_ij w mu_j into four accumulators: counted per alpha (at
# alpha = 500 64.3 v_fma, 49.2 v_mul, 9.0 v_add, 2.0 v_rsq)
FLOP_PER_PAIR_STOKES_GRAD = {5.0: 228.4, 50.0: 192.3, 500.0: 188.8}
# launch shapes (far-field source splits) chosen by the autotuner on MI355X for
# the plans of this benchmark
TUNED_SPLITS = os.path.join(ROOT, "paper_1908_07392_amd", "tuning", "mi355x_far_splits.json")
# HBM bytes per fused FP64 evaluation (FETCH_SIZE + WRITE_SIZE of far_eval_fp64
# and far_sk_finalize, each scaled by the same counter's reading for a plain
# 256 MiB copy), averaged over the three alphas, for the current kernels and
# launch shape (one stream launch of 4 x the resident blocks, numbered XCD by
# XCD) (profiles/far_eval_fp64_starfish4096_grid512_hbm_bytes.txt)
PROFILED_TRAFFIC = 49100000


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--grid", type=int, default=512)
    ap.add_argument("--cpu-seconds", type=float, default=25.0,
                    help="budget of the oracle CPU baseline (the whole config-2 evaluation takes ~18 s on 16 cores)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the batched, volume, warm-start and gradient legs")
    ap.add_argument("--legs", default="batched,volume,warm,gradient,stokes,fmm,step",
                    help="comma list of the extra legs to run (batched, volume, warm, gradient, stokes, fmm, step)")
    ap.add_argument("--tune-cache", default=TUNED_SPLITS,
                    help="JSON cache of the autotuned launch shapes (read; plans missing from it are tuned afresh)")
    ap.add_argument("--tune-write", action="store_true", help="add freshly tuned plans to the cache file")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(cfg, alpha, budget_s):
    """Oracle (FP64, OpenMP) SLP+DLP at the same targets, in random chunks of
    2048 until all are done or the budget is spent (then a bounded sample)."""
    import oracle
    g = cfg["geom"]
    rng = np.random.default_rng(7)
    sigma = np.cos(3 * g.theta)
    order = rng.permutation(len(cfg["tx"]))
    done, pairs, t_used = 0, 0, 0.0
    chunk = 2048
    while t_used < budget_s and done < len(order):
        idx = order[done:done + chunk]
        t0 = time.perf_counter()
        oracle.eval_potentials(g.x, g.y, alpha, cfg["tx"][idx], cfg["ty"][idx], sigma=sigma, mu=sigma)
        t_used += time.perf_counter() - t0
        done += len(idx)
        pairs += len(idx) * g.n_nodes
    return dict(value=pairs / t_used / 1e9, unit="GPair-evals/s", cores=oracle.max_threads(), kind="oracle",
                sample=(f"all {done} targets" if done == len(order) else f"{done} random targets") +
                       f" of the {len(cfg['tx'])} x {g.n_nodes} SLP+DLP evaluation at alpha={alpha:g} "
                       f"({pairs:.3g} pairs, {t_used:.1f} s)")


def cpu_baseline_legs(cfg2, wl):
    """The oracle on the other workloads, each in full or on its stated sample:
    the circle evaluation (all 2828 targets), GMRES to 1e-10 on the circle and
    on the starfish at alpha = 50 (dense oracle operator, assembly and solve
    timed separately), and the volume sum at the 2048-target sample."""
    import oracle
    legs = {}
    c1 = wl.config1()
    g1 = c1["geom"]
    t0 = time.perf_counter()
    oracle.eval_potentials(g1.x, g1.y, c1["alpha"], c1["tx"], c1["ty"], sigma=c1["sigma"], mu=c1["sigma"])
    dt = time.perf_counter() - t0
    legs["circle_eval"] = {"gpair_per_s": round(len(c1["tx"]) * g1.n_nodes / dt / 1e9, 5), "s": round(dt, 3),
                           "pairs": len(c1["tx"]) * g1.n_nodes}
    for name, geom, alpha, rhs in (("circle_gmres", g1, c1["alpha"], c1["sigma"]),
                                   ("starfish_gmres_alpha50", cfg2["geom"], 50.0, cfg2["data"][50.0]["g"])):
        t0 = time.perf_counter()
        _, D = oracle.onsurface_matrices(geom.x, geom.y, alpha)
        A = D + 0.5 * np.eye(geom.n_nodes)
        t1 = time.perf_counter()
        _, info = oracle.gmres(A, rhs, tol=1e-10)
        t2 = time.perf_counter()
        legs[name] = {"n": geom.n_nodes, "alpha": alpha, "assembly_s": round(t1 - t0, 3), "gmres_ms": round((t2 - t1) * 1e3, 2),
                      "iters": info["iters"], "residual": info["relres"]}
    c3 = wl.config3()
    t0 = time.perf_counter()
    oracle.volume_eval(c3["x"], c3["y"], c3["w"], c3["f"], c3["alpha"], c3["h"], c3["sample"])
    dt = time.perf_counter() - t0
    pairs3 = len(c3["sample"]) * c3["x"].size
    legs["volume_sample"] = {"gpair_per_s": round(pairs3 / dt / 1e9, 5), "s": round(dt, 3), "pairs": pairs3}
    return legs


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_1908_07392_amd import mhlp
    from paper_1908_07392_amd import workloads as wl

    dev = "cuda:0"
    torch.cuda.set_device(0)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)  # noqa: E731
    cfg = wl.config2(grid=args.grid)
    g = cfg["geom"]
    N, M = g.n_nodes, len(cfg["tx"])
    G = mhlp.Geometry(t(g.node_soa()))
    tx, ty = t(cfg["tx"]), t(cfg["ty"])
    plans = {}
    t0 = time.perf_counter()
    for a in cfg["alphas"]:
        print(f"# building plans alpha={a:g}", file=sys.stderr, flush=True)
        plans[a] = (mhlp.Plan(G, a), mhlp.Plan(G, a, tx, ty))
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    gdev = {a: t(cfg["data"][a]["g"]) for a in cfg["alphas"]}
    # launch shape of every plan from the autotuner (untimed set-up)
    from paper_1908_07392_amd import autotune
    tuned = {}
    for a in cfg["alphas"]:
        on, off = plans[a]
        kw = dict(use_cache=True, path=args.tune_cache, write=args.tune_write)
        # the FP64 operator and evaluation do not use source splits (symmetric
        # tiles; stream of (target block, panel) units): the splits serve the
        # mixed-precision leg's operator and evaluation, tuned for those
        r_on = autotune.tune(on, "bie", precision=mhlp.MIXED, reps=5, **kw)
        r_off = autotune.tune(off, "both", precision=mhlp.MIXED, reps=5, **kw)
        tuned[f"alpha={a:g}"] = {"bie_nsplit": r_on["nsplit"], "eval_nsplit": r_off["nsplit"],
                                 "from_cache": bool(r_on["cached"] and r_off["cached"])}
    print(f"# autotuned splits {tuned}", file=sys.stderr, flush=True)
    print(f"# plans built in {plan_ms:.0f} ms; near pairs "
          + ", ".join(f"alpha={a:g}: {plans[a][0].n_near_pairs}/{plans[a][1].n_near_pairs}" for a in cfg["alphas"]),
          file=sys.stderr, flush=True)

    stats = {}
    events = []  # (alpha, start, end) around every fused evaluation of the timed region

    def step(record=False):
        pairs = [0, 0]  # kernel evaluations, pair terms
        for a in cfg["alphas"]:
            on, off = plans[a]
            if record:
                torch.cuda.synchronize()  # attribute the previous evaluation to its own step
            t1 = time.perf_counter()
            mu, info = mhlp.gmres_solve(on, gdev[a], tol=1e-10, max_iter=400, restart=200)
            t2 = time.perf_counter()
            if record:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
            us, ud = mhlp.eval_layer(off, sigma=mu, mu=mu)
            if record:
                e1.record()
                events.append((a, e0, e1))
                stats.setdefault(a, []).append(dict(gmres_ms=(t2 - t1) * 1e3, iters=info["iters"],
                                                    residual=info["rel_residual"]))
            # operator applications of a zero-guess solve: one per Arnoldi step and
            # one true-residual check per cycle (the first residual is g itself);
            # the FP64 operator evaluates each unordered pair once (N(N-1)/2
            # kernel evaluations give its N^2 terms)
            napp = info["iters"] + info["restarts"]
            pairs[0] += napp * (N * (N - 1) // 2) + M * N
            pairs[1] += napp * N * N + M * N
        return pairs

    for _ in range(args.warmup):
        print("# warmup step", file=sys.stderr, flush=True)
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_pairs, total_terms = 0, 0
    for _ in range(args.steps):
        p_ev, p_terms = step(record=True)
        total_pairs += p_ev
        total_terms += p_terms
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    value = total_pairs / elapsed / 1e9

    # dominant kernel: fused SLP+DLP far-field evaluation at the targets; HIP events
    # on the launch stream around each evaluation of the timed region
    per_a = {}
    for a, e0, e1 in events:
        per_a.setdefault(a, []).append(e0.elapsed_time(e1))
    launch_ms = float(np.mean([v for a in per_a for v in per_a[a]]))
    eval_pairs = M * N
    # FLOPs and VALU instructions of every timed launch over the sum of their durations
    t_sum = sum(sum(v) for v in per_a.values()) * 1e-3
    flops = sum(len(v) * eval_pairs * FLOP_PER_PAIR_FP64[a] for a, v in per_a.items())
    valus = sum(len(v) * eval_pairs * VALU_PER_PAIR_FP64[a] for a, v in per_a.items())
    achieved_tf = flops / t_sum / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved_tf, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved_tf / FP64_PEAK_TFLOPS, 4),
                "traffic": PROFILED_TRAFFIC,
                "kernel": "far_eval_fp64<SLP,DLP> + far_sk_finalize",
                "launch_ms": round(launch_ms, 4),
                "launch_ms_by_alpha": {f"alpha={a:g}": round(float(np.mean(v)), 4) for a, v in per_a.items()},
                "pairs_per_launch": eval_pairs,
                "flop_per_pair_by_alpha": {f"alpha={a:g}": f for a, f in FLOP_PER_PAIR_FP64.items()},
                "eval_gpair_per_s": round(eval_pairs / (launch_ms * 1e-3) / 1e9, 3),
                "valu_per_pair_by_alpha": {f"alpha={a:g}": f for a, f in VALU_PER_PAIR_FP64.items()},
                "valu_issue_frac": round(valus / t_sum / VALU_ISSUE_PER_S, 4)}
    a_r = 50.0
    on, off = plans[a_r]
    mu, _ = mhlp.gmres_solve(on, gdev[a_r], tol=1e-10)
    reps = 20
    # context: the same evaluation launched back to back (steady clocks), alpha = 50
    mhlp.eval_layer(off, sigma=mu, mu=mu)
    eb0, eb1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    eb0.record()
    for _ in range(reps):
        mhlp.eval_layer(off, sigma=mu, mu=mu)
    eb1.record()
    torch.cuda.synchronize()
    roofline["back_to_back_launch_ms_alpha50"] = round(eb0.elapsed_time(eb1) / reps, 4)

    gm = {f"alpha={a:g}": {"gmres_ms": round(float(np.median([s["gmres_ms"] for s in stats[a]])), 3),
                           "iters": stats[a][-1]["iters"], "residual": stats[a][-1]["residual"]}
          for a in cfg["alphas"]}
    out = {"metric": METRIC, "value": round(value, 4), "unit": "GPair-evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"starfish 256x16 (N={N}), alpha 5/50/500, GMRES to 1e-10 + SLP+DLP at {M} "
                                  f"interior targets of a {args.grid}^2 grid",
                      "n_sources": N, "n_targets": M, "alphas": list(cfg["alphas"]), "precision": "fp64"},
           "pair_terms_per_s": round(total_terms / elapsed / 1e9, 4),
           "gmres": gm, "plan_build_ms": round(plan_ms, 1), "autotune": tuned, "roofline": roofline}
    # ---- mixed precision (FP32 far field, FP64 near/identity/Arnoldi, GMRES-IR) on the same step
    def mixed_step():
        tm = {}
        for a in cfg["alphas"]:
            on, off = plans[a]
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            mu_m, info_m = mhlp.gmres_solve(on, gdev[a], tol=1e-10, max_iter=400, restart=200, precision=mhlp.MIXED)
            t2 = time.perf_counter()
            mhlp.eval_layer(off, sigma=mu_m, mu=mu_m, precision=mhlp.MIXED)
            tm[a] = ((t2 - t1) * 1e3, info_m)
        return tm

    mixed_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tm = mixed_step()
    torch.cuda.synchronize()
    ms_mixed = (time.perf_counter() - t0) * 1e3 / args.steps
    mu64, _ = mhlp.gmres_solve(on, gdev[a_r], tol=1e-10)
    us64, ud64 = mhlp.eval_layer(off, sigma=mu64, mu=mu64)
    us32, ud32 = mhlp.eval_layer(off, sigma=mu64, mu=mu64, precision=mhlp.MIXED)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        mhlp.eval_layer(off, sigma=mu64, mu=mu64, precision=mhlp.MIXED)
    ev1.record()
    torch.cuda.synchronize()
    mixed_launch_ms = ev0.elapsed_time(ev1) / reps
    err_m = max(float((us32 - us64).abs().max() / us64.abs().max()), float((ud32 - ud64).abs().max() / ud64.abs().max()))
    out["mixed"] = {"ms_per_step": round(ms_mixed, 3), "speedup_vs_fp64": round(ms_per_step / ms_mixed, 3),
                    "eval_launch_ms": round(mixed_launch_ms, 4),
                    "eval_speedup_vs_fp64": round(launch_ms / mixed_launch_ms, 3),
                    "eval_gpair_per_s": round(eval_pairs / (mixed_launch_ms * 1e-3) / 1e9, 3),
                    "eval_max_rel_err_vs_fp64": err_m,
                    "gmres": {f"alpha={a:g}": {"gmres_ms": round(tm[a][0], 3), "iters": tm[a][1]["iters"],
                                               "refinements": tm[a][1]["restarts"],
                                               "residual": tm[a][1]["rel_residual"]} for a in cfg["alphas"]}}

    if args.copy_calibration:
        nbytes = 256 << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"bytes_read": nbytes, "bytes_written": nbytes, "launches": 3}
    legs = set() if args.no_extra else set(args.legs.split(","))
    if "batched" in legs:
        out["batched"] = bench_batched(mhlp, wl, t, torch)
    if "volume" in legs:
        out["volume"] = bench_volume(mhlp, wl, t, torch)
    if "warm" in legs:
        out["warm_start"] = bench_warm(mhlp, wl, t, torch)
    if "gradient" in legs:
        out["gradient"] = bench_grad(mhlp, plans, gdev, cfg, args, torch)
    if "stokes" in legs:
        out["stokes"] = bench_stokes(mhlp, wl, cfg, G, tx, ty, t, args, torch)
    if "fmm" in legs:
        out["fmm"] = bench_fmm(mhlp, wl, plans, gdev, cfg, G, tx, ty, t, torch)
    if "step" in legs:
        out["implicit_step"] = bench_step(mhlp, wl, cfg, G, t, torch)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, 50.0, args.cpu_seconds)
        out["cpu_baseline"]["legs"] = cpu_baseline_legs(cfg, wl)
    print(json.dumps(out), flush=True)


def _event_ms(torch, fn, reps):
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_fmm(mhlp, wl, plans, gdev, cfg, G, tx, ty, t, torch):
    """FMM far field (order 40, the paper's) against the direct tile sums on the
    same inputs: the fused SLP+DLP evaluation of the solved densities at the
    109,314 config-2 targets per alpha (own FMM plans, automatic leaf level), and
    the config-3 volume sum (65,536 points, 4.3e9 pairs).  Times per evaluation
    with HIP events; the tree build is reported separately."""
    print("# fmm leg", file=sys.stderr, flush=True)
    res = {"order": 40, "eval": {}}
    for a in cfg["alphas"]:
        on, off = plans[a]
        mu, _ = mhlp.gmres_solve(on, gdev[a], tol=1e-10)
        P = mhlp.Plan(G, a, tx, ty)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.set_fmm(40)
        build_ms = (time.perf_counter() - t0) * 1e3
        ds, dd = mhlp.eval_layer(off, sigma=mu, mu=mu)
        fs, fd = mhlp.eval_layer(P, sigma=mu, mu=mu)
        diff = max(float((fs - ds).abs().max() / ds.abs().max()), float((fd - dd).abs().max() / dd.abs().max()))
        fms = _event_ms(torch, lambda: mhlp.eval_layer(P, sigma=mu, mu=mu, out_slp=fs, out_dlp=fd), 10)
        dms = _event_ms(torch, lambda: mhlp.eval_layer(off, sigma=mu, mu=mu, out_slp=ds, out_dlp=dd), 10)
        res["eval"][f"alpha={a:g}"] = {"fmm_ms": round(fms, 4), "direct_ms": round(dms, 4),
                                       "speedup": round(dms / fms, 2), "leaf_level": P.fmm[1],
                                       "tree_build_ms": round(build_ms, 1), "max_rel_diff": diff}
    c = wl.config3()
    x, y, w, f = (t(c[k]) for k in ("x", "y", "w", "f"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    V = mhlp.VolumeFMM(x, y, w, c["alpha"], c["h"], order=40)
    build_ms = (time.perf_counter() - t0) * 1e3
    u = V.eval(f)
    ud, _ = mhlp.volume_eval(x, y, w, f, c["alpha"], c["h"])
    fms = _event_ms(torch, lambda: V.eval(f, out=u), 10)
    dms = _event_ms(torch, lambda: mhlp.volume_eval(x, y, w, f, c["alpha"], c["h"], out=ud), 3)
    res["volume"] = {"fmm_ms": round(fms, 4), "direct_ms": round(dms, 4), "speedup": round(dms / fms, 2),
                     "leaf_level": V.leaf_level, "tree_build_ms": round(build_ms, 1),
                     "max_rel_diff": float((u - ud).abs().max() / ud.abs().max()),
                     "gpair_equiv_per_s": round(c["x"].size ** 2 / (fms * 1e-3) / 1e9, 1)}
    return res


def bench_step(mhlp, wl, cfg, G, t, torch):
    """One implicit modified-Stokes step on the starfish (N = 4096): the particular
    solution of a smooth forcing on the periodic box [-1.6, 1.6)^2 with a 512^2
    grid (u, its gradient and the values at the 4096 boundary nodes), GMRES for
    (1/2 I + D + W) mu = g - u^P on the 8192 unknowns to 1e-10, and the double
    layer at the interior grid points; per alpha, after one untimed warm-up step."""
    print("# implicit step leg", file=sys.stderr, flush=True)
    g = cfg["geom"]
    M, x0, Lb = 512, -1.6, 3.2
    gx = x0 + np.arange(M) * Lb / M
    X, Y = np.meshgrid(gx, gx, indexing="xy")
    th = np.arctan2(Y, X)
    inside = np.hypot(X, Y) < 1.0 + 0.3 * np.cos(5 * th)
    ix = np.flatnonzero(inside.ravel())
    rng = np.random.default_rng(77)
    F = np.zeros((2, M, M))
    for _ in range(6):
        c = rng.uniform(-0.5, 0.5, 2)
        bump = np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2) / (2 * 0.15 ** 2))
        F[0] += rng.standard_normal() * bump
        F[1] += rng.standard_normal() * bump
    Fd = t(F)
    nx_, ny_ = t(g.x), t(g.y)
    gb = t(np.stack([np.cos(g.theta), np.sin(2 * g.theta)]))
    tx, ty = t(X.ravel()[ix]), t(Y.ravel()[ix])
    res = {"grid": M, "interior_points": int(ix.size), "by_alpha": {}}
    for a in cfg["alphas"]:
        box = mhlp.Box(M, x0, x0, Lb, a)
        on = mhlp.Plan(G, a, stokes=True)
        off = mhlp.Plan(G, a, tx, ty, stokes=True)

        def step():
            u, gr, ub = box.particular(Fd, want_u=True, want_grad=True, px=nx_, py=ny_)
            mu, info = mhlp.stokes_gmres_solve(on, gb - ub, tol=1e-10, restart=200)
            return u, gr, mhlp.stokes_eval(off, mu), info

        step()
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        t0 = time.perf_counter()
        e[0].record()
        u, gr, ub = box.particular(Fd, want_u=True, want_grad=True, px=nx_, py=ny_)
        e[1].record()
        mu, info = mhlp.stokes_gmres_solve(on, gb - ub, tol=1e-10, restart=200)
        e[2].record()
        uh = mhlp.stokes_eval(off, mu)
        e[3].record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        res["by_alpha"][f"alpha={a:g}"] = {"particular_ms": round(e[0].elapsed_time(e[1]), 3),
                                           "gmres_ms": round(e[1].elapsed_time(e[2]), 3), "iters": info["iters"],
                                           "eval_ms": round(e[2].elapsed_time(e[3]), 3), "step_ms": round(wall, 3)}
    # SISDC time steps of periodic Navier-Stokes on the same 512^2 grid (Re = 100,
    # dt = 0.01, orders K = 2 and 3: 2 and 6 implicit solves per step)
    Re, dtn = 100.0, 0.01
    gp = np.arange(M) * 2 * np.pi / M
    Xp, Yp = np.meshgrid(gp, gp, indexing="xy")
    u0 = np.stack([np.sin(Xp) * np.cos(2 * Yp), -0.5 * np.cos(Xp) * np.sin(2 * Yp)])
    g0 = np.stack([np.cos(Xp) * np.cos(2 * Yp), -2 * np.sin(Xp) * np.sin(2 * Yp), 0.5 * np.sin(Xp) * np.sin(2 * Yp),
                   -np.cos(Xp) * np.cos(2 * Yp)])
    res["sisdc_periodic"] = {"grid": M, "Re": Re, "dt": dtn}
    for K in (2, 3):
        box = mhlp.Box(M, 0.0, 0.0, 2 * np.pi, np.sqrt(Re * (K - 1) / dtn))
        u, gr, L = t(u0), t(g0), t(-5.0 * u0)
        box.sisdc_step(Re, dtn, K, u, gr, L)
        ms = _event_ms(torch, lambda: box.sisdc_step(Re, dtn, K, u, gr, L), 5)
        res["sisdc_periodic"][f"K={K}"] = {"ms_per_step": round(ms, 3), "implicit_solves": (K - 1) * K}
    return res


def bench_batched(mhlp, wl, t, torch):
    """64 geometries x 4 right-hand sides, GMRES to 1e-10: one batched solve vs the
    same 256 solves one by one (FP64 both)."""
    print("# batched leg", file=sys.stderr, flush=True)
    items = wl.config4()
    t0 = time.perf_counter()
    plans = []
    for it in items:
        G = mhlp.Geometry(t(it["geom"].node_soa()))
        plans.append(mhlp.Plan(G, it["alpha"]))
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    B = mhlp.Batch(plans, 4)
    target, _ = B.autotune(reps=3)
    tile = B.tile()
    rhs = [t(it["rhs"][r]) for it in items for r in range(4)]
    gb = B.pack(rhs)
    B.gmres(gb, tol=1e-10)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mu, infos = B.gmres(gb, tol=1e-10)
    torch.cuda.synchronize()
    batched_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    seq_iters = 0
    k = 0
    for p in plans:
        for r in range(4):
            _, inf = mhlp.gmres_solve(p, rhs[k], tol=1e-10, restart=64)
            seq_iters += inf["iters"]
            k += 1
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - t0) * 1e3
    n_nodes = sum(it["geom"].n_nodes for it in items)
    return {"systems": len(infos), "total_nodes": n_nodes, "plan_build_ms": round(plan_ms, 1), "block_target": target,
            "targets_per_lane": tile["targets_per_lane"], "sources_per_stage": tile["sources_per_stage"],
            "tile_candidates_ms": {f"{c[1]}x{c[2]}@{c[0]}": round(c[3], 3) for c in tile["candidates"]},
            "batched_ms": round(batched_ms, 2), "sequential_ms": round(seq_ms, 2),
            "speedup_vs_sequential": round(seq_ms / batched_ms, 2),
            "all_converged": all(i["converged"] for i in infos),
            "max_residual": max(i["rel_residual"] for i in infos),
            "max_iters": max(i["iters"] for i in infos), "sequential_total_iters": seq_iters}


def bench_grad(mhlp, plans, gdev, cfg, args, torch):
    """Target gradients grad S[mu] and grad D[mu] (both, one launch) of the solved
    density at the 109,314 interior grid targets, FP64, per alpha: first call
    (builds the 64 gradient weights per near pair) and the steady launch."""
    print("# gradient leg", file=sys.stderr, flush=True)
    from paper_1908_07392_amd import autotune
    res = {"flop_per_pair_by_alpha": {f"alpha={a:g}": f for a, f in FLOP_PER_PAIR_GRAD.items()}}
    launch = {}
    for a in cfg["alphas"]:
        on, off = plans[a]
        mu, _ = mhlp.gmres_solve(on, gdev[a], tol=1e-10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mhlp.eval_grad(off, sigma=mu, mu=mu)
        torch.cuda.synchronize()
        build_ms = (time.perf_counter() - t0) * 1e3
        r = autotune.tune(off, "grad", reps=5, use_cache=True, path=args.tune_cache, write=args.tune_write)
        reps = 10
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        mhlp.eval_grad(off, sigma=mu, mu=mu)
        e0.record()
        for _ in range(reps):
            mhlp.eval_grad(off, sigma=mu, mu=mu)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        launch[f"alpha={a:g}"] = {"launch_ms": round(ms, 4), "first_call_ms": round(build_ms, 2),
                                  "nsplit": r["nsplit"], "near_pairs": off.n_near_pairs}
    ms = float(np.mean([v["launch_ms"] for v in launch.values()]))
    pairs = off.n_targets * off.n_sources
    # the counted FLOPs of every alpha's launch over their summed durations
    tf = pairs * sum(FLOP_PER_PAIR_GRAD[a] for a in cfg["alphas"]) / (
        sum(launch[f"alpha={a:g}"]["launch_ms"] for a in cfg["alphas"]) * 1e-3) / 1e12
    res.update({"by_alpha": launch, "pairs_per_launch": pairs, "launch_ms": round(ms, 4),
                "gpair_per_s": round(pairs / (ms * 1e-3) / 1e9, 3), "achieved_tflops": round(tf, 3),
                "frac_of_fp64_peak": round(tf / FP64_PEAK_TFLOPS, 4),
                "kernel": "far_grad_fp64<gradS,gradD> (+ grad_finalize when split)"})
    return res


def bench_stokes(mhlp, wl, cfg, G, tx, ty, t, args, torch):
    """Modified-Stokes double layer (the paper's BIE kernel) on the same starfish and
    targets: Dirichlet data of two exterior point forces (modified stokeslets),
    GMRES for (1/2 I + D + W) mu = g to 1e-10 on the 2N = 8192 unknowns, then
    D[mu] and its target gradient (the velocity gradient) at the 109,314 targets;
    per alpha."""
    print("# stokes leg", file=sys.stderr, flush=True)
    import scipy.special as sp
    from paper_1908_07392_amd import autotune
    g = cfg["geom"]
    sources = [(2.2 + 0.4j, (1.0, 0.3)), (-0.5 - 2.1j, (-0.4, 0.8))]
    res = {"flop_per_pair_by_alpha": {f"alpha={a:g}": f for a, f in FLOP_PER_PAIR_STOKES.items()}}
    by = {}
    for a in cfg["alphas"]:
        gb = np.zeros((2, g.n_nodes))
        for x0, F in sources:
            rx, ry = g.x - x0.real, g.y - x0.imag
            z = a * np.hypot(rx, ry)
            K0, K1 = sp.k0(z), sp.k1(z)  # underflow to 0 at large alpha: the 1/z^2 parts remain
            S1 = (z * z * K0 + z * K1 - 1) / (2 * np.pi * z * z)
            S2 = -(z * z * K0 + 2 * z * K1 - 2) / (2 * np.pi * z ** 4)
            rF = rx * F[0] + ry * F[1]
            gb += np.array([S1 * F[0] + a * a * S2 * rx * rF, S1 * F[1] + a * a * S2 * ry * rF])
        gb /= np.abs(gb).max()
        gd = t(gb)
        t0 = time.perf_counter()
        on = mhlp.Plan(G, a, stokes=True)
        off = mhlp.Plan(G, a, tx, ty, stokes=True)
        torch.cuda.synchronize()
        build_ms = (time.perf_counter() - t0) * 1e3
        kw = dict(use_cache=True, path=args.tune_cache, write=args.tune_write)
        r_on = autotune.tune(on, "stokes", reps=3, **kw)
        r_off = autotune.tune(off, "stokes", reps=3, **kw)
        mhlp.stokes_gmres_solve(on, gd, tol=1e-10, restart=200)  # warm-up (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mu, info = mhlp.stokes_gmres_solve(on, gd, tol=1e-10, restart=200)
        torch.cuda.synchronize()
        gm_ms = (time.perf_counter() - t0) * 1e3
        mhlp.stokes_eval(off, mu)
        reps = 10
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            mhlp.stokes_eval(off, mu)
        e1.record()
        torch.cuda.synchronize()
        eval_ms = e0.elapsed_time(e1) / reps
        # velocity gradient of the same flow at the same targets: first call
        # (builds the 128 gradient weights per near pair), then steady launches
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mhlp.stokes_eval_grad(off, mu)
        torch.cuda.synchronize()
        gbuild_ms = (time.perf_counter() - t0) * 1e3
        r_g = autotune.tune(off, "stokes_grad", reps=3, **kw)
        mhlp.stokes_eval_grad(off, mu)
        e0.record()
        for _ in range(reps):
            mhlp.stokes_eval_grad(off, mu)
        e1.record()
        torch.cuda.synchronize()
        by[f"alpha={a:g}"] = {"gmres_ms": round(gm_ms, 3), "iters": info["iters"], "residual": info["rel_residual"],
                              "eval_launch_ms": round(eval_ms, 4), "plans_ms": round(build_ms, 1),
                              "nsplit_bie": r_on["nsplit"], "nsplit_eval": r_off["nsplit"],
                              "grad_launch_ms": round(e0.elapsed_time(e1) / reps, 4),
                              "grad_first_call_ms": round(gbuild_ms, 2), "nsplit_grad": r_g["nsplit"]}
    ms = float(np.mean([v["eval_launch_ms"] for v in by.values()]))
    gms = float(np.mean([v["grad_launch_ms"] for v in by.values()]))
    pairs = off.n_targets * off.n_sources
    al = [float(k.split("=")[1]) for k in by]
    tf = pairs * sum(FLOP_PER_PAIR_STOKES[a] for a in al) / (sum(v["eval_launch_ms"] for v in by.values()) * 1e-3) / 1e12
    gtf = pairs * sum(FLOP_PER_PAIR_STOKES_GRAD[a] for a in al) / (
        sum(v["grad_launch_ms"] for v in by.values()) * 1e-3) / 1e12
    res.update({"by_alpha": by, "pairs_per_launch": pairs, "eval_launch_ms": round(ms, 4),
                "eval_gpair_per_s": round(pairs / (ms * 1e-3) / 1e9, 3), "achieved_tflops": round(tf, 3),
                "frac_of_fp64_peak": round(tf / FP64_PEAK_TFLOPS, 4),
                "kernel": "far_stokes_fp64 (+ stk_finalize when split)",
                "grad": {"flop_per_pair_by_alpha": {f"alpha={a:g}": f for a, f in FLOP_PER_PAIR_STOKES_GRAD.items()},
                         "launch_ms": round(gms, 4),
                         "gpair_per_s": round(pairs / (gms * 1e-3) / 1e9, 3), "achieved_tflops": round(gtf, 3),
                         "frac_of_fp64_peak": round(gtf / FP64_PEAK_TFLOPS, 4),
                         "kernel": "far_stokes_grad_fp64 (+ stkg_finalize when split)"}})
    return res


def bench_volume(mhlp, wl, t, torch):
    """256^2 grid all-pairs K0 sum (4.3e9 pairs) with self-cell correction."""
    print("# volume leg", file=sys.stderr, flush=True)
    c = wl.config3()
    x, y, w, f = t(c["x"]), t(c["y"]), t(c["w"]), t(c["f"])
    res = {}
    for name, prec in (("fp64", mhlp.FP64), ("mixed", mhlp.MIXED)):
        u, _ = mhlp.volume_eval(x, y, w, f, c["alpha"], c["h"], precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            u, _ = mhlp.volume_eval(x, y, w, f, c["alpha"], c["h"], precision=prec)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        res[name] = {"ms": round(ms, 3), "gpair_per_s": round(len(c["x"]) ** 2 / (ms * 1e-3) / 1e9, 2)}
        res.setdefault("_u", {})[name] = u
    d = res.pop("_u")
    res["mixed_max_rel_err_vs_fp64"] = float((d["mixed"] - d["fp64"]).abs().max() / d["fp64"].abs().max())
    res["pairs"] = len(c["x"]) ** 2
    return res


def bench_warm(mhlp, wl, t, torch):
    """Multiply connected time series (outer circle + 3 starfish holes, 14,336 nodes,
    alpha 30, 200 steps): train the learned initial guess on the densities of steps
    1-100, then solve steps 101-200 to 1e-10 from five initial guesses (zero, the
    previous density, cubic extrapolation of the last four, the fitted recurrence
    alone, and the recurrence with the trained network)."""
    print("# warm-start leg", file=sys.stderr, flush=True)
    cfg = wl.config5()
    geom = cfg["geom"]
    plan = mhlp.Plan(mhlp.Geometry(t(geom.node_soa())), cfg["alpha"])
    g = t(cfg["g"])
    kw = dict(tol=1e-10, restart=100, max_iter=400)
    mus = []
    x0 = None
    for s in range(100):
        mu, _ = mhlp.gmres_solve(plan, g[s], x0=x0, **kw)
        mus.append(mu)
        x0 = mu
    # the model: per-coefficient recurrence fitted to the training densities
    # (base) and the network trained on what the recurrence leaves
    W = mhlp.WarmStart(t(geom.theta), t(geom.theta_w), geom.curve_node_ptr, n_modes=128, n_hist=4,
                       base_order=mhlp.WARM_RECURRENCE, width=256, seed=5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = W.train(torch.stack(mus).contiguous(), iters=2000, lr=1e-3)
    train_ms = (time.perf_counter() - t0) * 1e3
    # the same recurrence with a zero network: what the network itself adds
    R = mhlp.WarmStart(t(geom.theta), t(geom.theta_w), geom.curve_node_ptr, n_modes=128, n_hist=4,
                       base_order=mhlp.WARM_RECURRENCE, width=256, seed=5)
    R.train(torch.stack(mus).contiguous(), iters=0)
    R.mlp.set_params(torch.zeros(R.mlp.n_params, dtype=torch.float32, device=mus[0].device))
    hist = torch.stack(mus[-4:]).contiguous()

    def guess(kind):
        if kind == "zero":
            return None
        if kind == "previous":
            return hist[-1]
        if kind == "cubic":
            return 4 * hist[-1] - 6 * hist[-2] + 4 * hist[-3] - hist[-4]
        if kind == "recurrence":
            return R.predict(hist)
        return W.predict(hist)

    kinds = ("zero", "previous", "cubic", "recurrence", "learned")
    rec = {k: dict(iters=[], ms=[], res=[], x0res=[], used=[]) for k in kinds}
    pred_ms = []
    for s in range(100, 200):
        mu_true = None
        for k in kinds:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            x0 = guess(k)
            if k == "learned":
                torch.cuda.synchronize()
                pred_ms.append((time.perf_counter() - t1) * 1e3)
            mu, info = mhlp.gmres_solve(plan, g[s], x0=x0, **kw)
            torch.cuda.synchronize()
            r = rec[k]
            r["ms"].append((time.perf_counter() - t1) * 1e3)
            r["iters"].append(info["iters"])
            r["res"].append(info["rel_residual"])
            r["x0res"].append(info["x0_residual"])
            r["used"].append(info["used_x0"])
            if k == "zero":
                mu_true = mu
        hist = torch.cat([hist[1:], mu_true[None]]).contiguous()
    z_ms = float(np.mean(rec["zero"]["ms"]))
    res = {"steps": "101-200", "n_nodes": geom.n_nodes, "train_ms": round(train_ms, 1),
           "train_loss_first_last": [float(losses[0]), float(losses[-1])],
           "predict_ms_mean": round(float(np.mean(pred_ms)), 3)}
    for k in kinds:
        r = rec[k]
        res[k] = {"mean_iters": round(float(np.mean(r["iters"])), 3), "mean_ms": round(float(np.mean(r["ms"])), 3),
                  "speedup_vs_zero": round(z_ms / float(np.mean(r["ms"])), 3),
                  "max_residual": float(np.max(r["res"])),
                  "median_x0_residual": float(np.median(r["x0res"])) if k != "zero" else 1.0,
                  "x0_used": int(np.sum(r["used"])) if k != "zero" else 0}
    return res


if __name__ == "__main__":
    main()
