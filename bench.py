#!/usr/bin/env python3
"""Throughput of the plane-parallel formal solution + two-level ALI step.

One step = one operator-splitting iteration over the whole batch: the formal
solution of every atmosphere (both hemispheres, every angle and frequency,
difference form) fused with the J-bar and Lambda-bar* profile quadratures,
then the float64 source-function update and the per-atmosphere maximum
relative change.  The metric counts formal-solution points per second,
one point = one (depth, angle, frequency) triple with both I+ and I-.

Workload: 512 independent two-level atmospheres, depth points uniform in
48..256 (seed 3), 8 Gauss angles per hemisphere, 1024 frequencies across a
Doppler profile, eps log-uniform in 1e-6..1e-1, per-depth opacity
multipliers lognormal(0, 0.5).  All inputs are synthetic and resident in HBM
before the timed region.

Prints ONE JSON line.  Also reported beside the batched FP32 value: the plain
FP64 GPU path (one FP64 launch pair per atmosphere, no batching or tuning),
the FP32-vs-FP64 difference of the step, the roofline of the dominant kernel
measured with HIP events on its own stream, and the CPU oracle on a bounded
sample of the same workload.
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
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic work of the moments-mode sweep per point, fixed before measuring:
# bytes: q (or dtau) and S read, J - S and 1 - Lambda* written, 4 B each per
# (depth, frequency) in FP32 = 16 B per (d, k) = 16 / na B per point (2 B at na = 8);
# flops: per direction about 1 exp + 18 FP32 flops -> 36 flops + 2 exp per point.
# attainable = min(HBM / bytes, FP32 peak / flops) = min(4.0e12, 4.37e12) pts/s: HBM.
BYTES_PER_DK = 16.0
FLOPS_PER_POINT_ALG = 36.0
# What the fused kernel itself executes (FMA = 2 flops, exp = 1): per hemisphere
# and angle Delta (1), exp (1), 1 - e (1), times mu/dtau (2), D = e D + psi dS (3),
# J and Lambda* accumulations (4) -> 12, both hemispheres 24; and it moves only
# q once per (d, k) plus per-row data: about 0.5 B per point.
FLOPS_PER_POINT = 24.0
PEAK_FP32_VALU_NONPACKED = 78.6   # TFLOP/s: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
PEAK_FP32_VALU_PUBLISHED = 157.3  # TFLOP/s: the published FP32 vector figure (packed FP32, two FMAs per lane)
PEAK_HBM = 8000.0                 # GB/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=64,
                    help="atmospheres in the single-thread CPU sample")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="worker processes of the all-core oracle run (0: the host's CPU share, at most 16)")
    ap.add_argument("--settle-ms", type=float, default=150.0,
                    help="milliseconds of back-to-back steps before the warm-up (clock settle)")
    ap.add_argument("--stat-replays", type=int, default=50,
                    help="launches behind the median / p10 / p90 step and kernel times")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (read + write) 5 times and "
                         "exit: the reference for scaling FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--waves-per-block", type=int, default=0,
                    help="fix the waves per block (disables the autotuner)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--graph-chunk", type=int, default=25,
                    help="ALI iterations per captured graph in the graph-mode timing (0: skip)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic_fs_profile_c3a.json"))
    ap.add_argument("--workload", choices=["c3a", "spherical", "nonlocal", "voigt", "c3b", "adjoint", "vox3d",
                                           "c5"],
                    default="c3a",
                    help="c3a: the plane-parallel batch (default, the headline line); "
                         "spherical: the same batch shape as spheres (1D spherical symmetry); "
                         "nonlocal: c3a with the tri-diagonal approximate operator and Ng; "
                         "voigt: the multilevel atom with depth-dependent Voigt lines")
    ap.add_argument("--voigt-nb", type=int, default=64, help="voigt: atmospheres in the batch")
    ap.add_argument("--c5-steps", type=int, default=3, help="c5: timed multilevel iterations")
    ap.add_argument("--adj-k", type=int, default=16, choices=[1, 8, 16, 32],
                    help="adjoint: layer checkpoint interval")
    ap.add_argument("--conv-tol", type=float, default=1e-6,
                    help="nonlocal: tolerance of the convergence comparison")
    ap.add_argument("--conv-max-iter", type=int, default=4000)
    ap.add_argument("--sph-cpu-sample", type=int, default=8, help="spheres in the CPU sample")
    return ap.parse_args()


def cpu_baseline_one_thread(batch, nsample):
    """The oracle (numpy FP64, single thread) on a bounded sample of the same
    workload: every step of one ALI iteration for `nsample` atmospheres
    spread over the depth-count range."""
    from threadpoolctl import threadpool_limits
    from oracle import ali, formal
    from oracle.quadrature import gauss_legendre01
    order = np.argsort(batch.nd)
    idx = order[np.linspace(0, batch.nb - 1, nsample).astype(int)]
    sub = batch.subset(idx)
    mu, w = gauss_legendre01(sub.na)
    off = sub.off
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        jms = np.zeros(sub.tau.shape[0])
        olb = np.zeros_like(jms)
        S = sub.S_trial
        for b in range(sub.nb):
            s = slice(off[b], off[b + 1])
            out = formal.formal_solution(sub.tau[s], sub.q[s], S[s], mu, w, lower="diffusion",
                                         Bbot=np.full(sub.nf, sub.B[s][-1]),
                                         Bbot_prev=np.full(sub.nf, sub.B[s][-2]))
            Sg = np.broadcast_to(S[s][:, None], out["J"].shape)
            jms[s], olb[s] = ali.profile_moments(out, S[s], Sg, sub.phi, sub.wnu)
        ali.batch_two_level_update(sub.nd, S, sub.B, sub.eps, jms, olb)
        dt = time.perf_counter() - t0
    pts = sub.points
    return {"value": pts / dt, "unit": "pts/s", "cores": 1,
            "sample": f"one ALI step of {sub.nb} of the 512 atmospheres (nd {int(sub.nd.min())}.."
                      f"{int(sub.nd.max())}, {pts} points), numpy FP64, 1 thread, {dt:.1f} s"}


_CPU_BATCH = None


def _cpu_worker_init(seed):
    """Oracle worker (separate process): the same seeded workload, one thread."""
    global _CPU_BATCH
    from threadpoolctl import threadpool_limits
    from paper_0903_1949_amd import workloads as W
    threadpool_limits(limits=1)
    _CPU_BATCH = W.two_level_batch(seed=seed)


def _cpu_worker(idx):
    """Profile moments of the oracle's formal solution for atmospheres idx."""
    from oracle import ali, formal
    from oracle.quadrature import gauss_legendre01
    bt = _CPU_BATCH
    mu, w = gauss_legendre01(bt.na)
    off = bt.off
    t0 = time.perf_counter()
    res = []
    for b in idx:
        s = slice(off[b], off[b + 1])
        S = bt.S_trial[s]
        out = formal.formal_solution(bt.tau[s], bt.q[s], S, mu, w, lower="diffusion",
                                     Bbot=np.full(bt.nf, bt.B[s][-1]),
                                     Bbot_prev=np.full(bt.nf, bt.B[s][-2]))
        jms, olb = ali.profile_moments(out, S, np.broadcast_to(S[:, None], out["J"].shape),
                                       bt.phi, bt.wnu)
        res.append((int(b), jms, olb))
    return res, time.perf_counter() - t0


def cpu_share():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_allcore(batch, seed, nworkers):
    """The oracle on every atmosphere of the batch, spread over `nworkers`
    processes (one thread each, atmospheres dealt longest first), then the
    float64 update: one full ALI step of the workload on the host cores."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    from oracle import ali
    order = [int(b) for b in np.argsort(-batch.nd, kind="stable")]
    chunks = [order[i::nworkers * 4] for i in range(nworkers * 4)]
    with ProcessPoolExecutor(nworkers, mp_context=mp.get_context("spawn"),
                             initializer=_cpu_worker_init, initargs=(seed,)) as ex:
        list(ex.map(_cpu_worker, [[] for _ in range(nworkers)]))       # workers up and initialised
        t0 = time.perf_counter()
        parts = list(ex.map(_cpu_worker, chunks))
        jms = np.zeros(batch.tau.shape[0])
        olb = np.zeros_like(jms)
        off = batch.off
        for res, _ in parts:
            for b, j, o in res:
                jms[off[b]:off[b + 1]] = j
                olb[off[b]:off[b + 1]] = o
        ali.batch_two_level_update(batch.nd, batch.S_trial.copy(), batch.B, batch.eps, jms, olb)
        dt = time.perf_counter() - t0
    busy = sum(t for _, t in parts)
    return {"value": batch.points / dt, "unit": "pts/s", "cores": nworkers, "kind": "oracle",
            "sample": f"one ALI step of all {batch.nb} atmospheres ({batch.points} points), numpy FP64 "
                      f"oracle in {nworkers} processes of one thread each, {dt:.1f} s wall "
                      f"({busy:.1f} s of worker time)",
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def launch_times(fn, n, stream):
    """n back-to-back eager launches of fn with events between them: the
    average (first to last event / n) and the per-launch milliseconds."""
    import torch
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
    torch.cuda.synchronize()
    evs[0].record(stream)
    for i in range(n):
        fn()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(n)])
    return evs[0].elapsed_time(evs[n]) / n, per


def stats_ms(per):
    return {"median": round(float(np.median(per)), 5), "p10": round(float(np.percentile(per, 10)), 5),
            "p90": round(float(np.percentile(per, 90)), 5), "n": int(per.size)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {args.gpus}); the batched path "
              "shards over atmospheres or frequencies without communication but no multi-GPU "
              "run is part of this build", file=sys.stderr)
        sys.exit(2)
    if args.workload == "spherical":
        bench_spherical(args)
        return
    if args.workload == "nonlocal":
        bench_nonlocal(args)
        return
    if args.workload == "voigt":
        bench_voigt(args)
        return
    if args.workload == "c5":
        return bench_c5(args)
    if args.workload == "vox3d":
        bench_vox3d(args)
        return
    if args.workload == "c3b":
        bench_c3b(args)
        return
    if args.workload == "adjoint":
        bench_adjoint(args)
        return
    import torch
    from paper_0903_1949_amd import pprt
    from paper_0903_1949_amd import workloads as W

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 4, "launches": 5}), flush=True)
        return
    batch = W.two_level_batch(seed=3)
    pts = batch.points
    ctx = pprt.Context(0)
    stream = torch.cuda.current_stream()

    # ---------------- batched FP32 path: one ALI step captured in a hipGraph
    plan = pprt.Plan(ctx, batch.nd, batch.na, batch.nf, precision=pprt.FP32,
                     waves_per_block=args.waves_per_block)
    db = pprt.upload_two_level(batch, pprt.FP32)
    db.S.copy_(db.B)
    S0 = db.S.clone()
    mx = torch.zeros(batch.nb, dtype=torch.float64, device="cuda:0")

    def moments():
        plan.two_level_moments(db.tau, db.q, db.S, db.eps, db.B, db.wphi)

    def step():
        moments()
        plan.two_level_update(db.S, db.eps, db.B, db.wphi, mx)

    tune = None
    if not args.no_autotune and not args.waves_per_block:
        # the tuner's ~200 launches also bring the clocks up right before timing
        tune = plan.autotune(db.tau, db.q, db.S, db.eps, db.B, db.wphi, force=True)
    launch = plan.get_launch()
    # The timed steps are one launch of the library's persistent step graph
    # (pprt_two_level_graph_create: the K steps captured once), after the
    # warm-up steps launched as a graph of one step.
    G = max(1, min(args.steps, 4096))
    gG = plan.two_level_graph(db.tau, db.q, db.S, db.eps, db.B, db.wphi, mx, steps=G)
    g1 = plan.two_level_graph(db.tau, db.q, db.S, db.eps, db.B, db.wphi, mx, steps=1)
    # Clock settle: after host-side work the device runs the first ~100
    # sweeps up to 15% slower while its clock ramps; settle_ms of steps
    # back to back (no host synchronisation) bring it to its sustained rate
    # before the warm-up steps and the timed region.
    settle = 0
    if args.settle_ms > 0:
        est_ms = (tune or {}).get("best_ms") or 0.4
        settle = int(math.ceil(args.settle_ms / max(est_ms, 0.05)))
        for _ in range(settle):
            g1.launch()
    for _ in range(args.warmup):
        g1.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps // G):
        gG.launch()
    for _ in range(args.steps % G):
        g1.launch()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    value = pts / (wall / args.steps)
    # per-step and per-kernel spreads: back-to-back eager launches with an
    # event between steps (two small launches per step keep the host ahead)
    _, per_step = launch_times(step, args.stat_replays, stream)
    k_avg, per_k = launch_times(moments, args.stat_replays, stream)

    # ---------------- the same iterations through pprt_two_level_ali in graph mode
    graph = None
    if args.graph_chunk > 0:
        db.S.copy_(S0)
        torch.cuda.synchronize()
        tg = time.perf_counter()
        rep = plan.two_level_ali(db.tau, db.q, db.S, db.eps, db.B, db.wphi, tol=1e-300,
                                 max_iter=args.steps, iters_per_sync=args.graph_chunk,
                                 use_graph=True, raise_not_converged=False)
        torch.cuda.synchronize()
        wg = time.perf_counter() - tg
        graph = {"value": pts * rep["iterations"] / wg, "ms_per_step": wg * 1e3 / rep["iterations"],
                 "iterations": rep["iterations"], "chunk": args.graph_chunk,
                 "desc": "pprt_two_level_ali, chunks of iterations captured once and replayed "
                         "(includes capture, instantiation and a host check per chunk)"}

    # FP32 vs FP64 difference of one step from the same S (not timed)
    db.S.copy_(S0)
    step()
    torch.cuda.synchronize()
    S_fp32_one = db.S.clone()
    plan64 = pprt.Plan(ctx, batch.nd, batch.na, batch.nf, precision=pprt.FP64)
    db64 = pprt.upload_two_level(batch, pprt.FP64)
    db64.S.copy_(S0)
    mx64 = torch.zeros_like(mx)
    plan64.two_level_ali_step(db64.tau, db64.q, db64.S, db64.eps, db64.B, db64.wphi, mx64)
    torch.cuda.synchronize()
    d32 = (S_fp32_one - S0).double()
    d64 = (db64.S - S0)
    rel_step = float(((S_fp32_one - db64.S).abs() / db64.S.abs()).max())
    rel_update = float(((d32 - d64).abs() / torch.clamp(d64.abs(), min=1e-4 * float(d64.abs().max()))).max())

    # ---------------- roofline of the sweep kernel (moments mode)
    k_s = k_avg * 1e-3
    bytes_per_pt = BYTES_PER_DK / batch.na
    pts_per_s = pts / k_s
    attain_hbm = PEAK_HBM * 1e9 / bytes_per_pt
    attain_alu = PEAK_FP32_VALU_PUBLISHED * 1e12 / FLOPS_PER_POINT_ALG
    attainable = min(attain_hbm, attain_alu)
    gbs = pts * bytes_per_pt / k_s / 1e9
    traffic = measured_traffic(args.traffic_json, "fs_diag.hip")
    peaks = ctx.measure_peaks()
    roofline = {"bound": "hbm" if attain_hbm <= attain_alu else "alu",
                "achieved": round(gbs, 1), "peak": PEAK_HBM, "unit": "GB/s",
                "frac": round(pts_per_s / attainable, 4), "traffic": traffic,
                "kernel": "k_fs_profile<float,8>", "kernel_ms": round(k_avg, 5),
                "kernel_ms_stats": stats_ms(per_k),
                "bytes_per_point": bytes_per_pt, "flops_per_point": FLOPS_PER_POINT_ALG,
                "attainable_pts_per_s": attainable, "achieved_pts_per_s": pts_per_s,
                "alu_frac_published": round(pts_per_s * FLOPS_PER_POINT_ALG / (PEAK_FP32_VALU_PUBLISHED * 1e12), 4),
                "alu_frac_nonpacked": round(pts_per_s * FLOPS_PER_POINT_ALG / (PEAK_FP32_VALU_NONPACKED * 1e12), 4),
                "kernel_own_work": {
                    "flops_per_point": FLOPS_PER_POINT,
                    "tflops": round(pts_per_s * FLOPS_PER_POINT / 1e12, 3),
                    "frac_of_nonpacked_valu": round(pts_per_s * FLOPS_PER_POINT / (PEAK_FP32_VALU_NONPACKED * 1e12), 4),
                    "hbm_gbs_measured": round(traffic / k_s / 1e9, 1) if traffic else None},
                "peak_measured": {"fp32_tflops": round(peaks["fp32_tflops"], 2),
                                  "copy_gbs": round(peaks["copy_gbs"], 1)}}

    # ---------------- plain FP64 path: one FP64 launch pair per atmosphere
    fp64 = None
    fp64_batched = None
    if not args.no_fp64:
        off = batch.off
        plans, views = [], []
        for b in range(batch.nb):
            s = slice(int(off[b]), int(off[b + 1]))
            plans.append(pprt.Plan(ctx, batch.nd[b:b + 1], batch.na, batch.nf, precision=pprt.FP64,
                                   waves_per_block=1))
            views.append((db64.tau[s], db64.q[s], db64.S[s], db64.eps[b:b + 1], db64.B[s],
                          mx64[b:b + 1]))
        def step64():
            for p, (tau, q, S, eps, B, m) in zip(plans, views):
                p.two_level_ali_step(tau, q, S, eps, B, db64.wphi, m)
        step64()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.fp64_steps):
            step64()
        torch.cuda.synchronize()
        w64 = (time.perf_counter() - t1) / args.fp64_steps
        fp64 = {"value": pts / w64, "ms_per_step": w64 * 1e3,
                "desc": "FP64 sweep + update, one launch pair per atmosphere, untuned"}
        # the batched step itself in FP64: same plan layout, k_fs_profile<double,8>
        def step64b():
            plan64.two_level_ali_step(db64.tau, db64.q, db64.S, db64.eps, db64.B, db64.wphi, mx64)
        for _ in range(3):
            step64b()
        _, per64 = launch_times(step64b, max(args.fp64_steps, 10), stream)
        fp64_batched = {"value": pts / float(np.median(per64) * 1e-3),
                        "ms_per_step": stats_ms(per64)["median"], "step_ms_stats": stats_ms(per64),
                        "desc": "the same batched step in FP64 (k_fs_profile<double,8>: series for "
                                "thin layers, exp for thick ones; FP64 partials)"}

    cpu = None
    if not args.no_cpu_baseline:
        nw = args.cpu_workers or cpu_share()
        cpu = cpu_baseline_allcore(batch, 3, nw)
        cpu["one_thread"] = cpu_baseline_one_thread(batch, args.cpu_sample)

    line = {
        "metric": "formal-solution depth*angle*freq pts/s, batched FP32 (plain FP64 beside it)",
        "value": value, "unit": "pts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "512 two-level atmospheres, nd U{48..256}, na 8, nf 1024, "
                               "eps 1e-6..1e-1, seed 3 (one ALI step per step: sweep + moments "
                               "+ FP64 update; the timed steps are hipGraph replays)",
                   "graph_steps": G, "settle_steps": settle,
                   "nbatch": batch.nb, "rows": int(batch.nd.sum()), "na": batch.na,
                   "nf": batch.nf, "points_per_step": pts, "seed": 3,
                   "launch": {"waves_per_block": launch[0], "persistent_waves_per_cu": launch[1],
                              "autotune": tune}},
        "step_ms_stats": stats_ms(per_step),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "graph_mode": graph,
        "fp64_plain": fp64,
        "speedup_vs_fp64_plain": (value / fp64["value"]) if fp64 else None,
        "fp64_batched": fp64_batched,
        "speedup_vs_fp64_batched": (value / fp64_batched["value"]) if fp64_batched else None,
        "fp32_vs_fp64": {"S_after_one_step_rel": rel_step, "update_rel": rel_update},
    }
    print(json.dumps(line), flush=True)


# Spherical sweep, FP32 flops per (ray, shell, frequency) crossing: the
# 12 of one direction as above, both directions -> 24; plus, per outward
# segment of a tangent ray, the round trip through its tangent point:
# gamma (1), E^2 (1), e E^2 gamma (2), psi - that (1), alpha (1), the weighted
# term to the next node (2), E <- e E (1), accumulation (1) -> 10.
SPH_FLOPS_PER_POINT = 24.0
SPH_FLOPS_PER_TANGENT_SEGMENT = 10.0


def sph_cpu_baseline(c, S_trial, n_core, nsample):
    """The spherical oracle (numpy FP64, one thread): one ALI step for
    `nsample` spheres spread over the shell-count range."""
    from threadpoolctl import threadpool_limits
    from oracle import spherical
    order = np.argsort(c.nd)
    idx = order[np.linspace(0, c.nb - 1, nsample).astype(int)]
    pts = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for b in idx:
            s = c.rows(int(b))
            spherical.two_level_ali_sph(c.r[s], c.tau[s], c.q[s], c.phi, c.wnu, float(c.eps[b]),
                                        c.B[s], n_core, tol=0.0, max_iter=1, S0=S_trial[s])
            n = int(c.nd[b])
            pts += (n_core * n + n * (n + 1) // 2) * c.nf
        dt = time.perf_counter() - t0
    return {"value": pts / dt, "unit": "pts/s", "cores": 1, "kind": "oracle",
            "sample": f"one ALI step of {len(idx)} of the {c.nb} spheres (nd {int(c.nd[idx].min())}.."
                      f"{int(c.nd[idx].max())}, {pts} points), numpy FP64, 1 thread, {dt:.1f} s"}


def bench_spherical(args):
    """One two-level ALI step over 512 spheres: the ray-group sweep with the
    fused profile quadratures, then the float64 update.  A point is one
    (ray, shell, frequency) crossing, with both the inward and the outward
    intensity."""
    import torch
    from paper_0903_1949_amd import pprt
    from paper_0903_1949_amd import workloads as W

    torch.cuda.set_device(0)
    n_core = 16
    c = W.spherical_batch(nb=512, nd_lo=48, nd_hi=256, nf=1024, n_core=n_core, r_out=2.0,
                          tau_lo=1e-4, tau_hi=1e8, eps_lo=1e-6, eps_hi=1e-1, seed=3)
    nd = c.nd.astype(np.int64)
    pairs = n_core * nd + nd * (nd + 1) // 2
    pts = int(pairs.sum()) * c.nf
    flops = (SPH_FLOPS_PER_POINT * pairs.sum() +
             SPH_FLOPS_PER_TANGENT_SEGMENT * (nd * (nd - 1) // 2).sum()) * c.nf
    S_trial = np.empty_like(c.tau)
    for b in range(c.nb):
        s = c.rows(b)
        e = float(c.eps[b])
        S_trial[s] = 1.0 - (1.0 - math.sqrt(e)) * np.exp(-math.sqrt(3.0 * e) * c.tau[s])
    ctx = pprt.Context(0)
    stream = torch.cuda.current_stream()

    def upload(prec):
        dt = torch.float64 if prec == pprt.FP64 else torch.float32
        dev = lambda a, d: torch.as_tensor(np.ascontiguousarray(a), dtype=d, device="cuda:0")
        return dict(tau=dev(c.tau, torch.float64), q=dev(c.q, dt), eps=dev(c.eps, torch.float64),
                    B=dev(c.B, torch.float64), wphi=dev(c.wnu * c.phi, dt),
                    S=dev(S_trial, torch.float64))

    t_plan = time.perf_counter()
    plan = pprt.SphPlan(ctx, c.nd, c.nf, c.r, n_core, precision=pprt.FP32)
    t_plan = time.perf_counter() - t_plan
    d = upload(pprt.FP32)
    S0 = d["S"].clone()
    mx = torch.zeros(c.nb, dtype=torch.float64, device="cuda:0")

    def step(ev0=None, ev1=None):
        if ev0 is not None:
            ev0.record(stream)
        plan.two_level_moments(d["tau"], d["q"], d["S"], d["eps"], d["B"], d["wphi"])
        if ev1 is not None:
            ev1.record(stream)
        plan.two_level_update(d["S"], d["eps"], d["B"], d["wphi"], mx)

    # FP32 vs FP64 difference of one step from the same S (not timed)
    step()
    torch.cuda.synchronize()
    S32 = d["S"].clone()
    plan64 = pprt.SphPlan(ctx, c.nd, c.nf, c.r, n_core, precision=pprt.FP64)
    d64 = upload(pprt.FP64)
    mx64 = torch.zeros_like(mx)
    plan64.two_level_ali_step(d64["tau"], d64["q"], d64["S"], d64["eps"], d64["B"], d64["wphi"], mx64)
    torch.cuda.synchronize()
    rel_step = float(((S32 - d64["S"]).abs() / d64["S"].abs()).max())
    d["S"].copy_(S0)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in evs:
        step(e0, e1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    k_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
    value = pts / (wall / args.steps)
    print(f"[spherical] {args.steps} steps, {ms_per_step:.3f} ms/step, sweep {k_ms:.3f} ms",
          file=sys.stderr, flush=True)

    fp64 = None
    if not args.no_fp64:
        d64["S"].copy_(S0)
        plan64.two_level_ali_step(d64["tau"], d64["q"], d64["S"], d64["eps"], d64["B"], d64["wphi"], mx64)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.fp64_steps):
            plan64.two_level_ali_step(d64["tau"], d64["q"], d64["S"], d64["eps"], d64["B"],
                                      d64["wphi"], mx64)
        torch.cuda.synchronize()
        w64 = (time.perf_counter() - t1) / args.fp64_steps
        fp64 = {"value": pts / w64, "ms_per_step": w64 * 1e3,
                "desc": "the same step with the FP64 ray-group sweep (series / exp weights)"}

    achieved = flops / (k_ms * 1e-3) / 1e12
    peaks = ctx.measure_peaks()
    traffic = measured_traffic(os.path.join(ROOT, "profiles", "traffic_sph_fast_512spheres.json"), "sph.hip")
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_VALU_NONPACKED,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VALU_NONPACKED, 4),
                "traffic": traffic, "kernel": "k_sph_fast<float,10,true>", "kernel_ms": round(k_ms, 5),
                "hbm_gbs": round(traffic / (k_ms * 1e-3) / 1e9, 1) if traffic else None,
                "flops_per_launch": flops,
                "flops_per_point": SPH_FLOPS_PER_POINT,
                "flops_per_tangent_segment": SPH_FLOPS_PER_TANGENT_SEGMENT,
                "peak_measured": round(peaks["fp32_tflops"], 2),
                "frac_of_measured": round(achieved / peaks["fp32_tflops"], 4),
                "frac_of_published_packed": round(achieved / PEAK_FP32_VALU_PUBLISHED, 4)}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = sph_cpu_baseline(c, S_trial, n_core, args.sph_cpu_sample)
    line = {
        "metric": "spherical formal-solution ray*shell*freq pts/s, batched FP32",
        "value": value, "unit": "pts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "512 two-level spheres (r_out = 2 r_core, tau 1e-4..1e8), nd "
                               "U{48..256}, 16 core rays + one tangent ray per shell, nf 1024, "
                               "eps 1e-6..1e-1, seed 3 (one ALI step per step)",
                   "nbatch": c.nb, "rows": int(nd.sum()), "nf": c.nf, "n_core": n_core,
                   "points_per_step": pts, "seed": 3, "plan_build_s": round(t_plan, 3),
                   "group_size": 10},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp64": fp64,
        "speedup_vs_fp64": (value / fp64["value"]) if fp64 else None,
        "fp32_vs_fp64": {"S_after_one_step_rel": rel_step},
    }
    print(json.dumps(line), flush=True)


# Tri-diagonal sweep, FP32 flops per point: the 24 of the diagonal sweep plus,
# per angle and hemisphere, alpha (1), gamma (1), gamma + e alpha_prev (2) and
# the band accumulation (2) -> 36.
TRI_FLOPS_PER_POINT = 36.0


def nonlocal_cpu_baseline(batch, nsample):
    """The oracle's non-local step (numpy FP64, one thread) on the smallest
    atmospheres of the batch: the band of Lambda from nd unit-column formal
    solutions (its definition), one formal solution, the tri-diagonal solve
    and the Ng bookkeeping."""
    from threadpoolctl import threadpool_limits
    from oracle import ali
    from oracle.quadrature import gauss_legendre01
    idx = np.argsort(batch.nd)[:nsample]
    sub = batch.subset(idx)
    mu, w = gauss_legendre01(sub.na)
    off = sub.off
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for b in range(sub.nb):
            s = slice(off[b], off[b + 1])
            ali.two_level_ali_nonlocal(sub.tau[s], sub.q[s], sub.phi, sub.wnu, float(sub.eps[b]),
                                       sub.B[s], mu, w, tol=0.0, max_iter=1, operator="tri", ng=True,
                                       S0=sub.S_trial[s])
        dt = time.perf_counter() - t0
    pts = sub.points
    return {"value": pts / dt, "unit": "pts/s", "cores": 1, "kind": "oracle",
            "sample": f"one tri-diagonal ALI step of the {sub.nb} smallest of the 512 atmospheres "
                      f"(nd {int(sub.nd.min())}..{int(sub.nd.max())}, {pts} points; the band of Lambda "
                      f"from nd unit-column formal solutions each), numpy FP64, 1 thread, {dt:.1f} s"}


def bench_nonlocal(args):
    """The C3a batch with the tri-diagonal approximate operator and Ng
    acceleration: one ALI step is the sweep with the band quadratures, then
    the float64 tri-diagonal solve and Ng.  Also: iterations and wall time to
    the tolerance with the diagonal and with the tri-diagonal + Ng operator."""
    import torch
    from paper_0903_1949_amd import pprt
    from paper_0903_1949_amd import workloads as W

    torch.cuda.set_device(0)
    batch = W.two_level_batch(seed=3)
    pts = batch.points
    ctx = pprt.Context(0)
    stream = torch.cuda.current_stream()
    plan = pprt.Plan(ctx, batch.nd, batch.na, batch.nf, precision=pprt.FP32)
    plan.set_operator(pprt.LSTAR_TRI, ng=True)
    db = pprt.upload_two_level(batch, pprt.FP32)
    tune = None
    if not args.no_autotune:
        tune = plan.autotune(db.tau, db.q, db.S, db.eps, db.B, db.wphi, force=True)
    launch = plan.get_launch()
    db.S.copy_(db.B)
    plan.two_level_reset()
    mx = torch.zeros(batch.nb, dtype=torch.float64, device="cuda:0")

    def step(ev0=None, ev1=None):
        if ev0 is not None:
            ev0.record(stream)
        plan.two_level_moments(db.tau, db.q, db.S, db.eps, db.B, db.wphi)
        if ev1 is not None:
            ev1.record(stream)
        plan.two_level_update(db.S, db.eps, db.B, db.wphi, mx)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        step(e0, e1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    k_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
    value = pts / (wall / args.steps)
    print(f"[nonlocal] {args.steps} steps, {ms_per_step:.3f} ms/step, sweep {k_ms:.3f} ms",
          file=sys.stderr, flush=True)

    conv = {"tol": args.conv_tol, "max_iter": args.conv_max_iter, "start": "S = B",
            "desc": "pprt_two_level_ali in graph mode (chunks of 50 iterations), all 512 "
                    "atmospheres, until every one changes by less than tol"}
    for name, op, ng in (("diagonal", pprt.LSTAR_DIAG, False), ("tridiagonal_ng", pprt.LSTAR_TRI, True)):
        p2 = pprt.Plan(ctx, batch.nd, batch.na, batch.nf, precision=pprt.FP32)
        p2.set_operator(op, ng=ng)
        p2.set_launch(*launch)
        S = db.B.clone()
        torch.cuda.synchronize()
        tc = time.perf_counter()
        rep = p2.two_level_ali(db.tau, db.q, S, db.eps, db.B, db.wphi, tol=args.conv_tol,
                               max_iter=args.conv_max_iter, iters_per_sync=50, use_graph=True,
                               raise_not_converged=False)
        torch.cuda.synchronize()
        conv[name] = {"iterations": rep["iterations"], "n_converged": rep["n_converged"],
                      "max_rel": rep["max_rel"], "seconds": round(time.perf_counter() - tc, 4)}
        print(f"[nonlocal] {name}: {rep}", file=sys.stderr, flush=True)
        del p2

    achieved = pts * TRI_FLOPS_PER_POINT / (k_ms * 1e-3) / 1e12
    peaks = ctx.measure_peaks()
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_VALU_NONPACKED,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VALU_NONPACKED, 4),
                "traffic": None, "kernel": "k_fs_profile<float,8,true>", "kernel_ms": round(k_ms, 5),
                "flops_per_point": TRI_FLOPS_PER_POINT,
                "peak_measured": round(peaks["fp32_tflops"], 2),
                "frac_of_measured": round(achieved / peaks["fp32_tflops"], 4),
                "frac_of_published_packed": round(achieved / PEAK_FP32_VALU_PUBLISHED, 4)}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = nonlocal_cpu_baseline(batch, 4)
    line = {
        "metric": "formal-solution depth*angle*freq pts/s, batched FP32, tri-diagonal Lambda* + Ng",
        "value": value, "unit": "pts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "512 two-level atmospheres, nd U{48..256}, na 8, nf 1024, "
                               "eps 1e-6..1e-1, seed 3; tri-diagonal approximate operator with "
                               "Ng acceleration (one ALI step per step)",
                   "nbatch": batch.nb, "rows": int(batch.nd.sum()), "na": batch.na, "nf": batch.nf,
                   "points_per_step": pts, "seed": 3,
                   "launch": {"waves_per_block": launch[0], "persistent_waves_per_cu": launch[1],
                              "autotune": tune}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "convergence": conv,
    }
    print(json.dumps(line), flush=True)


# Multilevel step, FP64 flops.  Voigt function (Weideman, 40 terms): the
# complex Horner recursion 39 x 7, the Moebius map, the final products and
# four divisions (counted once each) -> 300 per evaluation; cross-section,
# opacity, emissivity and source per (row, frequency) -> 20 more.  Dense
# formal solution (omega > 0): 21 NA^3 per (layer, frequency).
VOIGT_FLOPS = 300.0
OPACITY_FLOPS = 20.0
PEAK_FP64_VALU = 78.6
PEAK_FP64_MFMA = 78.6    # TFLOP/s: dense FP64 matrix-core peak (the same as the FP64 vector rate)
DENSE_FLOPS_PER_LAYER = 21.0 * 8 ** 3   # the 21 NA^3 count per (layer, frequency) at NA = 8


def voigt_cpu_baseline(atom1, mu, w):
    """The oracle's multilevel iteration (numpy FP64, one thread) for one
    atmosphere of the batch."""
    from threadpoolctl import threadpool_limits
    from oracle import rates
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        rates.nlte_iteration(atom1, atom1.nstar.copy(), mu, w)
        dt = time.perf_counter() - t0
    pts = int(atom1.nd.sum()) * atom1.na * atom1.nf
    return {"value": pts / dt, "unit": "pts/s", "cores": 1, "kind": "oracle",
            "sample": f"one multilevel iteration of one atmosphere (nd {int(atom1.nd.sum())}, na "
                      f"{atom1.na}, nf {atom1.nf}, {pts} points), numpy FP64, 1 thread, {dt:.1f} s"}


def c3b_cpu_baseline(batch, mu, w, nsample=2):
    """The oracle's two-level step with the scattering continuum (dense
    formal solution, numpy FP64, one thread) on the smallest atmospheres."""
    from threadpoolctl import threadpool_limits
    from oracle import ali, dense
    order = np.argsort(batch.nd, kind="stable")[:nsample]
    off = batch.off
    pts = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for b in order:
            s = slice(int(off[b]), int(off[b + 1]))
            ali.two_level_ali(batch.tau[s], batch.q[s], batch.phi, batch.wnu, float(batch.eps[b]),
                              batch.B[s], mu, w, tol=1e-300, max_iter=1, S0=batch.S_trial[s],
                              pfrac=batch.pfrac[s], sg_const=batch.sg_const[s],
                              fs=dense.formal_solution_dense, fs_kwargs={"omega": batch.omega[s]})
            pts += int(batch.nd[b]) * batch.na * batch.nf
        dt = time.perf_counter() - t0
    return {"value": pts / dt, "unit": "pts/s", "cores": 1, "kind": "oracle",
            "sample": f"one step of the {nsample} smallest of the {batch.nb} atmospheres (nd "
                      f"{int(batch.nd[order].min())}..{int(batch.nd[order].max())}, {pts} points), "
                      f"numpy FP64, 1 thread, {dt:.1f} s"}


VOX_BYTES_PER_SEGMENT_FP32 = 12   # packed voxel index, path length, mean weight (read once per characteristic)


def vox3d_cpu_baseline(vs, ndir_sample=1, nmu=32, nphi=32):
    """The oracle (numpy FP64, one thread) on the same grid and frequencies
    for the first of the directions: its characteristics and formal
    solution."""
    from threadpoolctl import threadpool_limits
    from oracle import sph3d as O
    g = O.Grid(vs.r, vs.nt, vs.np_)
    dirs, w = O.directions(nmu, nphi)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        rs = O.ray_sets(g, dirs[:ndir_sample])
        O.formal_solution(g, dirs[:ndir_sample], w[:ndir_sample], rs, vs.chi, vs.B, I_core=vs.B[0])
        dt = time.perf_counter() - t0
    pts = g.nvox * ndir_sample * vs.nf
    nseg = sum(len(r.segs) for rays in rs for r in rays)
    return {"value": pts / dt, "unit": "voxel*angle*freq pts/s", "cores": 1, "kind": "oracle",
            "sample": f"{ndir_sample} of the {nmu * nphi} directions ({nseg} segments), all {g.nvox} voxels and "
                      f"{vs.nf} frequencies, characteristics and formal solution, numpy FP64, 1 thread, {dt:.1f} s"}


def bench_vox3d(args):
    """3D full characteristics on the paper's spherical voxel grid (65 x 33 x
    65 voxels, radial edges log in tau_std from 1e8 to 1e-4 with chi_c ~ r^-6,
    Sect. 3.1) with the line test's 32 wavelengths (line to continuum opacity
    1e6 at the centre, Sect. 3.2.2) and 32 x 32 solid angles, FP32: the
    formal solution (J over every voxel, direction and frequency) is the
    timed step; the Lambda* band and the operator-splitting step are timed
    beside it."""
    import torch
    from paper_0903_1949_amd import pprt
    from paper_0903_1949_amd import workloads as W

    torch.cuda.set_device(0)
    nmu = nphi = 32
    vs = W.voxel_sphere(nr=65, nt=33, np_=65, nf=32, continuum="r6", line_ratio=1e6, eps=1e-4)
    ctx = pprt.Context(0)
    stream = torch.cuda.current_stream()
    t_plan = time.perf_counter()
    plan = pprt.VoxPlan(ctx, vs.r, vs.nt, vs.np_, nmu, nphi, vs.nf, precision=pprt.FP32)
    t_plan = time.perf_counter() - t_plan
    info = plan.info
    print(f"[vox3d] plan {t_plan:.1f} s: {info}", file=sys.stderr, flush=True)
    d = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda:0")
    chi = d(vs.chi, torch.float32)
    S = d(vs.B, torch.float32)
    Ic = d(vs.B[0], torch.float32)
    out = plan.formal_solution(chi, S, None, Ic)
    pts = plan.nvox * plan.ndir * vs.nf

    def timed(fn, n):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for e0, e1 in evs:
            e0.record(stream)
            fn()
            e1.record(stream)
        torch.cuda.synchronize()
        return [e0.elapsed_time(e1) for e0, e1 in evs]

    fs = lambda: plan.formal_solution(chi, S, None, Ic, out=out)
    steps, warmup = max(1, min(args.steps, 20)), max(1, min(args.warmup, 3))
    timed(fs, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = timed(fs, steps)
    wall = time.perf_counter() - t0
    # the Lambda* band (once per ALI in the paper) and the operator-splitting step
    outL = plan.formal_solution(chi, S, None, Ic, lstar=True)
    msL = timed(lambda: plan.formal_solution(chi, S, None, Ic, lstar=True, out=outL), 2)
    Sd = d(vs.B, torch.float64)
    Bd, ed = d(vs.B, torch.float64), d(vs.eps, torch.float64)
    mx = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    msA = timed(lambda: plan.ali_step(chi, Sd, Bd, ed, mx, None, Ic), 3)
    torch.cuda.synchronize()
    J = out["J"].cpu().numpy()
    fs_ms = float(np.median(ms))
    nseg = int(info["nsegments"])
    seg_bytes = nseg * VOX_BYTES_PER_SEGMENT_FP32
    io_bytes = plan.nvox * vs.nf * (4 + 4 + 8 + 8)       # chi, S read; J cleared and accumulated
    achieved = (seg_bytes + io_bytes) / (fs_ms * 1e-3) / 1e9
    atom_rate = nseg * vs.nf / (fs_ms * 1e-3)
    pk = ctx.measure_peaks(256)
    # the formal solution's J adds: FP32 block sums (one add per segment and frequency)
    atom_peak = pk["atomic_f32_gadds"] * 1e9
    cpu = None if args.no_cpu_baseline else vox3d_cpu_baseline(vs, 1, nmu, nphi)
    line = {
        "metric": "3D formal-solution voxel*angle*freq pts/s (full characteristics, spherical voxel grid)",
        "value": pts / (fs_ms * 1e-3), "unit": "voxel*angle*freq pts/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": wall * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "spherical voxel grid 65 x 33 x 65 (r 1..2, tau_std 1e8..1e-4, chi_c ~ r^-6), "
                               "32 wavelengths (line/continuum 1e6), 32 x 32 solid angles, one formal solution "
                               "per step (J at every voxel, direction and frequency)",
                   "nvox": plan.nvox, "ndir": plan.ndir, "nf": vs.nf, "points_per_step": pts,
                   "characteristics": int(info["nrays"]), "segments": nseg,
                   "coverage_characteristics": int(info["ncoverage"]), "plan_s": round(t_plan, 1),
                   "geometry_gb": round(info["device_bytes"] / 1e9, 2)},
        "step_ms_stats": {"median": fs_ms, "min": float(np.min(ms)), "max": float(np.max(ms))},
        "roofline": {"bound": "atomic", "achieved": round(atom_rate / 1e9, 1),
                     "peak": round(atom_peak / 1e9, 1), "unit": "G atomic adds/s",
                     "frac": round(atom_rate / atom_peak, 4), "traffic": None,
                     "kernel": "k_vox_fs<float,float,0,8>", "kernel_ms": round(fs_ms, 3),
                     "adds_per_segment_and_frequency": 1,
                     "peak_note": "measured coalesced FP32 atomic-add rate (rows of 32 at hashed rows of a "
                                  "139425-row array); FP64 adds measured at "
                                  f"{pk['atomic_f64_gadds']:.1f} G/s",
                     "hbm_achieved_gbs": round(achieved, 1), "hbm_frac": round(achieved / 8000.0, 4),
                     "bytes_per_segment": VOX_BYTES_PER_SEGMENT_FP32},
        "lstar_band_ms": float(np.median(msL)), "ali_step_ms": float(np.median(msA)),
        "J_range": [float(J.min()), float(J.max())],
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_c3b(args):
    """The two-level step of the C3a batch with a grey coherent scattering
    continuum inside the layers (chi_c/chi_l = 1e-3 per unit tau, eps_c =
    1e-4): S^g assembly, the omega > 0 dense formal solution (FP64) at every
    point, the profile quadratures and the FP64 update."""
    import torch
    from paper_0903_1949_amd import pprt
    from paper_0903_1949_amd import workloads as W

    torch.cuda.set_device(0)
    batch = W.two_level_batch(seed=3, cont_ratio=1e-3, eps_c=1e-4)
    rows, nf, na = int(batch.nd.sum()), batch.nf, batch.na
    pts = rows * na * nf
    ctx = pprt.Context(0)
    plan = pprt.Plan(ctx, batch.nd, na, nf, precision=pprt.FP64)
    db = pprt.upload_two_level(batch, pprt.FP64)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")
    pf, sc, om = d(batch.pfrac), d(batch.sg_const), d(batch.omega)
    mx = torch.zeros(batch.nb, dtype=torch.float64, device="cuda:0")
    stream = torch.cuda.current_stream()

    def step(e0=None, e1=None):
        if e0 is not None:
            e0.record(stream)
        plan.two_level_ali_step_continuum(db.tau, db.q, db.S, db.eps, db.B, db.wphi, pf, sc, om,
                                          db.Bbot, db.Bbot_prev, mx)
        if e1 is not None:
            e1.record(stream)

    steps, warmup = max(1, min(args.steps, 5)), max(1, min(args.warmup, 2))
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    print(f"c3b: {warmup} warm-up steps done", file=sys.stderr, flush=True)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        step(e0, e1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
    flops = rows * nf * DENSE_FLOPS_PER_LAYER
    achieved = flops / (step_ms * 1e-3) / 1e12
    fp32 = c3b_fp32_bulk(ctx, batch, plan, db, pf, sc, om, steps, step_ms)
    cpu = None if args.no_cpu_baseline else c3b_cpu_baseline(batch, plan.mu, plan.w)
    line = {
        "metric": "formal-solution depth*angle*freq pts/s of the two-level step with coherent "
                  "continuum scattering, FP64 dense",
        "value": pts / (wall / steps), "unit": "pts/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": wall * 1e3 / steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "512 two-level atmospheres of the headline batch (nd U{48..256}, na 8, "
                               "nf 1024, seed 3) with a grey coherent continuum (r_c 1e-3, eps_c 1e-4): "
                               "omega > 0 at every point (one ALI step per step)",
                   "nbatch": batch.nb, "rows": rows, "na": na, "nf": nf, "points_per_step": pts,
                   "workspace_gb": round(plan_continuum_workspace_gb(plan), 1)},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_VALU,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_VALU, 4), "traffic": None,
                     "kernel": "k_fs_dense<8> (the whole step's event time, an upper bound on the "
                               "dense passes' own)",
                     "kernel_ms": round(step_ms, 3), "flops_per_layer_and_freq": DENSE_FLOPS_PER_LAYER,
                     "peak_note": "FP64 vector, 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz"},
        "fp32_bulk": fp32,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def c3b_fp32_bulk(ctx, batch, plan64, db64, pf64, sc64, om64, steps, fp64_step_ms):
    """The same step with an FP32 plan (FP64 layer operators, FP32 adding
    recursion, FP64 eliminations under the thick-layer rule): event time per
    step, the speed-up over the FP64 step, the share of eliminations that ran
    in FP64, and the error of one step's S against the FP64 step from the
    same S (and of the FP32-only eliminations beside it)."""
    import torch
    from paper_0903_1949_amd import pprt

    rows, nf, na = int(batch.nd.sum()), batch.nf, batch.na
    plan = pprt.Plan(ctx, batch.nd, na, nf, precision=pprt.FP32)
    db = pprt.upload_two_level(batch, pprt.FP32)
    f = lambda t: t.to(torch.float32).contiguous()
    pf, sc, om = f(pf64), f(sc64), f(om64)
    mx = torch.zeros(batch.nb, dtype=torch.float64, device="cuda:0")
    stream = torch.cuda.current_stream()

    def step(pl, d, a, b, c, m):
        pl.two_level_ali_step_continuum(d.tau, d.q, d.S, d.eps, d.B, d.wphi, a, b, c, d.Bbot,
                                        d.Bbot_prev, m)

    step(plan, db, pf, sc, om, mx)
    torch.cuda.synchronize()
    ctx.thick_counts(reset=True)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for e0, e1 in evs:
        e0.record(stream)
        step(plan, db, pf, sc, om, mx)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
    n64, ntot = ctx.thick_counts(reset=True)
    # one step from the same S in FP64, FP32 (rule) and FP32 (no FP64 eliminations)
    S0 = torch.as_tensor(batch.S_trial, dtype=torch.float64, device="cuda:0")
    mx64 = torch.zeros_like(mx)
    db64.S.copy_(S0)
    step(plan64, db64, pf64, sc64, om64, mx64)
    out = {}
    for mode, name in ((pprt.THICK_RULE, "rule"), (pprt.THICK_NEVER, "never")):
        plan.set_thick_mode(mode)
        db.S.copy_(S0)
        step(plan, db, pf, sc, om, mx)
        torch.cuda.synchronize()
        dS64 = (db64.S - S0).abs()
        err = ((db.S - db64.S).abs() / db64.S.abs()).max().item()
        err_d = ((db.S - db64.S).abs().max() / dS64.max()).item()
        out[name] = {"S_rel_err_vs_fp64": err, "dS_err_vs_fp64_scale": err_d}
    plan.set_thick_mode(pprt.THICK_RULE)
    return {"ms_per_step": round(ms, 3), "pts_per_s": rows * na * nf / (ms * 1e-3),
            "speedup_vs_fp64_step": round(fp64_step_ms / ms, 3),
            "fp64_eliminations": n64, "eliminations": ntot,
            "fp64_elimination_share": round(n64 / max(ntot, 1), 4),
            "one_step_errors": out,
            "workspace_gb": round(plan_continuum_workspace_gb(plan), 1)}


ADJ_FLOPS_PER_POINT = 48.0   # forward 12; reverse 2 x 12 (segment recompute) + 12 (adjoint)


def bench_adjoint(args):
    """Gradient of the emergent-spectrum loss L = sum I+(tau_1)^2 on the C4
    case (nd 256, na 16, nf 4096, FP32): the forward emergent intensity with
    layer checkpoints every 16 nodes and the hand-written vector-Jacobian
    product (dL/dq, dL/dS per depth and frequency), through the C ABI."""
    import torch
    from paper_0903_1949_amd import pprt
    from paper_0903_1949_amd import workloads as W

    torch.cuda.set_device(0)
    g = W.gradient_case()
    nd, na, nf = g.tau.shape[0], g.na, g.B.shape[1]
    pts = nd * na * nf
    ctx = pprt.Context(0)
    plan = pprt.Plan(ctx, [nd], na, nf, precision=pprt.FP32)
    d = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda:0")
    tau = d(g.tau, torch.float64)
    q = d(np.outer(g.c, g.f), torch.float32)
    B = d(g.B, torch.float32)
    Bb, Bp = B[-1:].contiguous(), B[-2:-1].contiguous()
    K = args.adj_k
    ws = torch.empty(max(plan.adjoint_workspace_bytes(K), 256), dtype=torch.uint8, device="cuda:0")
    stream = torch.cuda.current_stream()

    def step(e0=None, e1=None, e2=None):
        if e0 is not None:
            e0.record(stream)
        I, _ = plan.emergent_intensity(tau, q, B, Bb, Bp, checkpoint_interval=K, workspace=ws)
        if e1 is not None:
            e1.record(stream)
        gI = 2.0 * I
        plan.formal_solution_vjp(tau, q, B, gI, ws, Bb, Bp, checkpoint_interval=K)
        if e2 is not None:
            e2.record(stream)

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    steps = args.steps
    evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1, e2 in evs:
        step(e0, e1, e2)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1, _ in evs]))
    tot_ms = float(np.mean([e0.elapsed_time(e2) for e0, _, e2 in evs]))
    achieved = pts * ADJ_FLOPS_PER_POINT / (tot_ms * 1e-3) / 1e12

    # the same atmosphere with a grey coherent scatterer (albedo 0.5 at every
    # node), FP64: the forward with in-layer scattering and its hand-written VJP
    plan64 = pprt.Plan(ctx, [nd], na, nf, precision=pprt.FP64, outputs=pprt.OUT_IEMERG)
    q64, B64 = q.double(), B.double()
    om64 = torch.full_like(q64, 0.5)
    Bb64, Bp64 = B64[-1:].contiguous(), B64[-2:-1].contiguous()
    wsd, wsv = {}, {}

    def dense_step(e0=None, e1=None, e2=None):
        if e0 is not None:
            e0.record(stream)
        out = plan64.formal_solution_scattering(tau, q64, B64, om64, Bbot=Bb64, Bbot_prev=Bp64,
                                                workspace=wsd.get("w"))
        wsd["w"] = out["_workspace"]
        if e1 is not None:
            e1.record(stream)
        gv = plan64.formal_solution_scattering_vjp(tau, q64, B64, om64, 2.0 * out["Iemerg"], Bbot=Bb64,
                                                   Bbot_prev=Bp64, workspace=wsv.get("w"))
        wsv["w"] = gv["_workspace"]
        if e2 is not None:
            e2.record(stream)

    dense_step()
    torch.cuda.synchronize()
    devs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(3)]
    for e0, e1, e2 in devs:
        dense_step(e0, e1, e2)
    torch.cuda.synchronize()
    dense_leg = {"forward_ms": round(float(np.median([e0.elapsed_time(e1) for e0, e1, _ in devs])), 3),
                 "vjp_ms": round(float(np.median([e1.elapsed_time(e2) for _, e1, e2 in devs])), 3),
                 "what": "albedo 0.5 at every node, FP64: pprt_formal_solution_scattering (Iemerg) and "
                         "pprt_formal_solution_scattering_vjp (dL/dq, dL/dS^g)"}
    del wsd, wsv
    cpu = None
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits
        from oracle import grad
        ks = slice(0, nf)
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            grad.emergent_intensity(g.tau, np.outer(g.c, g.f)[:, ks], g.B[:, ks], plan.mu,
                                    Bbot=g.B[-1, ks], Bbot_prev=g.B[-2, ks])
            dt = time.perf_counter() - t1
        cpu = {"value": pts / dt, "unit": "pts/s", "cores": 1, "kind": "oracle",
               "sample": f"the oracle's FP64 forward emergent intensity at all {nf} frequencies "
                         f"({pts} points, {dt:.1f} s, numpy, 1 thread); it differentiates by complex "
                         "step, one complex forward per parameter depth, and has no adjoint"}
    line = {
        "metric": "formal-solution depth*angle*freq pts/s of the emergent-spectrum gradient (forward + VJP), FP32",
        "value": pts / (wall / steps), "unit": "pts/s", "n_gpus": 1, "steps": steps,
        "warmup": max(1, args.warmup), "ms_per_step": wall * 1e3 / steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "one atmosphere, nd 256, tau 1e-4..1e4, na 16, nf 4096 (nu 1.5e14..3e15 Hz), "
                               "lognormal per-depth opacity, B_nu of a grey Eddington T(tau), seed 4; "
                               f"loss sum of I+(tau_1)^2, checkpoints every {K} nodes",
                   "nd": nd, "na": na, "nf": nf, "points_per_step": pts, "checkpoint_interval": K},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_VALU_NONPACKED,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VALU_NONPACKED, 4),
                     "traffic": None, "kernel": "k_emergent + k_emergent_vjp (forward + VJP launches)",
                     "kernel_ms": round(tot_ms, 4), "forward_ms": round(fwd_ms, 4),
                     "flops_per_point": ADJ_FLOPS_PER_POINT,
                     "note": "a single atmosphere: 4096 x 16 lanes, one wave per SIMD; latency-bound"},
        "with_scattering": dense_leg,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def plan_continuum_workspace_gb(plan):
    import ctypes as C
    nbytes = C.c_size_t()
    plan.ctx._check(plan.lib.pprt_plan_continuum_workspace_bytes(plan.h, C.byref(nbytes)),
                    "continuum_workspace_bytes")
    return nbytes.value / 1e9


def bench_voigt(args):
    """One multilevel iteration over a batch of atmospheres whose line
    profiles depend on depth: opacities and sources from the populations with
    device Voigt profiles, the omega > 0 formal solution (FP64 dense), the
    preconditioned rates (Voigt profiles again) and the per-depth FP64 solve.
    Each stage is also timed on its own with HIP events."""
    import torch
    from paper_0903_1949_amd import pprt
    from paper_0903_1949_amd import workloads as W

    torch.cuda.set_device(0)
    nb = args.voigt_nb
    atom = W.multilevel_atom(nbound=6, ncont=5, nd=128, na=8, nline_pts=100, ncont_pts=100,
                             nb=nb, seed=2, depth_profiles=True)
    rows, nf, na = int(atom.nd.sum()), atom.nf, atom.na
    pts = rows * na * nf
    ctx = pprt.Context(0)
    stream = torch.cuda.current_stream()
    plan = pprt.Plan(ctx, atom.nd, na, nf, precision=pprt.FP64, outputs=pprt.OUT_J | pprt.OUT_LSTAR)
    da = pprt.DeviceAtom(atom)
    pops = da.nstar.clone()
    mx = torch.zeros(nb, dtype=torch.float64, device="cuda:0")
    for _ in range(args.warmup):
        plan.nlte_step(da.tau, da, pops, mx)
    torch.cuda.synchronize()
    steps = args.steps
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.nlte_step(da.tau, da, pops, mx)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / steps
    value = pts / (wall / steps)

    # the stages one by one, from the same populations
    off = np.concatenate([[0], np.cumsum(atom.nd)])
    Bnu = np.asarray(atom.Bnu)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")
    Bb, Bp = dev(Bnu[off[1:] - 1]), dev(Bnu[off[1:] - 2])

    def timed(fn, n=5):
        fn()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        out = None
        for e0, e1 in evs:
            e0.record(stream)
            out = fn()
            e1.record(stream)
        torch.cuda.synchronize()
        return float(np.median([e0.elapsed_time(e1) for e0, e1 in evs])), out

    t_op, (q, om, Sg) = timed(lambda: plan.nlte_opacity(da, pops))
    ws = {}
    t_fs, fs = timed(lambda: fs_reusing(ws, lambda w: plan.formal_solution_scattering(
        da.tau, q, Sg, om, Bbot=Bb, Bbot_prev=Bp, workspace=w)))
    t_ra, (dRlu, dRul, Rsul) = timed(lambda: plan.rates_assemble(da, pops, fs["J"], fs["lstar"]))
    t_so, _ = timed(lambda: plan.rates_solve(da, pops, dRlu, dRul, Rsul))
    line_pts = int(np.count_nonzero(np.asarray(atom.line_nu0)[np.asarray(atom.owner)] > 0)) * rows
    op_flops = line_pts * VOIGT_FLOPS + rows * nf * OPACITY_FLOPS
    fs_flops = 21.0 * na ** 3 * rows * nf
    stages = {
        "opacity_voigt": {"ms": round(t_op, 4), "flops": op_flops,
                          "tflops": round(op_flops / (t_op * 1e-3) / 1e12, 3),
                          "line_points": line_pts},
        "formal_solution_dense": {"ms": round(t_fs, 4), "flops": fs_flops,
                                  "tflops": round(fs_flops / (t_fs * 1e-3) / 1e12, 3)},
        "rates_assemble_voigt": {"ms": round(t_ra, 4)},
        "rates_solve": {"ms": round(t_so, 4)},
    }
    print(f"[voigt] {ms_per_step:.3f} ms/step; stages {stages}", file=sys.stderr, flush=True)
    dom = max(("opacity_voigt", "formal_solution_dense"), key=lambda k: stages[k]["ms"])
    kern = {"opacity_voigt": "k_ml_opacity", "formal_solution_dense": "k_fs_dense<8>"}[dom]
    ach = stages[dom]["tflops"]
    peaks = ctx.measure_peaks()
    roofline = {"bound": "alu", "achieved": ach, "peak": PEAK_FP64_VALU, "unit": "TFLOP/s",
                "frac": round(ach / PEAK_FP64_VALU, 4), "traffic": None, "kernel": kern,
                "kernel_ms": stages[dom]["ms"], "peak_measured": round(peaks["fp64_tflops"], 2),
                "frac_of_measured": round(ach / peaks["fp64_tflops"], 4)}
    cpu = None
    if not args.no_cpu_baseline:
        from oracle.quadrature import gauss_legendre01
        a1 = W.multilevel_atom(nbound=6, ncont=5, nd=128, na=8, nline_pts=100, ncont_pts=100,
                               nb=1, seed=2, depth_profiles=True)
        cpu = voigt_cpu_baseline(a1, *gauss_legendre01(na))
    line = {
        "metric": "formal-solution depth*angle*freq pts/s of the multilevel iteration, FP64",
        "value": value, "unit": "pts/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{nb} atmospheres of the 6+1-level hydrogen-like atom (15 lines, "
                               "5 continua, depth-dependent Voigt lines), nd 128, na 8, nf 2000, "
                               "grey scattering continuum eps_c 1e-2, seed 2 (one multilevel "
                               "iteration per step)",
                   "nbatch": nb, "rows": rows, "na": na, "nf": nf, "points_per_step": pts, "seed": 2},
        "roofline": roofline,
        "stages": stages,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_c5(args):
    """The large angle-coupled case: one multilevel iteration of the 20-level
    atom (100 depth-dependent Voigt lines, 4 continua) on 512 depths, 32
    angles per hemisphere (the 64 x 64 block layer operators on the FP64
    matrix cores) and 16384 frequencies: opacities, the omega > 0 formal
    solution, the preconditioned rates and the 20-level FP64 solve per depth.
    Each stage is also timed on its own with HIP events."""
    import torch
    from paper_0903_1949_amd import pprt
    from paper_0903_1949_amd import workloads as W

    torch.cuda.set_device(0)
    atom = W.c5_atom()
    rows, nf, na = int(atom.nd.sum()), atom.nf, atom.na
    pts = rows * na * nf
    ctx = pprt.Context(0)
    stream = torch.cuda.current_stream()
    plan = pprt.Plan(ctx, atom.nd, na, nf, precision=pprt.FP64, outputs=pprt.OUT_J | pprt.OUT_LSTAR)
    da = pprt.DeviceAtom(atom)
    pops = da.nstar.clone()
    mx = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")
    Bnu = np.asarray(atom.Bnu)
    Bb, Bp = dev(Bnu[-1:]), dev(Bnu[-2:-1])

    def timed(fn, n=3):
        fn()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        out = None
        for e0, e1 in evs:
            e0.record(stream)
            out = fn()
            e1.record(stream)
        torch.cuda.synchronize()
        return float(np.median([e0.elapsed_time(e1) for e0, e1 in evs])), out

    # the stages one by one from the LTE populations (the formal solution's
    # workspace is released before the iterations allocate their own)
    t_op, (q, om, Sg) = timed(lambda: plan.nlte_opacity(da, pops))
    ws = {}
    t_fs, fs = timed(lambda: fs_reusing(ws, lambda w: plan.formal_solution_scattering(
        da.tau, q, Sg, om, Bbot=Bb, Bbot_prev=Bp, workspace=w)))
    ws_gb = ws["w"].numel() * ws["w"].element_size() / 1e9
    t_ra, (dRlu, dRul, Rsul) = timed(lambda: plan.rates_assemble(da, pops, fs["J"], fs["lstar"]))
    t_so, _ = timed(lambda: plan.rates_solve(da, pops, dRlu, dRul, Rsul))
    J64, L64 = fs["J"].clone(), fs["lstar"].clone()
    del fs, ws, dRlu, dRul, Rsul
    torch.cuda.empty_cache()
    # the same formal solution on an FP32 plan (FP32 arrays and workspace,
    # FP64 arithmetic): time and per-output error against the FP64 stage
    plan32 = pprt.Plan(ctx, atom.nd, na, nf, precision=pprt.FP32, outputs=pprt.OUT_J | pprt.OUT_LSTAR)
    q32, Sg32, om32, Bb32, Bp32 = (x.float() for x in (q, Sg, om, Bb, Bp))
    ws32 = {}
    t_fs32, fs32 = timed(lambda: fs_reusing(ws32, lambda w: plan32.formal_solution_scattering(
        da.tau, q32, Sg32, om32, Bbot=Bb32, Bbot_prev=Bp32, workspace=w)))

    def arr_err(a, b):
        return float(((a.double() - b).abs() / torch.maximum(b.abs(), 1e-4 * b.abs().max())).max())

    fp32_leg = {"ms": round(t_fs32, 2), "J_err": arr_err(fs32["J"], J64), "lstar_err": arr_err(fs32["lstar"], L64),
                "workspace_gb": round(ws32["w"].numel() * ws32["w"].element_size() / 1e9, 1),
                "metric": "max |FP32 - FP64| / max(|FP64|, 1e-4 max |FP64|), inputs rounded to FP32"}
    del fs32, ws32, plan32, q32, Sg32, om32, J64, L64, q, om, Sg
    torch.cuda.empty_cache()
    print(f"[c5] stages: opacity {t_op:.2f} ms, formal solution {t_fs:.1f} ms (FP32 plan {t_fs32:.1f} ms), "
          f"rates {t_ra:.2f} ms, solve {t_so:.2f} ms", file=sys.stderr, flush=True)

    warmup, steps = min(args.warmup, 2), args.c5_steps      # about a second per iteration
    for _ in range(warmup):
        plan.nlte_step(da.tau, da, pops, mx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.nlte_step(da.tau, da, pops, mx)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / steps
    value = pts / (wall / steps)
    fs_flops = 21.0 * na ** 3 * (rows - 1) * nf
    stages = {
        "opacity_voigt": {"ms": round(t_op, 3)},
        "formal_solution_dense": {"ms": round(t_fs, 2), "flops": fs_flops,
                                  "tflops": round(fs_flops / (t_fs * 1e-3) / 1e12, 3),
                                  "workspace_gb": round(ws_gb, 1)},
        "rates_assemble_voigt": {"ms": round(t_ra, 3)},
        "rates_solve_20_levels": {"ms": round(t_so, 3)},
        "formal_solution_fp32_plan": fp32_leg,
    }
    ach = stages["formal_solution_dense"]["tflops"]
    roofline = {"bound": "mfma", "achieved": ach, "peak": PEAK_FP64_MFMA, "unit": "TFLOP/s",
                "frac": round(ach / PEAK_FP64_MFMA, 4), "traffic": None,
                "kernel": "k_fs_dense_mfma<2,1> + <2,2>", "kernel_ms": stages["formal_solution_dense"]["ms"],
                "flops_per_unit": "21 NA^3 per (layer, frequency)"}
    cpu = None
    if not args.no_cpu_baseline:
        from oracle.quadrature import gauss_legendre01
        cpu = c5_cpu_baseline(W.c5_atom(nd=24, nline_pts=5, ncont_pts=4), *gauss_legendre01(na))
    line = {
        "metric": "formal-solution depth*angle*freq pts/s of the multilevel iteration, FP64",
        "value": value, "unit": "pts/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "20-level hydrogen-like atom (100 depth-dependent Voigt lines, damping "
                               "log-uniform 1e-4..1e-1, 4 continua), nd 512, tau 1e-6..1e2, na 32 "
                               "(64 x 64 block layer operators), nf 16384, grey scattering continuum "
                               "eps_c 1e-2, seed 5 (one multilevel iteration per step)",
                   "rows": rows, "na": na, "nf": nf, "levels": int(atom.nl), "transitions": int(atom.nt),
                   "points_per_step": pts, "seed": 5},
        "roofline": roofline,
        "stages": stages,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def c5_cpu_baseline(atom1, mu, w):
    """The oracle's multilevel iteration (numpy FP64, one thread) for the
    same atom on a reduced grid."""
    from threadpoolctl import threadpool_limits
    from oracle import rates
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        rates.nlte_iteration(atom1, atom1.nstar.copy(), mu, w)
        dt = time.perf_counter() - t0
    pts = int(atom1.nd.sum()) * atom1.na * atom1.nf
    return {"value": pts / dt, "unit": "pts/s", "cores": 1, "kind": "oracle",
            "sample": f"one multilevel iteration of the same 20-level atom on a reduced grid (nd "
                      f"{int(atom1.nd.sum())}, na {atom1.na}, nf {atom1.nf}: 5 points per line, 4 per "
                      f"continuum; {pts} points), numpy FP64, 1 thread, {dt:.1f} s"}


def kernel_hash(name: str = "fs_diag.hip") -> str:
    """Hash of a kernel source: traffic counters are only reported while the
    kernel they were taken on is unchanged."""
    import hashlib
    src = os.path.join(ROOT, "paper_0903_1949_amd", "csrc", name)
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def fs_reusing(ws: dict, call):
    """call(workspace) for a formal solution that returns its workspace under
    "_workspace": the first call allocates it, later calls reuse it (a second
    allocation while the first result is alive would double the footprint;
    the 32-angle FP64 case needs 214 GiB)."""
    out = call(ws.get("w"))
    ws["w"] = out["_workspace"]
    return out


def measured_traffic(path: str, source: str):
    """HBM bytes per launch from a committed counter summary, if it was taken
    on the current kernel source."""
    try:
        tj = json.load(open(path))
    except (OSError, ValueError):
        return None
    if tj.get("kernel_source_hash") != kernel_hash(source):
        return None
    return tj.get("bytes_per_launch", {}).get("total")


if __name__ == "__main__":
    main()
