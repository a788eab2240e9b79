"""Benchmark: cell x ordinate x band updates/s of the source-iteration sweep on
the 2D nongray square (256 x 256 cells, 15 bands, 128 directions of which 64
distinct in-plane projections are swept, FP32 sweeps with FP64 band sums),
plus the adjoint/forward time ratio and batched solves/s as extra fields.

One step is one source iteration of the whole hot path on the whole problem:
the fused transport sweep of every (band, direction) pair with the band /
direction reduction and the new temperature, replayed from a captured
hipGraph. The timed run is K iterations with the convergence test once at
the end (tolerance 0, as the paper times a fixed iteration count): the heat
flux and the residuals of Eq. 22 are formed in the last two iterations, as in
any solve that checks every K iterations. Inputs are resident in HBM before
the timed region.

Prints one JSON line. --gpus N with N > 1 exits: the benchmark measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def flops_per_update(dim: int, with_q: bool) -> float:
    # f = S + sum_d a_d f_d (dim FMAs), one FMA into the temperature sum, dim FMAs
    # into the flux sums on flux iterations
    return 2.0 * (dim + 1 + (dim if with_q else 0))


def cpu_baseline(p, iters: int, m_swept: int, iters_single: int = 2):
    """The FP64 oracle timed on the host over a bounded number of iterations,
    as a rate in the metric's own counting (swept projections per band), on
    all host threads and, over fewer iterations, on one thread."""
    import oracle
    threads = oracle.num_threads()
    upd = p.n_active * m_swept * p.B
    t0 = time.perf_counter()
    oracle.solve(p, tol=0.0, max_iters=iters, threads=threads)
    dt = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.solve(p, tol=0.0, max_iters=iters_single, threads=1)
    dt1 = time.perf_counter() - t0
    return dict(value=upd * iters / dt, unit="updates/s", cores=threads, kind="oracle",
                sample=f"{iters} source iterations of the full 256x256 problem in FP64 ({dt:.1f} s; the oracle "
                       f"sweeps all {p.M} directions, counted as the {m_swept} swept projections per band)",
                single_thread=dict(value=upd * iters_single / dt1, unit="updates/s", cores=1,
                                   sample=f"{iters_single} source iterations, same problem ({dt1:.1f} s)"))


SWEEP_SOURCES = ("bte_sweep2d.hip", "bte_sweep2d_launch.h", "bte_kutil.h")


def sweep_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(ROOT, "paper_2503_23657_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when it holds none for this kernel or the sweep sources changed since
    the counters were taken. The summary lists `- sweep source hash: ...` and
    one `- hbm bytes per launch of <kernel>: <bytes>` line per kernel."""
    path = os.path.join(ROOT, "profiles", "sweep2d_square256_hbm_counters.md")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].rsplit(":", 1)
                kv[k.strip().replace("`", "")] = v.strip().strip("`")
    if kv.get("sweep source hash") != sweep_source_hash():
        return None
    try:
        return float(kv[f"hbm bytes per launch of {kernel}"])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=12)
    ap.add_argument("--batch-kn-min", type=float, default=0.3)
    ap.add_argument("--plan", type=str, default=None,
                    help="fixed kernel plan 'G,R,P,NR' instead of the autotuned one")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of 256 MiB three times (calibrates the HBM byte counters)")
    ap.add_argument("--sweep3d", choices=("finfet", "finfet_mixed"), default=None,
                    help="only time the 3D sweep on the full FinFET-like domain (diffuse walls, or the paper's "
                         "specular/diffuse/isothermal mix) and print one JSON line; not the benchmark metric")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        x = torch.ones(64 * 1024 * 1024, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": x.numel() * 4, "copies": 3}))
        return
    if args.sweep3d:
        import torch

        import bte_inputs as bi
        import paper_2503_23657_amd as bte
        p = bi.finfet_3d(scale=1) if args.sweep3d == "finfet" else bi.finfet_3d_mixed(scale=1)
        solver = bte.Solver(p, precision="fp32")
        Q = torch.tensor(p.Q, dtype=torch.float64, device="cuda")
        solver.solve(Q, tol=0.0, max_iters=2, check_every=2)
        ms, upd = solver.time_sweep(n_launches=max(1, args.steps // 60))
        print(json.dumps({"workload": f"3D {args.sweep3d} 96x96x120 ({p.n_active} cells), 15 bands, 128 directions",
                          "plan": solver.plan(), "sweep_ms": ms, "updates_per_s": upd / (ms * 1e-3),
                          "dtype": "f32"}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import bte_inputs as bi
    import paper_2503_23657_amd as bte

    dev = torch.device("cuda:0")
    p = bi.square_2d(256)  # 1 um square, 15 bands, 8x2 per octant z-polar (128 dirs)
    M_swept = 64
    solver = bte.Solver(p, precision="fp32")
    Q = torch.tensor(p.Q, dtype=torch.float64, device=dev)
    if args.plan:
        G_, R_, P_, NR_ = (int(x) for x in args.plan.split(","))
        solver.set_plan(G=G_, R=R_, P=P_, NR=NR_)
        plan = solver.plan()
    else:
        # whole iterations, the flux carried by the last two as in a long solve
        plan = solver.autotune(Q, n_iters=30)
    log("plan", plan)
    K = max(8, args.steps)
    # warm-up (also captures the graphs)
    solver.solve(Q, tol=0.0, max_iters=max(args.warmup, 2), check_every=K)
    solver.solve(Q, tol=0.0, max_iters=K, check_every=K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T, q, rep = solver.solve(Q, tol=0.0, max_iters=K, check_every=K)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_upd = p.n_active * M_swept * p.B
    value = n_upd * K / dt
    ms_per_step = dt / K * 1e3
    log(f"forward: {K} iterations in {dt:.4f} s -> {value:.4e} updates/s")

    # dominant kernel: the sweep, timed with HIP events on the stream it runs on
    sweep_ms, _ = solver.time_sweep(n_launches=50)
    flop = n_upd * flops_per_update(2, False)
    achieved_tf = flop / (sweep_ms * 1e-3) / 1e12
    kname = f"sweep2d_kernel<float, {plan['G']}, {plan['NR']}, {plan['P']}, 1, 0>"
    traffic = profiled_traffic(kname)
    roofline = dict(bound="alu", achieved=achieved_tf, peak=FP32_VALU_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=achieved_tf / FP32_VALU_PEAK_TFLOPS, traffic=traffic,
                    kernel=kname, kernel_ms=sweep_ms, sweep_updates_per_s=n_upd / (sweep_ms * 1e-3))
    if traffic is not None:
        # the measured HBM bytes of one launch over its event-timed duration,
        # against the published HBM peak
        gbs = traffic / (sweep_ms * 1e-3) / 1e9
        roofline.update(hbm_gbs=gbs, hbm_peak_gbs=HBM_PEAK_GBS, hbm_frac=gbs / HBM_PEAK_GBS)

    extra = {}
    if not args.no_extra:
        # adjoint / forward time ratio at equal tolerance (inverse-problem case on the square)
        s64 = solver
        tol = 1e-6
        t0 = time.perf_counter()
        T, _, rf = s64.solve(Q, tol=tol, check_every=8, store_state=True)
        torch.cuda.synchronize()
        tf = time.perf_counter() - t0
        case = bi.adjoint_case(p)
        probes = torch.tensor(case["probes"], device=dev)
        Tt = T.detach().clone().requires_grad_(True)
        target = T.detach()[probes] + 1.0
        J = ((Tt[probes] - target) ** 2).mean()
        (gT,) = torch.autograd.grad(J, Tt)
        t0 = time.perf_counter()
        dtau, dQ, ra = s64.adjoint(gT.contiguous(), tol=tol, check_every=8)
        torch.cuda.synchronize()
        ta = time.perf_counter() - t0
        extra["adjoint_forward_ratio"] = ta / tf
        extra["forward_solve_s"] = tf
        extra["forward_iters"] = rf["iters"]
        extra["adjoint_solve_s"] = ta
        extra["adjoint_iters"] = ra["iters"]
        log(f"adjoint/forward = {ta / tf:.3f} ({ra['iters']} vs {rf['iters']} iterations)")

    if not args.no_extra:
        # batched solves/s vs a sequential loop of single solves at equal accuracy
        insts = [q for q in bi.batch_instances() if q.Kn >= args.batch_kn_min]
        tol_b = 1e-6
        Qs = [torch.tensor(q.Q, dtype=torch.float64, device=dev) for q in insts]
        bs = bte.BatchSolver(insts, precision="fp32")
        bs.solve(Qs, tol=tol_b, check_every=8)  # warm-up (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Ts, _, reps = bs.solve(Qs, tol=tol_b, check_every=8)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        singles = [bte.Solver(q, precision="fp32", plan=bs.plan()) for q in insts]
        for s1, q1 in zip(singles, Qs):
            s1.solve(q1, tol=tol_b, check_every=8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        worst = 0.0
        for s1, q1, Tb in zip(singles, Qs, Ts):
            T1, _, _ = s1.solve(q1, tol=tol_b, check_every=8)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        for s1, q1, Tb, q in zip(singles, Qs, Ts, insts):
            T1, _, _ = s1.solve(q1, tol=tol_b, check_every=8)
            worst = max(worst, float((T1 - Tb).abs().max() / (Tb - 300.0).abs().max()))
        n_ok = sum(r["status"] == "ok" for r in reps)
        extra["batch"] = dict(instances=len(insts), kn_min=args.batch_kn_min, converged=n_ok, tol=tol_b,
                              batched_solves_per_s=len(insts) / tb, sequential_solves_per_s=len(insts) / ts,
                              speedup=ts / tb, max_rel_diff_batched_vs_single=worst,
                              iters_min=min(r["iters"] for r in reps), iters_max=max(r["iters"] for r in reps))
        log(f"batch: {len(insts)} instances, {len(insts)/tb:.1f} solves/s batched vs {len(insts)/ts:.1f} sequential")

    out = {
        "metric": "cell-ordinate-band updates/s",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D nongray square 256x256, 15 bands, 128 directions "
                               "(64 in-plane projections swept), Gaussian hot spot, isothermal edges",
                   "cells": p.n_active, "bands": p.B, "directions": p.M, "directions_swept": M_swept,
                   "plan": plan, "parallelism": "single GPU"},
        "roofline": roofline,
    }
    out.update(extra)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_iters, M_swept)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
