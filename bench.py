"""Benchmark: cell x ordinate x band updates/s of whole source iterations on
the 3D FinFET-like domain (96 x 96 x 120 voxel mask, 876,544 active cells,
15 bands, 128 directions, FP32 sweeps with FP64 band sums; isothermal
substrate bottom, every other wall diffusely reflecting), the largest
workload of the benchmark set on one GPU. Extra fields: the same rate on the
2D nongray square (256 x 256, 15 bands, 64 in-plane projections swept), the
adjoint/forward time ratio, and batched vs sequential solves/s over all 256
instances of the batch workload.

One step is one source iteration of the whole hot path on the whole problem:
the fused transport sweep of every (band, direction) pair with the band /
direction reduction, the new temperature and the lagged diffuse-wall values,
replayed from a captured hipGraph. The timed run is K iterations with the
convergence test once at the end (tolerance 0, as the paper times a fixed
iteration count): the heat flux and the residuals of Eq. 22 are formed in the
last two iterations, as in any solve that checks every K iterations. Inputs
are resident in HBM before the timed region.

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
# algorithmic flop per (cell, ordinate, band) update, as the scope's measurement
# section counts them: temperature-only iterations / iterations with the flux
FLOP_PER_UPDATE = {2: (7.0, 11.0), 3: (9.0, 15.0)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(p, iters: int, m_swept: int, single=None):
    """The FP64 oracle timed on the host over a bounded number of iterations,
    as a rate in the metric's own counting, on all host threads; `single`
    (problem, iterations, note) adds a one-thread rate on a smaller sample."""
    import oracle
    threads = oracle.num_threads()
    upd = p.n_active * m_swept * p.B
    t0 = time.perf_counter()
    oracle.solve(p, tol=0.0, max_iters=iters, threads=threads)
    dt = time.perf_counter() - t0
    out = dict(value=upd * iters / dt, unit="updates/s", cores=threads, kind="oracle",
               sample=f"{iters} source iterations of the full problem ({p.n_active} cells, {p.B} bands, "
                      f"{p.M} directions) in FP64, {dt:.1f} s")
    if single is not None:
        q, it1, note = single
        t0 = time.perf_counter()
        oracle.solve(q, tol=0.0, max_iters=it1, threads=1)
        dt1 = time.perf_counter() - t0
        out["single_thread"] = dict(value=q.n_active * m_swept * q.B * it1 / dt1, unit="updates/s", cores=1,
                                    sample=f"{it1} source iterations of {note}, {dt1:.1f} s")
    return out


def source_hash(files) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2503_23657_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


SOURCES_2D = ("bte_sweep2d.hip", "bte_sweep2d_launch.h", "bte_kutil.h", "bte_device.h", "bte_strips.h")
SOURCES_3D = ("bte_sweep2d.hip", "bte_sweep2d_launch.h", "bte_sweep3r_f.hip", "bte_kutil.h", "bte_device.h",
              "bte_strips.h")


def profiled_traffic(summary: str, kernel: str, files):
    """HBM bytes per launch of `kernel` from a committed counter summary under
    profiles/, or None when it holds none for this kernel or the kernel's
    sources changed since the counters were taken. The summary lists
    `- sweep source hash: ...` and `- hbm bytes per launch of <kernel>: <bytes>`."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].rsplit(":", 1)
                kv[k.strip().replace("`", "")] = v.strip().strip("`")
    try:
        if kv.get("sweep source hash") != source_hash(files):
            return None
        return float(kv[f"hbm bytes per launch of {kernel}"])
    except (KeyError, ValueError, OSError):
        return None


def timed_iterations(solver, Q, K, warmup):
    """K whole iterations from a graph replay, after `warmup` untimed ones (which
    also capture the graphs); returns seconds."""
    import torch
    solver.solve(Q, tol=0.0, max_iters=max(warmup, 2), check_every=K)
    solver.solve(Q, tol=0.0, max_iters=K, check_every=K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.solve(Q, tol=0.0, max_iters=K, check_every=K)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def roofline_of(solver, n_upd, dim, summary, files):
    """The dominant kernel (the forward sweep) timed with HIP events on the
    solver's stream; achieved = algorithmic flop per launch / that time."""
    sweep_ms, _ = solver.time_sweep(n_launches=20)
    flop = n_upd * FLOP_PER_UPDATE[dim][0]
    achieved = flop / (sweep_ms * 1e-3) / 1e12
    kname = solver.sweep_kernel_name()
    traffic = profiled_traffic(summary, kname, files)
    r = dict(bound="alu", achieved=achieved, peak=FP32_VALU_PEAK_TFLOPS, unit="TFLOP/s",
             frac=achieved / FP32_VALU_PEAK_TFLOPS, traffic=traffic, kernel=kname, kernel_ms=sweep_ms,
             flop_per_update=FLOP_PER_UPDATE[dim][0], sweep_updates_per_s=n_upd / (sweep_ms * 1e-3))
    if traffic is not None:
        gbs = traffic / (sweep_ms * 1e-3) / 1e9
        r.update(hbm_gbs=gbs, hbm_peak_gbs=HBM_PEAK_GBS, hbm_frac=gbs / HBM_PEAK_GBS)
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=2)
    ap.add_argument("--workload", choices=("finfet", "square"), default="finfet",
                    help="headline workload (the square runs as an extra field of the default line)")
    ap.add_argument("--plan", type=str, default=None,
                    help="fixed kernel plan 'G,R,P,C,NR' for the headline workload")
    ap.add_argument("--order", type=int, choices=(1, 2), default=1,
                    help="face reconstruction of the headline workload (2: second-order faces; for profiling)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of 256 MiB three times (calibrates the HBM byte counters)")
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
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import bte_inputs as bi
    import paper_2503_23657_amd as bte

    dev = torch.device("cuda:0")
    K = max(4, args.steps)

    def plan_arg(s):
        if args.plan:
            G_, R_, P_, C_, NR_ = (int(x) for x in args.plan.split(","))
            s.set_plan(G=G_, R=R_, P=P_, C=C_, NR=NR_)

    # ------------------------------------------------ headline workload
    if args.workload == "finfet":
        p = bi.finfet_3d(scale=1)
        M_swept = p.M
        wl = dict(workload="3D FinFET-like voxel domain 96x96x120 (substrate slab + seeded fin), 15 bands, "
                           "128 directions, fin-top heat source, isothermal bottom, diffuse other walls",
                  cells=p.n_active, bands=p.B, directions=p.M, directions_swept=M_swept)
        summary, files, dim = "sweep3d_finfet_hbm_counters.md", SOURCES_3D, 3
    else:
        p = bi.square_2d(256)
        M_swept = 64
        wl = dict(workload="2D nongray square 256x256, 15 bands, 128 directions (64 in-plane projections "
                           "swept), Gaussian hot spot, isothermal edges",
                  cells=p.n_active, bands=p.B, directions=p.M, directions_swept=M_swept)
        summary, files, dim = "sweep2d_square256_hbm_counters.md", SOURCES_2D, 2
    solver = bte.Solver(p, precision="fp32")
    Q = torch.tensor(p.Q, dtype=torch.float64, device=dev)
    if args.order == 2:
        solver.set_order(2)
    plan_arg(solver)
    plan = solver.plan()
    log("plan", plan)
    dt = timed_iterations(solver, Q, K, args.warmup)
    n_upd = p.n_active * M_swept * p.B
    value = n_upd * K / dt
    ms_per_step = dt / K * 1e3
    log(f"{args.workload}: {K} iterations in {dt:.4f} s -> {value:.4e} updates/s")
    roofline = roofline_of(solver, n_upd, dim, summary, files)
    log(f"sweep {roofline['kernel']}: {roofline['kernel_ms']:.3f} ms")
    extra = {}
    if args.workload == "finfet" and not args.no_extra:
        solver.close()
        # ------------------------- the same domain with second-order faces
        s3o = bte.Solver(p, precision="fp32")
        s3o.set_order(2)
        K3o = 8
        dt3o = timed_iterations(s3o, Q, K3o, 2)
        extra["finfet_second_order"] = dict(updates_per_s=n_upd * K3o / dt3o, ms_per_step=dt3o / K3o * 1e3,
                                            steps=K3o, plan=s3o.plan(), sweep_ms=s3o.time_sweep(n_launches=3)[0])
        s3o.close()
        log(f"finfet, second order: {n_upd * K3o / dt3o:.4e} updates/s")
        # ------------------------------------------- the 2D square
        p2 = bi.square_2d(256)
        s2 = bte.Solver(p2, precision="fp32", plan=dict(G=1, R=1, P=4, NR=4))
        Q2 = torch.tensor(p2.Q, dtype=torch.float64, device=dev)
        K2 = max(20, K)
        dt2 = timed_iterations(s2, Q2, K2, args.warmup)
        n2 = p2.n_active * 64 * p2.B
        extra["square_2d"] = dict(
            workload="2D nongray square 256x256, 15 bands, 64 in-plane projections swept, FP32 sweeps",
            updates_per_s=n2 * K2 / dt2, ms_per_step=dt2 / K2 * 1e3, steps=K2, plan=s2.plan(),
            roofline=roofline_of(s2, n2, 2, "sweep2d_square256_hbm_counters.md", SOURCES_2D))
        log(f"square: {n2 * K2 / dt2:.4e} updates/s")
        # the same square with second-order faces (deferred correction: the
        # sweep reads each ordinate's correction and stores its field, and a
        # correction kernel runs after every iteration)
        s2o = bte.Solver(p2, precision="fp32", plan=dict(G=1, R=1, P=4, NR=4))
        s2o.set_order(2)
        dt2o = timed_iterations(s2o, Q2, K2, args.warmup)
        extra["square_2d_second_order"] = dict(updates_per_s=n2 * K2 / dt2o, ms_per_step=dt2o / K2 * 1e3, steps=K2,
                                               sweep_ms=s2o.time_sweep(n_launches=10)[0])
        s2o.close()
        log(f"square, second order: {n2 * K2 / dt2o:.4e} updates/s")
        # ------------------------- adjoint / forward time at equal tolerance
        tol = 1e-6
        t0 = time.perf_counter()
        T, _, rf = s2.solve(Q2, tol=tol, check_every=8, store_state=True)
        torch.cuda.synchronize()
        tf = time.perf_counter() - t0
        case = bi.adjoint_case(p2)
        probes = torch.tensor(case["probes"], device=dev)
        Tt = T.detach().clone().requires_grad_(True)
        target = T.detach()[probes] + 1.0
        (gT,) = torch.autograd.grad(((Tt[probes] - target) ** 2).mean(), Tt)
        t0 = time.perf_counter()
        _, _, ra = s2.adjoint(gT.contiguous(), tol=tol, check_every=8)
        torch.cuda.synchronize()
        ta = time.perf_counter() - t0
        extra.update(adjoint_forward_ratio=ta / tf, forward_solve_s=tf, forward_iters=rf["iters"],
                     adjoint_solve_s=ta, adjoint_iters=ra["iters"],
                     adjoint_workload="the 2D square at tolerance 1e-6, loss on 64 probe cells")
        log(f"adjoint/forward = {ta / tf:.3f} ({ra['iters']} vs {rf['iters']} iterations)")
        s2.close()
        # ------------------------------ batched vs sequential, all 256 instances
        insts = bi.batch_instances()
        tol_b = 1e-6
        Qs = [torch.tensor(q.Q, dtype=torch.float64, device=dev) for q in insts]
        bs = bte.BatchSolver(insts, precision="fp32")
        bs.solve(Qs, tol=tol_b, check_every=16, max_iters=20000)  # warm-up (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Ts, _, reps = bs.solve(Qs, tol=tol_b, check_every=16, max_iters=20000)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        bplan = bs.plan()
        bs.close()
        singles = [bte.Solver(q, precision="fp32", plan=bplan) for q in insts]
        for s1, q1 in zip(singles, Qs):
            s1.solve(q1, tol=tol_b, check_every=16, max_iters=20000)  # warm-up (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = [s1.solve(q1, tol=tol_b, check_every=16, max_iters=20000) for s1, q1 in zip(singles, Qs)]
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        worst = max(float((o[0] - Tb).abs().max() / (Tb - 300.0).abs().max()) for o, Tb in zip(outs, Ts))
        for s1 in singles:
            s1.close()
        its = np.array([r["iters"] for r in reps])
        kn = np.array([q.Kn for q in insts])
        status = {}
        for r in reps:
            status[r["status"]] = status.get(r["status"], 0) + 1
        extra["batch"] = dict(
            instances=len(insts), kn_range=[float(kn.min()), float(kn.max())], cells=int(sum(q.n_active for q in insts)),
            tol=tol_b, status=status, batched_solves_per_s=len(insts) / tb, sequential_solves_per_s=len(insts) / ts,
            batched_s=tb, sequential_s=ts, speedup=ts / tb, max_rel_diff_batched_vs_single=worst, plan=bplan,
            iters_min=int(its.min()), iters_median=float(np.median(its)), iters_max=int(its.max()),
            iters_kn_below_0p05=int(its[kn < 0.05].sum()), iters_total=int(its.sum()))
        log(f"batch: {len(insts)} instances, {len(insts) / tb:.1f} solves/s batched vs {len(insts) / ts:.1f} "
            f"sequential; status {status}; iterations {its.min()}..{its.max()}")

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
        "config": dict(wl, plan=plan, parallelism="single GPU"),
        "roofline": roofline,
    }
    out.update(extra)
    if not args.no_cpu:
        if args.workload == "finfet":
            q = bi.finfet_3d(scale=4)
            out["cpu_baseline"] = cpu_baseline(p, args.cpu_iters, M_swept,
                                               single=(q, 2, "the same domain at a quarter of its size per axis"))
        else:
            out["cpu_baseline"] = cpu_baseline(p, 12, M_swept, single=(p, 2, "the same problem"))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
