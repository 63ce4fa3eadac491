#!/usr/bin/env python3
"""Benchmark of the RS canonical/Tucker potential path on one MI355X.

One step = one RS assembly of the workload's particle system: side matrices,
charge-weighted Gram GEMMs, eigensolve and rank rule, projection, core,
short-range windows and the full n^3 grid, followed by the interaction
energy and the forces.  Inputs (positions, charges, quadrature table) are
resident on the device before the timed region.  Prints one JSON line.

Default workload: 10x10x10 lattice, spacing 1.0, 100 vacancies, jitter
N(0, 0.05^2), alternating +-1 charges (N = 900); box [-12,12]^3, n = 512,
R = 24, R_l = 10, n_s = 17, Tucker tolerance 1e-6, FP64.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RS assemblies/sec at rel-L∞≤1e-5 vs plain FP64 on GPU; p50/p99 latency"
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "fp16": 2500.0}


def workload(name: str):
    import workloads
    if name == "cfg2":
        s = workloads.cfg2_lattice()
        cfg = {"workload": "lattice10^3_vac100_N900_n512_R24_Rl10_ns17",
               "N": s.N, "n": s.n, "b": s.b, "R": s.R, "R_l": s.R_l, "n_s": s.n_s,
               "eps_tucker": s.eps_tucker, "kernel": s.kernel, "r_max": 112}
        return s, cfg, 112
    if name == "cfg1":
        s = workloads.cfg1_plain_small()
        cfg = {"workload": "uniform64_n128_R20_Rl8_ns9", "N": s.N, "n": s.n, "b": s.b, "R": s.R,
               "R_l": s.R_l, "n_s": s.n_s, "eps_tucker": s.eps_tucker, "kernel": s.kernel,
               "r_max": 128}
        return s, cfg, 128
    raise SystemExit(f"unknown workload {name}")


def kernel_source_hash() -> str:
    """Hash of the source file of the FP64 GEMM kernels: traffic counters
    taken on another version of it are stale."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1606_09218_amd", "csrc")
    for f in ("k_gemm64.hip",):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_tag: str, workload_tag: str):
    """HBM bytes per launch of the dominant kernel from committed rocprofv3
    --pmc summaries, if they were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_tag}_{workload_tag}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(s, budget_s: float = 20.0):
    """The oracle (plain FP64 NumPy), timed on this host on a bounded sample
    of one step: the full RS-Tucker build (side matrices, SVD of the weighted
    side matrices, core), grid values on a few i1-planes, and energy and
    forces for a subset of particles; scaled to one full step."""
    import numpy as np
    from oracle import canonical, pointeval, rs
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [os.cpu_count() or 1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    T = rs.assemble_system(s)
    t_build = time.perf_counter() - t0
    n = s.n
    planes = 2
    t0 = time.perf_counter()
    for i1 in range(n // 2, n // 2 + planes):
        long_plane = np.einsum("abc,a,jb,kc->jk", T.beta, T.Q[0][i1], T.Q[1], T.Q[2], optimize=True)
        ii = np.stack(np.meshgrid([i1], np.arange(n), np.arange(n), indexing="ij"), -1).reshape(-1, 3)
        short_plane = canonical.short_range_at(ii, s.b, n, T.pos, T.q, T.t, T.a, T.R_l, T.n_s)
        _ = long_plane.ravel() + short_plane
    t_grid = (time.perf_counter() - t0) * n / planes
    m = min(16, s.N)
    sub = rs.RSTucker(T.b, T.n, T.t, T.a, T.R_l, T.n_s, T.pos[:m], T.q[:m], T.Q, T.beta,
                      T.sigma, T.ranks)
    t0 = time.perf_counter()
    pointeval.energy(sub)
    pointeval.forces(sub)
    t_ef = (time.perf_counter() - t0) * s.N / m
    total = t_build + t_grid + t_ef
    return {"value": 1.0 / total, "unit": "assemblies/s", "cores": cores, "kind": "oracle",
            "sample": (f"oracle RS-Tucker build of the full system ({t_build:.1f} s) + grid on "
                       f"{planes} of {n} i1-planes (scaled x{n // planes}) + energy/forces for "
                       f"{m} of {s.N} particles (scaled); one step = {total:.1f} s")}


def cpu_baseline_child(workload_name: str):
    """cpu_baseline in a child process started before this process touches
    the GPU, so that the oracle's BLAS threads never share a process with
    the HIP runtime; returns its result (or the child's error)."""
    import subprocess
    print("cpu baseline: oracle sample in a child process", file=sys.stderr, flush=True)
    try:
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only",
                            "--workload", workload_name], capture_output=True, text=True,
                           timeout=900)
    except subprocess.TimeoutExpired:
        return {"error": "oracle child did not finish within 900 s"}
    if r.returncode != 0 or not r.stdout.strip():
        return {"error": f"oracle child exited with status {r.returncode}: {r.stderr[-400:]}"}
    try:
        return json.loads(r.stdout.strip().splitlines()[-1])
    except ValueError:
        return {"error": "oracle child printed no result line"}


def timed_steps(step, steps, stream, starts=None, ends=None):
    """Run `steps` steps back to back and return (wall seconds, per-step stage
    times, ranks of the first step).  Each step's result is released as soon
    as the next step has passed its rank readback (which orders it after the
    whole previous step), so its device memory is reused as in a serving loop
    rather than held until the end."""
    import torch
    stages, ranks, prev = [], None, None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        if starts is not None:
            starts[i].record(stream)
        h = step()
        if ends is not None:
            ends[i].record(stream)
        if prev is not None:
            stages.append(prev.stage_ms())
            if ranks is None:
                ranks = list(prev.info().ranks)
            prev.free()
        prev = h
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stages.append(prev.stage_ms())
    if ranks is None:
        ranks = list(prev.info().ranks)
    prev.free()
    return wall, stages, ranks


def mixed_leg(rsm, ctx, f, pos, q, s, r_max, grid64, steps, warmup, stream):
    """The same step with split-FP16 core and grid expansion (FP32 grid):
    throughput and its error against the FP64 GPU result of the same input."""
    import numpy as np
    import torch
    out = {}
    E64 = torch.empty(1, dtype=torch.float64, device=grid64.device)
    T = rsm.assemble(ctx, f, pos, q, grid64, rsm.make_aopts(s.eps_tucker, r_max=r_max), stream=stream)
    rsm.energy(T, E64, stream=stream)
    ranks = list(T.info().ranks)
    T.free()
    for prec in ("mixed_fp16", "mixed_bf16"):
        g32 = torch.empty(s.n ** 3, dtype=torch.float32, device=grid64.device)
        E = torch.empty(1, dtype=torch.float64, device=grid64.device)
        F = torch.empty(3 * s.N, dtype=torch.float64, device=grid64.device)
        # same options as the FP64 step: the eigen stage is FP64 in both paths,
        # so ranks and subspace size agree
        opts = rsm.make_aopts(s.eps_tucker, r_max=r_max, prec=prec)

        def step():
            T = rsm.assemble(ctx, f, pos, q, g32, opts, stream=stream)
            rsm.energy_forces(T, E, F, 1.0, stream=stream)
            return T

        for _ in range(warmup):
            step().free()
        ctx.set_timing(2)
        wall, st, ranks_m = timed_steps(step, steps, stream)
        ctx.set_timing(1)
        _, st1, _ = timed_steps(step, min(steps, 5), stream)
        same_ranks = ranks_m == ranks
        err = float((g32.double() - grid64).abs().max() / grid64.abs().max())
        e_err = abs(E.item() - E64.item()) / abs(E64.item())
        out[prec] = {"value": round(steps / wall, 4), "unit": "assemblies/s",
                     "ms_per_step": round(wall / steps * 1e3, 3),
                     "grid_rel_linf_vs_fp64": err, "energy_rel_err_vs_fp64": e_err,
                     "meets_1e-5": bool(err <= 1e-5), "same_ranks_as_fp64": same_ranks,
                     "core_ms": round(float(np.mean([x["core"] for x in st1])), 4),
                     "grid_ms": round(float(np.mean([x["grid"] for x in st])), 4)}
    return out


def serving_leg(n_requests: int, n_slots: int = 4, prec: str = "mixed_fp16"):
    """The first `n_requests` requests of the seeded Poisson serving trace
    (rate 200/s; N log-uniform in [32, 20000]; n in {256, 512, 1024}; R in
    24..32), replayed in real time through the continuous-batching server,
    then the same requests all present at t = 0 (saturating).  Latency is
    arrival to result (energy and ranks on the host)."""
    import torch

    import workloads
    from paper_1606_09218_amd.serve import GpuExecutor, Server, summarize
    trace = workloads.cfg5_trace(seed=5, n_requests=n_requests)
    ex = GpuExecutor(0, prec=prec, r_max=384)
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.85 * free)
    # factors of every (n, R) in the trace are built before the clock starts
    # (device-resident tables, as in a long-running server)
    for r in trace:
        ex.factors(r.system())
    out = {"requests": n_requests, "slots": n_slots, "prec": prec, "hbm_budget_GB": round(budget / 2**30, 1),
           "trace": "Poisson 200/s, seed 5 (first requests of the 2000-request trace)"}
    for label, scale in (("poisson", 1.0), ("saturating", 0.0)):
        print(f"serving leg: {label} replay of {n_requests} requests", file=sys.stderr, flush=True)
        srv = Server(ex, n_slots=n_slots, hbm_budget=budget)
        recs = srv.run_trace(trace, time_scale=scale)
        sm = summarize(recs)
        sm["peak_concurrency"] = srv.peak_concurrency
        out[label] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in sm.items()}
        errs = [r.error for r in recs if r.error]
        if errs:
            out[label]["first_error"] = errs[0]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests of the serving trace to replay (0: skip the serving leg)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain device copy of known size (for PMC scaling)")
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="print only the oracle CPU baseline (no GPU use)")
    args = ap.parse_args()
    if args.cpu_baseline_only:
        s, _, _ = workload(args.workload)
        print(json.dumps(cpu_baseline(s)), flush=True)
        return False
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(every workload here runs on a single MI355X).", file=sys.stderr)
        sys.exit(2)

    cpu = None if args.no_cpu_baseline else cpu_baseline_child(args.workload)

    import numpy as np
    import torch

    import paper_1606_09218_amd as rsm

    s, cfg, r_max = workload(args.workload)
    dev = torch.device("cuda:0")
    ctx = rsm.Context(0)
    ctx.set_timing(True)
    f = rsm.Factors(ctx, s.b, s.n, s.R, s.R_l, s.n_s, kernel=s.kernel, lam=s.lam,
                    delta_rel=s.delta_rel)
    pos = torch.tensor(s.pos, dtype=torch.float64, device=dev)
    q = torch.tensor(s.q, dtype=torch.float64, device=dev)
    grid = torch.empty(s.n ** 3, dtype=torch.float64, device=dev)
    E = torch.empty(1, dtype=torch.float64, device=dev)
    F = torch.empty(3 * s.N, dtype=torch.float64, device=dev)
    opts = rsm.make_aopts(s.eps_tucker, r_max=r_max)
    stream = torch.cuda.current_stream()

    def step():
        T = rsm.assemble(ctx, f, pos, q, grid, opts, stream=stream)
        rsm.energy_forces(T, E, F, 1.0, stream=stream)
        return T

    for _ in range(args.warmup):
        step().free()
    torch.cuda.synchronize()

    # the timed steps carry only the two events around the grid kernel (the
    # roofline kernel); the per-stage breakdown comes from separate steps
    # after the timed region, so that its markers do not slow the value
    ctx.set_timing(2)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    wall, grid_stages, ranks = timed_steps(step, args.steps, stream, starts, ends)
    lat = np.array([a.elapsed_time(b) for a, b in zip(starts, ends)])
    ctx.set_timing(1)
    _, stages, _ = timed_steps(step, min(args.steps, 5), stream)

    stage_avg = {k: float(np.mean([st[k] for st in stages])) for k in stages[0]}
    n, r3 = s.n, ranks[2]
    # dominant single kernel: the grid expansion (one launch), timed over the timed steps
    grid_ms = float(np.mean([st["grid"] for st in grid_stages]))
    t_grid = grid_ms * 1e-3
    flops_grid = 2.0 * n ** 3 * r3
    bytes_grid = 8.0 * (n ** 3 + n * n * r3 + n * r3)
    achieved = flops_grid / t_grid / 1e12
    traffic = traffic_from_profiles("grid64_stream", args.workload)
    # the streaming grid kernel's column panel: the widest whose V3 rows fit 150 KB of LDS
    kp = (r3 + 31) // 32 * 32
    bn = next((b for b in (128, 64, 32) if kp * (b + 2) * 8 <= 150 * 1024), None)
    kname = (f"rs::grid64_stream_kernel<{bn}, 16>" if bn else
             "rs::gemm_kernel<rs::Cfg<4, 2, 2, 4, 16, 16>, false, false>")
    roofline = {"kernel": kname + " (grid = T2 x_3 V3)",
                "bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS["f64"],
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS["f64"], 4),
                "traffic": traffic,
                "algorithmic_flops_per_launch": flops_grid,
                "algorithmic_bytes_per_launch": bytes_grid,
                "achieved_hbm_GBs_algorithmic": round(bytes_grid / t_grid / 1e9, 1),
                "avg_launch_ms": round(grid_ms, 4)}

    if args.calibrate_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    ms_per_step = wall / args.steps * 1e3
    out = {
        "metric": METRIC,
        "value": round(args.steps / wall, 4),
        "unit": "assemblies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": cfg,
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "ranks": ranks,
        "stage_ms": {k: round(v, 4) for k, v in stage_avg.items()},
        "roofline": roofline,
    }
    if not args.no_mixed:
        out["mixed"] = mixed_leg(rsm, ctx, f, pos, q, s, r_max, grid, args.steps, args.warmup, stream)
    if args.serve_requests > 0:
        try:
            out["serving"] = serving_leg(args.serve_requests)
        except Exception as e:  # reported in the line rather than losing it
            out["serving"] = {"error": f"{type(e).__name__}: {e}"}
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    return args.serve_requests > 0


if __name__ == "__main__":
    if main():
        # after the serving leg the line is out: leave without the
        # interpreter's and the runtimes' teardown (one full run with the
        # serving leg crashed there, after every result had been printed).
        # Runs without it end normally, so that a profiler attached to them
        # still writes its output at exit.
        sys.stdout.flush()
        sys.stderr.flush()
        os._exit(0)
