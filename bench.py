"""Benchmark: RK-stage cell-updates/s of WCNS-T on one MI355X.

Default workload (`--workload quadrant2d`): 2D Euler four-quadrant Riemann problem (Sec. 3.6.1 states) on
[0,1]^2, 2048 x 2048 cells, FP64, characteristic-wise TENO-5 interpolation,
Roe flux, MND difference, SSP-RK3, CFL 0.5, zero-gradient boundaries.  One
benchmark step = one SSP-RK3 step (three fused stage kernels, CFL reduction
fused into the third) over the whole grid.  The state is reset to the
initial condition after warm-up, so the timed region is steps 1..K of the
problem (K = 200 by default, the full fixed-step run).

Prints one JSON line.  `roofline` prices the stage kernel against the FP64
vector peak with the algorithmic flop count per stage-cell-update (see
`flops_per_stage_cell`); `cpu_baseline` times the CPU oracle on one full
SSP-RK3 step of the same grid on the host cores.  The default line also
carries the two systems workloads as sub-records, `tubes` and `serve`
(below), each with its per-solve comparison on the same GPU (leave them out
with `--no-systems`).

`--workload serve`: a Poisson stream of mixed requests (70 % 1D tubes with
N in [512, 16384] to t = 0.15, 30 % 2D random four-quadrant problems of
side 256-1024 to t = 0.1) served with continuous batching from an HBM
arena; the arrival rate is `--load` x the capacity measured with all
requests queued at once.  Reports p50/p99 time-to-solution and throughput,
beside the plain path (one wcnst_solve per request, FIFO) on the same
arrival times.

`--workload tubes`: 4096 independent 1D Euler shock tubes of uneven length
(N log-uniform in [256, 8192], random left/right states, t = 0.15, Roe,
characteristic TENO, MND) advanced to their final times by the batched
solver (graph-captured ticks of multi-instance stage launches).  One benchmark step = the
whole batch solved once.  Also times the plain one-solve-per-instance path
on a seeded subset of the same tubes and the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
N_SIDE = 2048


TRAFFIC_FILE = os.path.join(ROOT, "paper_1810_07806_amd", "traffic.json")


def kernel_source_hash() -> str:
    """Hash of the sources of the stage kernels (counter figures taken on
    another build of them are not reported)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("wcnst_kernels.hip", "wcnst_device.hpp"):
        with open(os.path.join(ROOT, "paper_1810_07806_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_record(workload: str):
    """Counter figures of the dominant kernel (HBM bytes per launch from
    FETCH_SIZE and WRITE_SIZE runs scaled by the same counters on a plain
    copy of known size; VALU busy fraction from SQ counters), or None when
    they were taken on other kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        rec = json.load(f).get(workload)
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec


def measured_traffic(workload: str):
    """HBM bytes per launch of the dominant kernel (see counter_record)."""
    rec = counter_record(workload)
    return rec["hbm_bytes_per_launch"] if rec else None


def flops_per_stage_cell() -> dict:
    """Algorithmic flops of one stage-cell-update of 2D Euler WCNS-T (Roe,
    TENO, characteristic-wise, MND), counting +, -, *, /, sqrt as written in
    the method (Sec. 2-3), a 4-term dot product as 7.  Per midpoint:"""
    interp = 42 + 46          # candidates + beta (Eqs. 9-11, 15); TENO Eqs. 16-19
    eigen = 85                # Roe average, c, b1, b2, R and L entries
    midpoint = (eigen         # projection basis at nodes j, j+1
                + 6 * 4 * 7   # project six nodes
                + 2 * 4 * interp
                + 2 * 4 * 7   # back-project u_L, u_R
                + 2 * 14 + eigen + 4 + 4 * 7 + 4 + 4 * 7 + 12)  # Roe flux
    per_cell = (2 * midpoint  # one x- and one y-midpoint per cell
                + 2 * 14      # node fluxes f(U_i), g(U_i)
                + 2 * 4 * 8   # MND, Eq. (5)
                + 4           # R = R_x + R_y
                + 16          # Shu-Osher stage combination (mean of 8, 20, 20)
                + 6)          # CFL speed (18 per cell per step)
    return dict(interp=interp, midpoint=midpoint, per_stage_cell=per_cell)


def bytes_per_stage_cell() -> float:
    """Minimum HBM bytes of the fused stage: read U^(k) (32 B), read U^n in
    stages 2 and 3 (32 B), write U^(k+1) (32 B)."""
    return (3 * 32 + 2 * 32 + 3 * 32) / 3.0


def flops_per_stage_cell_1d() -> dict:
    """Algorithmic flops of one stage-cell-update of 1D Euler WCNS-T (Roe,
    TENO, characteristic-wise, MND), counted as for 2D with 3 variables and
    3-term dot products (5 flops).  Per midpoint:"""
    interp = 42 + 46
    eigen = 55                # Roe average, c, R and L entries (1D)
    midpoint = (eigen
                + 6 * 3 * 5   # project six nodes
                + 2 * 3 * interp
                + 2 * 3 * 5   # back-project u_L, u_R
                + 2 * 9 + eigen + 3 + 3 * 5 + 3 + 3 * 5 + 9)  # Roe flux
    per_cell = (midpoint
                + 9           # node flux f(U_i)
                + 3 * 8       # MND, Eq. (5)
                + 12          # Shu-Osher stage combination (mean of 6, 15, 15)
                + 6)          # CFL speed (18 per cell per step)
    return dict(interp=interp, midpoint=midpoint, per_stage_cell=per_cell)


def cpu_baseline(steps: int = 1) -> dict:
    import numpy as np

    import oracle
    from paper_1810_07806_amd import workloads as W
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    d, U = W.riemann2d_config3(N_SIDE)
    p = oracle.problem(d)
    oracle.lib()
    t0 = time.perf_counter()
    V = U
    for k in range(steps):
        dt = 0.5 / oracle.max_speed(p, V)
        V, st, _, _ = oracle.rk3_step(p, V, dt, stage_base=3 * k, nthreads=cores)
        assert st == 0
    el = time.perf_counter() - t0
    units = 3.0 * steps * N_SIDE * N_SIDE
    return {"value": units / el, "unit": "stage-cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} SSP-RK3 step(s) of the {N_SIDE}x{N_SIDE} four-quadrant state "
                      f"({el:.1f} s wall on {cores} threads)"}


def _oracle_tube_steps(job):
    """Worker: `steps` oracle RK3 steps of one tube (process pool)."""
    import oracle
    d, U, steps = job
    p = oracle.problem(d)
    done = 0
    for k in range(steps):
        s = oracle.max_speed(p, U)
        if not (s > 0 and math.isfinite(s)):
            break
        U, st, _, _ = oracle.rk3_step(p, U, 0.5 / s, stage_base=3 * k, nthreads=1)
        if st != 0:
            break
        done += 1
    return 3 * done * d["nx"]


def cpu_baseline_tubes(items, idx, steps: int) -> dict:
    from concurrent.futures import ProcessPoolExecutor
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    jobs = [(items[int(i)][0], items[int(i)][1], steps) for i in idx]
    t0 = time.perf_counter()
    with ProcessPoolExecutor(cores) as ex:
        units = sum(ex.map(_oracle_tube_steps, jobs))
    el = time.perf_counter() - t0
    return {"value": units / el, "unit": "stage-cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} SSP-RK3 steps of each of {len(jobs)} seeded tubes of the batch, one process "
                      f"per core ({el:.1f} s wall incl. pool start-up)"}


def bench_tubes(args):
    import numpy as np
    import torch

    from paper_1810_07806_amd import autotune
    from paper_1810_07806_amd import workloads as W
    from paper_1810_07806_amd.wcnst import Batch, Solver

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    count, seed, t_final = args.count, args.seed, 0.15
    items = W.shock_tube_batch(count=count, seed=seed, t_final=t_final, n_min=args.n_min, n_max=args.n_max)
    descs = [d for d, _ in items]
    b = Batch(descs)
    U0 = b.pack([U for _, U in items])
    Ug = torch.empty_like(U0)
    log(f"tubes: {count} instances, {int(sum(d['nx'] for d in descs))} cells")
    if args.steps_per_tick:
        b.set_tuning(args.steps_per_tick)
        b.set_persist(args.switch_strips, args.persist_waves, args.persist_group)
        tune = dict(steps_per_tick=args.steps_per_tick, switch_strips=args.switch_strips,
                    waves_per_group=args.persist_waves, instances_per_group=args.persist_group, cached=False, table=[])
    else:
        tune = autotune.tune_batch(b, U0, t_final, cfl=0.5, cache=args.tune_cache,
                                   device_name=torch.cuda.get_device_name(0), log=log)
    log(f"tuning: steps/tick={tune['steps_per_tick']} persistent switch={tune['switch_strips']} strips "
        f"({tune['waves_per_group']} waves x {tune['instances_per_group']} per workgroup)")
    for _ in range(args.warmup):
        Ug.copy_(U0)
        b.solve(Ug, t_final * 0.05, cfl=0.5)
    units = 0.0
    wall = 0.0
    kernel_ms = []
    for k in range(args.steps):
        Ug.copy_(U0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = b.solve(Ug, t_final, cfl=0.5)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        kernel_ms.append(b.kernel_ms())
        stats = b.stats()
        units += float(np.sum(3.0 * res["steps"] * np.array([d["nx"] for d in descs])))
        log(f"batch solve {k}: {kernel_ms[-1]:.1f} ms kernel")
    failed = int(np.count_nonzero(res["status"]))
    units_per_solve = units / args.steps
    avg_kernel_s = float(np.mean(kernel_ms)) / 1e3

    # plain path: one wcnst_solve per instance, on a seeded subset
    rng = np.random.default_rng(seed + 1)
    sub = np.sort(rng.choice(count, size=min(args.per_solve, count), replace=False))
    ps_units, ps_wall = 0.0, 0.0
    for i in sub:
        d, U = items[int(i)]
        s = Solver(d)
        V = s.new_state(U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            _, n = s.solve(V, t_final=t_final, cfl=0.5)
        except Exception:
            n = s.status()["steps"]
        torch.cuda.synchronize()
        ps_wall += time.perf_counter() - t0
        ps_units += 3.0 * n * d["nx"]
        s.close()
    log(f"per-solve subset: {len(sub)} tubes in {ps_wall:.2f} s")

    fl = flops_per_stage_cell_1d()
    achieved = fl["per_stage_cell"] * units_per_solve / avg_kernel_s / 1e12
    rec = {
        "metric": "RK-stage cell-updates/s",
        "value": units / wall,
        "unit": "stage-cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded random shock tubes)",
        "config": {"workload": f"batched 1D Euler shock tubes: {count} instances, N log-uniform in "
                               f"[{args.n_min}, {args.n_max}], "
                               f"t = {t_final}, WCNS-T TENO C_T=1e-5, Roe, MND, SSP-RK3 CFL 0.5, seed {seed}",
                   "instances": count, "cells": int(sum(d["nx"] for d in descs)),
                   "stage_cell_updates_per_solve": units_per_solve, "failed_instances": failed,
                   "kernel_ms_avg": avg_kernel_s * 1e3, "steps_per_tick": tune["steps_per_tick"],
                   "tuning_cached": tune.get("cached", False), "ticks": stats["ticks"],
                   "graphs_captured": stats["graphs"], "persistent_switch_strips": tune["switch_strips"],
                   "persistent_shape": [tune["waves_per_group"], tune["instances_per_group"]],
                   "persistent_instances": stats["persist_instances"]},
        "per_solve": {"value": ps_units / ps_wall, "unit": "stage-cell-updates/s", "instances": int(len(sub)),
                      "wall_s": ps_wall, "speedup_batched": (units / wall) / (ps_units / ps_wall)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                     "flops_per_unit": fl["per_stage_cell"]},
    }
    if not args.no_cpu_baseline:
        idx = np.random.default_rng(seed + 2).choice(count, size=min(64, count), replace=False)
        rec["cpu_baseline"] = cpu_baseline_tubes(items, idx, steps=args.cpu_steps)
    return rec


def bench_serve(args):
    import numpy as np
    import torch

    from paper_1810_07806_amd import workloads as W
    from paper_1810_07806_amd.serve import Server, fifo_latencies, per_solve_service, percentiles

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.75 * free) if args.budget_gb <= 0 else int(args.budget_gb * 2**30)
    budget = min(budget, int(0.75 * free))
    count, seed = args.count, args.seed
    unit = W.serving_trace(count=count, seed=seed, rate=1.0)  # arrivals in units of 1 / rate

    def work(done):
        return sum(3.0 * c["steps"] * c["cells"] for c in done)

    # warm-up: the first few requests, all at once
    srv = Server(budget_bytes=budget, capacity=args.capacity, tick_ms=args.tick_ms)
    srv.run(unit[:min(4, count)], realtime=False)
    # capacity: everything queued at t = 0
    log(f"serve: {count} requests, arena {budget / 2**30:.1f} GiB")
    t0 = time.perf_counter()
    done_cap = srv.run(unit, realtime=False)
    cap_s = time.perf_counter() - t0
    capacity = count / cap_s
    log(f"capacity run: {cap_s:.2f} s, {capacity:.2f} requests/s, {srv.ticks} ticks")
    # served run at load x capacity
    rate = args.load * capacity
    trace = [dict(r, arrival=r["arrival"] / rate) for r in unit]
    rng = np.random.default_rng(seed + 7)
    keep = set(int(i) for i in rng.choice(count, size=min(6, count), replace=False))
    t0 = time.perf_counter()
    done = srv.run(trace, realtime=True, keep=keep)
    served_s = time.perf_counter() - t0
    ticks = srv.ticks
    srv.close()
    lat = percentiles([c["latency"] for c in done])
    failed = sum(1 for c in done if c["status"] != 0)
    log(f"served run: {served_s:.2f} s, p50 {lat['p50']:.3f} s, p99 {lat['p99']:.3f} s")
    # plain path: each request alone, one after the other (FIFO on the same arrivals)
    ps = per_solve_service(trace, keep=keep)
    ps_lat = percentiles(fifo_latencies([r["arrival"] for r in trace], [c["service"] for c in ps]))
    ps_busy = sum(c["service"] for c in ps)
    log(f"per-solve: {ps_busy:.2f} s of service, p50 {ps_lat['p50']:.3f} s, p99 {ps_lat['p99']:.3f} s")
    byid = {c["rid"]: c for c in done}
    same = all(np.array_equal(byid[c["rid"]]["U"].ravel(), c["U"].ravel()) for c in ps if c["rid"] in keep)
    w = work(done)
    rec = {
        "metric": "RK-stage cell-updates/s",
        "value": w / served_s,
        "unit": "stage-cell-updates/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": served_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Poisson stream of random shock tubes and four-quadrant problems)",
        "config": {"workload": f"served mixed requests: {count} (70 % 1D tubes N 512-16384 to t 0.15, 30 % 2D "
                               f"four-quadrant 256^2-1024^2 to t 0.1), Poisson arrivals at {args.load} x capacity "
                               f"({rate:.2f}/s), WCNS-T TENO, Roe, MND, SSP-RK3 CFL 0.5, seed {seed}",
                   "requests": count, "failed": failed, "arena_GiB": budget / 2**30, "ticks": ticks,
                   "tick_ms_target": args.tick_ms, "capacity_req_s": capacity, "rate_req_s": rate},
        "latency_s": {"p50": lat["p50"], "p99": lat["p99"], "mean": lat["mean"], "max": lat["max"]},
        "throughput_req_s": count / served_s,
        "per_solve": {"latency_s": {"p50": ps_lat["p50"], "p99": ps_lat["p99"]},
                      "capacity_req_s": count / ps_busy, "service_s": ps_busy,
                      "stage_cell_updates_per_s": w / ps_busy},
        "sampled_results_bitwise_equal": bool(same),
    }
    return rec


def bench_copy(args):
    """Plain device copy of a known size: the reference for scaling the
    FETCH_SIZE / WRITE_SIZE counters to HBM bytes."""
    import torch
    torch.cuda.set_device(0)
    n = (args.copy_mib << 20) // 8
    src = torch.rand(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(max(1, args.warmup)):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    nbytes = 2 * 8 * n
    print(json.dumps({"metric": "copy GB/s", "value": nbytes / ms / 1e6, "unit": "GB/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
                      "dtype": "f64", "config": {"workload": f"device copy of {args.copy_mib} MiB",
                                                 "bytes_read_per_launch": 8 * n, "bytes_written_per_launch": 8 * n}}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("quadrant2d", "tubes", "serve", "copy"), default="quadrant2d")
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 200; tubes: 1 batch solve)")
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--n", type=int, default=N_SIDE, help="grid side (default: the 2048^2 workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-systems", action="store_true",
                    help="default workload only: leave out the tubes and serve sub-records")
    ap.add_argument("--rows", type=int, default=0, help="rows per 2D segment (0: library default)")
    ap.add_argument("--tune-rows", action="store_true", help="2D: autotune the rows per segment first")
    ap.add_argument("--count", type=int, default=4096, help="tubes: instances")
    ap.add_argument("--seed", type=int, default=0, help="tubes: generator seed")
    ap.add_argument("--steps-per-tick", type=int, default=0, help="tubes: fixed tick length (default: autotune)")
    ap.add_argument("--tune-cache", default=None, help="tubes: JSON autotune cache")
    ap.add_argument("--n-min", type=int, default=256, help="tubes: smallest N")
    ap.add_argument("--n-max", type=int, default=8192, help="tubes: largest N")
    ap.add_argument("--switch-strips", type=int, default=0,
                    help="tubes with --steps-per-tick: persistent finish below this many running strips")
    ap.add_argument("--persist-waves", type=int, default=8, help="tubes: waves per persistent workgroup")
    ap.add_argument("--persist-group", type=int, default=1, help="tubes: instances per persistent workgroup")
    ap.add_argument("--per-solve", type=int, default=32, help="tubes: instances timed on the per-solve path")
    ap.add_argument("--cpu-steps", type=int, default=200, help="tubes: oracle steps per sampled tube")
    ap.add_argument("--load", type=float, default=0.7, help="serve: arrival rate / measured capacity")
    ap.add_argument("--tick-ms", type=float, default=10.0, help="serve: target tick duration")
    ap.add_argument("--capacity", type=int, default=256, help="serve: pool slots")
    ap.add_argument("--budget-gb", type=float, default=0.0, help="serve: arena GiB (0: 75 %% of free)")
    ap.add_argument("--copy-mib", type=int, default=1024, help="copy: bytes copied per launch (MiB)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "copy":
        args.steps = 20 if args.steps is None else args.steps
        args.warmup = 2 if args.warmup is None else args.warmup
        return bench_copy(args)
    if args.workload == "serve":
        args.count = 80 if args.count == 4096 else args.count
        print(json.dumps(bench_serve(args)), flush=True)
        return
    if args.workload == "tubes":
        args.steps = 1 if args.steps is None else args.steps
        args.warmup = 1 if args.warmup is None else args.warmup
        print(json.dumps(bench_tubes(args)), flush=True)
        return
    args.steps = 200 if args.steps is None else args.steps
    args.warmup = 3 if args.warmup is None else args.warmup

    import torch

    from paper_1810_07806_amd import workloads as W
    from paper_1810_07806_amd.wcnst import Solver

    torch.cuda.set_device(0)
    d, U0 = W.riemann2d_config3(args.n)
    s = Solver(d)
    if args.rows > 0:
        s.set_tuning(args.rows)
    U0g = s.new_state(U0)
    tuned = None
    if args.tune_rows and args.rows == 0:
        from paper_1810_07806_amd import autotune

        def log(msg):
            print(msg, file=sys.stderr, flush=True)

        tuned = autotune.tune_rows(s, U0g, cache=args.tune_cache, device_name=torch.cuda.get_device_name(0),
                                   log=log)
        args.rows = tuned["rows"]
    U = U0g.clone()
    if args.warmup > 0:
        s.solve(U, t_final=math.inf, cfl=0.5, max_steps=args.warmup)
    U.copy_(U0g)
    s.reset(0.0, 0)
    torch.cuda.synchronize()
    s.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_end, nsteps = s.solve(U, t_final=math.inf, cfl=0.5, max_steps=args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms, launches = s.profile_read()
    shape = s.stage_shape()
    s.profile_enable(False)
    st = s.status()
    assert st["status"] == 0, st
    assert nsteps == args.steps

    cells = args.n * args.n
    units = 3.0 * nsteps * cells
    fl = flops_per_stage_cell()
    avg_launch_s = stage_ms / 1e3 / max(1, launches)
    achieved = fl["per_stage_cell"] * cells / avg_launch_s / 1e12
    rec = {
        "metric": "RK-stage cell-updates/s",
        "value": units / wall,
        "unit": "stage-cell-updates/s",
        "n_gpus": 1,
        "steps": nsteps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / nsteps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (analytic four-quadrant initial state)",
        "config": {"workload": f"2D Euler four-quadrant Riemann (Lax-Liu 3), {args.n}x{args.n} cells, "
                               f"WCNS-T TENO C_T=1e-5, Roe, MND, SSP-RK3 CFL 0.5, {nsteps} steps",
                   "nx": args.n, "ny": args.n, "t_reached": t_end, "kernel_ms_avg": avg_launch_s * 1e3,
                   "stage_launches": launches, "rows_per_segment": args.rows or None,
                   "rows_autotuned": tuned is not None, "stage_shape": shape},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": measured_traffic(f"quadrant2d_{args.n}") if not args.rows else None,
                     "flops_per_unit": fl["per_stage_cell"],
                     "bytes_per_launch_algorithmic": bytes_per_stage_cell() * cells,
                     "hbm_GBs_algorithmic": bytes_per_stage_cell() * cells / avg_launch_s / 1e9},
    }
    crec = counter_record(f"quadrant2d_{args.n}") if not args.rows else None
    if crec:
        # counter-measured figures of the same kernel (profiles/ summaries)
        rec["roofline"]["hbm_GBs_measured"] = crec["hbm_bytes_per_launch"] / avg_launch_s / 1e9
        rec["roofline"]["valu_busy_counters"] = crec.get("valu_busy_frac")
    if not args.no_cpu_baseline and args.n == N_SIDE:
        rec["cpu_baseline"] = cpu_baseline()
    if not args.no_systems and args.n == N_SIDE:
        # the two systems workloads on the same GPU, each beside its
        # per-solve comparison: the batched shock tubes and the served mix
        rec["tubes"] = systems_record(bench_tubes, args, steps=1, warmup=1, count=4096)
        rec["serve"] = systems_record(bench_serve, args, steps=1, warmup=1, count=80)
        rec["singles"] = bench_singles()
    print(json.dumps(rec), flush=True)


def bench_singles() -> dict:
    """Time-to-solution of the two 1D single-solve workloads on the
    single-solve path (wcnst_solve, inputs resident, one synchronising call):
    linear advection of a sine plus a square pulse (N = 200, periodic, to
    t = 2) and the Shu-Osher problem (N = 2048, zero gradient, to t = 1.8),
    both WCNS-T TENO with MND and SSP-RK3 at CFL 0.5.  One grid fills a
    handful of CUs, so there is no roofline claim: each stage costs about
    one wavefront's latency."""
    import torch

    from paper_1810_07806_amd import workloads as W
    from paper_1810_07806_amd.wcnst import Solver
    out = {}
    for name, (d, U0), tf in (("advection_sine_square_200", W.advection_sine_square(200), 2.0),
                              ("shu_osher_2048", W.shu_osher(2048), 1.8)):
        s = Solver(d)
        U = s.new_state(U0)
        s.solve(U.clone(), t_final=math.inf, cfl=0.5, max_steps=20)  # warm-up
        # the time to solution without per-launch events, then the kernel
        # time of the same solve with them
        s.reset(0.0, 0)
        V = U.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t, n = s.solve(V, t_final=tf, cfl=0.5)
        wall = time.perf_counter() - t0
        s.reset(0.0, 0)
        s.profile_enable(True)
        s.solve(U, t_final=tf, cfl=0.5)
        stage_ms, launches = s.profile_read()
        s.profile_enable(False)
        units = 3.0 * n * int(d["nx"])
        out[name] = {"time_to_solution_s": wall, "steps": n, "t_final": t, "cells": int(d["nx"]),
                     "stage_cell_updates_per_s": units / wall,
                     "kernel_us_per_stage": stage_ms * 1e3 / max(1, launches)}
        s.close()
    return out


def systems_record(fn, args, steps, warmup, count):
    """One systems workload as a sub-record of the default line (its own
    step counts; the per-solve comparison and CPU baseline inside)."""
    sub = argparse.Namespace(**vars(args))
    sub.steps, sub.warmup, sub.count = steps, warmup, count
    rec = fn(sub)
    for k in ("n_gpus", "steps", "warmup", "higher_is_better", "scaling", "vs_baseline", "dtype"):
        rec.pop(k, None)
    return rec


if __name__ == "__main__":
    main()
