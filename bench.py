"""Benchmark: RK-stage cell-updates/s of WCNS-T on one MI355X.

Workload: 2D Euler four-quadrant Riemann problem (Sec. 3.6.1 states) on
[0,1]^2, 2048 x 2048 cells, FP64, characteristic-wise TENO-5 interpolation,
Roe flux, MND difference, SSP-RK3, CFL 0.5, zero-gradient boundaries.  One
benchmark step = one SSP-RK3 step (three fused stage kernels, CFL reduction
fused into the third) over the whole grid.  The state is reset to the
initial condition after warm-up, so the timed region is steps 1..K of the
problem (K = 200 by default, the full fixed-step run).

Prints one JSON line.  `roofline` prices the stage kernel against the FP64
vector peak with the algorithmic flop count per stage-cell-update (see
`flops_per_stage_cell`); `cpu_baseline` times the CPU oracle on one full
SSP-RK3 step of the same grid on the host cores.
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=N_SIDE, help="grid side (default: the 2048^2 workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rows", type=int, default=0, help="rows per 2D segment (0: library default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1810_07806_amd import workloads as W
    from paper_1810_07806_amd.wcnst import Solver

    torch.cuda.set_device(0)
    d, U0 = W.riemann2d_config3(args.n)
    s = Solver(d)
    if args.rows > 0:
        s.set_tuning(args.rows)
    U0g = s.new_state(U0)
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
                   "stage_launches": launches, "rows_per_segment": args.rows or None},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                     "flops_per_unit": fl["per_stage_cell"],
                     "hbm_GBs_algorithmic": bytes_per_stage_cell() * cells / avg_launch_s / 1e9},
    }
    if not args.no_cpu_baseline and args.n == N_SIDE:
        rec["cpu_baseline"] = cpu_baseline()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
