"""Autotuners for the launch decomposition of 2D solves and batched solves.

2D solves (`tune_rows`): the height of the row segment that one 64-lane
wavefront marches up in a strip of 61 columns.  Taller segments compute
fewer halo y-midpoints (3 per segment and column), shorter ones give more
wavefronts; the default two-height shape (0) balances the two wavefronts
that share a SIMD.  A copy of the state is first advanced by `pre_steps`
steps with the default shape (the ranking of the shapes changes as the
solution develops: timed at the initial state alone, 35-row segments beat
the default by 3 % and then lose by 5 % over 200 steps of the 2048^2
benchmark); each candidate then runs a few steps with a fixed,
tiny dt on that state, and a candidate replaces the default only when it
is faster by `margin`.  The solver's step record is restored afterwards.

Batched solves (`tune_batch`): three choices never change results, only
time:

* the tick length (steps between the host's retirement of finished
  instances from the launch table): short ticks retire finished instances
  sooner, long ticks replay one captured graph longer between host round
  trips;
* the switch to the persistent finish: once the running instances hold at
  most `switch_strips` strips, one persistent launch runs them to their
  final times with no kernel boundary between stages (0 = never);
* the persistent launch's workgroup shape: waves per workgroup (which
  share the strips of a stage) and instances per workgroup.

Candidates are timed on a proxy of the real batch: the same instances run
to a fraction of their final times.  Step counts scale with t_final, so the
proxy keeps the relative lengths of the instances while costing a few
percent of the real run.  The search is greedy: the tick length first
(stage launches only), then the switch point at 8 waves x 1 instance, then
the workgroup shape at the best switch point (skipped when stage launches
to the end win).  A persistent winner is confirmed on a longer proxy
against stage launches to the end: on the short one its share of the run
(the tail) is larger than on the real run, and measured batches of shock
tubes (N in [256, 8192] and in [64, 512]) ran slower with it.

The winner can be cached in a JSON file keyed by device name and a
signature of the batch (instance count, total cells, largest instance).
"""
from __future__ import annotations

import json
import os
import time

DEFAULT_TICKS = (16, 32, 64, 128, 256)
DEFAULT_SWITCH = (0, 64, 256, 1024)
DEFAULT_SHAPES = ((8, 1), (4, 1), (8, 2), (4, 4))


def signature(descs, t_final) -> str:
    import numpy as np
    n = np.array([int(d["nx"]) for d in descs])
    tf = np.broadcast_to(np.asarray(t_final, dtype=float), n.shape)
    return f"n={len(n)},cells={int(n.sum())},nmax={int(n.max())},tmax={float(tf.max()):.6g}"


def _load(path):
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


DEFAULT_ROWS = (0, 12, 16, 21, 24, 28, 32, 35, 40, 48, 64)


def tune_rows(solver, U, steps: int = 3, pre_steps: int = 60, dt: float = 1e-9, margin: float = 0.02,
              rows=DEFAULT_ROWS, cfl: float = 0.5, cache: str | None = None, device_name: str = "", log=None):
    """Time each segment height (0: the default shape) over `steps` steps
    with a fixed dt on a copy of U advanced by `pre_steps` CFL steps, and
    set the fastest on `solver` (the default unless another is faster by
    `margin`).  U is not modified.  Returns dict(rows, ms_per_launch, table,
    cached)."""
    import torch
    d = solver.desc
    key = f"{device_name}|2d|nx={int(d['nx'])},ny={int(d['ny'])}|rows"
    db = _load(cache)
    if key in db:
        solver.set_tuning(int(db[key]["rows"]))
        return dict(db[key], cached=True, table=[])
    st = solver.status()
    base = U.clone()
    if pre_steps > 0:
        solver.set_tuning(0)
        solver.reset(0.0, 0)
        solver.solve(base, cfl=cfl, max_steps=pre_steps)
    Ut = torch.empty_like(U)
    table = []
    for r in rows:
        solver.set_tuning(int(r))
        Ut.copy_(base)
        solver.step(Ut, dt=dt)  # untimed: first launch of this shape
        solver.profile_enable(True)
        for _ in range(steps):
            solver.step(Ut, dt=dt)
        ms, n = solver.profile_read()
        solver.profile_enable(False)
        row = dict(rows=int(r), ms_per_launch=ms / max(1, n), shape=solver.stage_shape())
        table.append(row)
        if log:
            log(f"tune rows={r}: {row['ms_per_launch'] * 1e3:.1f} us per stage launch {row['shape']}")
    solver.reset(st["t"], st["steps"])
    torch.cuda.synchronize()
    best = min(table, key=lambda x: x["ms_per_launch"])
    default = next((x for x in table if x["rows"] == 0), None)
    if default is not None and best["ms_per_launch"] > (1.0 - margin) * default["ms_per_launch"]:
        best = default
    solver.set_tuning(best["rows"])
    out = dict(rows=best["rows"], ms_per_launch=best["ms_per_launch"])
    if cache:
        db = _load(cache)
        db[key] = dict(out, when=time.strftime("%Y-%m-%d %H:%M:%S"))
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
    return dict(out, cached=False, table=table)


def _apply(batch, cfg):
    batch.set_tuning(cfg["steps_per_tick"])
    batch.set_persist(cfg["switch_strips"], cfg["waves_per_group"], cfg["instances_per_group"])


def tune_batch(batch, Ug_init, t_final, cfl: float = 0.5, proxy: float = 0.05, ticks=DEFAULT_TICKS,
               switches=DEFAULT_SWITCH, shapes=DEFAULT_SHAPES, confirm: float = 0.25, cache: str | None = None,
               device_name: str = "", log=None):
    """Time the candidates on the proxy run and set the fastest on `batch`.
    `Ug_init` (packed initial states) is not modified.  Returns dict(
    steps_per_tick, switch_strips, waves_per_group, instances_per_group, ms,
    table, cached)."""
    import numpy as np
    import torch
    key = f"{device_name}|{signature(batch.descs, t_final)}|cfl={cfl}|persist"
    db = _load(cache)
    if key in db:
        best = db[key]
        _apply(batch, best)
        return dict(best, cached=True, table=[])
    tf = np.broadcast_to(np.asarray(t_final, dtype=float), (batch.n,)) * proxy
    U = torch.empty_like(Ug_init)
    table = []

    def trial(cfg):
        _apply(batch, cfg)
        U.copy_(Ug_init)
        torch.cuda.synchronize()
        batch.solve(U, tf, cfl=cfl)
        row = dict(cfg, ms=batch.kernel_ms(), proxy=float(tf.max() / max(1e-300, float(np.max(t_final)))))
        table.append(row)
        if log:
            log("tune " + ", ".join(f"{k}={v}" for k, v in cfg.items()) + f": {row['ms']:.2f} ms")
        return row

    base = dict(steps_per_tick=ticks[0], switch_strips=0, waves_per_group=8, instances_per_group=1)
    best = min([trial(dict(base, steps_per_tick=spt)) for spt in ticks], key=lambda r: r["ms"])
    for sw in switches:
        if sw > 0:
            cfg = {k: best[k] for k in ("steps_per_tick", "waves_per_group", "instances_per_group")}
            r = trial(dict(cfg, switch_strips=sw, waves_per_group=8, instances_per_group=1))
            best = r if r["ms"] < best["ms"] else best
    if best["switch_strips"] > 0:
        for w, g in shapes:
            if (w, g) != (best["waves_per_group"], best["instances_per_group"]):
                cfg = {k: best[k] for k in ("steps_per_tick", "switch_strips")}
                r = trial(dict(cfg, waves_per_group=w, instances_per_group=g))
                best = r if r["ms"] < best["ms"] else best
        # the short proxy favours the persistent finish (its tail is a larger
        # share of the run): confirm against stage launches to the end on a
        # proxy of `confirm` of the final times
        tf_short = tf
        tf = tf_short / proxy * confirm
        ticks_only = trial(dict({k: best[k] for k in ("steps_per_tick", "waves_per_group", "instances_per_group")},
                                switch_strips=0))
        persistent = trial({k: best[k] for k in ("steps_per_tick", "switch_strips", "waves_per_group",
                                                 "instances_per_group")})
        best = persistent if persistent["ms"] < ticks_only["ms"] else ticks_only
    best = {k: best[k] for k in ("steps_per_tick", "switch_strips", "waves_per_group", "instances_per_group", "ms")}
    _apply(batch, best)
    if cache:
        db = _load(cache)
        db[key] = dict(best, proxy=proxy, when=time.strftime("%Y-%m-%d %H:%M:%S"))
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
    return dict(best, cached=False, table=table)
