"""Autotuner for the batched solver's tick length.

The tick length (steps between the host's retirement of finished instances
from the launch table) never changes results, only time: short ticks retire
finished instances sooner, long ticks replay one captured graph longer
between host round trips.  Candidates are timed on a proxy of the real
batch: the same instances run to a fraction of their final times.  Step
counts scale with t_final, so the proxy keeps the relative lengths of the
instances while costing a few percent of the real run.

The winner can be cached in a JSON file keyed by device name and a
signature of the batch (instance count, total cells, largest instance).
"""
from __future__ import annotations

import json
import os
import time

DEFAULT_TICKS = (16, 32, 64, 128, 256)


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


def tune_batch(batch, Ug_init, t_final, cfl: float = 0.5, proxy: float = 0.05, ticks=DEFAULT_TICKS,
               cache: str | None = None, device_name: str = "", log=None):
    """Time every steps-per-tick candidate on the proxy run and set the
    fastest on `batch`.  `Ug_init` (packed initial states) is not modified.
    Returns dict(steps_per_tick, ms, table, cached)."""
    import numpy as np
    import torch
    key = f"{device_name}|{signature(batch.descs, t_final)}|cfl={cfl}"
    db = _load(cache)
    if key in db:
        best = db[key]
        batch.set_tuning(best["steps_per_tick"])
        return dict(best, cached=True, table=[])
    tf = np.broadcast_to(np.asarray(t_final, dtype=float), (batch.n,)) * proxy
    U = torch.empty_like(Ug_init)
    table = []
    for spt in ticks:
        batch.set_tuning(spt)
        U.copy_(Ug_init)
        torch.cuda.synchronize()
        batch.solve(U, tf, cfl=cfl)
        ms = batch.kernel_ms()
        table.append(dict(steps_per_tick=spt, ms=ms))
        if log:
            log(f"tune steps/tick={spt}: {ms:.2f} ms")
    best = min(table, key=lambda r: r["ms"])
    batch.set_tuning(best["steps_per_tick"])
    if cache:
        db = _load(cache)
        db[key] = dict(steps_per_tick=best["steps_per_tick"], ms=best["ms"], proxy=proxy,
                       when=time.strftime("%Y-%m-%d %H:%M:%S"))
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
    return dict(best, cached=False, table=table)
