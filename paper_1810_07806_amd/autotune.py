"""Autotuner for the batched solver's work decomposition.

The decomposition (parts per instance via `split`, wavefronts per workgroup,
persistent grid size) never changes results, only time, so it is chosen by
measurement.  Candidates are timed on a proxy of the real batch: the same
instances run to a fraction of their final times.  Step counts scale with
t_final, so the proxy keeps the relative costs of the instances (and hence
the load-balance problem) while costing a few percent of the real run.

The winner can be cached in a JSON file keyed by device name and a
signature of the batch (instance count, total cells, largest instance).
"""
from __future__ import annotations

import json
import os
import time

DEFAULT_SPLITS = (0.0, 0.5, 1.0, 2.0, 4.0)
DEFAULT_WPG = (1, 2, 4)


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


def tune_batch(batch, Ug_init, t_final, cfl: float = 0.5, proxy: float = 0.05, splits=DEFAULT_SPLITS,
               wpgs=DEFAULT_WPG, cache: str | None = None, device_name: str = "", log=None):
    """Time every (split, waves_per_group) candidate on the proxy run and set
    the fastest on `batch`.  `Ug_init` (packed initial states) is not
    modified.  Returns dict(split, waves_per_group, ms, table, cached)."""
    import numpy as np
    import torch
    key = f"{device_name}|{signature(batch.descs, t_final)}|cfl={cfl}"
    db = _load(cache)
    if key in db:
        best = db[key]
        batch.set_tuning(best["split"], 0, best["waves_per_group"])
        return dict(best, cached=True, table=[])
    tf = np.broadcast_to(np.asarray(t_final, dtype=float), (batch.n,)) * proxy
    U = torch.empty_like(Ug_init)
    table = []
    for wpg in wpgs:
        for split in splits:
            batch.set_tuning(split, 0, wpg)
            U.copy_(Ug_init)
            torch.cuda.synchronize()
            batch.solve(U, tf, cfl=cfl)
            ms = batch.kernel_ms()
            table.append(dict(split=split, waves_per_group=wpg, ms=ms))
            if log:
                log(f"tune split={split} waves/group={wpg}: {ms:.2f} ms")
    best = min(table, key=lambda r: r["ms"])
    batch.set_tuning(best["split"], 0, best["waves_per_group"])
    if cache:
        db = _load(cache)
        db[key] = dict(split=best["split"], waves_per_group=best["waves_per_group"], ms=best["ms"],
                       proxy=proxy, when=time.strftime("%Y-%m-%d %H:%M:%S"))
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
    return dict(best, cached=False, table=table)
