"""Host logic of the launch-shape autotuners, on stand-in solver and batch
objects whose timings are given functions of the candidate (no GPU): the
search order, the confirmation of a persistent winner on the longer proxy,
the margin by which a segment height must beat the default, the restored
step record, and the JSON cache."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from paper_1810_07806_amd import autotune


@pytest.fixture(autouse=True)
def _no_device_sync(monkeypatch):
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)


class FakeBatch:
    """Batch stand-in: kernel_ms() is cost(config, fraction of t_final)."""

    def __init__(self, cost, n=4):
        self.cost, self.n = cost, n
        self.descs = [dict(nx=100 + 10 * i) for i in range(n)]
        self.cfg = {}
        self.calls = []

    def set_tuning(self, spt):
        self.cfg["steps_per_tick"] = spt

    def set_persist(self, sw, w, g):
        self.cfg.update(switch_strips=sw, waves_per_group=w, instances_per_group=g)

    def solve(self, U, tf, cfl=0.5):
        self.frac = float(np.max(tf)) / 0.15
        self.calls.append((dict(self.cfg), round(self.frac, 6)))

    def kernel_ms(self):
        return self.cost(self.cfg, self.frac)


def _ticks_cost(cfg, frac):
    # 32 steps per tick is best; the persistent finish costs per its shape
    return frac * 1000.0 * (1.0 + abs(cfg["steps_per_tick"] - 32) / 256.0)


def test_batch_tuner_picks_the_fastest_tick_and_keeps_stage_launches():
    b = FakeBatch(lambda c, f: _ticks_cost(c, f) * (1.2 if c["switch_strips"] else 1.0))
    res = autotune.tune_batch(b, torch.zeros(8), 0.15)
    assert res["steps_per_tick"] == 32 and res["switch_strips"] == 0 and not res["cached"]
    assert b.cfg["steps_per_tick"] == 32 and b.cfg["switch_strips"] == 0
    # every tick length, then every switch point, on the 5 % proxy only
    assert {c["steps_per_tick"] for c, f in b.calls if f == 0.05} == set(autotune.DEFAULT_TICKS)
    assert all(f == 0.05 for _, f in b.calls)


def test_batch_tuner_rejects_a_persistent_finish_that_only_wins_on_the_short_proxy():
    def cost(c, f):
        base = _ticks_cost(c, f)
        if not c["switch_strips"]:
            return base
        return base * (0.95 if f < 0.1 else 1.05)  # wins at 5 %, loses at 25 %
    b = FakeBatch(cost)
    res = autotune.tune_batch(b, torch.zeros(8), 0.15)
    assert res["switch_strips"] == 0 and b.cfg["switch_strips"] == 0
    longer = [(c, f) for c, f in b.calls if f == 0.25]
    assert len(longer) == 2 and {c["switch_strips"] > 0 for c, _ in longer} == {True, False}


def test_batch_tuner_keeps_a_persistent_finish_that_wins_on_both_proxies():
    def cost(c, f):
        base = _ticks_cost(c, f)
        if not c["switch_strips"]:
            return base
        shape = 0.9 if (c["waves_per_group"], c["instances_per_group"]) == (4, 4) else 0.95
        return base * shape * (1.0 if c["switch_strips"] == 256 else 1.02)
    b = FakeBatch(cost)
    res = autotune.tune_batch(b, torch.zeros(8), 0.15)
    assert (res["switch_strips"], res["waves_per_group"], res["instances_per_group"]) == (256, 4, 4)
    assert b.cfg == dict(steps_per_tick=32, switch_strips=256, waves_per_group=4, instances_per_group=4)


def test_batch_tuner_cache_round_trip(tmp_path):
    cache = str(tmp_path / "tune.json")
    b = FakeBatch(lambda c, f: _ticks_cost(c, f) * (1.2 if c["switch_strips"] else 1.0))
    first = autotune.tune_batch(b, torch.zeros(8), 0.15, cache=cache, device_name="dev")
    n = len(b.calls)
    again = autotune.tune_batch(b, torch.zeros(8), 0.15, cache=cache, device_name="dev")
    assert again["cached"] and len(b.calls) == n
    assert again["steps_per_tick"] == first["steps_per_tick"] == 32
    other = autotune.tune_batch(b, torch.zeros(8), 0.15, cache=cache, device_name="other device")
    assert not other["cached"] and len(b.calls) > n


class FakeSolver:
    """Solver stand-in: each stage launch of shape `rows` takes cost[rows] ms."""

    def __init__(self, cost):
        self.cost = cost
        self.desc = dict(nx=256, ny=256)
        self.rows = 0
        self.t, self.steps = 0.125, 7
        self.prof = False
        self.ms = 0.0
        self.launches = 0

    def status(self):
        return dict(t=self.t, steps=self.steps, status=0)

    def reset(self, t, steps):
        self.t, self.steps = t, steps

    def set_tuning(self, rows):
        self.rows = rows

    def solve(self, U, cfl=0.5, max_steps=0, t_final=np.inf):
        self.steps += max_steps
        U.add_(1.0)

    def step(self, U, dt=0.0):
        self.steps += 1
        if self.prof:
            self.ms += 3 * self.cost[self.rows]
            self.launches += 3

    def profile_enable(self, on=True):
        self.prof = on
        self.ms, self.launches = 0.0, 0

    def profile_read(self):
        return self.ms, self.launches

    def stage_shape(self):
        return dict(rows1=self.rows)


def test_rows_tuner_needs_a_margin_over_the_default_and_restores_the_record():
    rows = (0, 16, 32)
    s = FakeSolver({0: 1.00, 16: 0.99, 32: 1.10})  # 16 rows: 1 % faster, inside the 2 % margin
    U = torch.zeros(4)
    res = autotune.tune_rows(s, U, rows=rows)
    assert res["rows"] == 0 and s.rows == 0
    assert (s.t, s.steps) == (0.125, 7) and torch.equal(U, torch.zeros(4))
    s = FakeSolver({0: 1.00, 16: 0.95, 32: 1.10})  # 5 % faster: taken
    res = autotune.tune_rows(s, U, rows=rows)
    assert res["rows"] == 16 and s.rows == 16
    assert [r["rows"] for r in res["table"]] == list(rows)
