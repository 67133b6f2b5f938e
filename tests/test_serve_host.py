"""Host logic of the serving loop: arena allocator, FIFO latency model,
request stream generator (no GPU)."""
from __future__ import annotations

import numpy as np

from paper_1810_07806_amd import workloads as W
from paper_1810_07806_amd.serve import ALIGN, Arena, fifo_latencies, percentiles, request_bytes


def test_arena_first_fit_and_coalescing():
    a = Arena(10 * ALIGN)
    x = a.alloc(3 * ALIGN)
    y = a.alloc(1)
    z = a.alloc(2 * ALIGN)
    assert (x, y, z) == (0, 3 * ALIGN, 4 * ALIGN)
    assert a.alloc(5 * ALIGN) is None
    a.free(y)
    assert a.alloc(2 * ALIGN) == 6 * ALIGN  # the 1-block hole is too small
    a.free(x)
    assert a.alloc(4 * ALIGN) == 0  # x and y coalesced
    a.free(z)
    a.free(0)
    a.free(6 * ALIGN)
    assert a._free == [(0, 10 * ALIGN)] and a.used_bytes == 0


def test_arena_random_against_byte_map():
    """Random alloc/free sequence checked against a brute-force byte map:
    blocks never overlap, stay in range and every freed byte is reusable."""
    rng = np.random.default_rng(5)
    size = 64 * ALIGN
    a = Arena(size)
    owner = np.full(size // ALIGN, -1)
    live = {}
    for step in range(3000):
        if live and rng.uniform() < 0.45:
            off = list(live)[rng.integers(len(live))]
            n = live.pop(off)
            assert (owner[off // ALIGN: (off + n) // ALIGN] == off).all()
            owner[off // ALIGN: (off + n) // ALIGN] = -1
            a.free(off)
        else:
            want = int(rng.integers(1, 9 * ALIGN))
            off = a.alloc(want)
            nb = (want + ALIGN - 1) // ALIGN
            # first fit: None exactly when no run of nb free blocks exists
            runs = np.flatnonzero(np.convolve(owner == -1, np.ones(nb, dtype=int), "valid") == nb)
            if off is None:
                assert runs.size == 0
                continue
            assert off % ALIGN == 0 and off // ALIGN == runs[0]
            assert (owner[off // ALIGN: off // ALIGN + nb] == -1).all()
            owner[off // ALIGN: off // ALIGN + nb] = off
            live[off] = nb * ALIGN
        assert a.used_bytes == (owner != -1).sum() * ALIGN


def test_fifo_latencies():
    # idle server: latency = service; busy server: waits for the previous one
    assert fifo_latencies([0.0, 10.0], [1.0, 2.0]) == [1.0, 2.0]
    assert fifo_latencies([0.0, 0.5, 0.6], [1.0, 1.0, 1.0]) == [1.0, 1.5, 2.4]
    p = percentiles([1.0] * 99 + [100.0])
    assert p["p50"] == 1.0 and p["max"] == 100.0


def test_serving_trace_mix_and_sizes():
    tr = W.serving_trace(count=300, seed=3, rate=5.0)
    arr = np.array([r["arrival"] for r in tr])
    assert (np.diff(arr) > 0).all()
    assert abs(np.mean(np.diff(arr)) - 0.2) < 0.05  # mean inter-arrival 1 / rate
    one = [r for r in tr if r["desc"]["ndim"] == 1]
    two = [r for r in tr if r["desc"]["ndim"] == 2]
    assert 0.6 < len(one) / len(tr) < 0.8
    assert all(512 <= r["desc"]["nx"] <= 16384 and r["t_final"] == 0.15 for r in one)
    assert all(r["desc"]["nx"] == r["desc"]["ny"] and r["desc"]["nx"] % 64 == 0 and 256 <= r["desc"]["nx"] <= 1024
               and r["t_final"] == 0.1 for r in two)
    r = two[0]
    assert request_bytes(r["desc"]) == 3 * 4 * r["desc"]["nx"] ** 2 * 8
    assert r["U0"].shape == (4, r["desc"]["ny"], r["desc"]["nx"])


def test_admission_backfills_and_bounds_skips():
    """A request that does not fit yet lets later ones that fit pass it, at
    most max_skips times; after that nothing passes it until memory frees."""
    from collections import deque

    from paper_1810_07806_amd.serve import Arena, plan_admissions, request_bytes

    def req(rid, n):
        return dict(rid=rid, desc=dict(ndim=1, nx=n))
    small, big = request_bytes(req(0, 100)["desc"]), request_bytes(req(0, 4000)["desc"])
    arena = Arena(big)                              # room for one big or several small
    held = arena.alloc(small)                       # part of the arena in use: the big one waits
    queue = deque([req(1, 4000), req(2, 100), req(3, 100), req(4, 100)])
    skips = {}
    got = plan_admissions(queue, arena, 10, skips, max_skips=2)
    assert [r["rid"] for r, off in got] == [2, 3, 4] and all(off is not None for _, off in got)
    assert [r["rid"] for r in queue] == [1] and skips == {1: 1}
    for _, off in got:
        arena.free(off)
    queue.extend([req(5, 100), req(6, 100)])
    assert [r["rid"] for r, _ in plan_admissions(queue, arena, 10, skips, max_skips=2)] == [5, 6]
    for r in list(arena._used):
        if r != held:
            arena.free(r)
    queue.extend([req(7, 100)])
    # third skip: over the limit, request 1 now holds the queue
    assert plan_admissions(queue, arena, 10, skips, max_skips=2) == []
    assert [r["rid"] for r in queue] == [1, 7]
    arena.free(held)
    got = plan_admissions(queue, arena, 10, skips, max_skips=2)
    assert [r["rid"] for r, _ in got] == [1] and [r["rid"] for r in queue] == [7]  # 1 fills the arena
    # slot limit
    queue.extend([req(8, 10), req(9, 10)])
    for _, off in got:
        arena.free(off)
    assert [r["rid"] for r, _ in plan_admissions(queue, arena, 1, skips, max_skips=2)] == [7]
    assert [r["rid"] for r in queue] == [8, 9]
