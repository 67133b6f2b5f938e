"""Serving loop with continuous batching over the request pool.

Requests (1D or 2D Euler solves of any size) arrive over time.  The server
keeps an HBM arena of a fixed byte budget; a request is admitted as soon as
its three state buffers (U, U1, U2: 3 x nvar x cells x 8 bytes) fit in the
arena and a pool slot is free, in arrival order except that a request that
does not fit yet lets later ones that fit pass it (a bounded number of
times, after which it holds the queue until memory frees up).  Its initial
state is copied into the arena and it joins the pool, which advances all
resident requests together, a tick at a time.  After each tick finished
requests are retired: the result is copied back, the slot and the memory
are freed, and waiting requests are admitted before the next tick.  The
1D and the 2D requests take separate step counts per tick (their launches
run side by side on two streams): each is sized so that its launches take
about `tick_ms`, from its measured device time per step in the last tick,
rescaled to the cells active in the next one.  So a small 1D request that
needs many steps is not held to the pace of large 2D ones, and a large
arrival shortens the next tick at once, which bounds how long a new
arrival waits for admission.

`per_solve_latencies` is the comparison: the plain path, one wcnst_solve
per request in arrival order on the same GPU.
"""
from __future__ import annotations

import bisect
import time
from collections import deque

import numpy as np

ALIGN = 256


class Arena:
    """First-fit allocator over [0, size) with coalescing of free blocks
    (offsets in bytes, ALIGN-aligned)."""

    def __init__(self, size: int):
        self.size = int(size) // ALIGN * ALIGN
        self._free = [(0, self.size)]  # sorted (offset, length)
        self._used = {}

    @staticmethod
    def _round(n: int) -> int:
        return (int(n) + ALIGN - 1) // ALIGN * ALIGN

    def alloc(self, nbytes: int):
        n = self._round(max(1, nbytes))
        for i, (off, ln) in enumerate(self._free):
            if ln >= n:
                if ln == n:
                    self._free.pop(i)
                else:
                    self._free[i] = (off + n, ln - n)
                self._used[off] = n
                return off
        return None

    def free(self, off: int):
        n = self._used.pop(off)
        i = bisect.bisect_left(self._free, (off, 0))
        self._free.insert(i, (off, n))
        # merge with the right, then the left neighbour
        if i + 1 < len(self._free) and off + n == self._free[i + 1][0]:
            self._free[i] = (off, n + self._free[i + 1][1])
            self._free.pop(i + 1)
        if i > 0 and self._free[i - 1][0] + self._free[i - 1][1] == off:
            self._free[i - 1] = (self._free[i - 1][0], self._free[i - 1][1] + self._free[i][1])
            self._free.pop(i)

    @property
    def used_bytes(self) -> int:
        return sum(self._used.values())

    def largest_free(self) -> int:
        return max((ln for _, ln in self._free), default=0)


def request_values(desc: dict) -> int:
    """FP64 values of one state buffer of the request."""
    nd = int(desc.get("ndim", 1))
    nv = 3 if nd == 1 else 4
    return nv * int(desc["nx"]) * (int(desc["ny"]) if nd == 2 else 1)


def request_bytes(desc: dict) -> int:
    """HBM bytes the server reserves for a request: U, U1, U2."""
    return 3 * Arena._round(8 * request_values(desc))


def percentiles(lat):
    a = np.asarray(lat, dtype=float)
    if a.size == 0:
        return dict(p50=None, p99=None, mean=None, max=None)
    return dict(p50=float(np.percentile(a, 50)), p99=float(np.percentile(a, 99)), mean=float(a.mean()),
                max=float(a.max()))


def plan_admissions(queue, arena, free_slots: int, skips: dict, max_skips: int):
    """One admission round over `queue` (a deque of requests by arrival,
    modified in place): requests are placed in the arena in order while
    slots are free; one that does not fit stays queued and lets later ones
    pass, until it has been passed max_skips times (counted in `skips` by
    rid), after which nothing passes it.  Returns [(request, arena offset)]
    of the admitted requests, plus (request, None) for a request that does
    not fit at all while the queue holds nothing else that could run (the
    caller decides whether that is an error)."""
    admitted, waiting = [], deque()
    while queue and free_slots > 0:
        r = queue.popleft()
        off = arena.alloc(request_bytes(r["desc"]))
        if off is None:
            skips[r["rid"]] = skips.get(r["rid"], 0) + 1
            waiting.append(r)
            if skips[r["rid"]] > max_skips:
                break  # it has waited long enough: nothing passes it
            continue
        admitted.append((r, off))
        free_slots -= 1
    queue.extendleft(reversed(waiting))
    if not admitted and waiting and arena.used_bytes == 0:
        admitted.append((waiting[0], None))
    return admitted


def _active_cells(active) -> list:
    """Cells of the active 1D and 2D requests."""
    cells = [0, 0]
    for a in active.values():
        d = a["req"]["desc"]
        nd = int(d.get("ndim", 1))
        cells[nd - 1] += int(d["nx"]) * (int(d["ny"]) if nd == 2 else 1)
    return cells


class Server:
    """Continuous-batching server over one Pool and one arena tensor."""

    def __init__(self, budget_bytes: int, capacity: int = 256, cfl: float = 0.5, tick_ms: float = 10.0,
                 min_steps: int = 4, max_steps: int = 2048, device: str = "cuda", scheme: dict | None = None,
                 max_skips: int = 8):
        import torch

        from .wcnst import Pool
        self.torch = torch
        self.arena = Arena(budget_bytes)
        self.buf = torch.empty(self.arena.size // 8, dtype=torch.float64, device=device)
        self.pool = Pool(scheme=scheme, capacity=capacity, device=device)
        self.capacity = capacity
        self.cfl = cfl
        self.tick_ms = tick_ms
        self.min_steps, self.max_steps = min_steps, max_steps
        # admission backfills: a request that does not fit the arena yet lets
        # later ones that fit go first, at most max_skips times; then it
        # holds the queue until memory frees up for it
        self.max_skips = max_skips

    def _views(self, off: int, nvals: int):
        per = Arena._round(8 * nvals) // 8
        base = off // 8
        return tuple(self.buf[base + k * per: base + k * per + nvals] for k in range(3))

    def run(self, trace, realtime: bool = True, keep=None, log=None):
        """Serve `trace` (list of dict(rid, arrival, desc, U0, t_final), by
        arrival).  With realtime, requests become visible at their arrival
        times on the wall clock; otherwise all at once.  Returns a list of
        completion records; `keep` = set of rids whose final states are
        copied into the records."""
        torch = self.torch
        keep = keep or set()
        pending = deque(sorted(trace, key=lambda r: r["arrival"]))
        queue = deque()
        active = {}
        done = []
        skips = {}                # rid -> admissions it let later requests pass
        steps = [32, 32]          # per tick, for the 1D and the 2D requests
        per_step = [None, None]   # ms per step per active cell in the last tick
        ticks = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while pending or queue or active:
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0]["arrival"] <= now):
                queue.append(pending.popleft())
            for r, off in plan_admissions(queue, self.arena, self.capacity - len(active), skips, self.max_skips):
                if off is None:
                    if not active:
                        raise RuntimeError(f"request {r['rid']} needs {request_bytes(r['desc'])} bytes, more than "
                                           f"the arena's {self.arena.size}")
                    continue
                nvals = request_values(r["desc"])
                U, U1, U2 = self._views(off, nvals)
                U.copy_(torch.from_numpy(np.ascontiguousarray(r["U0"], dtype=np.float64).ravel()))
                slot = self.pool.admit(r["desc"], U, U1, U2, r["t_final"], self.cfl)
                active[slot] = dict(req=r, off=off, U=U, admitted=time.perf_counter() - t0)
            if not active:
                if pending and realtime:
                    time.sleep(max(0.0, min(0.01, pending[0]["arrival"] - (time.perf_counter() - t0))))
                continue
            cells = _active_cells(active)
            steps = [self._steps_for(k, cells[k], per_step[k], steps[k]) for k in range(2)]
            self.pool.tick(steps[0], steps[1])
            ticks += 1
            for k, ms in enumerate(self.pool.tick_ms()):
                if cells[k] and ms > 0.0:
                    per_step[k] = ms / steps[k] / cells[k]
            for slot in list(active):
                res = self.pool.result(slot)
                if not res["finished"]:
                    continue
                a = active.pop(slot)
                r = a["req"]
                out = a["U"].cpu().numpy().copy() if r["rid"] in keep else None
                self.pool.release(slot)
                self.arena.free(a["off"])
                t_done = time.perf_counter() - t0
                d = r["desc"]
                cells = int(d["nx"]) * (int(d["ny"]) if int(d.get("ndim", 1)) == 2 else 1)
                done.append(dict(rid=r["rid"], arrival=r["arrival"] if realtime else 0.0, admitted=a["admitted"],
                                 done=t_done, latency=t_done - (r["arrival"] if realtime else 0.0),
                                 status=res["status"], steps=res["steps"], t=res["t"], cells=cells,
                                 ndim=int(d.get("ndim", 1)), U=out))
                if log:
                    log(f"done rid={r['rid']} ndim={d.get('ndim', 1)} cells={cells} steps={res['steps']} "
                        f"latency={done[-1]['latency']:.3f}s active={len(active)} queued={len(queue)}")
        self.ticks = ticks
        return done

    def _steps_for(self, k, cells, per_cell, last):
        """Steps of dimension k (0: 1D, 1: 2D) for the next tick: about
        tick_ms of device time at the last measured cost per step and cell,
        or the last count when nothing was measured yet."""
        if not cells or per_cell is None:
            return last
        ms = per_cell * cells
        return int(min(self.max_steps, max(self.min_steps, self.tick_ms / max(ms, 1e-6))))

    def close(self):
        self.pool.close()


def per_solve_service(trace, cfl: float = 0.5, keep=None, log=None):
    """Plain path: each request solved alone with wcnst_solve, one after the
    other; returns per-request service times (H2D, solve, D2H) and results."""
    import torch

    from .wcnst import Solver, WcnstError
    keep = keep or set()
    out = []
    for r in trace:
        d = r["desc"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = Solver(d)
        U = s.new_state(r["U0"])
        status = 0
        try:
            _, n = s.solve(U, t_final=r["t_final"], cfl=cfl)
        except WcnstError as e:
            status = e.status
            n = s.status()["steps"]
        res = U.cpu().numpy().copy() if r["rid"] in keep else None
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        s.close()
        cells = int(d["nx"]) * (int(d["ny"]) if int(d.get("ndim", 1)) == 2 else 1)
        out.append(dict(rid=r["rid"], service=el, status=status, steps=n, cells=cells, U=res))
        if log:
            log(f"per-solve rid={r['rid']} cells={cells} steps={n} {el:.3f}s")
    return out


def fifo_latencies(arrivals, services):
    """Completion latencies of a single FIFO server with the given arrival
    and service times (the per-solve path serves one request at a time)."""
    t = 0.0
    lat = []
    for a, s in zip(arrivals, services):
        t = max(t, a) + s
        lat.append(t - a)
    return lat
