"""Continuous-batching solve service over several resident SLR preconditioners.

Each preloaded matrix owns one batch (``slr_batch_*``: per-column Krylov
state on the device) on its own HIP stream.  Requests (an RHS block of
1..16 columns for one of the matrices) are admitted by device bytes
against one budget shared by all matrices: into a batch with free column
slots, or into a new batch when its bytes fit, and batches left idle are
destroyed to free memory for other matrices.  The loop advances every
batch that has work by a few iterations (the launches of different batches
overlap on the device), retires finished requests, and admits waiting ones
as slots and memory free up.  A column's arithmetic
does not depend on the other columns of its batch, so a request's result is
the same alone and in the mix.

The plain comparison form solves each request on its own with ``slr_solve``
(one request at a time, no batching).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

import paper_1505_04340_amd as P


@dataclass
class Request:
    tag: int
    matrix: int
    b: object                  # torch tensor (n, r) on the device
    arrival: float             # seconds, relative to the start of the run
    admitted: float = -1.0
    done: float = -1.0
    info: dict = field(default_factory=dict)
    x: object = None


class Service:
    """Continuous batching over preloaded SLR contexts, admitted by device
    bytes against one budget shared by every matrix.

    The budget covers the resident preconditioners (slr_query's
    device_bytes, which also counts the scratch a context keeps) and every
    live batch (slr_batch_bytes).  A request goes into a batch of its matrix
    with free column slots; if none has room, a new batch is created when
    its bytes fit what the budget has left (estimated from the bytes per
    column measured on that matrix's first batch, and checked after
    creation).  A batch with no columns in flight is destroyed when its
    matrix has nothing queued and memory is wanted elsewhere (or the matrix
    has another batch), so memory freed by one matrix admits another
    matrix's requests."""

    def __init__(self, slrs, method: str = "fcg", rtol: float = 1e-8, maxit: int = 300,
                 hbm_budget_bytes: int = 8 << 30, max_cols: int = 64, batch_cols: int = 32,
                 iters_per_round: int = 16):
        import torch
        self.slrs = slrs
        self.method, self.rtol, self.maxit = method, rtol, maxit
        self.iters = iters_per_round
        self.budget = int(hbm_budget_bytes)
        self.max_cols = max_cols
        self.batch_cols = max(1, min(batch_cols, max_cols))
        self.streams = [torch.cuda.Stream() for _ in slrs]
        self.batches = [[] for _ in slrs]          # per matrix: [Batch, ...]
        self.inflight = [dict() for _ in slrs]     # per matrix: tag -> (Request, Batch)
        self.per_col = [None] * len(slrs)          # measured batch bytes per column
        self.queues = [collections.deque() for _ in slrs]
        self.peak_bytes = 0
        self.batches_made = 0
        if self.resident_bytes() > self.budget:
            raise ValueError("the resident preconditioners alone exceed the budget")

    def resident_bytes(self) -> int:
        return int(sum(s.query()["device_bytes"] for s in self.slrs))

    def batch_bytes(self) -> int:
        return int(sum(b.bytes() for bl in self.batches for b in bl))

    def device_bytes(self) -> int:
        return self.resident_bytes() + self.batch_bytes()

    def close(self):
        for bl in self.batches:
            for b in bl:
                b.close()
            bl.clear()

    def _new_batch(self, i: int, cols: int):
        """A batch of `cols` columns for matrix i if it fits the budget."""
        cap = min(self.max_cols, max(self.batch_cols, cols))
        used = self.device_bytes()
        if self.per_col[i] is not None and used + self.per_col[i] * cap > self.budget:
            cap = cols      # the smallest batch that takes the request
            if used + self.per_col[i] * cap > self.budget:
                return None
        bt = P.Batch(self.slrs[i], cap, self.method, self.rtol, self.maxit)
        nb = bt.bytes()
        if self.per_col[i] is None:
            self.per_col[i] = nb / cap
        if used + nb > self.budget:
            bt.close()
            return None
        self.batches[i].append(bt)
        self.batches_made += 1
        return bt

    def _admit(self, i: int, rq, stream, t_now: float) -> bool:
        cols = int(rq.b.shape[1])
        for bt in self.batches[i]:
            x = bt.admit(rq.b, rq.tag, stream=stream)
            if x is not None:
                break
        else:
            bt = self._new_batch(i, cols)
            if bt is None:
                return False
            x = bt.admit(rq.b, rq.tag, stream=stream)
            if x is None:
                return False
        rq.admitted = t_now
        rq.x = x
        self.inflight[i][rq.tag] = (rq, bt)
        return True

    def _release_idle(self, memory_wanted: bool):
        """Destroy batches with no columns in flight whose matrix has nothing
        queued; one idle batch per matrix is kept unless memory is wanted."""
        for i, bl in enumerate(self.batches):
            if self.queues[i]:
                continue
            busy = {id(bt) for _, bt in self.inflight[i].values()}
            keep = [bt for bt in bl if id(bt) in busy]
            idle = [bt for bt in bl if id(bt) not in busy]
            if idle and not keep and not memory_wanted:
                keep.append(idle.pop(0))
            for bt in idle:
                bt.close()
            self.batches[i] = keep

    def run(self, requests, clock=time.perf_counter):
        """Serve `requests` (sorted by arrival).  Returns them completed."""
        import torch
        for rq in requests:
            if rq.b.shape[1] > self.max_cols:
                raise ValueError(f"request {rq.tag}: {rq.b.shape[1]} columns exceed max_cols {self.max_cols}")
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        t0 = clock()
        left = len(requests)
        while left:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                rq = pending.popleft()
                self.queues[rq.matrix].append(rq)
            waiting = False
            for i in range(len(self.slrs)):
                q = self.queues[i]
                with torch.cuda.stream(self.streams[i]):
                    while q and self._admit(i, q[0], self.streams[i], clock() - t0):
                        q.popleft()
                waiting = waiting or bool(q)
            self.peak_bytes = max(self.peak_bytes, self.device_bytes())
            progressed = False
            for i in range(len(self.slrs)):
                live = {id(bt): bt for _, bt in self.inflight[i].values()}
                with torch.cuda.stream(self.streams[i]):
                    for bt in live.values():
                        bt.step(self.iters, stream=self.streams[i])
                        progressed = True
            for i in range(len(self.slrs)):
                live = {id(bt): bt for _, bt in self.inflight[i].values()}
                for bt in live.values():
                    for tag, x, info in bt.poll(stream=self.streams[i]):
                        rq, _ = self.inflight[i].pop(tag)
                        rq.done = clock() - t0
                        rq.info = info
                        rq.x = x
                        left -= 1
            self._release_idle(waiting)
            if waiting and not any(self.inflight) and not any(self.batches):
                stuck = [q[0].tag for q in self.queues if q]
                raise ValueError(f"requests {stuck} do not fit the memory budget even alone")
            if not progressed and pending:
                # idle until the next arrival
                wait = pending[0].arrival - (clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
        torch.cuda.synchronize()
        return requests


def serve_plain(slrs, requests, method: str = "pcg", rtol: float = 1e-8, maxit: int = 300,
                clock=time.perf_counter):
    """One request at a time with slr_solve, in arrival order (no batching)."""
    import torch
    t0 = clock()
    for rq in sorted(requests, key=lambda r: r.arrival):
        now = clock() - t0
        if rq.arrival > now:
            time.sleep(rq.arrival - now)
        rq.admitted = clock() - t0
        x, infos = slrs[rq.matrix].solve(rq.b, method, rtol=rtol, maxit=maxit)
        torch.cuda.synchronize()
        rq.done = clock() - t0
        rq.x = x
        rq.info = {"iters": max(i["iters"] for i in infos), "status": min(i["status"] for i in infos),
                   "relres": max(i["relres"] for i in infos)}
    return requests


def make_requests(ns, count: int, rate: float, seed: int, max_rhs: int = 16, device="cuda"):
    """Poisson arrivals (rate per second; rate <= 0: all at t = 0), matrix
    uniform over the preloaded ones, 1..max_rhs right-hand sides U[-1, 1]."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for tag in range(count):
        if rate > 0:
            t += rng.exponential(1.0 / rate)
        mi = int(rng.integers(0, len(ns)))
        r = int(rng.integers(1, max_rhs + 1))
        b = rng.uniform(-1.0, 1.0, size=(ns[mi], r))
        out.append(Request(tag, mi, torch.tensor(b, dtype=torch.float64, device=device), t))
    return out


def summarize(requests, wall: float) -> dict:
    lat = np.array([r.done - r.arrival for r in requests])
    cols = sum(int(r.b.shape[1]) for r in requests)
    ok = all(r.info.get("status", -1) == 0 for r in requests)
    worst = max(r.info.get("relres", np.inf) for r in requests)
    per = {}
    for r in requests:
        e = per.setdefault(r.matrix, {"requests": 0, "max_iters": 0, "worst_relres": 0.0})
        e["requests"] += 1
        e["max_iters"] = max(e["max_iters"], int(r.info.get("iters", -1)))
        e["worst_relres"] = max(e["worst_relres"], float(r.info.get("relres", np.inf)))
    return {"requests": len(requests), "rhs": cols, "wall_s": round(wall, 4),
            "solves_per_s": round(cols / wall, 3), "requests_per_s": round(len(requests) / wall, 3),
            "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
            "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
            "all_converged": ok, "worst_relres": worst, "per_matrix": [per[i] for i in sorted(per)]}
