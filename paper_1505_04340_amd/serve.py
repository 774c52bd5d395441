"""Continuous-batching solve service over several resident SLR preconditioners.

Each preloaded matrix owns one batch (``slr_batch_*``: per-column Krylov
state on the device) on its own HIP stream.  Requests (an RHS block of
1..16 columns for one of the matrices) are admitted while the batch has
free column slots; a batch's column capacity is sized from an HBM budget.
The loop advances every batch that has work by a few iterations (the
launches of different batches overlap on the device), retires finished
requests, and admits waiting ones as slots free up.  A column's arithmetic
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
    """Continuous batching over preloaded SLR contexts."""

    def __init__(self, slrs, method: str = "fcg", rtol: float = 1e-8, maxit: int = 300,
                 hbm_budget_bytes: int = 8 << 30, max_cols: int = 64, iters_per_round: int = 4):
        import torch
        self.slrs = slrs
        self.method = method
        self.iters = iters_per_round
        self.streams = [torch.cuda.Stream() for _ in slrs]
        self.batches = []
        self.cols = []
        share = hbm_budget_bytes // max(1, len(slrs))
        for s in slrs:
            # per-column device bytes of a batch: Krylov vectors plus apply scratch
            per_col = 8 * (6 * s.n + 3 * s.query()["s"] + 64)
            cap = int(max(1, min(max_cols, share // per_col)))
            self.batches.append(P.Batch(s, cap, method, rtol, maxit))
            self.cols.append(cap)
        self.queues = [collections.deque() for _ in slrs]
        self.inflight = [dict() for _ in slrs]

    def close(self):
        for b in self.batches:
            b.close()

    def device_bytes(self) -> int:
        return int(sum(b.bytes() for b in self.batches))

    def run(self, requests, clock=time.perf_counter):
        """Serve `requests` (sorted by arrival).  Returns them completed."""
        import torch
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        t0 = clock()
        left = len(requests)
        while left:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                rq = pending.popleft()
                if rq.b.shape[1] > self.cols[rq.matrix]:
                    raise ValueError(f"request {rq.tag}: {rq.b.shape[1]} columns exceed the batch "
                                     f"capacity {self.cols[rq.matrix]} of matrix {rq.matrix}")
                self.queues[rq.matrix].append(rq)
            progressed = False
            for i, bt in enumerate(self.batches):
                q = self.queues[i]
                with torch.cuda.stream(self.streams[i]):
                    while q:
                        rq = q[0]
                        x = bt.admit(rq.b, rq.tag, stream=self.streams[i])
                        if x is None:
                            break
                        rq.admitted = clock() - t0
                        rq.x = x
                        self.inflight[i][rq.tag] = rq
                        q.popleft()
                    if self.inflight[i]:
                        bt.step(self.iters, stream=self.streams[i])
                        progressed = True
            for i, bt in enumerate(self.batches):
                if not self.inflight[i]:
                    continue
                for tag, x, info in bt.poll(stream=self.streams[i]):
                    rq = self.inflight[i].pop(tag)
                    rq.done = clock() - t0
                    rq.info = info
                    rq.x = x
                    left -= 1
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
