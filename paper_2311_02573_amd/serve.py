"""Continuous-batching request loop over the group-testing range search.

Requests (query batches of uneven size, each with its own threshold) arrive
over time.  A fixed set of device workspaces (gt_batch), each on its own HIP
stream, bounds the work in flight; their number follows from a device-memory
budget.  Whenever a workspace is free, the waiting requests are admitted in
arrival order, packed into one call up to the workspace's query limit, and
launched at once, while calls admitted earlier are still running: their
kernels overlap on the device.  Inserts (the paper's streaming setting, Sec. 4)
are applied between steps; a request sees the vectors indexed when it was
admitted.  Latency = completion time - arrival time on the host clock.

The scheduler only needs a backend with `workspace(max_queries)` returning
objects with submit / poll / finish, plus `insert(rows)` and `n`; the GPU
backend wraps paper_2311_02573_amd.gt, and the tests drive the scheduler with
a CPU stand-in.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    queries: object            # [nq, d] float32 (device tensor for the GPU backend)
    rho: np.ndarray            # [nq] float64
    arrival: float             # seconds on the server clock
    admitted: float | None = None
    done: float | None = None
    epoch_n: int | None = None  # vectors visible to the request
    results: list | None = None  # per query: (ids int64, sims float32)

    @property
    def nq(self) -> int:
        return len(self.rho)

    @property
    def latency(self) -> float | None:
        return None if self.done is None else self.done - self.arrival


@dataclasses.dataclass
class _Call:
    ws: object
    requests: list
    sizes: list


class Server:
    """Admission, packing and completion of requests over workspaces."""

    def __init__(self, backend, n_workspaces: int = 4, max_queries: int = 2048,
                 pool: str = "bf16", clock=time.perf_counter):
        self.backend = backend
        self.pool = pool
        self.max_queries = max_queries
        self.free = [backend.workspace(max_queries) for _ in range(n_workspaces)]
        self.busy: list[_Call] = []
        self.waiting: collections.deque[Request] = collections.deque()
        self.finished: list[Request] = []
        self.clock = clock
        self.t0 = clock()

    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: Request):
        if req.nq > self.max_queries:
            raise ValueError(f"request of {req.nq} queries exceeds the workspace limit {self.max_queries}")
        self.waiting.append(req)

    @property
    def idle(self) -> bool:
        return not self.busy and not self.waiting

    def step(self) -> int:
        """Admits what fits, completes what is done; returns completed requests."""
        self._admit()
        return self._complete()

    def _admit(self):
        while self.free and self.waiting:
            group, total = [], 0
            while self.waiting and total + self.waiting[0].nq <= self.max_queries:
                r = self.waiting.popleft()
                group.append(r)
                total += r.nq
            ws = self.free.pop()
            now = self.now()
            n = self.backend.n
            for r in group:
                r.admitted = now
                r.epoch_n = n
            q = self.backend.concat([r.queries for r in group])
            rho = np.concatenate([r.rho for r in group])
            ws.submit(q, rho, self.pool)
            self.busy.append(_Call(ws, group, [r.nq for r in group]))

    def _complete(self) -> int:
        done = 0
        still = []
        for call in self.busy:
            if not call.ws.poll():
                still.append(call)
                continue
            lists = call.ws.finish().to_lists()
            now = self.now()
            off = 0
            for r, k in zip(call.requests, call.sizes):
                r.results = lists[off:off + k]
                r.done = now
                off += k
                self.finished.append(r)
                done += 1
            self.free.append(call.ws)
        self.busy = still
        return done

    def drain(self, timeout_s: float = 60.0):
        t_end = self.now() + timeout_s
        while not self.idle:
            if self.now() > t_end:
                raise TimeoutError("requests still in flight after the drain timeout")
            if self.step() == 0:
                time.sleep(0.0002)


def latency_summary(reqs) -> dict:
    lat = np.array([r.latency for r in reqs if r.latency is not None]) * 1e3
    nq = sum(r.nq for r in reqs if r.latency is not None)
    if len(lat) == 0:
        return {"requests": 0}
    return {"requests": int(len(lat)), "queries": int(nq),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3)}


def run_poisson(server: Server, schedule, make_queries, rho_of, duration_s: float,
                insert_every_s: float | None = None, insert_rows=None):
    """Drives `server` in wall-clock time.  schedule: [(arrival s, batch size)];
    make_queries(i, size) -> queries; rho_of(i, size) -> thresholds;
    insert_rows(k) -> rows for the k-th insert group (applied every
    insert_every_s between steps).  Returns (requests, wall seconds, inserts)."""
    reqs = []
    nxt = 0
    k_ins = 0
    t_start = server.now()
    while True:
        now = server.now() - t_start
        while nxt < len(schedule) and schedule[nxt][0] <= now:
            t, size = schedule[nxt]
            r = Request(nxt, make_queries(nxt, size), rho_of(nxt, size), arrival=t_start + t)
            server.submit(r)
            reqs.append(r)
            nxt += 1
        if insert_every_s and insert_rows is not None and now >= (k_ins + 1) * insert_every_s \
                and now < duration_s:
            server.backend.insert(insert_rows(k_ins))
            k_ins += 1
        server.step()
        if nxt >= len(schedule) and server.idle:
            break
        if now > duration_s + 30.0:
            raise TimeoutError("serving run did not drain")
        if not server.busy and nxt < len(schedule) and not server.waiting:
            time.sleep(max(0.0, min(0.0005, schedule[nxt][0] - now)))
    return reqs, server.now() - t_start, k_ins


class GpuBackend:
    """Backend over a GTIndex (device tensors, one workspace per stream)."""

    def __init__(self, index):
        import torch

        self.index = index
        self.torch = torch

    @property
    def n(self) -> int:
        return self.index.n

    def workspace(self, max_queries: int):
        from paper_2311_02573_amd import gt

        return gt.Workspace(self.index, max_queries)

    def concat(self, parts):
        return parts[0] if len(parts) == 1 else self.torch.cat(parts, 0)

    def insert(self, rows):
        self.index.insert(rows)
