"""Continuous-batching request loop with admission by device memory.

Requests (query batches of uneven size, each query with its own threshold)
arrive over time.  The server holds one device arena of a fixed byte budget
and a few workspaces, each on its own HIP stream, whose calls take their
device memory from the arena (gt_batch_submit_external).  Whenever a stream is
free, the waiting requests are packed in arrival order into one call (up to
max_queries queries); the call's memory is estimated -- frontier entries and
candidate pairs per query, from what earlier calls measured, with a margin --
and the call is admitted only if that many bytes are free in the arena.  If
not, the packed group is cut back (later requests stay queued), and if not
even its first request fits, the requests wait until running calls return
their memory.  A call whose frontier outgrows its estimate still completes
(the library then runs it one query tile at a time), only later, and raises
the estimate for the calls after it.  Running calls overlap on the device.

Inserts (the paper's streaming setting, Sec. 4) are applied between steps; a
request sees the vectors indexed when it was admitted.  Latency = completion
time - arrival time on the host clock.

The scheduler only needs a backend with `slot(max_queries)` (a workspace with
submit / poll / finish / info), `reserve(nbytes)`, `call_bytes(nq, entries,
pairs)`, `submit(slot, queries, rho, pool, offset, nbytes, pairs)`,
`insert(rows)`, `concat(parts)` and `n`; the GPU backend wraps
paper_2311_02573_amd.gt, and the tests drive the scheduler with a CPU
stand-in.
"""
from __future__ import annotations

import bisect
import collections
import dataclasses
import math
import time

import numpy as np

ALIGN = 256


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
    timeout_s: float | None = None  # longest wait for admission (None: no limit)
    status: str = "waiting"      # waiting, running, done, cancelled, timeout

    @property
    def nq(self) -> int:
        return len(self.rho)

    @property
    def latency(self) -> float | None:
        return None if self.done is None else self.done - self.arrival


class Arena:
    """First-fit allocator of byte ranges of a fixed-size region (offsets
    aligned to 256 bytes).  Free ranges are kept sorted and merged."""

    def __init__(self, size: int):
        self.size = int(size)
        self.free = [(0, self.size)]   # (offset, length), sorted by offset
        self.used = 0
        self.peak = 0

    @staticmethod
    def _round(n: int) -> int:
        return (int(n) + ALIGN - 1) // ALIGN * ALIGN

    def alloc(self, nbytes: int):
        n = self._round(nbytes)
        for k, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(k)
                else:
                    self.free[k] = (off + n, ln - n)
                self.used += n
                self.peak = max(self.peak, self.used)
                return off
        return None

    def release(self, off: int, nbytes: int):
        n = self._round(nbytes)
        k = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(k, (off, n))
        # merge with the neighbours
        if k + 1 < len(self.free) and off + n == self.free[k + 1][0]:
            self.free[k] = (off, n + self.free[k + 1][1])
            self.free.pop(k + 1)
        if k > 0 and self.free[k - 1][0] + self.free[k - 1][1] == off:
            po, pl = self.free[k - 1]
            self.free[k - 1] = (po, pl + self.free[k][1])
            self.free.pop(k)
        self.used -= n


class Estimator:
    """Memory figures of a call: frontier entries at its largest level per
    query tile (an entry is a (pool, tile) pair, so a tile of a few queries
    holds nearly as many as a full one) and candidate pairs per query (about
    the results), each scaled by a margin.  Starts from a prior and follows
    what finished calls report: a larger figure is taken at once, a smaller
    one slowly."""

    def __init__(self, entries_per_tile: float = 8192.0, pairs_per_query: float = 512.0,
                 margin: float = 2.0, pairs_margin: float = 1.5, tile_queries: int = 64):
        self.entries = float(entries_per_tile)
        self.pairs_q = float(pairs_per_query)
        self.margin = margin            # entries spread unevenly over the frontier's slots
        self.pairs_margin = pairs_margin
        self.tile = tile_queries

    def tiles(self, nq: int) -> int:
        return (nq + self.tile - 1) // self.tile

    def frontier(self, nq: int) -> int:
        return int(math.ceil(self.tiles(nq) * self.entries * self.margin))

    def pairs(self, nq: int) -> int:
        return int(math.ceil(nq * self.pairs_q * self.pairs_margin)) + 1024

    def observe(self, nq: int, max_level_entries: int, results: int):
        if nq <= 0:
            return
        for name, v in (("entries", max_level_entries / self.tiles(nq)), ("pairs_q", results / nq)):
            old = getattr(self, name)
            setattr(self, name, v if v > old else 0.9 * old + 0.1 * v)


@dataclasses.dataclass
class _Call:
    ws: object
    requests: list
    sizes: list
    offset: int
    nbytes: int


class Server:
    """Admission by memory, packing and completion of requests."""

    def __init__(self, backend, memory_budget: int, streams: int = 4, max_queries: int = 2048,
                 pool: str = "bf16", estimator: Estimator | None = None, clock=time.perf_counter):
        self.backend = backend
        self.pool = pool
        self.max_queries = max_queries
        self.arena = Arena(memory_budget)
        backend.reserve(self.arena.size)
        self.free = [backend.slot(max_queries) for _ in range(streams)]
        self.busy: list[_Call] = []
        self.waiting: collections.deque[Request] = collections.deque()
        self.finished: list[Request] = []
        self.dropped: list[Request] = []   # cancelled or timed out
        self.est = estimator or Estimator()
        self.clock = clock
        self.t0 = clock()
        self.memory_waits = 0        # admission passes that found no memory for the next request
        self.continued_calls = 0     # calls whose frontier outgrew their memory
        self.calls = 0

    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: Request):
        if req.nq > self.max_queries:
            raise ValueError(f"request of {req.nq} queries exceeds the call limit {self.max_queries}")
        req.status = "waiting"
        self.waiting.append(req)

    def cancel(self, req: Request) -> bool:
        """Withdraws a request.  A waiting one leaves the queue at once; a
        running one cannot be stopped on the device, so its call completes
        and its results are dropped.  Returns False if it had already ended."""
        if req.status == "waiting":
            self.waiting.remove(req)
            self._end(req, "cancelled")
            return True
        if req.status == "running":
            req.status = "cancelling"
            return True
        return False

    def _end(self, req: Request, status: str):
        req.status = status
        req.done = self.now()
        if status != "done":
            req.results = None
            self.dropped.append(req)
        else:
            self.finished.append(req)

    def _expire(self):
        """Requests that waited past their admission timeout end unserved."""
        if not self.waiting:
            return
        now = self.now()
        keep = collections.deque()
        for r in self.waiting:
            if r.timeout_s is not None and now - r.arrival > r.timeout_s:
                self._end(r, "timeout")
            else:
                keep.append(r)
        self.waiting = keep

    @property
    def idle(self) -> bool:
        return not self.busy and not self.waiting

    def step(self) -> int:
        """Completes what is done, admits what fits; returns completed requests."""
        done = self._complete()
        self._expire()
        self._admit()
        return done

    def _memory_for(self, nq: int, least_ok: bool = False):
        """(offset, bytes, pairs) reserved in the arena for a call of nq
        queries at its estimated memory (or at the least memory the call
        accepts, with least_ok), or None."""
        pairs = self.est.pairs(nq)
        need, least = self.backend.call_bytes(nq, self.est.frontier(nq), pairs)
        nbytes = least if least_ok else need
        off = self.arena.alloc(nbytes)
        return None if off is None else (off, nbytes, pairs)

    def _admit(self):
        while self.free and self.waiting:
            k, total = 0, 0
            while k < len(self.waiting) and total + self.waiting[k].nq <= self.max_queries:
                total += self.waiting[k].nq
                k += 1
            got = None
            while k > 0:
                nq = sum(self.waiting[i].nq for i in range(k))
                got = self._memory_for(nq)
                if got is not None:
                    break
                k -= 1          # later requests stay queued
            if got is None and not self.busy:
                # nothing running will return memory: the first request alone,
                # with the least memory it accepts (its frontier may then run
                # tile by tile)
                k = 1
                got = self._memory_for(self.waiting[0].nq, least_ok=True)
                if got is None:
                    raise MemoryError(f"a request of {self.waiting[0].nq} queries does not fit "
                                      f"the serving memory budget of {self.arena.size} bytes")
            if got is None:
                self.memory_waits += 1
                return
            off, nbytes, pairs = got
            group = [self.waiting.popleft() for _ in range(k)]
            ws = self.free.pop()
            now = self.now()
            n = self.backend.n
            for r in group:
                r.admitted = now
                r.epoch_n = n
                r.status = "running"
            q = self.backend.concat([r.queries for r in group])
            rho = np.concatenate([r.rho for r in group])
            self.backend.submit(ws, q, rho, self.pool, off, nbytes, pairs)
            self.busy.append(_Call(ws, group, [r.nq for r in group], off, nbytes))
            self.calls += 1

    def _complete(self) -> int:
        done = 0
        still = []
        for call in self.busy:
            if not call.ws.poll():
                still.append(call)
                continue
            lists = call.ws.finish().to_lists()
            info = call.ws.info()
            self.arena.release(call.offset, call.nbytes)
            nq = sum(call.sizes)
            self.est.observe(nq, info["max_level_entries"], info["results"])
            if info["continued_tiles"]:
                self.continued_calls += 1
            now = self.now()
            off = 0
            for r, k in zip(call.requests, call.sizes):
                if r.status == "cancelling":
                    self._end(r, "cancelled")
                else:
                    r.results = lists[off:off + k]
                    self._end(r, "done")
                    r.done = now
                off += k
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

    def summary(self) -> dict:
        return {"memory_budget_bytes": self.arena.size, "memory_peak_bytes": self.arena.peak,
                "calls": self.calls, "memory_waits": self.memory_waits,
                "continued_calls": self.continued_calls,
                "estimate_entries_per_tile": round(self.est.entries, 1),
                "estimate_pairs_per_query": round(self.est.pairs_q, 1)}


def latency_summary(reqs) -> dict:
    """Latency percentiles over the requests served (cancelled and timed-out
    requests are counted apart)."""
    served = [r for r in reqs if r.status == "done" and r.latency is not None]
    lat = np.array([r.latency for r in served]) * 1e3
    nq = sum(r.nq for r in served)
    if len(lat) == 0:
        return {"requests": 0}
    return {"requests": int(len(lat)), "queries": int(nq),
            "cancelled": sum(r.status == "cancelled" for r in reqs),
            "timed_out": sum(r.status == "timeout" for r in reqs),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3)}


def run_poisson(server: Server, schedule, make_queries, rho_of, duration_s: float,
                insert_every_s: float | None = None, insert_rows=None, progress=None):
    """Drives `server` in wall-clock time.  schedule: [(arrival s, batch size)];
    make_queries(i, size) -> queries; rho_of(i, size) -> thresholds;
    insert_rows(k) -> rows for the k-th insert group, due every insert_every_s
    up to duration_s; the groups that are due are applied together between
    steps, so a long step delays them but none is skipped.  progress(s) is
    called about every 10 s of the run.  Returns (requests, wall seconds,
    insert groups applied)."""
    reqs = []
    nxt = 0
    k_ins = 0
    n_groups = int(duration_s / insert_every_s + 1e-9) if insert_every_s and insert_rows else 0
    next_report = 10.0
    t_start = server.now()
    while True:
        now = server.now() - t_start
        while nxt < len(schedule) and schedule[nxt][0] <= now:
            t, size = schedule[nxt]
            r = Request(nxt, make_queries(nxt, size), rho_of(nxt, size), arrival=t_start + t)
            server.submit(r)
            reqs.append(r)
            nxt += 1
        # every insert group that is due is applied now, in one call: a step
        # that ran long must not let the inserts fall behind their schedule
        due = []
        while k_ins < n_groups and now >= (k_ins + 1) * insert_every_s:
            due.append(insert_rows(k_ins))
            k_ins += 1
        if due:
            server.backend.insert(due[0] if len(due) == 1 else server.backend.concat(due))
        server.step()
        if progress is not None and now >= next_report:
            progress(now)
            next_report += 10.0
        if nxt >= len(schedule) and server.idle:
            break
        if now > duration_s + 60.0:
            raise TimeoutError("serving run did not drain")
        if not server.busy and nxt < len(schedule) and not server.waiting:
            time.sleep(max(0.0, min(0.0005, schedule[nxt][0] - now)))
    return reqs, server.now() - t_start, k_ins


class GpuBackend:
    """Backend over a GTIndex: one device arena (a uint8 tensor) and external
    workspaces, one stream each."""

    def __init__(self, index, pool: str = "bf16"):
        import torch

        self.index = index
        self.torch = torch
        self.pool = pool
        self.arena = None

    @property
    def n(self) -> int:
        return self.index.n

    def reserve(self, nbytes: int):
        self.arena = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device="cuda")

    def slot(self, max_queries: int):
        from paper_2311_02573_amd import gt

        return gt.ExternalWorkspace(self.index, max_queries)

    def call_bytes(self, nq: int, entries: int, pairs: int):
        from paper_2311_02573_amd import gt

        return gt.call_bytes(self.index, nq, self.pool, entries, pairs)

    def submit(self, ws, q, rho, pool, offset, nbytes, pairs):
        ws.submit(q, rho, pool, self.arena.data_ptr() + offset, nbytes, pairs)

    def concat(self, parts):
        return parts[0] if len(parts) == 1 else self.torch.cat(parts, 0)

    def insert(self, rows):
        self.index.insert(rows)
