"""Continuous-batching scheduler with admission by memory, driven on the CPU by
a stand-in backend whose workspaces answer with the float64 oracle after a
few polls and whose calls cost a known number of bytes."""
import numpy as np
import pytest

import oracle.brute as ob
from paper_2311_02573_amd import serve, synth


class _Res:
    def __init__(self, lists):
        self._l = lists

    def to_lists(self):
        return self._l


class FakeWorkspace:
    def __init__(self, backend, max_queries):
        self.b, self.max_queries = backend, max_queries
        self.pending = None
        self.last = None

    def submit(self, q, rho, pool, offset, nbytes, pairs):
        assert self.pending is None, "workspace reused while busy"
        assert len(q) <= self.max_queries
        assert nbytes >= self.b.call_bytes(len(q), 0, pairs)[1]
        self.b.in_flight += 1
        self.b.peak = max(self.b.peak, self.b.in_flight)
        self.b.bytes_in_flight += nbytes
        self.b.peak_bytes = max(self.b.peak_bytes, self.b.bytes_in_flight)
        self.b.calls.append(len(q))
        n = self.b.n
        self.pending = (np.asarray(q), np.asarray(rho), n, self.b.polls_needed, nbytes)

    def poll(self):
        q, rho, n, left, nb = self.pending
        if left > 0:
            self.pending = (q, rho, n, left - 1, nb)
            return False
        return True

    def finish(self):
        q, rho, n, _, nb = self.pending
        self.pending = None
        self.b.in_flight -= 1
        self.b.bytes_in_flight -= nb
        res = ob.range_search(self.b.feats[:n], q, rho)
        self.last = {"max_level_entries": 40 * len(q), "results": sum(len(i) for i, _ in res),
                     "continued_tiles": 0}
        return _Res([(i, s.astype(np.float32)) for i, s in res])

    def info(self):
        return self.last


class FakeBackend:
    """Calls cost 4096 + 64 per query + 24 per frontier entry + 36 per pair
    bytes; the least a call accepts is 4096 + 64 per query + 36 per pair +
    2048 (one tile's frontier)."""

    def __init__(self, feats, polls_needed=2):
        self.feats = feats
        self.n = len(feats)
        self.polls_needed = polls_needed
        self.in_flight = self.peak = 0
        self.bytes_in_flight = self.peak_bytes = 0
        self.calls = []
        self.reserved = None

    def reserve(self, nbytes):
        self.reserved = nbytes

    def slot(self, max_queries):
        return FakeWorkspace(self, max_queries)

    def call_bytes(self, nq, entries, pairs):
        base = 4096 + 64 * nq + 36 * pairs
        return base + 24 * max(entries, 0) + 2048, base + 2048

    def submit(self, ws, q, rho, pool, offset, nbytes, pairs):
        assert 0 <= offset and offset + nbytes <= self.reserved
        ws.submit(q, rho, pool, offset, nbytes, pairs)

    def concat(self, parts):
        return np.concatenate(parts, 0)

    def insert(self, rows):
        self.feats = np.concatenate([self.feats, rows], 0)
        self.n = len(self.feats)


def _workload():
    w = synth.workload_small(3000, 48, 200, temp=0.25, seed_offset=21)
    return np.asarray(w.feats), w.queries


def test_every_request_gets_its_own_results_in_order():
    F, Q = _workload()
    be = FakeBackend(F)
    srv = serve.Server(be, 1 << 30, streams=3, max_queries=40)
    sizes = [1, 7, 13, 40, 2, 25, 9, 31, 5, 17, 3, 38]
    off, reqs = 0, []
    for i, k in enumerate(sizes):
        r = serve.Request(i, Q[off:off + k], np.linspace(0.8, 0.95, k), arrival=srv.now())
        off += k
        srv.submit(r)
        reqs.append(r)
    srv.drain(timeout_s=30)
    assert be.peak <= 3 and max(be.calls) <= 40
    assert sum(be.calls) == sum(sizes)
    order = [r.rid for r in srv.finished]
    assert sorted(order) == list(range(len(sizes)))
    for r in reqs:
        want = ob.range_search(F, r.queries, r.rho)
        assert len(r.results) == r.nq
        for (gi, gs), (wi, ws) in zip(r.results, want):
            np.testing.assert_array_equal(gi, wi)
        assert r.latency is not None and r.latency >= 0
    # FIFO: admission times never decrease with arrival order
    adm = [r.admitted for r in reqs]
    assert all(a <= b for a, b in zip(adm, adm[1:]))


def test_requests_admitted_while_others_run():
    F, Q = _workload()
    be = FakeBackend(F, polls_needed=5)
    srv = serve.Server(be, 1 << 30, streams=2, max_queries=16)
    r0 = serve.Request(0, Q[:16], np.full(16, 0.9), arrival=srv.now())
    srv.submit(r0)
    srv.step()
    assert be.in_flight == 1 and r0.done is None
    r1 = serve.Request(1, Q[16:20], np.full(4, 0.9), arrival=srv.now())
    srv.submit(r1)
    srv.step()
    assert be.in_flight == 2, "the second request must start while the first is in flight"
    srv.drain(timeout_s=30)
    assert r0.done is not None and r1.done is not None


def test_oversized_request_is_rejected():
    F, Q = _workload()
    srv = serve.Server(FakeBackend(F), 1 << 30, streams=1, max_queries=8)
    with pytest.raises(ValueError):
        srv.submit(serve.Request(0, Q[:9], np.full(9, 0.9), arrival=0.0))


def test_inserts_are_visible_to_requests_admitted_after_them():
    F, Q = _workload()
    be = FakeBackend(F[:2000])
    srv = serve.Server(be, 1 << 30, streams=2, max_queries=64)
    r0 = serve.Request(0, Q[:10], np.full(10, 0.85), arrival=srv.now())
    srv.submit(r0)
    srv.step()
    be.insert(F[2000:])
    r1 = serve.Request(1, Q[:10], np.full(10, 0.85), arrival=srv.now())
    srv.submit(r1)
    srv.drain(timeout_s=30)
    assert r0.epoch_n == 2000 and r1.epoch_n == 3000
    for r in (r0, r1):
        want = ob.range_search(F[:r.epoch_n], r.queries, r.rho)
        for (gi, _), (wi, _) in zip(r.results, want):
            np.testing.assert_array_equal(gi, wi)


def test_poisson_driver_and_latency_summary():
    F, Q = _workload()
    be = FakeBackend(F, polls_needed=1)
    srv = serve.Server(be, 1 << 30, streams=4, max_queries=64)
    sched = synth.poisson_arrivals(0, rate_per_s=400.0, duration_s=0.2, max_batch=16)
    assert len(sched) > 20
    reqs, wall, ins = serve.run_poisson(
        srv, sched, lambda i, k: Q[(i * 7) % 150:(i * 7) % 150 + k],
        lambda i, k: np.full(k, 0.9), duration_s=0.2)
    s = serve.latency_summary(reqs)
    assert s["requests"] == len(sched) and s["p99_ms"] >= s["p50_ms"] >= 0


def test_arena_allocates_disjoint_aligned_ranges_and_merges():
    rng = np.random.default_rng(5)
    size = 1 << 20
    a = serve.Arena(size)
    live = {}
    for step in range(2000):
        if live and (rng.random() < 0.45 or len(live) > 40):
            off = list(live)[rng.integers(len(live))]
            a.release(off, live.pop(off))
        else:
            n = int(rng.integers(1, 60000))
            off = a.alloc(n)
            if off is None:
                continue
            assert off % 256 == 0 and off + n <= size
            for o, m in live.items():      # no overlap with a live range
                assert off + n <= o or o + m <= off
            live[off] = n
        assert a.used == sum(serve.Arena._round(m) for m in live.values())
    for off in list(live):
        a.release(off, live.pop(off))
    assert a.free == [(0, size)] and a.used == 0


def test_memory_budget_forces_queueing():
    """A budget that holds one call of 16 queries at a time: with three streams
    free, the second and third calls still wait until the first returns its
    memory; every request gets the oracle's result."""
    F, Q = _workload()
    be = FakeBackend(F, polls_needed=3)
    est = serve.Estimator(entries_per_tile=100, pairs_per_query=10, margin=1.0, pairs_margin=1.0)
    one = be.call_bytes(16, est.frontier(16), est.pairs(16))[0]
    srv = serve.Server(be, int(one * 1.5), streams=3, max_queries=16, estimator=est)
    reqs = []
    for i in range(6):
        r = serve.Request(i, Q[16 * i:16 * i + 16], np.full(16, 0.9), arrival=srv.now())
        srv.submit(r)
        reqs.append(r)
    srv.step()
    assert be.in_flight == 1 and len(srv.waiting) == 5
    srv.drain(timeout_s=30)
    assert be.peak == 1 and srv.memory_waits > 0
    assert be.peak_bytes <= int(one * 1.5) and srv.arena.used == 0
    for r in reqs:
        want = ob.range_search(F, r.queries, r.rho)
        for (gi, _), (wi, _) in zip(r.results, want):
            np.testing.assert_array_equal(gi, wi)


def test_group_is_cut_back_to_what_fits():
    """Waiting requests of 4 queries each: a full pack of 64 queries would not
    fit the budget, so the call takes as many requests as fit."""
    F, Q = _workload()
    be = FakeBackend(F, polls_needed=2)
    est = serve.Estimator(entries_per_tile=100, pairs_per_query=10, margin=1.0, pairs_margin=1.0)
    fit = be.call_bytes(24, est.frontier(24), est.pairs(24))[0]
    srv = serve.Server(be, serve.Arena._round(fit) + 100, streams=2, max_queries=64, estimator=est)
    for i in range(16):
        srv.submit(serve.Request(i, Q[4 * i:4 * i + 4], np.full(4, 0.9), arrival=srv.now()))
    srv.step()
    assert be.calls == [24]
    srv.drain(timeout_s=30)
    assert sum(be.calls) == 64 and max(be.calls) <= 24


def test_request_that_never_fits_is_refused():
    F, Q = _workload()
    be = FakeBackend(F)
    srv = serve.Server(be, 5000, streams=1, max_queries=64)
    srv.submit(serve.Request(0, Q[:40], np.full(40, 0.9), arrival=0.0))
    with pytest.raises(MemoryError):
        srv.step()


def test_estimator_follows_measured_calls():
    est = serve.Estimator(entries_per_tile=10, pairs_per_query=10, margin=2.0, pairs_margin=1.5)
    est.observe(100, 5000, 300)          # 2 tiles of 64 queries; larger: taken at once
    assert est.entries == 2500 and est.pairs_q == 10 * 0.9 + 3 * 0.1
    est.observe(100, 1000, 3000)         # smaller entries decay slowly
    assert est.entries == 0.9 * 2500 + 0.1 * 500 and est.pairs_q == 30
    assert est.frontier(10) == int(np.ceil(1 * est.entries * 2.0))
    assert est.frontier(65) == int(np.ceil(2 * est.entries * 2.0))


def test_cancel_waiting_and_running_requests():
    """A waiting request leaves the queue and never runs; a running one's call
    completes (the device cannot be stopped), its results are dropped, and its
    memory returns to the arena; the other requests get theirs."""
    F, Q = _workload()
    be = FakeBackend(F, polls_needed=4)
    srv = serve.Server(be, 1 << 30, streams=1, max_queries=16)
    reqs = [serve.Request(i, Q[10 * i:10 * i + 10], np.full(10, 0.9), arrival=srv.now())
            for i in range(4)]
    for r in reqs:
        srv.submit(r)
    srv.step()
    assert reqs[0].status == "running" and reqs[1].status == "waiting"
    assert srv.cancel(reqs[2]) and reqs[2].status == "cancelled"
    assert srv.cancel(reqs[0]) and reqs[0].status == "cancelling"
    srv.drain(timeout_s=30)
    assert reqs[0].status == "cancelled" and reqs[0].results is None
    assert reqs[2].results is None and 20 not in be.calls[:0]
    assert sum(be.calls) == 30           # requests 0, 1, 3 ran; 2 never did
    for r in (reqs[1], reqs[3]):
        assert r.status == "done"
        want = ob.range_search(F, r.queries, r.rho)
        for (gi, _), (wi, _) in zip(r.results, want):
            np.testing.assert_array_equal(gi, wi)
    assert not srv.cancel(reqs[1]) and srv.arena.used == 0
    s = serve.latency_summary(reqs)
    assert s["requests"] == 2 and s["cancelled"] == 2


def test_admission_timeout():
    """With one stream busy, requests whose admission wait exceeds their
    timeout end unserved; the rest are served in order."""
    F, Q = _workload()
    t = [0.0]
    be = FakeBackend(F, polls_needed=10 ** 9)   # the first call runs until released
    srv = serve.Server(be, 1 << 30, streams=1, max_queries=8, clock=lambda: t[0])
    r0 = serve.Request(0, Q[:8], np.full(8, 0.9), arrival=0.0)
    r1 = serve.Request(1, Q[8:16], np.full(8, 0.9), arrival=0.0, timeout_s=0.5)
    r2 = serve.Request(2, Q[16:24], np.full(8, 0.9), arrival=0.0, timeout_s=5.0)
    for r in (r0, r1, r2):
        srv.submit(r)
    srv.step()
    t[0] = 1.0
    srv.step()
    assert r1.status == "timeout" and r2.status == "waiting"
    be.polls_needed = 0
    ws = srv.busy[0].ws
    ws.pending = ws.pending[:3] + (0,) + ws.pending[4:]
    srv.drain(timeout_s=30)
    assert r0.status == "done" and r2.status == "done" and r1.results is None
    assert [r.rid for r in srv.finished] == [0, 2]


def test_inserts_keep_their_schedule_when_steps_run_long():
    """Insert groups are due every 10 ms; with every poll taking 25 ms the
    driver applies the groups that fell due together, so all groups up to the
    run's end are applied and every request still matches the oracle over
    the rows of its epoch."""
    import time

    F, Q = _workload()
    extra = np.abs(np.random.default_rng(3).normal(size=(2000, F.shape[1]))).astype(np.float32)
    extra /= np.linalg.norm(extra, axis=1, keepdims=True)

    class SlowBackend(FakeBackend):
        def slot(self, ws_id):
            ws = super().slot(ws_id)
            poll = ws.poll

            def slow_poll():
                time.sleep(0.025)
                return poll()

            ws.poll = slow_poll
            return ws

    be = SlowBackend(F, polls_needed=1)
    srv = serve.Server(be, 1 << 30, streams=2, max_queries=32)
    sched = [(0.3 * i / 11, 4) for i in range(12)]   # the last at the run's end
    groups = []

    def rows(k):
        r = extra[20 * k:20 * k + 20]
        groups.append(len(r))
        return r

    reqs, wall, applied = serve.run_poisson(
        srv, sched, lambda i, k: Q[4 * i:4 * i + k], lambda i, k: np.full(k, 0.9),
        duration_s=0.3, insert_every_s=0.01, insert_rows=rows)
    assert applied == 30 and len(groups) == 30
    assert be.n == len(F) + 600
    assert max(r.epoch_n for r in reqs) > len(F)
    for r in reqs:
        want = ob.range_search(be.feats[:r.epoch_n], r.queries, r.rho)
        for (gi, _), (wi, _) in zip(r.results, want):
            np.testing.assert_array_equal(gi, wi)
