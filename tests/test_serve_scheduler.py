"""Continuous-batching scheduler, driven on the CPU by a stand-in backend whose
workspaces answer with the float64 oracle after a few polls."""
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

    def submit(self, q, rho, pool):
        assert self.pending is None, "workspace reused while busy"
        assert len(q) <= self.max_queries
        self.b.in_flight += 1
        self.b.peak = max(self.b.peak, self.b.in_flight)
        self.b.calls.append(len(q))
        n = self.b.n
        self.pending = (np.asarray(q), np.asarray(rho), n, self.b.polls_needed)

    def poll(self):
        q, rho, n, left = self.pending
        if left > 0:
            self.pending = (q, rho, n, left - 1)
            return False
        return True

    def finish(self):
        q, rho, n, _ = self.pending
        self.pending = None
        self.b.in_flight -= 1
        res = ob.range_search(self.b.feats[:n], q, rho)
        return _Res([(i, s.astype(np.float32)) for i, s in res])


class FakeBackend:
    def __init__(self, feats, polls_needed=2):
        self.feats = feats
        self.n = len(feats)
        self.polls_needed = polls_needed
        self.in_flight = self.peak = 0
        self.calls = []

    def workspace(self, max_queries):
        return FakeWorkspace(self, max_queries)

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
    srv = serve.Server(be, n_workspaces=3, max_queries=40)
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
    srv = serve.Server(be, n_workspaces=2, max_queries=16)
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
    srv = serve.Server(FakeBackend(F), n_workspaces=1, max_queries=8)
    with pytest.raises(ValueError):
        srv.submit(serve.Request(0, Q[:9], np.full(9, 0.9), arrival=0.0))


def test_inserts_are_visible_to_requests_admitted_after_them():
    F, Q = _workload()
    be = FakeBackend(F[:2000])
    srv = serve.Server(be, n_workspaces=2, max_queries=64)
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
    srv = serve.Server(be, n_workspaces=4, max_queries=64)
    sched = synth.poisson_arrivals(0, rate_per_s=400.0, duration_s=0.2, max_batch=16)
    assert len(sched) > 20
    reqs, wall, ins = serve.run_poisson(
        srv, sched, lambda i, k: Q[(i * 7) % 150:(i * 7) % 150 + k],
        lambda i, k: np.full(k, 0.9), duration_s=0.2)
    s = serve.latency_summary(reqs)
    assert s["requests"] == len(sched) and s["p99_ms"] >= s["p50_ms"] >= 0
