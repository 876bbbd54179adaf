"""Serving on the GPU: continuous batching with admission by memory over
external workspaces on their own streams.  Every request's result in the mix
must equal its result run alone (ids identical, similarities within 1e-6;
they are in fact bit-identical), and with inserts between steps, the oracle's
result over the rows indexed when the request was admitted.  A call whose
frontier outgrows its memory runs again tile by tile with the same results."""
import numpy as np
import pytest
import torch

import oracle.brute as ob
from paper_2311_02573_amd import serve, synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def gt():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2311_02573_amd import gt as g

    g.lib()
    return g


def test_mix_equals_alone(gt):
    w = synth.workload_small(60000, 256, 600, temp=0.2, seed_offset=31)
    F = np.asarray(w.feats)
    idx = gt.GTIndex(torch.from_numpy(F).cuda(), pools=("f32", "bf16"))
    Q = torch.from_numpy(w.queries).cuda()
    rng = np.random.default_rng(3)
    srv = serve.Server(serve.GpuBackend(idx), 2 << 30, streams=3, max_queries=192, pool="bf16")
    reqs, off = [], 0
    while off < len(w.queries):
        k = int(min(rng.integers(1, 97), len(w.queries) - off))
        rho = rng.uniform(0.75, 0.95, size=k)
        reqs.append(serve.Request(len(reqs), Q[off:off + k], rho, arrival=srv.now()))
        off += k
    say(f"{len(reqs)} requests")
    for r in reqs:
        srv.submit(r)
        srv.step()
    srv.drain(timeout_s=120)
    assert len(srv.finished) == len(reqs)
    for r in reqs:
        alone = idx.query(r.queries, r.rho, pool="bf16").to_lists()
        for (gi, gs), (ai, as_) in zip(r.results, alone):
            np.testing.assert_array_equal(gi, ai)
            assert np.max(np.abs(gs.astype(np.float64) - as_), initial=0.0) <= 1e-6
    sample = [reqs[0], reqs[len(reqs) // 2], reqs[-1]]
    for r in sample:
        ora = ob.range_search(F, r.queries.cpu().numpy(), r.rho)
        for (gi, _), (oi, _) in zip(r.results, ora):
            np.testing.assert_array_equal(gi, oi)
    idx.close()


def test_inserts_between_steps(gt):
    w = synth.workload_small(40000, 128, 240, temp=0.25, seed_offset=32)
    F = np.asarray(w.feats)
    n0 = 25000
    idx = gt.GTIndex(torch.from_numpy(F[:n0]).cuda(), capacity=65536, pools=("f32", "bf16"))
    Q = torch.from_numpy(w.queries).cuda()
    srv = serve.Server(serve.GpuBackend(idx), 1 << 30, streams=2, max_queries=64, pool="bf16")
    reqs = []
    lo = n0
    for i in range(12):
        r = serve.Request(i, Q[20 * i:20 * i + 20], np.full(20, 0.88), arrival=srv.now())
        srv.submit(r)
        reqs.append(r)
        srv.step()
        if lo < len(F):
            hi = min(len(F), lo + 1500)
            idx.insert(torch.from_numpy(F[lo:hi]).cuda())
            lo = hi
    srv.drain(timeout_s=120)
    epochs = sorted({r.epoch_n for r in reqs})
    assert len(epochs) > 3
    for r in reqs:
        say(f"request {r.rid} epoch {r.epoch_n}")
        ora = ob.range_search(F[:r.epoch_n], r.queries.cpu().numpy(), r.rho)
        for (gi, gs), (oi, os_) in zip(r.results, ora):
            np.testing.assert_array_equal(gi, oi)
            if len(gs):
                assert np.max(np.abs(gs.astype(np.float64) - os_)) <= 1e-6
    idx.close()


def test_workspace_memory_is_reserved_once(gt):
    """A workspace with a query limit allocates its score records for its
    largest call on first use: later calls of other sizes neither grow nor
    reallocate device memory (growing per call used to free and reallocate
    buffers while other calls ran), and their results equal the oracle's."""
    w = synth.workload_small(40000, 128, 256, temp=0.2, seed_offset=33)
    F = np.asarray(w.feats)
    idx = gt.GTIndex(torch.from_numpy(F).cuda(), pools=("f32", "bf16"))
    ws = gt.Workspace(idx, 256)
    Q = torch.from_numpy(w.queries).cuda()
    sizes = (3, 70, 256, 1, 129)
    seen = []
    for k in sizes:
        say(f"workspace call of {k} queries")
        ws.submit(Q[:k], 0.9, pool="bf16")
        res = ws.finish()
        torch.cuda.synchronize()
        seen.append(idx.stats()["bytes_device"])
        ora = ob.range_search(F, w.queries[:k], 0.9)
        for (gi, _), (oi, _) in zip(res.to_lists(), ora):
            assert np.array_equal(gi, oi)
    assert len(set(seen)) == 1, seen
    ws.close()
    idx.close()


def test_serving_shape_against_oracle(gt):
    """The serving index at its full shape: N0 = 2^22 float16 rows, d = 512,
    capacity 2^23 (depth 23), bfloat16 pools; requests of 512, 300, 77 and 1
    queries admitted between inserts of 100 rows, so they see three epochs.
    A sample of every request's queries against the oracle over the rows of
    its epoch, ids element by element, similarities within 1e-6."""
    say("generate N0=2^22 d=512 float16")
    w = synth.workload3()
    idx = gt.GTIndex(w.feats.cuda(), capacity=w.capacity, pools=("f32", "bf16"))
    Q = torch.from_numpy(w.queries).cuda()
    srv = serve.Server(serve.GpuBackend(idx), 8 << 30, streams=2, max_queries=512, pool="bf16")
    added = []
    reqs, off = [], 0
    for i, k in enumerate((512, 300, 77, 1)):
        r = serve.Request(i, Q[off:off + k], np.full(k, 0.9), arrival=srv.now())
        off += k
        srv.submit(r)
        reqs.append(r)
        srv.step()
        if i < 2:
            rows = synth.insert_rows(3, 100, w.d, w.temp, offset=500 + i)
            rt = torch.from_numpy(rows).to(torch.float16)
            idx.insert(rt.cuda())
            added.append(rt)
    srv.drain(timeout_s=120)
    assert len({r.epoch_n for r in reqs}) == 3
    F = torch.cat([w.feats] + added, 0)
    rng = np.random.default_rng(40)
    for r in reqs:
        pick = np.sort(rng.choice(r.nq, size=min(r.nq, 24), replace=False))
        say(f"request {r.rid}: {r.nq} queries, epoch {r.epoch_n}, oracle on {len(pick)}")
        qs = r.queries.cpu().numpy()[pick]
        ora = ob.range_search(F[:r.epoch_n], qs, r.rho[pick])
        for j, b in enumerate(pick):
            gi, gs = r.results[b]
            oi, os_ = ora[j]
            np.testing.assert_array_equal(gi, oi, err_msg=f"request {r.rid} query {b}")
            if len(gs):
                assert np.max(np.abs(gs.astype(np.float64) - os_)) <= 1e-6
    assert sum(len(x[0]) for r in reqs for x in r.results) > 0
    idx.close()


@pytest.mark.parametrize("pool", ["bf16", "fp8", "f32", "max_bf16"])
def test_external_memory_continuation(gt, pool):
    """Calls given far less memory than their frontier needs: a level
    overflows, the call runs again one tile at a time within the same memory,
    and every query's result is the oracle's; with ample memory no tile runs
    alone.  A result overflow during the continuation (more results than the
    first output buffers) is finished again with room, as for any call."""
    w = synth.workload_small(30000, 200, 300, temp=0.2, seed_offset=34)
    F = np.asarray(w.feats)
    idx = gt.GTIndex(torch.from_numpy(F).cuda(), pools=("f32", "bf16", "fp8", "max_bf16"))
    Q = torch.from_numpy(w.queries).cuda()
    rng = np.random.default_rng(9)
    try:
        for rho, entries in ((np.linspace(0.75, 0.95, 300), 10), (0.4, 10), (0.9, 1 << 22)):
            want = ob.range_search(F, w.queries, rho)
            total = sum(len(i) for i, _ in want)
            need, least = gt.call_bytes(idx, 300, pool, entries, total + 4096)
            # the least memory the call accepts: the first pass gets a frontier
            # of 64 entries per tile and overflows
            give = least if entries == 10 else need
            mem = torch.empty(give, dtype=torch.uint8, device="cuda")
            ws = gt.ExternalWorkspace(idx, 300)
            say(f"{pool} external, {give} bytes (least {least}, estimate {need})")
            ws.submit(Q, rho, pool, mem.data_ptr(), give, total + 4096)
            res = ws.finish().to_lists()
            info = ws.info()
            for (gi, gs), (oi, os_) in zip(res, want):
                np.testing.assert_array_equal(gi, oi)
                if len(gs):
                    assert np.max(np.abs(gs.astype(np.float64) - os_)) <= 1e-6
            assert info["results"] == total
            if entries == 10:
                assert info["continued_tiles"] > 0, info
            else:
                assert info["continued_tiles"] == 0, info
            ws.close()
            del mem
    finally:
        idx.close()


def test_memory_admission_queues_clustered_requests(gt):
    """The stress shape at a reduced size (bfloat16 rows, clusters of
    near-duplicates, per-query thresholds in [0.75, 0.95], requests of 1-256
    queries): a memory budget that holds about one call at a time makes
    requests wait for memory while streams are free; every request's result
    equals the same queries run alone through gt_query_batch."""
    w = synth.workload4(n=1 << 17, d=256, nq=600, clusters=8, per_cluster=2000)
    idx = gt.GTIndex(w.feats.cuda(), pools=("f32", "bf16"))
    Q = torch.from_numpy(w.queries).cuda()
    be = serve.GpuBackend(idx)
    est = serve.Estimator(entries_per_tile=20000, pairs_per_query=500)
    one, _ = be.call_bytes(256, est.frontier(256), est.pairs(256))
    srv = serve.Server(be, int(one * 1.3), streams=3, max_queries=256, estimator=est)
    rng = np.random.default_rng(4)
    reqs, off = [], 0
    while off < len(w.queries):
        k = int(min(rng.integers(1, 257), len(w.queries) - off))
        reqs.append(serve.Request(len(reqs), Q[off:off + k], w.rho[off:off + k], arrival=srv.now()))
        off += k
    say(f"{len(reqs)} requests, budget {int(one * 1.3)} bytes")
    for r in reqs:
        srv.submit(r)
    srv.drain(timeout_s=120)
    summ = srv.summary()
    say(f"summary {summ}")
    assert len(srv.finished) == len(reqs)
    assert summ["memory_waits"] > 0 and summ["memory_peak_bytes"] <= int(one * 1.3)
    for r in reqs:
        alone = idx.query(r.queries, r.rho, pool="bf16").to_lists()
        for (gi, gs), (ai, as_) in zip(r.results, alone):
            np.testing.assert_array_equal(gi, ai)
            assert np.max(np.abs(gs.astype(np.float64) - as_), initial=0.0) <= 1e-6
    ora = ob.range_search(w.feats, w.queries[:60], w.rho[:60])
    flat = [x for r in reqs for x in r.results][:60]
    for (gi, _), (oi, _) in zip(flat, ora):
        np.testing.assert_array_equal(gi, oi)
    idx.close()


def test_continuation_keeps_the_calls_epoch(gt):
    """A call whose frontier overflows runs again at finish time; rows
    inserted between its submit and its finish (here copies of its own
    queries, which would match) stay invisible to it, as to any call."""
    w = synth.workload_small(20000, 128, 128, temp=0.2, seed_offset=35)
    F = np.asarray(w.feats)
    idx = gt.GTIndex(torch.from_numpy(F).cuda(), capacity=1 << 15, pools=("f32", "bf16"))
    Q = torch.from_numpy(w.queries).cuda()
    try:
        want = ob.range_search(F, w.queries, 0.85)
        total = sum(len(i) for i, _ in want)
        _, least = gt.call_bytes(idx, 128, "bf16", 10, total + 4096)
        mem = torch.empty(least, dtype=torch.uint8, device="cuda")
        ws = gt.ExternalWorkspace(idx, 128)
        ws.submit(Q, 0.85, "bf16", mem.data_ptr(), least, total + 4096)
        idx.insert(torch.from_numpy(np.repeat(w.queries[:8], 3, axis=0)).cuda())
        res = ws.finish().to_lists()
        assert ws.info()["continued_tiles"] > 0
        for (gi, _), (oi, _) in zip(res, want):
            np.testing.assert_array_equal(gi, oi)
        ws.close()
    finally:
        idx.close()
