"""GPU parity tests: the HIP path (through the C ABI) against the CPU oracle.

Id sets must be bit-identical to the float64 brute-force oracle and reported
similarities within 1e-6 of the oracle's float64 cosines.  Inputs are seeded
synthetic softmax features (paper Sec. 4 uses VGG softmax features; see
paper_2311_02573_amd.synth).
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle.brute as ob
from oracle import formats, pools
from paper_2311_02573_amd import synth

pytestmark = pytest.mark.gpu

SIM_TOL = 1e-6
FORMATS = ("f32", "bf16", "fp8")


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gtmod():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2311_02573_amd import gt

    gt.lib()  # raises if the HIP library is missing
    return gt


def _dev(x, dtype=None):
    t = torch.as_tensor(np.asarray(x)) if not isinstance(x, torch.Tensor) else x
    if dtype is not None:
        t = t.to(dtype)
    return t.contiguous().cuda()


def assert_same(got, want, label, tol=SIM_TOL):
    assert len(got) == len(want), label
    for b, ((gi, gs), (oi, os_)) in enumerate(zip(got, want)):
        if not np.array_equal(gi, oi):
            miss = sorted(set(oi.tolist()) - set(gi.tolist()))[:10]
            extra = sorted(set(gi.tolist()) - set(oi.tolist()))[:10]
            raise AssertionError(f"{label} query {b}: {len(gi)} ids vs oracle {len(oi)}; "
                                 f"missing {miss} extra {extra}")
        if len(gs):
            err = np.max(np.abs(gs.astype(np.float64) - os_))
            assert err <= tol, f"{label} query {b}: similarity error {err}"


def run_all(gtmod, feats_cpu, queries, rho, capacity=0, formats_=FORMATS, exhaustive=True,
            label=""):
    ora = ob.range_search(feats_cpu, queries, rho)
    idx = gtmod.GTIndex(_dev(feats_cpu), capacity=capacity)
    q = _dev(queries, torch.float32)
    try:
        for f in formats_:
            say(f"{label} walk {f}")
            assert_same(idx.query(q, rho, pool=f).to_lists(), ora, f"{label} {f}")
        if exhaustive:
            say(f"{label} exhaustive")
            assert_same(idx.exhaustive(q, rho).to_lists(), ora, f"{label} exhaustive")
    finally:
        idx.close()
    return ora


# ------------------------------------------------------------------ workloads
@pytest.mark.parametrize("rho", [0.8, 0.9, 0.95])
def test_workload0_all_paths(gtmod, rho):
    """N=16384, d=128, 32 queries with planted neighbours."""
    w = synth.workload0()
    ora = run_all(gtmod, w.feats, w.queries, rho, label=f"w0 rho={rho}")
    if rho == 0.9:
        assert sum(len(i) for i, _ in ora) > 100


@pytest.mark.parametrize("n,d,nq,cap", [
    (1, 5, 3, 0), (3, 1, 2, 0), (1000, 100, 33, 0), (4097, 130, 65, 0),
    (3000, 257, 130, 8192), (2048, 1000, 70, 0), (777, 64, 1, 1024),
])
def test_ragged_shapes(gtmod, n, d, nq, cap):
    """Non-power-of-two sizes, several tiles and a ragged tail, odd dimensions."""
    w = synth.workload_small(n, d, nq, temp=0.25, seed_offset=n + d)
    for rho in (0.7, 0.9):
        run_all(gtmod, w.feats, w.queries, rho, capacity=cap, label=f"ragged n={n} d={d} nq={nq} rho={rho}")


def test_odd_size_index_last_vectors(gtmod):
    """An index of odd size N = 2^k + 1 (capacity 2^(k+1)): the last pool of
    the last tested level pairs vector N - 1 with a slot past the epoch.
    Queries equal to the last four vectors find them, against the oracle for
    every pool format and the exhaustive path."""
    for n in (1025, 4097):
        w = synth.workload_small(n, 96, 8, temp=0.25, seed_offset=70 + n % 13)
        F = np.asarray(w.feats)
        Q = w.queries.copy()
        Q[:4] = F[n - 4:]
        rho = np.full(len(Q), 0.9)
        say(f"odd-size index n={n}")
        ora = run_all(gtmod, F, Q, rho, label=f"odd-size n={n}")
        assert all(n - 4 + i in set(ora[i][0].tolist()) for i in range(4))


def test_mixed_thresholds_and_edge_rows(gtmod):
    """Zero rows, duplicated rows, queries equal to rows (cosine 1), per-query
    thresholds including rho <= 0 (every non-zero row) and rho > 1."""
    w = synth.workload_small(3000, 96, 40, temp=0.25, seed_offset=7)
    F = np.asarray(w.feats).copy()
    F[[5, 77, 2999]] = 0.0
    F[100:110] = F[200]
    Q = w.queries.copy()
    Q[3] = F[200]
    Q[4] = F[1234]
    Q[5] = 0.0                         # zero query: empty result
    rho = np.full(len(Q), 0.9)
    rho[0], rho[1], rho[2] = 0.0, -0.5, 1.0
    rho[6], rho[7] = 1.0 + 1e-12, 0.3
    run_all(gtmod, F, Q, rho, label="edge rows")


def test_band_recheck_decides_exactly(gtmod):
    """Thresholds placed exactly on oracle cosines: the float32 test cannot
    decide them, so the float64 recheck must reproduce the oracle bit for bit."""
    w = synth.workload_small(5000, 200, 24, temp=0.25, seed_offset=9)
    F = np.asarray(w.feats)
    base = ob.range_search(F, w.queries, 0.5)
    rho = np.empty(len(w.queries))
    for b, (ids, sims) in enumerate(base):
        rho[b] = sims[len(sims) // 2] if len(sims) else 0.95
    idx = gtmod.GTIndex(_dev(F))
    q = _dev(w.queries)
    ora = ob.range_search(F, w.queries, rho)
    for f in FORMATS:
        say(f"band {f}")
        assert_same(idx.query(q, rho, pool=f).to_lists(), ora, f"band {f}")
    st = idx.stats()
    assert st["rechecked"] > 0
    idx.close()


def test_half_precision_features(gtmod):
    w = synth.workload_small(4000, 128, 50, temp=0.2, dtype="f16", seed_offset=11)
    run_all(gtmod, w.feats, w.queries, 0.85, label="f16 features")
    w = synth.workload_small(4000, 256, 50, temp=0.3, dtype="bf16", seed_offset=12)
    run_all(gtmod, w.feats, w.queries, 0.8, label="bf16 features")


def test_clustered_near_duplicates_per_query_thresholds(gtmod):
    """Stress shape at a reduced size: bfloat16 rows with 8 clusters of 2000
    near-duplicates, a tenth of the queries inside a cluster (thousands of
    neighbours each, many pools live down to the leaves), per-query
    thresholds in [0.75, 0.95]; every path against the oracle."""
    w = synth.workload4()
    say("clustered workload: oracle")
    ora = run_all(gtmod, w.feats, w.queries, w.rho, label="clusters")
    big = [len(ora[b][0]) for b in range(20)]
    assert min(big) >= 1000, big
    # every near-duplicate whose oracle cosine reaches the threshold is found
    for b in range(20):
        want = set(ora[b][0].tolist())
        assert set(w.planted[b].tolist()) & want, b


# --------------------------------------------------------------- tree contents
def test_pool_sums_are_upper_bounds_and_rounded_up(gtmod):
    """Stored float32 pools bracket the exact member sums from above within
    depth ulps; bfloat16 / float8 copies are the least representable values
    >= the float32 pool (converters checked against the format tables)."""
    w = synth.workload_small(3000, 72, 4, temp=0.25, seed_offset=13)
    F = np.asarray(w.feats)
    idx = gtmod.GTIndex(_dev(F))
    st = idx.stats()
    D, dp = st["depth"], st["d_pad"]
    lv = pools.pool_tree(F)
    bvals, _ = formats.bf16_nonneg_values()
    evals, _ = formats.e4m3_nonneg_values()
    for level in range(D + 1):
        say(f"pools level {level}")
        m = idx.read_pools(level, pool="f32").astype(np.float64)[:, :72]
        lo, hi = pools.exact_bounds(lv, level)
        h = D - level
        assert np.all(m >= lo), level
        assert np.all(m <= hi * (1 + 2.0 ** -23) ** h + 1e-300), level
        if level == D:
            continue
        mf = idx.read_pools(level, pool="f32")
        b = idx.read_pools(level, pool="bf16").astype(np.uint32)
        bv = (b << 16).view(np.float32).astype(np.float64)
        want = np.maximum(mf.astype(np.float64), np.where(mf > 0, 2.0 ** -126, 0.0))
        k = formats.least_geq(want, bvals)
        np.testing.assert_array_equal(bv, bvals[k])
        e8 = idx.read_pools(level, pool="fp8")
        scale = 2.0 ** st["fp8_exp"][level]
        ev = evals[e8.astype(np.int64)] * scale
        k8 = formats.least_geq(mf.astype(np.float64) / scale, evals)
        np.testing.assert_array_equal(ev, evals[k8] * scale)
    idx.close()


def test_insert_equals_rebuild(gtmod):
    """Streaming inserts (paper Sec. 4): build on a prefix, insert the rest in
    uneven groups; pools equal a fresh build bit for bit and queries match the
    oracle over every inserted row."""
    w = synth.workload_small(5000, 80, 20, temp=0.25, seed_offset=14)
    F = np.asarray(w.feats)
    idx = gtmod.GTIndex(_dev(F[:1500]), capacity=8192)
    lo = 1500
    for g in (1, 99, 900, 2500):
        first = idx.insert(_dev(F[lo:lo + g]))
        assert first == lo
        lo += g
    assert idx.stats()["n"] == 5000 and idx.stats()["epoch"] == 4
    fresh = gtmod.GTIndex(_dev(F), capacity=8192)
    for level in range(idx.stats()["depth"]):
        a = idx.read_pools(level, pool="f32")
        b = fresh.read_pools(level, pool="f32")
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(idx.read_pools(level, pool="bf16"),
                                      fresh.read_pools(level, pool="bf16"))
    q = _dev(w.queries)
    ora = ob.range_search(F, w.queries, 0.85)
    for f in FORMATS:
        say(f"insert {f}")
        assert_same(idx.query(q, 0.85, pool=f).to_lists(), ora, f"insert {f}")
    with pytest.raises(gtmod.GTError) as e:
        idx.insert(_dev(np.ones((4000, 80), np.float32)))
    assert e.value.status == gtmod.GT_ERR_CAPACITY
    bad = F[:10].copy()
    bad[3, 5] = -1.0
    with pytest.raises(gtmod.GTError) as e:
        idx.insert(_dev(bad))
    assert e.value.status == gtmod.GT_ERR_INVALID_INPUT
    assert idx.stats()["n"] == 5000
    assert_same(idx.query(q, 0.85, pool="bf16").to_lists(), ora, "after rejected insert")
    idx.close()
    fresh.close()


# -------------------------------------------------------------- error handling
def test_errors_and_overflow(gtmod):
    w = synth.workload_small(2000, 64, 10, temp=0.25, seed_offset=15)
    F = np.asarray(w.feats)
    bad = F.copy()
    bad[7, 3] = float("nan")
    with pytest.raises(gtmod.GTError) as e:
        gtmod.GTIndex(_dev(bad))
    assert e.value.status == gtmod.GT_ERR_INVALID_INPUT
    idx = gtmod.GTIndex(_dev(F))
    q = _dev(w.queries)
    qn = w.queries.copy()
    qn[2, 1] = -0.5
    with pytest.raises(gtmod.GTError) as e:
        idx.query(_dev(qn), 0.9)
    assert e.value.status == gtmod.GT_ERR_INVALID_INPUT
    ora = ob.range_search(F, w.queries, 0.0)
    total = sum(len(i) for i, _ in ora)
    with pytest.raises(gtmod.GTError) as e:
        idx.query(q, 0.0, pool="bf16", max_results=total - 1)
    assert e.value.status == gtmod.GT_ERR_RESULT_OVERFLOW
    res = idx.query(q, 0.0, pool="bf16")  # the binding regrows and retries
    assert res.total == total
    assert_same(res.to_lists(), ora, "rho=0 all rows")
    empty = idx.query(_dev(np.zeros((0, 64), np.float32)), 0.9)
    assert empty.total == 0 and empty.offsets.cpu().tolist() == [0]
    idx.close()


def test_workspace_overflow_keeps_results(gtmod):
    """gt_batch_finish with too small buffers reports the size and keeps the
    call's results; a second finish with room returns them without a rerun."""
    import ctypes

    w = synth.workload_small(3000, 96, 12, temp=0.25, seed_offset=17)
    F = np.asarray(w.feats)
    idx = gtmod.GTIndex(_dev(F))
    q = _dev(w.queries)
    ora = ob.range_search(F, w.queries, 0.3)
    total = sum(len(i) for i, _ in ora)
    assert total > 1
    ws = gtmod.Workspace(idx, 64)
    ws.submit(q, 0.3, "bf16")
    lib = gtmod.lib()
    offs = torch.empty(13, dtype=torch.int64, device="cuda")
    ids = torch.empty(total, dtype=torch.int64, device="cuda")
    sims = torch.empty(total, dtype=torch.float32, device="cuda")
    got = ctypes.c_int64(0)
    st = lib.gt_batch_finish(ws._h, 1, ctypes.c_void_p(offs.data_ptr()), ctypes.c_void_p(ids.data_ptr()),
                             ctypes.c_void_p(sims.data_ptr()), ctypes.byref(got))
    assert st == gtmod.GT_ERR_RESULT_OVERFLOW and got.value == total
    st = lib.gt_batch_finish(ws._h, total, ctypes.c_void_p(offs.data_ptr()), ctypes.c_void_p(ids.data_ptr()),
                             ctypes.c_void_p(sims.data_ptr()), ctypes.byref(got))
    assert st == gtmod.GT_OK and got.value == total
    torch.cuda.synchronize()
    res = gtmod.Results(offs, ids, sims, total)
    assert_same(res.to_lists(), ora, "workspace finish after overflow")
    # the workspace is free again; the binding's own retry path gives the same
    ws._max_results = 1
    ws.submit(q, 0.3, "bf16")
    assert_same(ws.finish().to_lists(), ora, "binding retry")
    ws.close()
    idx.close()


# --------------------------------------------------------- determinism / mixes
def test_result_of_a_query_does_not_depend_on_its_batch(gtmod):
    w = synth.workload_small(20000, 200, 150, temp=0.2, seed_offset=16)
    F = np.asarray(w.feats)
    idx = gtmod.GTIndex(_dev(F))
    Q = w.queries
    rho = np.linspace(0.75, 0.95, len(Q))
    for f in FORMATS:
        say(f"mix {f}")
        full = idx.query(_dev(Q), rho, pool=f).to_lists()
        again = idx.query(_dev(Q), rho, pool=f).to_lists()
        for (a, sa), (b, sb) in zip(full, again):
            np.testing.assert_array_equal(a, b)
            np.testing.assert_array_equal(sa, sb)
        perm = np.random.default_rng(0).permutation(len(Q))[:37]
        sub = idx.query(_dev(Q[perm]), rho[perm], pool=f).to_lists()
        for j, p in enumerate(perm):
            np.testing.assert_array_equal(sub[j][0], full[p][0])
            np.testing.assert_array_equal(sub[j][1], full[p][1])
        alone = idx.query(_dev(Q[perm[:1]]), rho[perm[:1]], pool=f).to_lists()[0]
        np.testing.assert_array_equal(alone[0], full[perm[0]][0])
        np.testing.assert_array_equal(alone[1], full[perm[0]][1])
    idx.close()


@pytest.mark.parametrize("dense_last,head", [(-1, -1), (-2, -1), ("deepest", -1),
                                             ("deepest", 2), (-2, 0), (11, 6)])
def test_dense_and_sparse_level_steps_agree(gtmod, dense_last, head):
    """The walk may test the first levels densely (every pool x every query) and
    the rest with per-tile frontiers; any split gives the oracle's result.  An
    explicit head chains several dense steps (each masked by its parent's
    result); the automatic head tests only the last dense level."""
    w = synth.workload_small(20000, 300, 200, temp=0.2, seed_offset=17)
    F = np.asarray(w.feats)
    idx = gtmod.GTIndex(_dev(F))
    depth = idx.stats()["depth"]
    idx.set_option("dense_last", depth - 1 if dense_last == "deepest" else dense_last)
    idx.set_option("head_level", head)
    q = _dev(w.queries)
    for rho in (0.6, 0.9):
        ora = ob.range_search(F, w.queries, rho)
        for f in FORMATS:
            say(f"dense_last={dense_last} head={head} {f} rho={rho}")
            assert_same(idx.query(q, rho, pool=f).to_lists(), ora,
                        f"dense_last={dense_last} head={head} {f}")
            st = idx.stats()
            if head >= 0:
                assert st["head_level"] == head
            elif f != "f32" and dense_last != -1:
                # only the last dense level is tested
                h = st["head_level"]
                assert st["pairs"][h] == 0 and st["pairs"][h + 1] > 0
    idx.close()


@pytest.mark.parametrize("ws", [0, 1, 2])
def test_subtraction_step_agrees(gtmod, ws):
    """The bfloat16 walk may bound each left child's score by its pool's bound
    minus a lower bound of the right child's score (paper Sec. 2 and Alg. 1:
    one dot product per split) instead of reading the left child.  Any setting
    (0 off, 1 every sparse level, 2 all but the last) and any split between
    dense and sparse steps gives the oracle's result.  The row count is not a
    multiple of the pool sizes, so pools straddle the end of the data, where
    the step falls back to the pool's own bound; inserted rows move that end."""
    w = synth.workload_small(20077, 300, 200, temp=0.2, seed_offset=18)
    F = np.asarray(w.feats)
    idx = gtmod.GTIndex(_dev(F), capacity=1 << 15)
    idx.set_option("walk_subtract", ws)
    q = _dev(w.queries)
    try:
        for dl in (-2, 9, 12):
            idx.set_option("dense_last", dl)
            for rho in (0.5, 0.8, 0.9, 0.95):
                say(f"walk_subtract={ws} dense_last={dl} rho={rho}")
                ora = ob.range_search(F, w.queries, rho)
                assert_same(idx.query(q, rho, pool="bf16").to_lists(), ora,
                            f"walk_subtract={ws} dense_last={dl} rho={rho}")
        extra = synth.insert_rows(w.index, 1500, 300, 0.2)
        idx.insert(_dev(extra))
        F2 = np.concatenate([F, extra])
        idx.set_option("dense_last", -2)
        for rho in (0.8, 0.9):
            say(f"walk_subtract={ws} after insert rho={rho}")
            ora = ob.range_search(F2, w.queries, rho)
            assert_same(idx.query(q, rho, pool="bf16").to_lists(), ora,
                        f"walk_subtract={ws} after insert rho={rho}")
    finally:
        idx.close()


# ------------------------------------------------------------ Our-Max pools
MAX_POOLS = ("f32", "bf16", "max_f32", "max_bf16")


def test_max_pool_tree_is_the_elementwise_maximum(gtmod):
    """Our-Max pools (paper Sec. 2): every stored float32 max pool equals the
    element-wise maximum of its members (the oracle's max tree, exactly), and
    the bfloat16 copy is the least bfloat16 >= it (values below 2^-126
    raised to 2^-126, as for sum pools)."""
    w = synth.workload_small(3000, 72, 4, temp=0.25, seed_offset=20)
    F = np.asarray(w.feats)
    idx = gtmod.GTIndex(_dev(F), pools=MAX_POOLS)
    st = idx.stats()
    D = st["depth"]
    lv = pools.max_pool_tree(F)
    bvals, _ = formats.bf16_nonneg_values()
    for level in range(D + 1):
        say(f"max pools level {level}")
        m = idx.read_pools(level, pool="max_f32")[:, :72]
        np.testing.assert_array_equal(m.astype(np.float64), lv[level])
        if level == D:
            continue
        mf = idx.read_pools(level, pool="max_f32")
        b = idx.read_pools(level, pool="max_bf16").astype(np.uint32)
        bv = (b << 16).view(np.float32).astype(np.float64)
        want = np.maximum(mf.astype(np.float64), np.where(mf > 0, 2.0 ** -126, 0.0))
        np.testing.assert_array_equal(bv, bvals[formats.least_geq(want, bvals)])
    idx.close()


@pytest.mark.parametrize("dense_last", [-2, -1, "deepest"])
def test_max_pool_walk_agrees(gtmod, dense_last):
    """The walk over Our-Max pools returns the oracle's set for float32 and
    bfloat16 max pools, with and without dense steps, on softmax data with
    planted neighbours, a ragged row count and per-query thresholds."""
    w = synth.workload_small(20077, 300, 203, temp=0.2, seed_offset=21)
    F = np.asarray(w.feats)
    idx = gtmod.GTIndex(_dev(F), pools=MAX_POOLS)
    depth = idx.stats()["depth"]
    idx.set_option("dense_last", depth - 1 if dense_last == "deepest" else dense_last)
    q = _dev(w.queries)
    try:
        rhos = [0.6, 0.9, np.linspace(0.7, 0.97, len(w.queries))]
        for rho in rhos:
            ora = ob.range_search(F, w.queries, rho)
            for f in ("max_f32", "max_bf16"):
                say(f"max pools {f} dense_last={dense_last}")
                assert_same(idx.query(q, rho, pool=f).to_lists(), ora, f"{f} dense_last={dense_last}")
                assert idx.stats()["last_format"] == gtmod.POOLS[f]
    finally:
        idx.close()


def test_max_pool_inserts_equal_rebuild(gtmod):
    """Inserts update the max pools on the new rows' root-to-leaf paths: the
    tree equals a fresh build and queries match the oracle."""
    w = synth.workload_small(5000, 80, 20, temp=0.25, seed_offset=22)
    F = np.asarray(w.feats)
    idx = gtmod.GTIndex(_dev(F[:1700]), capacity=8192, pools=MAX_POOLS)
    lo = 1700
    for g in (1, 333, 2966):
        idx.insert(_dev(F[lo:lo + g]))
        lo += g
    fresh = gtmod.GTIndex(_dev(F), capacity=8192, pools=MAX_POOLS)
    for level in range(idx.stats()["depth"]):
        np.testing.assert_array_equal(idx.read_pools(level, pool="max_f32"),
                                      fresh.read_pools(level, pool="max_f32"))
        np.testing.assert_array_equal(idx.read_pools(level, pool="max_bf16"),
                                      fresh.read_pools(level, pool="max_bf16"))
    q = _dev(w.queries)
    ora = ob.range_search(F, w.queries, 0.85)
    for f in ("max_f32", "max_bf16"):
        say(f"max insert {f}")
        assert_same(idx.query(q, 0.85, pool=f).to_lists(), ora, f"max insert {f}")
    idx.close()
    fresh.close()


def test_max_pools_clustered_near_duplicates(gtmod):
    """The clustered stress workload (thousands of neighbours per query for a
    tenth of the queries, per-query thresholds) through the max-pool walk."""
    w = synth.workload4()
    ora = ob.range_search(w.feats, w.queries, w.rho)
    idx = gtmod.GTIndex(_dev(w.feats), pools=MAX_POOLS)
    q = _dev(w.queries, torch.float32)
    try:
        for f in ("max_f32", "max_bf16"):
            say(f"clusters {f}")
            assert_same(idx.query(q, w.rho, pool=f).to_lists(), ora, f"clusters {f}")
    finally:
        idx.close()


def test_adaptive_dense_level_keeps_results(gtmod):
    """The automatic dense level moves from call to call with the frontier
    density of the previous call (rows of 512+ columns): on a clustered index
    with thousands of neighbours for some queries, every call, whatever level
    it chose, returns the oracle's set."""
    w = synth.workload4(n=1 << 15, d=512, nq=64, clusters=4, per_cluster=2000)
    ora = ob.range_search(w.feats, w.queries, w.rho)
    idx = gtmod.GTIndex(_dev(w.feats), pools=("f32", "bf16"))
    q = _dev(w.queries, torch.float32)
    heads = []
    try:
        for call in range(4):
            say(f"adaptive dense level, call {call}")
            assert_same(idx.query(q, w.rho, pool="bf16").to_lists(), ora, f"adaptive call {call}")
            heads.append(idx.stats()["head_level"])
        say(f"dense levels chosen: {[h + 1 for h in heads]}")
        assert all(0 <= h < idx.stats()["depth"] for h in heads)
        # the first call uses the fixed rule; its dense frontier moves the
        # following calls' dense level down (entry counts are exact, so this
        # is deterministic for the seeded workload: levels 11 -> 14)
        assert heads[1] > heads[0] and heads[2] == heads[1]
    finally:
        idx.close()


# ------------------------------------------------- launch shapes and big segments
@pytest.mark.parametrize("grid", [8, 16, 24])
def test_more_tiles_than_workgroups_per_xcd(gtmod, grid):
    """The persistent walk kernels split the query tiles over the workgroups
    of each XCD; with fewer workgroups per XCD than tiles (grid / 8 < tiles)
    each workgroup walks several tiles in turn.  A small grid reaches that
    branch with a few hundred queries: every pool format, the subtraction step
    on and off, dense steps on and off, against the oracle."""
    w = synth.workload_small(12000, 200, 300, temp=0.2, seed_offset=30)
    F = np.asarray(w.feats)
    idx = gtmod.GTIndex(_dev(F))
    idx.set_option("grid", grid)
    q = _dev(w.queries)
    rho = np.linspace(0.7, 0.95, len(w.queries))
    ora = ob.range_search(F, w.queries, rho)
    try:
        for dl, ws in ((-2, -1), (-2, 0), (-1, 0), (9, 2)):
            idx.set_option("dense_last", dl)
            idx.set_option("walk_subtract", ws)
            for f in FORMATS:
                say(f"grid={grid} dense_last={dl} walk_subtract={ws} {f}")
                assert_same(idx.query(q, rho, pool=f).to_lists(), ora,
                            f"grid={grid} dense_last={dl} walk_subtract={ws} {f}")
                st = idx.stats()
                assert st["last_tiles"] * 8 > grid  # tiles outnumber workgroups per XCD
    finally:
        idx.close()


def test_maximum_queries_per_call(gtmod):
    """The largest call a format takes: 1024 query tiles (65,536 queries for
    bf16 and fp8 pools, 32,768 for float32 rows), on a small index so that
    every tile's frontier is short; the oracle on every 16th query and the
    whole last tile.  One query more is refused."""
    n, d = 8192, 64
    w = synth.workload_small(n, d, 64, temp=0.25, seed_offset=33)
    F = np.asarray(w.feats)
    g = np.random.default_rng(33)
    idx = gtmod.GTIndex(_dev(F))
    try:
        for fmt, nq in (("bf16", 65536), ("fp8", 65536), ("f32", 32768)):
            # queries near random rows, so that most have a few neighbours
            base = F[g.integers(0, n, nq)].astype(np.float64)
            Q = base * np.exp(g.normal(0.0, 0.08, size=base.shape))
            Q = (Q / np.linalg.norm(Q, axis=1, keepdims=True)).astype(np.float32)
            sample = np.unique(np.concatenate([np.arange(0, nq, 16), np.arange(nq - 64, nq)]))
            ora = ob.range_search(F, Q[sample], 0.9)
            say(f"maximum call {fmt} nq={nq}")
            got = idx.query(_dev(Q), 0.9, pool=fmt).to_lists()
            assert len(got) == nq
            assert_same([got[i] for i in sample], ora, f"max call {fmt}")
            assert sum(len(o[0]) for o in ora) > len(sample)
            with pytest.raises(gtmod.GTError):
                idx.query(_dev(np.concatenate([Q, Q[:1]])), 0.9, pool=fmt)
    finally:
        idx.close()


def test_result_segments_beyond_4096(gtmod):
    """Queries with more than 4096 results each take the radix-sort branch of
    the per-query sort: rho <= 0 on 6500 rows (every non-zero row), and a
    cluster of 6000 near-duplicates of one query at rho = 0.9 (walked down to
    the leaves through thousands of live pools).  Ids and similarities
    against the oracle, element by element."""
    n, d = 9000, 96
    w = synth.workload_small(n, d, 6, temp=0.25, seed_offset=31)
    F = np.asarray(w.feats).copy()
    Q = w.queries.copy()
    g = np.random.default_rng(31)
    # near-duplicates of query 0: its logits' softmax plus a small perturbation
    pos = g.choice(n, size=6000, replace=False)
    noise = np.exp(g.normal(0.0, 0.02, size=(6000, d)))
    dup = Q[0][None, :].astype(np.float64) * noise
    dup /= np.linalg.norm(dup, axis=1, keepdims=True)
    F[pos] = dup.astype(np.float32)
    F[[17, 4000]] = 0.0
    rho = np.array([0.9, 0.0, -0.25, 0.9, 0.5, 0.95])
    ora = ob.range_search(F, Q, rho)
    sizes = [len(o[0]) for o in ora]
    assert sizes[0] > 4096 and sizes[1] > 4096 and sizes[2] > 4096, sizes
    run_all(gtmod, F, Q, rho, label="segments > 4096")
