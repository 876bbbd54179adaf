"""GPU parity for vectors of any sign (paper Sec. 2, negative descriptors):
max/min pools, walked through the C ABI, against the CPU oracle.

Id sets must be bit-identical to the float64 brute-force oracle and reported
similarities within 1e-6 of its cosines.  Inputs: centred softmax rows
unit(softmax(z/T) - 1/d) with planted neighbours (paper_2311_02573_amd.synth).
"""
import sys

import numpy as np
import pytest
import torch

import oracle.brute as ob
from oracle import formats, pools
from paper_2311_02573_amd import synth

pytestmark = pytest.mark.gpu

SIM_TOL = 1e-6
SIGNED = ("max_f32", "max_bf16", "signed")


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


def _f32_up_sum(v, B):
    """Least float32 >= v + B (exact real sum) for float32-exact v with |v| <=
    B, B a power of two.  The float64 sum s may be rounded; Fast2Sum gives its
    exact error e = (v + B) - s.  If s is not a float32 the answer is the least
    float32 above s (the error is far below a float32 ulp); if s is one, the
    answer moves one float32 up when e > 0."""
    v = np.asarray(v, np.float64)
    s = v + B
    e = v - (s - B)
    f = s.astype(np.float32)
    below = f.astype(np.float64) < s
    f[below] = np.nextafter(f[below], np.float32(np.inf))
    bump = (f.astype(np.float64) == s) & (e > 0)
    f[bump] = np.nextafter(f[bump], np.float32(np.inf))
    return f


def test_shifted_max_min_rows(gtmod):
    """Every stored row of a signed index is [max + B | B - min] over the
    pool's members (the oracle's max/min tree), each entry the least float32
    >= the exact value, zero past d and for pools without members; B is the
    least power of two >= the largest |value|; the bfloat16 copy is the least
    bfloat16 >= the float32 row."""
    w = synth.workload_signed(3000, 72, 4, seed_offset=1)
    F = np.asarray(w.feats)
    idx = gtmod.GTIndex(_dev(F), capacity=4096, pools=SIGNED)
    st = idx.stats()
    D, dp = st["depth"], st["d_pad"]
    assert st["pool_width"] == 2 * dp
    B = 2.0 ** np.ceil(np.log2(np.abs(F).max()))
    assert st["shift_bound"] == B
    assert st["pool_formats"] & gtmod.POOL_SIGNED and not st["pool_formats"] & gtmod.POOL_F32
    maxes, mins = pools.max_min_pool_tree(F, 4096)
    bvals, _ = formats.bf16_nonneg_values()
    for level in range(D):
        say(f"signed rows level {level}")
        m = idx.read_pools(level, pool="max_f32")
        empty = np.isinf(maxes[level]).all(axis=1)
        hi = _f32_up_sum(np.where(empty[:, None], 0.0, maxes[level]), B)
        lo = _f32_up_sum(np.where(empty[:, None], 0.0, -mins[level]), B)
        hi[empty] = 0.0
        lo[empty] = 0.0
        np.testing.assert_array_equal(m[:, :72], hi)
        np.testing.assert_array_equal(m[:, dp:dp + 72], lo)
        assert not m[:, 72:dp].any() and not m[:, dp + 72:].any()
        b = idx.read_pools(level, pool="max_bf16").astype(np.uint32)
        bv = (b << 16).view(np.float32).astype(np.float64)
        want = np.maximum(m.astype(np.float64), np.where(m > 0, 2.0 ** -126, 0.0))
        np.testing.assert_array_equal(bv, bvals[formats.least_geq(want, bvals)])
    leaves = idx.read_pools(D, 0, 3000, pool="max_f32")[:, :72]
    np.testing.assert_array_equal(leaves, F)
    idx.close()


@pytest.mark.parametrize("n,d,nq,dense_last", [
    (20077, 300, 203, -2), (20077, 300, 203, -1), (20077, 300, 203, "deepest"),
    (4097, 130, 65, -2), (1, 5, 3, -2), (2, 512, 9, -2), (70000, 512, 130, -2)])
def test_signed_walk_matches_oracle(gtmod, n, d, nq, dense_last):
    """The max/min walk (float32 and bfloat16 rows, with and without dense
    steps) and the exhaustive path on a signed index return the oracle's set,
    for one threshold and for per-query thresholds."""
    w = synth.workload_signed(n, d, nq, seed_offset=2 + n % 7)
    F = np.asarray(w.feats)
    idx = gtmod.GTIndex(_dev(F), pools=SIGNED)
    depth = idx.stats()["depth"]
    idx.set_option("dense_last", depth - 1 if dense_last == "deepest" else dense_last)
    q = _dev(w.queries)
    try:
        for rho in (0.6, 0.9, np.linspace(0.55, 0.97, nq)):
            ora = ob.range_search(F, w.queries, rho)
            for f in ("max_f32", "max_bf16"):
                say(f"signed n={n} d={d} nq={nq} {f} dense_last={dense_last}")
                assert_same(idx.query(q, rho, pool=f).to_lists(), ora, f"signed {f}")
            say(f"signed n={n} exhaustive")
            assert_same(idx.exhaustive(q, rho).to_lists(), ora, "signed exhaustive")
    finally:
        idx.close()


def test_signed_edge_rows(gtmod):
    """Zero rows (never members), exact and scaled duplicates of a query, its
    negation (cosine -1), a one-hot of either sign, a zero query (no result),
    a query equal to a row at rho = 1."""
    w = synth.workload_signed(1500, 40, 12, seed_offset=3)
    F = np.array(w.feats)
    Q = np.array(w.queries)
    F[0] = 0.0
    F[1] = Q[0]
    F[2] = 3.0 * Q[0]
    F[3] = -Q[0]
    F[4] = 0.0
    F[4, 7] = -0.5
    F[5] = 0.0
    F[5, 7] = 0.25
    Q[11] = 0.0
    Q[10] = F[900]
    idx = gtmod.GTIndex(_dev(F), pools=SIGNED)
    q = _dev(Q)
    try:
        for rho in (0.3, 0.9, 1.0):
            ora = ob.range_search(F, Q, rho)
            for f in ("max_f32", "max_bf16"):
                say(f"signed edges {f} rho={rho}")
                got = idx.query(q, rho, pool=f).to_lists()
                assert_same(got, ora, f"signed edges {f}")
                assert len(got[11][0]) == 0
        assert {1, 2} <= set(idx.query(q, 0.99, pool="max_bf16").to_lists()[0][0].tolist())
    finally:
        idx.close()


def test_signed_inserts_equal_rebuild(gtmod):
    """Inserts re-derive the shifted rows on the new rows' paths: the tree
    equals a fresh build over the same rows (same B) and queries match the
    oracle.  A row beyond B is refused with INVALID_INPUT and leaves the
    index as it was."""
    w = synth.workload_signed(5000, 80, 20, seed_offset=4)
    F = np.asarray(w.feats)
    idx = gtmod.GTIndex(_dev(F[:1700]), capacity=8192, pools=SIGNED)
    lo = 1700
    for g in (1, 333, 2966):
        idx.insert(_dev(F[lo:lo + g]))
        lo += g
    fresh = gtmod.GTIndex(_dev(F), capacity=8192, pools=SIGNED)
    assert idx.stats()["shift_bound"] == fresh.stats()["shift_bound"]
    for level in range(idx.stats()["depth"]):
        np.testing.assert_array_equal(idx.read_pools(level, pool="max_f32"),
                                      fresh.read_pools(level, pool="max_f32"))
        np.testing.assert_array_equal(idx.read_pools(level, pool="max_bf16"),
                                      fresh.read_pools(level, pool="max_bf16"))
    B = idx.stats()["shift_bound"]
    bad = np.array(F[:2])
    bad[1, 3] = -2.0 * B
    with pytest.raises(gtmod.GTError) as e:
        idx.insert(_dev(bad))
    assert e.value.status == gtmod.GT_ERR_INVALID_INPUT
    assert idx.stats()["n"] == 5000
    q = _dev(w.queries)
    ora = ob.range_search(F, w.queries, 0.85)
    for f in ("max_f32", "max_bf16"):
        say(f"signed insert {f}")
        assert_same(idx.query(q, 0.85, pool=f).to_lists(), ora, f"signed insert {f}")
    idx.close()
    fresh.close()


def test_signed_errors(gtmod):
    """Sum formats, d > 4096, rho <= 0 and non-finite values are refused; a
    negative value without the signed flag is refused as before."""
    w = synth.workload_signed(600, 16, 3, seed_offset=5)
    F = _dev(w.feats)
    for p in (("f32", "signed"), ("bf16", "max_f32", "signed"), ("fp8", "signed")):
        with pytest.raises(gtmod.GTError) as e:
            gtmod.GTIndex(F, pools=p)
        assert e.value.status == gtmod.GT_ERR_INVALID_ARG, p
    with pytest.raises(gtmod.GTError) as e:
        gtmod.GTIndex(_dev(np.zeros((4, 4097), np.float32)), pools=SIGNED)
    assert e.value.status == gtmod.GT_ERR_INVALID_ARG
    with pytest.raises(gtmod.GTError) as e:
        gtmod.GTIndex(F, pools=("f32", "max_f32"))
    assert e.value.status == gtmod.GT_ERR_INVALID_INPUT
    nan = np.array(w.feats)
    nan[5, 5] = np.nan
    with pytest.raises(gtmod.GTError) as e:
        gtmod.GTIndex(_dev(nan), pools=SIGNED)
    assert e.value.status == gtmod.GT_ERR_INVALID_INPUT
    idx = gtmod.GTIndex(F, pools=SIGNED)
    q = _dev(w.queries)
    try:
        for rho in (0.0, -0.5, [0.9, 0.0, 0.9]):
            with pytest.raises(gtmod.GTError) as e:
                idx.query(q, rho, pool="max_f32")
            assert e.value.status == gtmod.GT_ERR_INVALID_ARG
            with pytest.raises(gtmod.GTError) as e:
                idx.exhaustive(q, rho)
            assert e.value.status == gtmod.GT_ERR_INVALID_ARG
        with pytest.raises(gtmod.GTError) as e:
            idx.query(q, 0.9, pool="bf16")
        assert e.value.status == gtmod.GT_ERR_INVALID_ARG
        qn = w.queries.copy()
        qn[1, 2] = np.inf
        with pytest.raises(gtmod.GTError) as e:
            idx.query(_dev(qn), 0.9, pool="max_bf16")
        assert e.value.status == gtmod.GT_ERR_INVALID_INPUT
        ora = ob.range_search(w.feats, w.queries, 0.9)
        assert_same(idx.query(q, 0.9, pool="max_bf16").to_lists(), ora, "after errors")
    finally:
        idx.close()
