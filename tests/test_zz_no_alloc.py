"""gt_query_batch_noalloc (every per-call buffer carved out of the library's
fixed device scratch) against gt_query_batch on the same index: ids
identical, similarities within 1e-6 (they are the same kernels, so in fact
identical), on consecutive calls whose second is smaller than the first, so
that what the first left in the scratch must not leak into the second."""
import ctypes

import numpy as np
import pytest
import torch

import oracle.brute as ob
from paper_2311_02573_amd import synth

pytestmark = pytest.mark.gpu

SIM_TOL = 1e-6


def say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def gt():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2311_02573_amd import gt as g

    g.lib()
    return g


def _same(a, b, label):
    assert len(a) == len(b), label
    for j, ((ai, asim), (bi, bsim)) in enumerate(zip(a, b)):
        np.testing.assert_array_equal(ai, bi, err_msg=f"{label} query {j}")
        if len(asim):
            assert np.max(np.abs(asim.astype(np.float64) - bsim.astype(np.float64))) <= SIM_TOL


def test_noalloc_equals_query_batch(gt):
    w = synth.workload_small(20077, 300, 300, temp=0.2, seed_offset=60)
    F = np.asarray(w.feats)
    idx = gt.GTIndex(torch.from_numpy(F).cuda(), pools=("f32", "bf16", "fp8", "max_bf16"))
    Q = torch.from_numpy(w.queries).cuda()
    rho = np.linspace(0.7, 0.95, len(w.queries))
    try:
        for pool in ("bf16", "f32", "fp8", "max_bf16"):
            for k in (300, 45):  # second call smaller than the first
                say(f"noalloc {pool} {k} queries")
                got = idx.query_noalloc(Q[:k], rho[:k], pool=pool).to_lists()
                want = idx.query(Q[:k], rho[:k], pool=pool).to_lists()
                _same(got, want, f"{pool} nq={k}")
        ora = ob.range_search(F, w.queries[:45], rho[:45])
        got = idx.query_noalloc(Q[:45], rho[:45], pool="bf16").to_lists()
        for (gi, gs), (oi, os_) in zip(got, ora):
            np.testing.assert_array_equal(gi, oi)
            if len(gs):
                assert np.max(np.abs(gs.astype(np.float64) - os_)) <= SIM_TOL
    finally:
        idx.close()


def test_noalloc_through_the_c_abi_and_its_limits(gt):
    """Direct C-ABI calls: a result overflow reports the size and valid
    offsets; a call whose worst-case frontier exceeds the scratch is refused
    with GT_ERR_CAPACITY and leaves the next call correct."""
    w = synth.workload_small(3000, 96, 200, temp=0.25, seed_offset=61)
    F = np.asarray(w.feats)
    # capacity 2^20: depth 20, a frontier of 12.6 MB per tile of 64 queries
    idx = gt.GTIndex(torch.from_numpy(F).cuda(), capacity=1 << 20)
    Q = torch.from_numpy(w.queries).cuda()
    lib = gt.lib()
    rho = np.full(200, 0.5)
    ora = ob.range_search(F, w.queries, rho)
    total_want = sum(len(i) for i, _ in ora)
    offs = torch.empty(201, dtype=torch.int64, device="cuda")
    ids = torch.empty(total_want, dtype=torch.int64, device="cuda")
    sims = torch.empty(total_want, dtype=torch.float32, device="cuda")
    total = ctypes.c_int64(0)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def call(nq, max_results):
        r = np.ascontiguousarray(rho[:nq])
        return lib.gt_query_batch_noalloc(idx.handle, ctypes.c_void_p(Q.data_ptr()), nq,
                                          ctypes.c_void_p(r.ctypes.data), gt.POOL_BF16,
                                          max_results, ctypes.c_void_p(offs.data_ptr()),
                                          ctypes.c_void_p(ids.data_ptr()),
                                          ctypes.c_void_p(sims.data_ptr()), ctypes.byref(total),
                                          stream)

    try:
        say("result overflow")
        st = call(200, 0)
        assert st == gt.GT_ERR_RESULT_OVERFLOW and total.value == total_want
        counts = np.diff(offs.cpu().numpy())
        np.testing.assert_array_equal(counts, [len(i) for i, _ in ora])
        say("full call")
        assert call(200, total_want) == gt.GT_OK and total.value == total_want
        res = gt.Results(offs, ids, sims, total.value).to_lists()
        for (gi, gs), (oi, os_) in zip(res, ora):
            np.testing.assert_array_equal(gi, oi)
            if len(gs):
                assert np.max(np.abs(gs.astype(np.float64) - os_)) <= SIM_TOL
        say("too many queries for the scratch")
        big = torch.from_numpy(np.tile(w.queries, (11, 1))).cuda()  # 2200 queries: 35 tiles
        r = np.full(len(big), 0.5)
        big_offs = torch.empty(len(big) + 1, dtype=torch.int64, device="cuda")
        st = lib.gt_query_batch_noalloc(idx.handle, ctypes.c_void_p(big.data_ptr()), len(big),
                                        ctypes.c_void_p(r.ctypes.data), gt.POOL_BF16, 0,
                                        ctypes.c_void_p(big_offs.data_ptr()), None, None,
                                        ctypes.byref(total), stream)
        assert st == gt.GT_ERR_CAPACITY, st
        assert b"scratch" in lib.gt_last_error()
        say("smaller call after the refusal")
        got = idx.query_noalloc(Q[:33], rho[:33], pool="bf16").to_lists()
        _same(got, [(i, s.astype(np.float32)) for i, s in ora[:33]], "after refusal")
    finally:
        idx.close()
