"""GPU parity for wide rows: d up to 4096, the boundary's limit.  Rows of
more than 1152 padded columns (2304 for float8) no longer fit the walk's
query tile in LDS; the walk then streams the tile through LDS in windows.
Every pool format, with and without dense steps, the exhaustive GEMM, and
vectors of any sign (max/min rows of 2 d_pad columns), against the float64
oracle: ids element by element, similarities within 1e-6."""
import sys

import numpy as np
import pytest
import torch

import oracle.brute as ob
from paper_2311_02573_amd import synth

pytestmark = pytest.mark.gpu

SIM_TOL = 1e-6
POOLS = ("f32", "bf16", "fp8", "max_f32", "max_bf16")


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gtmod():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2311_02573_amd import gt

    gt.lib()
    return gt


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


@pytest.mark.parametrize("d", [1153, 2048, 2305, 4096])
def test_wide_rows_every_path(gtmod, d):
    """n = 6000 rows (a ragged tree), 130 queries (3 tiles of 64, 5 of 32)
    with planted neighbours, per-query thresholds; automatic dense level,
    dense steps off, and a grid with more tiles than workgroups per XCD."""
    w = synth.workload_small(6000, d, 130, temp=0.1, seed_offset=80 + d % 97)
    F = np.asarray(w.feats)
    rho = np.linspace(0.55, 0.95, len(w.queries))
    say(f"d={d}: oracle")
    ora = ob.range_search(F, w.queries, rho)
    assert sum(len(i) for i, _ in ora) > 100
    idx = gtmod.GTIndex(torch.from_numpy(F).cuda(), pools=POOLS)
    q = torch.from_numpy(w.queries).cuda()
    try:
        for dl, grid in ((-2, 0), (-1, 0), (-2, 16)):
            idx.set_option("dense_last", dl)
            idx.set_option("grid", grid)
            for f in POOLS:
                say(f"d={d} dense_last={dl} grid={grid} {f}")
                assert_same(idx.query(q, rho, pool=f).to_lists(), ora,
                            f"d={d} dense_last={dl} grid={grid} {f}")
        say(f"d={d} exhaustive")
        assert_same(idx.exhaustive(q, rho).to_lists(), ora, f"d={d} exhaustive")
    finally:
        idx.close()


def test_wide_rows_inserts_and_noalloc(gtmod):
    """Inserts into a d = 3000 index update the wide pools; the walk and the
    allocation-free entry point agree with the oracle over every row."""
    d = 3000
    w = synth.workload_small(5000, d, 70, temp=0.1, seed_offset=91)
    F = np.asarray(w.feats)
    idx = gtmod.GTIndex(torch.from_numpy(F[:3100]).cuda(), capacity=8192)
    q = torch.from_numpy(w.queries).cuda()
    try:
        idx.insert(torch.from_numpy(F[3100:]).cuda())
        ora = ob.range_search(F, w.queries, 0.8)
        for f in ("f32", "bf16", "fp8"):
            say(f"d={d} after insert {f}")
            assert_same(idx.query(q, 0.8, pool=f).to_lists(), ora, f"insert {f}")
            assert_same(idx.query_noalloc(q, 0.8, pool=f).to_lists(), ora, f"noalloc {f}")
    finally:
        idx.close()


@pytest.mark.parametrize("d", [700, 2100])
def test_wide_signed_rows(gtmod, d):
    """Vectors of any sign beyond the LDS tile: a signed index keeps max/min
    rows of 2 d_pad columns (1536 and 4352 here), walked in windows."""
    w = synth.workload_signed(4000, d, 90, seed_offset=d % 89)
    F = np.asarray(w.feats)
    rho = np.linspace(0.6, 0.95, len(w.queries))
    ora = ob.range_search(F, w.queries, rho)
    assert sum(len(i) for i, _ in ora) > 50
    idx = gtmod.GTIndex(torch.from_numpy(F).cuda(), pools=("max_f32", "max_bf16", "signed"))
    q = torch.from_numpy(w.queries).cuda()
    try:
        assert idx.stats()["pool_width"] == 2 * ((d + 127) // 128 * 128)
        for dl in (-2, -1):
            idx.set_option("dense_last", dl)
            for f in ("max_f32", "max_bf16"):
                say(f"signed d={d} dense_last={dl} {f}")
                assert_same(idx.query(q, rho, pool=f).to_lists(), ora, f"signed d={d} {f}")
        assert_same(idx.exhaustive(q, rho).to_lists(), ora, f"signed d={d} exhaustive")
    finally:
        idx.close()
