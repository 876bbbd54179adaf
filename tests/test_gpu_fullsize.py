"""Full-size parity: N = 2^20 softmax vectors, d = 1000, 1024 queries per batch
(the benchmark's workload and launch configuration).

The oracle cannot scan all 1024 queries in test time, so it checks a sample of
queries one by one; for the whole batch, the properties that hold at any size
are checked: every walk format and the exhaustive GEMM return identical id sets
and identical similarities, planted neighbours whose cosine reaches rho are
returned, and every returned id is a valid row.
"""
import numpy as np
import pytest
import torch

import oracle.brute as ob
from paper_2311_02573_amd import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2311_02573_amd import gt

    say("generate N=2^20 d=1000")
    w = synth.workload1(nq=1024)
    idx = gt.GTIndex(torch.from_numpy(w.feats).cuda())
    q = torch.from_numpy(w.queries).cuda()
    yield gt, w, idx, q
    idx.close()


def test_fullsize_sampled_oracle_and_cross_path_identity(setup):
    gt, w, idx, q = setup
    rng = np.random.default_rng(5)
    sample = np.concatenate([np.arange(4), rng.choice(np.arange(4, 1024), 6, replace=False)])
    say("oracle sample at rho=0.8")
    ora = ob.range_search(w.feats, w.queries[sample], 0.8)
    for rho in (0.8, 0.9, 0.95):
        runs = {}
        for f in ("bf16", "f32", "fp8"):
            say(f"walk {f} rho={rho}")
            runs[f] = idx.query(q, rho, pool=f).to_lists()
        say(f"exhaustive rho={rho}")
        runs["exh"] = idx.exhaustive(q, rho).to_lists()
        ref = runs["bf16"]
        for name, lists in runs.items():
            for b in range(1024):
                np.testing.assert_array_equal(lists[b][0], ref[b][0], err_msg=f"{name} q{b} rho={rho}")
                np.testing.assert_array_equal(lists[b][1], ref[b][1], err_msg=f"{name} q{b} rho={rho}")
        for j, b in enumerate(sample):
            oi, os_ = ora[j]
            keep = os_ >= rho
            np.testing.assert_array_equal(ref[b][0], oi[keep], err_msg=f"oracle q{b} rho={rho}")
            if keep.any():
                assert np.max(np.abs(ref[b][1].astype(np.float64) - os_[keep])) <= 1e-6
        nres = sum(len(x[0]) for x in ref)
        assert all(len(x[0]) == 0 or (x[0].min() >= 0 and x[0].max() < w.n) for x in ref)
        say(f"rho={rho}: {nres} results")
        assert nres > 0


def test_fullsize_planted_neighbours_found(setup):
    gt, w, idx, q = setup
    res = idx.query(q, 0.9, pool="bf16").to_lists()
    found = total = 0
    for b in range(1024):
        p = w.planted[b]
        if len(p) == 0:
            continue
        c = ob.pair_cos(w.feats, w.queries, np.full(len(p), b), p)
        for pid, cv in zip(p, c):
            if cv >= 0.9:
                total += 1
                found += int(pid in set(res[b][0].tolist()))
    assert total > 100 and found == total
