"""The exact leaf test's float32 similarity, bit for bit, against a CPU
emulation of its documented summation order (paper Sec. 2: the leaves get an
exact cosine test; the float32 form and its bound are this implementation's,
with float64 deciding the band near rho).

Order, per row pair (x: query, y: vector, both padded with zeros to d_pad):
in 1024-element chunk c, lane l owns elements 1024 c + 256 v + 4 l + j;
slice v = fma(x0, y0, x1 y1) + fma(x2, y2, x3 y3); chunk = (s0 + s1) +
(s2 + s3); chunks added in order; the 64 lane values summed by the tree of
partners 32, 16, 8, 4, 2, 1; similarity = (dot * 1/|q|) * 1/|f| in float32,
the inverse norms rounded from float64.

Queries are multiples of 2^-12 in [0, 1), so that their float64 squared norm
is exact in any summation order; the vectors are generic float32.  A result
whose emulated float32 value lies within 1e-5 of rho was re-decided in
float64 and reports that value instead (checked against the float64 oracle).
The walk's leaf test and the exhaustive path's pair test share the function,
so both are checked.
"""
import sys

import numpy as np
import pytest
import torch

import oracle.brute as ob
from leaf_order import inv_norm, leaf_dot
from paper_2311_02573_amd import synth

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("n,d,nq", [(20000, 1000, 48), (12000, 300, 40), (8000, 2100, 24)])
def test_leaf_similarity_bits(gtmod, n, d, nq):
    w = synth.workload_small(n, d, nq, temp=0.2, seed_offset=60 + d % 89)
    F = np.asarray(w.feats, dtype=np.float32)
    # queries rounded down to multiples of 2^-12 (still near their planted
    # neighbours); their squared norms are then exact in any order
    Q = (np.floor(w.queries.astype(np.float64) * 4096.0) / 4096.0).astype(np.float32)
    rho = np.full(nq, 0.8)
    ora = ob.range_search(F, Q, rho)
    assert sum(len(o[0]) for o in ora) > 50
    dp = (d + 127) // 128 * 128
    Fp = np.zeros((n, dp), np.float32)
    Fp[:, :d] = F
    Qp = np.zeros((nq, dp), np.float32)
    Qp[:, :d] = Q
    invf, invq = inv_norm(F), inv_norm(Q)
    idx = gtmod.GTIndex(torch.from_numpy(F).cuda())
    q = torch.from_numpy(Q).cuda()
    try:
        paths = [("walk bf16", lambda: idx.query(q, rho, pool="bf16")),
                 ("walk f32", lambda: idx.query(q, rho, pool="f32")),
                 ("exhaustive", lambda: idx.exhaustive(q, rho))]
        for label, run in paths:
            say(f"n={n} d={d} nq={nq} {label}")
            got = run().to_lists()
            checked = band = 0
            for b, ((gi, gs), (oi, os_)) in enumerate(zip(got, ora)):
                assert np.array_equal(gi, oi), f"{label} query {b}: ids differ from the oracle"
                if not len(gi):
                    continue
                dot = leaf_dot(np.repeat(Qp[b:b + 1], len(gi), axis=0), Fp[gi])
                cs = ((dot * invq[b]).astype(np.float32) * invf[gi]).astype(np.float32)
                inband = np.abs(cs.astype(np.float64) - rho[b]) < 1e-5
                same = gs.view(np.uint32) == cs.view(np.uint32)
                assert np.all(same | inband), \
                    f"{label} query {b}: {np.sum(~(same | inband))} similarities differ from the emulated order"
                assert np.all(np.abs(gs[inband].astype(np.float64) - os_[inband]) <= 1e-6)
                checked += int(np.sum(~inband))
                band += int(np.sum(inband))
            assert checked > 50, (label, checked)
    finally:
        idx.close()
