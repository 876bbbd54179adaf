"""The shifted max/min rows of a signed index never prune a neighbour, under
the worst rounding the device arithmetic allows (no GPU).

Paper Sec. 2 (negative descriptors): a pool keeps the element-wise maximum and
minimum of its members, and a query scores it with the maximum where q_k >= 0
and the minimum where q_k < 0; that score U bounds every member's q.f.  The
index stores R = [max + B | B - min] (B >= every |value|, each entry rounded
up, then rounded up to bfloat16) and walks Q = [max(q,0) | max(-q,0)]
(rounded up to bfloat16) against tau' = (tau + B |q|_1)(1 - (K+2) 2^-22) -
2K 2^-126, K = 2 d_pad products, tau = rho |q| m_min.  This test models that
arithmetic in numpy, independently of the HIP code: every float32 partial
sum of Q.R truncated (products below 2^-126 flushed), and checks that every
pool holding a member with cos >= rho passes, and that dropping the B |q|_1
term from the threshold is caught.
"""
import numpy as np
import pytest

from paper_2311_02573_amd import synth


def _f32_up(x64):
    f = np.asarray(x64, np.float64).astype(np.float32)
    lo = f.astype(np.float64) < x64
    f[lo] = np.nextafter(f[lo], np.float32(np.inf))
    return f


def _f32_down(x64):
    f = np.asarray(x64, np.float64).astype(np.float32)
    hi = f.astype(np.float64) > x64
    f[hi] = np.nextafter(f[hi], np.float32(-np.inf))
    return f


def _bf16_up(x):
    """Least bfloat16 >= x (x >= 0 float32), values below 2^-126 raised to it."""
    u = np.asarray(x, np.float32).view(np.uint32).copy()
    u[(u != 0) & (u < 0x00800000)] = 0x00800000
    hi = (u >> 16) + ((u & 0xFFFF) != 0)
    return (hi.astype(np.uint32) << 16).view(np.float32)


def _accumulate_down(q, r):
    """Float32 accumulation of q . r (both >= 0, bfloat16 values: products
    exact) with every partial sum truncated and tiny products flushed."""
    prod = q.astype(np.float64)[:, None, :] * r.astype(np.float64)[None, :, :]
    prod = np.where(prod < 2.0 ** -126, 0.0, prod)
    s = np.zeros(prod.shape[:-1], np.float32)
    for k in range(prod.shape[-1]):
        s = _f32_down(s.astype(np.float64) + prod[..., k])
    return s


def _case(seed, n=256, d=24, nq=12):
    w = synth.workload_signed(n, d, nq, seed_offset=40 + seed)
    F = np.asarray(w.feats, np.float32)
    Q = np.asarray(w.queries, np.float32)
    # a few queries that are members' near copies, so that neighbours exist
    Q[:4] = F[[3, 50, 128, 200]] + np.float32(1e-3)
    return F, Q


def _thresholds(F, Q, rho, with_shift=True):
    dp = 128 * ((F.shape[1] + 127) // 128)
    K = 2 * dp
    nrm = np.sqrt((Q.astype(np.float64) ** 2).sum(1))
    fn = np.sqrt((F.astype(np.float64) ** 2).sum(1))
    m_min = fn[fn > 0].min()
    B = 2.0 ** np.ceil(np.log2(np.abs(F).max()))
    reff = rho * (1 - 4e-11)
    tau = reff * nrm * m_min * (1 - 4e-11)
    kappa = B * np.abs(Q.astype(np.float64)).sum(1) * (1 - 1e-12) if with_shift else 0.0
    sl = (K + 2) * 2.0 ** -22
    return _f32_down((tau + kappa) * (1 - sl) - 2.0 * K * 2.0 ** -126), B


def _pools(F, B, span):
    """Shifted rows of the pools of `span` consecutive members, as stored:
    float32 rounded up (add_up of f and B), maximum over members, bf16 up."""
    hi = _f32_up(F.astype(np.float64) + B)
    lo = _f32_up(B - F.astype(np.float64))
    n = F.shape[0]
    rows = []
    for a in range(0, n, span):
        rows.append(np.concatenate([hi[a:a + span].max(0), lo[a:a + span].max(0)]))
    return _bf16_up(np.array(rows, np.float32))


def _split_query(Q):
    return _bf16_up(np.concatenate([np.maximum(Q, 0), np.maximum(-Q, 0)], 1).astype(np.float32))


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("span", [2, 8, 32])
def test_pools_with_a_neighbour_pass(seed, span):
    F, Q = _case(seed)
    rho = 0.9
    cos = (Q.astype(np.float64) @ F.astype(np.float64).T) / (
        np.linalg.norm(Q.astype(np.float64), axis=1)[:, None] *
        np.linalg.norm(F.astype(np.float64), axis=1)[None, :])
    assert (cos >= rho).sum() >= 4
    thr, B = _thresholds(F, Q, rho)
    score = _accumulate_down(_split_query(Q), _pools(F, B, span))   # [nq, pools]
    for b in range(Q.shape[0]):
        for i in np.nonzero(cos[b] >= rho)[0]:
            assert score[b, i // span] >= thr[b], (b, i, span)


def test_dropping_the_shift_from_the_threshold_is_caught():
    """Without + B |q|_1 the threshold is far too low and nothing is pruned;
    the check that some pool is pruned fails (a planted mistake in the model
    the GPU path follows)."""
    F, Q = _case(0)
    thr_ok, B = _thresholds(F, Q, 0.9)
    thr_bad, _ = _thresholds(F, Q, 0.9, with_shift=False)
    score = _accumulate_down(_split_query(Q), _pools(F, B, 8))
    assert (score < thr_ok[:, None]).mean() > 0.5      # the real bound prunes
    assert not (score < thr_bad[:, None]).any()        # the mistaken one never does
