"""The score bounds of the subtraction step hold under the worst rounding the
device arithmetic allows (no GPU).

Paper Sec. 2 and Alg. 1 derive one child's score as the pool's score minus the
other child's.  The walk keeps that as bounds: an upper bound of the pool's
real score (the record), a lower bound of the right child's real score from
its computed score, and their difference rounded up.  These tests take the
constants from the device header, model the stored operands exactly as the
build rounds them (float32 master sums rounded up, bfloat16 rounded up with
values below 2^-126 raised to it) and the float32 accumulation at both
extremes (every partial sum truncated, every partial sum rounded up, products
below 2^-126 flushed), and check that the bounds bracket the exact score.
"""
import os
import re
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NUMERICS = os.path.join(ROOT, "paper_2311_02573_amd", "csrc", "gt_numerics.h")


def _const(name):
    m = re.search(rf"constexpr float {name} = ([0-9.eE+-]+)f;", open(NUMERICS).read())
    assert m, name
    return np.float32(float(m.group(1)))


K_UP = _const("kScoreUp")
K_LOW = _const("kScoreLow")


def test_constants_cover_the_derived_factors():
    """kScoreUp and kScoreLow (as float32 values) against the factors the
    derivation needs for K <= 4096 products, with room for one rounding."""
    u = 2.0 ** -23
    for K in (1, 128, 1024, 1152, 4096):
        up_needed = 1.0 / (1.0 - (K + 1) * u)
        low_needed = 1.0 / ((1.0 + (K + 1) * u) * (1.0 + 2.0 ** -7) ** 2 * (1.0 + 40 * u))
        assert float(K_UP) * (1.0 - 2.0 ** -24) > up_needed, K
        assert float(K_LOW) * (1.0 + 2.0 ** -24) < low_needed, K


def _f32_up(x64):
    f = x64.astype(np.float32)
    lo = f.astype(np.float64) < x64
    f[lo] = np.nextafter(f[lo], np.float32(np.inf))
    return f


def _f32_down(x64):
    f = x64.astype(np.float32)
    hi = f.astype(np.float64) > x64
    f[hi] = np.nextafter(f[hi], np.float32(-np.inf))
    return f


def _bf16_up(x):
    """Least bfloat16 >= x (x >= 0 float32), values below 2^-126 raised to it."""
    u = x.view(np.uint32).copy()
    u[(u != 0) & (u < 0x00800000)] = 0x00800000
    hi = (u >> 16) + ((u & 0xFFFF) != 0)
    return (hi.astype(np.uint32) << 16).view(np.float32)


def _master(rows):
    """Pool sum of float32 rows, built pairwise as the tree is, each addition
    rounded up (the build's add_up)."""
    level = [r.astype(np.float32) for r in rows]
    while len(level) > 1:
        level = [_f32_up(level[i].astype(np.float64) + level[i + 1].astype(np.float64))
                 for i in range(0, len(level), 2)]
    return level[0]


def _accumulate(a, b, mode):
    """Float32 accumulation of a . b over the last axis, every partial sum
    rounded toward zero ('down') or up ('up'); products below 2^-126 are
    flushed in 'down' mode (the device may do so) and kept in 'up' mode."""
    prod = a.astype(np.float64) * b.astype(np.float64)     # exact: bf16 x bf16
    if mode == "down":
        prod = np.where(prod < 2.0 ** -126, 0.0, prod)
    s = np.zeros(prod.shape[:-1], np.float32)
    for k in range(prod.shape[-1]):
        x = s.astype(np.float64) + prod[..., k]
        s = _f32_down(x) if mode == "down" else _f32_up(x)
    return s


def _score_upper(s, K):
    # device: fma(s, kScoreUp, K 2^-125), one rounding to nearest (the worst
    # case here: rounded down)
    return _f32_down(s.astype(np.float64) * float(K_UP) + K * 2.0 ** -125)


def _score_lower(s, a):
    # device: max(fma(s, kScoreLow, -a), 0), one rounding (worst case: up)
    return np.maximum(_f32_up(s.astype(np.float64) * float(K_LOW) - a.astype(np.float64)), 0)


def _abs_term(q, root, K):
    # query preparation: 2^-125 (1.01 (|q|_1 + |root|_1) + K 2^-126) + 2^-126
    l1 = q.astype(np.float64).sum(-1) + root.astype(np.float64).sum()
    return _f32_up(np.ldexp(1.01 * l1 + K * 2.0 ** -126, -125) + 2.0 ** -126)


def _case(rng, K, tiny):
    """8 member rows of a pool (two children of 4), 16 queries."""
    rows = rng.random((8, K)) ** 4
    q = rng.random((16, K)) ** 4
    if tiny:
        # components around and below the smallest normal, and exact zeros
        mask = rng.random(rows.shape) < 0.5
        rows[mask] *= 2.0 ** -130
        q[rng.random(q.shape) < 0.5] *= 2.0 ** -128
        rows[rng.random(rows.shape) < 0.1] = 0.0
    return rows.astype(np.float32), q.astype(np.float32)


@pytest.mark.parametrize("K,tiny", [(64, False), (256, False), (64, True), (512, True)])
def test_bounds_bracket_the_real_scores(K, tiny):
    rng = np.random.default_rng(1000 * K + tiny)
    for _ in range(4):
        rows, q = _case(rng, K, tiny)
        real = q.astype(np.float64) @ rows.astype(np.float64).T      # [16, 8]
        S_pool, S_right = real.sum(1), real[:, 4:].sum(1)
        S_left = real[:, :4].sum(1)
        pool = _bf16_up(_master(list(rows)))
        right = _bf16_up(_master(list(rows[4:])))
        qb = _bf16_up(q)
        root = _master(list(rows))          # the pool stands in for the root
        a = _abs_term(q, root, K)
        # the record comes from the lowest computed pool score
        rec = _bf16_up(_score_upper(_accumulate(qb, pool[None, :], "down"), K))
        assert np.all(rec.astype(np.float64) >= S_pool)
        # the right child's lower bound from the highest computed score
        low = _score_lower(_accumulate(qb, right[None, :], "up"), a)
        assert np.all(low.astype(np.float64) <= S_right)
        # left bound: record minus lower bound, rounded up
        d = rec.astype(np.float64) - low.astype(np.float64)
        ub = np.maximum(_f32_up(d), 0)
        assert np.all(ub.astype(np.float64) >= S_left)


def test_a_planted_mistake_is_caught(monkeypatch):
    """The bracket check fails for a lower-bound factor without the slack for
    the operands' upward rounding (0.995 instead of 0.9839): a wrong constant
    in the header would be seen."""
    monkeypatch.setattr(sys.modules[__name__], "K_LOW", np.float32(0.995))
    with pytest.raises(AssertionError):
        for K, tiny in [(64, False), (256, False)]:
            test_bounds_bracket_the_real_scores(K, tiny)
