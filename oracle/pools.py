"""Explicit pool-sum tree in float64 -- test infrastructure only.

A pool is the element-wise sum of its member vectors (Sec. 2, sum pooling); the
binary-splitting pools over a power-of-two capacity form a complete binary tree
whose node j at level l (level 0 = root, 2^l nodes) holds rows
[j * 2^(D-l), (j+1) * 2^(D-l)) with zero rows past N.  With the cumulative sums
of Eq. 1 the same pool is C[end] - C[start]; here each node is summed directly.

float64 error bound: a node of height h is a pairwise sum of 2^h non-negative
float32-exact values, so its float64 value S64 satisfies
    |S64 - S_exact| <= ((1 + 2^-53)^h - 1) * S_exact  <=  h * 2^-52 * S_exact,
which is what `exact_bounds` returns as an interval around S_exact.
"""
from __future__ import annotations

import numpy as np


def pool_tree(feats, capacity: int | None = None):
    """levels[l] = float64 array [2^l, d]; levels[D] are the (padded) leaves."""
    f = np.asarray(feats, dtype=np.float64)
    n, d = f.shape
    cap = capacity or 1 << max(0, (n - 1).bit_length())
    assert cap >= n and cap & (cap - 1) == 0
    leaves = np.zeros((cap, d), np.float64)
    leaves[:n] = f
    levels = [leaves]
    while levels[0].shape[0] > 1:
        below = levels[0]
        levels.insert(0, below[0::2] + below[1::2])
    return levels


def exact_bounds(levels, level: int):
    """(lo, hi) float64 arrays bracketing the exact pool sums at `level`."""
    D = len(levels) - 1
    h = D - level
    s = levels[level]
    rel = h * 2.0 ** -52
    return s * (1.0 - rel), s * (1.0 + rel)


def pool_scores(levels, q):
    """Dot product of query q with every pool, per level (float64)."""
    qv = np.asarray(q, dtype=np.float64)
    return [lv @ qv for lv in levels]


def max_pool_tree(feats, capacity: int | None = None):
    """Our-Max pools (Sec. 2): levels[l] = float64 [2^l, d], node j the
    element-wise maximum of its members (exact: a maximum of float32 values is
    one of them); levels[D] are the (zero-padded) leaves."""
    f = np.asarray(feats, dtype=np.float64)
    n, d = f.shape
    cap = capacity or 1 << max(0, (n - 1).bit_length())
    assert cap >= n and cap & (cap - 1) == 0
    leaves = np.zeros((cap, d), np.float64)
    leaves[:n] = f
    levels = [leaves]
    while levels[0].shape[0] > 1:
        below = levels[0]
        levels.insert(0, np.maximum(below[0::2], below[1::2]))
    return levels



def max_min_pool_tree(feats, capacity: int | None = None):
    """Max/min pools for vectors of any sign (Sec. 2, negative descriptors):
    (maxes, mins), each a list of float64 levels [2^l, d] like `pool_tree`;
    node j holds the element-wise maximum / minimum over its members (exact).
    Padding slots past N are not members: a node without members holds -inf
    in `maxes` and +inf in `mins`."""
    f = np.asarray(feats, dtype=np.float64)
    n, d = f.shape
    cap = capacity or 1 << max(0, (n - 1).bit_length())
    assert cap >= n and cap & (cap - 1) == 0
    hi = np.full((cap, d), -np.inf)
    lo = np.full((cap, d), np.inf)
    hi[:n] = f
    lo[:n] = f
    maxes, mins = [hi], [lo]
    while maxes[0].shape[0] > 1:
        maxes.insert(0, np.maximum(maxes[0][0::2], maxes[0][1::2]))
        mins.insert(0, np.minimum(mins[0][0::2], mins[0][1::2]))
    return maxes, mins


def signed_pool_scores(maxes, mins, q):
    """Per level, the max/min pool score of every node for query q (float64):
    sum_k q_k max_k over q_k >= 0 plus q_k min_k over q_k < 0 (-inf for a node
    without members)."""
    qv = np.asarray(q, dtype=np.float64)
    pos, neg = np.maximum(qv, 0.0), np.minimum(qv, 0.0)
    out = []
    for hi, lo in zip(maxes, mins):
        with np.errstate(invalid="ignore"):
            a = np.where(pos > 0, hi, 0.0) @ pos + np.where(neg < 0, lo, 0.0) @ neg
        a[np.isinf(hi).all(axis=1)] = -np.inf
        out.append(a)
    return out
