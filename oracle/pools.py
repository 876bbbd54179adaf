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


def members(level: int, node: int, depth: int):
    """Row range [lo, hi) covered by node `node` of `level` in a depth-`depth` tree."""
    span = 1 << (depth - level)
    return node * span, (node + 1) * span


def max_pool_tree(feats, capacity: int | None = None):
    """Our-Max pools (Sec. 3): levels[l] = float64 [2^l, d], node j the
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

