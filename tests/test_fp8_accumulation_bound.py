"""Soundness of the float8 pruning threshold under the float8 matrix cores'
accumulation (no GPU).

Measured on gfx950 (the fp8 32x32x16 / 16x16x32 and f8f6f4 forms alike): the
products of a group of 8 consecutive dimensions are summed with truncation
about 13 bits below the group's largest product, and each group sum is then
added to the float32 accumulator.  This file models that accumulation on
e4m3 operands -- random ones, softmax-shaped ones and adversarial groups (one
large product beside seven just below the truncation step) -- and checks that
the computed score never falls below the real one by the factor the float8
threshold is lowered by (kFp8ThrFactor = 1 - 2^-8 in gt_numerics.h), while
the float32-only slack used before does not cover the adversarial case."""
import math
import os
import re

import numpy as np
import pytest

from oracle import formats

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_factor():
    src = open(os.path.join(ROOT, "paper_2311_02573_amd", "csrc", "gt_numerics.h")).read()
    m = re.search(r"kFp8ThrFactor\s*=\s*1\.0f\s*-\s*0x1p-(\d+)f", src)
    assert m, "kFp8ThrFactor not found"
    return 1.0 - 2.0 ** -int(m.group(1))


def _pool_slack(K):
    return (K + 2) * 2.0 ** -22


def mfma_fp8_score(a, b, group=8, keep_bits=13):
    """Modelled matrix-core score of two non-negative e4m3-valued vectors:
    per group of `group` products, each product truncated to a multiple of
    2^(E - keep_bits) with E = floor(log2(largest product of the group)),
    the group summed exactly, then the groups added in float32."""
    p = np.asarray(a, np.float64) * np.asarray(b, np.float64)
    acc = np.float32(0.0)
    for g in range(0, len(p), group):
        grp = p[g:g + group]
        m = grp.max()
        if m > 0:
            step = 2.0 ** (math.floor(math.log2(m)) - keep_bits)
            grp = np.floor(grp / step) * step
        acc = np.float32(acc + np.float32(grp.sum()))
    return float(acc)


def _e4m3_values():
    vals, _ = formats.e4m3_nonneg_values()
    return vals[np.isfinite(vals)]


def test_model_reproduces_the_measured_cases():
    """The model gives the measured outcomes: a 2^13 product keeps its seven
    unit neighbours, a 2^14 product drops them (32x32x64: 56 of 63 kept)."""
    a = np.ones(64)
    b = np.ones(64)
    a[0], b[0] = 2.0 ** 7, 2.0 ** 6
    assert mfma_fp8_score(a, b) == 2.0 ** 13 + 63
    a[0], b[0] = 2.0 ** 7, 2.0 ** 7
    assert mfma_fp8_score(a, b) == 2.0 ** 14 + 56


def test_threshold_factor_covers_the_accumulation_loss():
    vals = _e4m3_values()
    factor = _header_factor()
    rng = np.random.default_rng(3)
    worst = 0.0
    K = 1024
    for trial in range(300):
        if trial < 100:       # arbitrary e4m3 codes
            a = rng.choice(vals, K)
            b = rng.choice(vals, K)
        elif trial < 200:     # a peaky softmax-like query against pool rows
            a = vals[np.minimum(len(vals) - 1, rng.geometric(0.08, K))][::-1].copy()
            rng.shuffle(a)
            b = rng.choice(vals[len(vals) // 3:], K)
        else:                 # adversarial: per group one large product and seven
            a = np.empty(K)   # just below the truncation step
            b = np.ones(K)
            big = vals[-1]
            small = big * 2.0 ** -13 * (1 - 2.0 ** -4)
            sv = vals[vals <= small].max()
            for g in range(0, K, 8):
                a[g] = big
                a[g + 1:g + 8] = sv
        real = float(np.dot(a, b))
        got = mfma_fp8_score(a, b)
        assert got <= real * (1 + 2.0 ** -20)
        worst = max(worst, 1 - got / real)
    # every modelled score clears the lowered threshold
    assert worst < 1 - factor, (worst, 1 - factor)
    # and the float32-only slack alone (the constant before) does not
    assert worst > _pool_slack(K), worst
