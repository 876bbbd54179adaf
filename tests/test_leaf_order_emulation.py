"""The CPU emulation of the leaf test's float32 order (tests/leaf_order.py)
against exact rational arithmetic: the fused multiply-add rounds the exact
a b + c once to float32, and the vectorised order equals a scalar loop that
follows its definition element by element."""
from fractions import Fraction

import numpy as np

from leaf_order import fma32, inv_norm, leaf_dot


def round_f32(x: Fraction) -> np.float32:
    """float32 nearest to the rational x, ties to even."""
    f = np.float32(float(x))
    best = None
    for v in (np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))):
        key = (abs(Fraction(float(v)) - x), int(np.float32(v).view(np.uint32)) & 1)
        if best is None or key < best[0]:
            best = (key, v)
    return np.float32(best[1])


def test_fma32_rounds_once():
    g = np.random.default_rng(7)
    n = 3000
    a = g.standard_normal(n).astype(np.float32)
    b = g.standard_normal(n).astype(np.float32)
    c = (g.standard_normal(n) * g.choice([1e-9, 1e-3, 1.0, 1e3, 1e9], n)).astype(np.float32)
    # products landing exactly on float32 midpoints after a tiny addend
    a[:300] = np.float32(1.0) + np.float32(2.0 ** -23)
    b[:300] = np.float32(1.0) + np.float32(2.0 ** -23)
    c[:300] = np.float32(0.0)
    c[300:400] = np.float32(2.0 ** -60)
    a[300:400] = np.float32(1.0) + np.float32(2.0 ** -12)
    b[300:400] = np.float32(1.0) + np.float32(2.0 ** -12)
    got = fma32(a, b, c)
    for i in range(n):
        want = round_f32(Fraction(float(a[i])) * Fraction(float(b[i])) + Fraction(float(c[i])))
        assert got[i].view(np.uint32) == want.view(np.uint32), (i, a[i], b[i], c[i], got[i], want)


def scalar_dot(x, y):
    """The order written out element by element, every operation rounded
    exactly once to float32 (fused multiply-adds from rationals)."""
    dp = len(x)
    chunks = (dp + 1023) // 1024
    lanes = []
    for l in range(64):
        acc = None
        for c in range(chunks):
            sv = []
            for v in range(4):
                e0 = 1024 * c + 256 * v + 4 * l
                if e0 >= dp:
                    sv.append(np.float32(0.0))
                    continue
                p1 = np.float32(x[e0 + 1] * y[e0 + 1])
                p3 = np.float32(x[e0 + 3] * y[e0 + 3])
                t01 = round_f32(Fraction(float(x[e0])) * Fraction(float(y[e0])) + Fraction(float(p1)))
                t23 = round_f32(Fraction(float(x[e0 + 2])) * Fraction(float(y[e0 + 2])) + Fraction(float(p3)))
                sv.append(np.float32(t01 + t23))
            part = np.float32(np.float32(sv[0] + sv[1]) + np.float32(sv[2] + sv[3]))
            acc = part if acc is None else np.float32(acc + part)
        lanes.append(acc)
    vals = lanes
    for d in (32, 16, 8, 4, 2, 1):
        vals = [np.float32(vals[i] + vals[i + d]) for i in range(d)]
    return vals[0]


def test_vectorised_order_equals_scalar_definition():
    g = np.random.default_rng(11)
    for dp in (128, 384, 1152):
        x = np.abs(g.standard_normal((3, dp))).astype(np.float32)
        y = np.abs(g.standard_normal((3, dp))).astype(np.float32)
        got = leaf_dot(x, y)
        for i in range(3):
            assert got[i].view(np.uint32) == scalar_dot(x[i], y[i]).view(np.uint32), (dp, i)


def test_inverse_norm_is_rounded_from_float64():
    g = np.random.default_rng(3)
    rows = g.random((5, 200)).astype(np.float32)
    got = inv_norm(rows)
    for i in range(5):
        s = 0.0
        for v in rows[i].astype(np.float64):
            s += v * v
        assert got[i] == np.float32(1.0 / np.sqrt(s))
    assert inv_norm(np.zeros((1, 8), np.float32))[0] == 0.0
