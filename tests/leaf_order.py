"""CPU emulation of the exact leaf test's float32 summation order (test
infrastructure: the GPU tests compare the kernels' similarities with it bit
for bit; tests/test_leaf_order_emulation.py checks it against exact
rational arithmetic).  Shares nothing with the HIP sources.
"""
import numpy as np


def fma32(a, b, c):
    """Correctly rounded float32 fused multiply-add, elementwise: the product
    is exact in float64, the sum is split exactly (two-sum) and rounded once
    to float32 (a float64 value on a float32 midpoint is resolved by the
    sign of the remainder)."""
    a64, b64, c64 = a.astype(np.float64), b.astype(np.float64), c.astype(np.float64)
    p = a64 * b64
    hi = p + c64
    bb = hi - p
    lo = (p - (hi - bb)) + (c64 - bb)
    r = hi.astype(np.float32)
    r64 = r.astype(np.float64)
    up = np.nextafter(r, np.float32(np.inf)).astype(np.float64)
    dn = np.nextafter(r, np.float32(-np.inf)).astype(np.float64)
    mid_up = (hi > r64) & (hi == (r64 + up) / 2)
    mid_dn = (hi < r64) & (hi == (r64 + dn) / 2)
    out = r.copy()
    # hi sits on a midpoint that float32 rounding resolved by evenness; the
    # exact value is hi + lo
    sel = mid_up & (lo > 0)
    out[sel] = up[sel].astype(np.float32)
    sel = mid_up & (lo < 0)
    out[sel] = r[sel]
    sel = mid_dn & (lo < 0)
    out[sel] = dn[sel].astype(np.float32)
    sel = mid_dn & (lo > 0)
    out[sel] = r[sel]
    return out


def leaf_dot(x, y):
    """float32 dot products of rows x[i] and y[i] (each of length d_pad, a
    multiple of 128) in the kernel's order."""
    n, dp = x.shape
    chunks = (dp + 1023) // 1024
    acc = None
    for c in range(chunks):
        sv = []
        for v in range(4):
            lane_vals = np.zeros((n, 64), np.float32)
            e0 = 1024 * c + 256 * v + 4 * np.arange(64)
            ok = e0 < dp
            idx = np.minimum(e0, dp - 4)
            xs = [x[:, idx + j] for j in range(4)]
            ys = [y[:, idx + j] for j in range(4)]
            t01 = fma32(xs[0], ys[0], (xs[1] * ys[1]).astype(np.float32))
            t23 = fma32(xs[2], ys[2], (xs[3] * ys[3]).astype(np.float32))
            s = (t01 + t23).astype(np.float32)
            lane_vals[:, ok] = s[:, ok]
            sv.append(lane_vals)
        part = ((sv[0] + sv[1]).astype(np.float32) + (sv[2] + sv[3]).astype(np.float32)).astype(np.float32)
        acc = part if acc is None else (acc + part).astype(np.float32)
    arr = acc
    for d in (32, 16, 8, 4, 2, 1):
        arr = (arr[:, :d] + arr[:, d:2 * d]).astype(np.float32)
    return arr[:, 0]


def inv_norm(rows):
    """float32(1 / sqrt(sum of squares)), the sum sequential in float64."""
    sq = np.cumsum(rows.astype(np.float64) ** 2, axis=1)[:, -1]
    out = np.zeros(len(rows), np.float32)
    nz = sq > 0
    out[nz] = (1.0 / np.sqrt(sq[nz])).astype(np.float32)
    return out
