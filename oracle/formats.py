"""Value sets of the reduced-precision pool formats -- test infrastructure only.

bfloat16: the upper 16 bits of an IEEE binary32.
float8 e4m3 (OCP "E4M3FN"): 1 sign, 4 exponent bits with bias 7, 3 mantissa
bits; exponent field 0 is subnormal (m * 2^-9); no infinities; code 0x7F is NaN,
so the largest finite value is 0x7E = 1.75 * 2^8 = 448.

`least_geq(x, table)` is the rounded-up conversion used for pool sums and
queries: the smallest representable value >= x (None past the largest).
"""
from __future__ import annotations

import numpy as np


def bf16_nonneg_values():
    """All finite non-negative bfloat16 values, ascending, with their codes."""
    codes = np.arange(0, 0x7F80, dtype=np.uint32)  # 0 .. largest finite (0x7F7F)
    vals = (codes << 16).view(np.float32).astype(np.float64)
    return vals, codes.astype(np.uint16)


def e4m3_value(code: int) -> float:
    s = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    m = code & 0x7
    if e == 0xF and m == 0x7:
        return float("nan")
    if e == 0:
        return s * m * 2.0 ** -9
    return s * (1.0 + m / 8.0) * 2.0 ** (e - 7)


def e4m3_nonneg_values():
    codes = np.arange(0, 0x7F, dtype=np.uint8)
    vals = np.array([e4m3_value(int(c)) for c in codes], dtype=np.float64)
    return vals, codes


def least_geq(x, table_vals):
    """Index into the ascending table of the least value >= x (len(table) if none)."""
    return np.searchsorted(table_vals, np.asarray(x, dtype=np.float64), side="left")
