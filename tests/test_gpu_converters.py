"""The device's upward-rounded conversions, exhaustively: every finite
non-negative bfloat16 value and its float32 neighbours, random float32
inputs, and every e4m3 code a level's scale can reach with its neighbours.

An index of capacity 2 with one all-zero row has a single pool whose float32
sum is the other row itself (x + 0 rounded upward is x), so its stored
bfloat16 and float8 copies are bf16_up(x) and e4m3_up(x / 2^e), e the level's
scale exponent.  Expected codes come from the format tables of the oracle
(the least representable value >= x; for bfloat16, values below 2^-126 are
first raised to 2^-126)."""
import numpy as np
import pytest
import torch

from oracle import formats

pytestmark = pytest.mark.gpu

D = 4096


@pytest.fixture(scope="module")
def gt():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2311_02573_amd import gt as g

    g.lib()
    return g


def _pool_codes(gt, row):
    F = np.zeros((2, D), np.float32)
    F[0, :len(row)] = row
    idx = gt.GTIndex(torch.from_numpy(F).cuda(), capacity=2, pools=("f32", "bf16", "fp8"))
    try:
        st = idx.stats()
        master = idx.read_pools(0, pool="f32")[0, :len(row)]
        b = idx.read_pools(0, pool="bf16")[0, :len(row)]
        e = idx.read_pools(0, pool="fp8")[0, :len(row)]
        return master, b, e, st["fp8_exp"][0]
    finally:
        idx.close()


def _check(gt, vals):
    bvals, _ = formats.bf16_nonneg_values()
    evals, _ = formats.e4m3_nonneg_values()
    for k in range(0, len(vals), D):
        row = vals[k:k + D].astype(np.float32)
        master, b, e, ex = _pool_codes(gt, row)
        np.testing.assert_array_equal(master, row)           # x + 0 upward is x
        x = row.astype(np.float64)
        want_b = formats.least_geq(np.maximum(x, np.where(x > 0, 2.0 ** -126, 0.0)), bvals)
        got_b = (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        np.testing.assert_array_equal(got_b, bvals[want_b])
        want_e = formats.least_geq(x / 2.0 ** ex, evals)
        np.testing.assert_array_equal(evals[e.astype(np.int64)], evals[want_e])


def test_every_bfloat16_value_and_its_neighbours(gt):
    bvals, _ = formats.bf16_nonneg_values()
    v = bvals.astype(np.float32)
    up = np.nextafter(v, np.float32(np.inf))
    down = np.nextafter(v[1:], np.float32(0))
    # (above the largest finite bfloat16 the upward conversion is infinite)
    vals = np.concatenate([v, up[up <= v[-1]], down])
    _check(gt, vals)


def test_random_float32_inputs(gt):
    rng = np.random.default_rng(12)
    bits = rng.integers(0, 0x7F7F0000, size=65536, dtype=np.uint32)
    _check(gt, bits.view(np.float32))
    # and the range pool sums live in
    _check(gt, rng.exponential(scale=1e-2, size=16384).astype(np.float32))


def test_every_reachable_e4m3_code_and_its_neighbours(gt):
    """The level's scale puts twice its largest value at or below 448, so
    scaled values reach 224; each code's value times the scale, and the
    float32 values just above and below it."""
    evals, _ = formats.e4m3_nonneg_values()
    for ex in (-20, 0, 7):
        scale = 2.0 ** ex
        v = (evals[evals <= 224.0] * scale).astype(np.float32)
        # (v ascends to 224 * scale, the row's maximum, which fixes the scale)
        row = np.concatenate([v, np.nextafter(v[:-1], np.float32(np.inf)),
                              np.nextafter(v[1:], np.float32(0))])
        master, b, e, got_ex = _pool_codes(gt, row)
        assert got_ex == ex, (got_ex, ex)
        _check(gt, row)


def test_e4m3_codes_above_the_build_range_after_insert(gt):
    """Codes between 224 and 448 are reached when inserts grow a pool up to
    twice its build-time maximum without a new scale.  Row 0 holds half of
    each target (largest 224 * scale), the inserted row the exact rest (a
    difference of floats within a factor of two of each other), so the pool
    sum is the target itself."""
    evals, _ = formats.e4m3_nonneg_values()
    for ex in (-20, 0, 7):
        scale = 2.0 ** ex
        v = (evals[evals > 224.0] * scale).astype(np.float32)
        targets = np.concatenate([v, np.nextafter(v[:-1], np.float32(np.inf)),
                                  np.nextafter(v, np.float32(0))])
        halves = np.concatenate([v, v[:-1], v]) / np.float32(2)
        rest = targets - halves
        assert np.all(rest.astype(np.float64) == targets.astype(np.float64) - halves)
        k = len(targets)
        F = np.zeros((1, D), np.float32)
        F[0, :k] = halves
        idx = gt.GTIndex(torch.from_numpy(F).cuda(), capacity=2, pools=("f32", "bf16", "fp8"))
        try:
            assert idx.stats()["fp8_exp"][0] == ex
            R = np.zeros((1, D), np.float32)
            R[0, :k] = rest
            idx.insert(torch.from_numpy(R).cuda())
            assert idx.stats()["fp8_exp"][0] == ex
            master = idx.read_pools(0, pool="f32")[0, :k]
            e = idx.read_pools(0, pool="fp8")[0, :k]
        finally:
            idx.close()
        np.testing.assert_array_equal(master, targets)
        want = formats.least_geq(targets.astype(np.float64) / scale, evals)
        np.testing.assert_array_equal(e.astype(np.int64), want)
