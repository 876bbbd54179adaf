"""Pins for the CPU oracle, independent of the oracle itself (no GPU).

Each test checks the oracle against something the paper or the mathematics
fixes: exact rational decisions, hand-computed closed forms, the paper's own
binary-splitting algorithm run in exact arithmetic (Sec. 2, Alg. 1), the toy
pooling example of Sec. 2, special cases, a float64 BLAS computation of the
same definition, and invariances.  `test_planted_mistakes_are_caught` rebuilds
the oracle with deliberate mistakes and checks that the pins catch each one.
"""
import json
import math
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle.brute as ob
from oracle import exact, pools
from paper_2311_02573_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_nonneg(rng, n, d, zero_frac=0.3):
    a = rng.random((n, d)).astype(np.float32)
    a[rng.random((n, d)) < zero_frac] = 0.0
    return a


def _tiny_cases(seed=0):
    """Small inputs with zero rows, zero queries, duplicates, scaled copies and
    one-hots, plus thresholds placed on constructed values."""
    rng = np.random.default_rng(seed)
    cases = []
    for n, d in [(1, 1), (2, 3), (5, 2), (17, 4), (33, 8), (64, 5)]:
        F = _rand_nonneg(rng, n, d)
        Q = _rand_nonneg(rng, 4, d)
        F[0] = 0.0                      # zero row: never a member
        if n > 2:
            F[1] = Q[0]                 # exact duplicate of query 0
            F[2] = 2.0 * Q[0]           # scaled duplicate: same cosine
        Q[3] = 0.0                      # zero query: empty result
        oh = np.zeros(d, np.float32)
        oh[d - 1] = 0.5
        F[-1] = oh
        for rho in (0.0, -0.5, 0.3, 0.7, 0.9, 1.0, 1.0 + 2 ** -52):
            cases.append((F, Q, rho))
    return cases


# ----------------------------------------------------------------- closed forms
def test_closed_forms_golden():
    with open(os.path.join(GOLDEN, "closed_forms.json")) as fh:
        g = json.load(fh)
    for c in g["cases"]:
        q = np.array([c["q"]], np.float32)
        f = np.array([c["f"]], np.float32)
        got = ob.pair_cos(f, q, [0], [0])[0]
        if "cos_num" in c:
            want = c["cos_num"] / c["cos_den"]
        else:
            want = math.sqrt(c["cos_sq_num"] / c["cos_sq_den"])
        assert abs(got - want) <= 4e-16, (c, got, want)
        # membership just below / above the exact value
        ids_lo = ob.range_search(f, q, want - 1e-12)[0][0]
        ids_hi = ob.range_search(f, q, want + 1e-12)[0][0]
        assert list(ids_lo) == [0] and list(ids_hi) == [], c


# ------------------------------------------------------- exact rational decision
def _check_against_exact(feats, queries, rho, lib_path=None):
    """Returns a list of failure strings (empty when the oracle agrees)."""
    got = ob.range_search(feats, queries, rho, lib_path=lib_path)
    want = exact.exact_range_search(feats, queries, rho)
    fails = []
    for j, ((ids, sims), w) in enumerate(zip(got, want)):
        if sorted(w) == list(ids):
            continue
        for i in set(w) ^ set(ids.tolist()):
            c = exact.cos_decimal(queries[j], feats[i])
            # only a tie within rounding of rho may be decided either way
            if c.is_nan() or abs(float(c) - rho) > 1e-14:
                fails.append(f"q{j} row{i} rho={rho} exact_cos={c}")
    return fails


@pytest.mark.parametrize("case", range(len(_tiny_cases())))
def test_brute_matches_exact_rationals(case):
    F, Q, rho = _tiny_cases()[case]
    assert _check_against_exact(F, Q, rho) == []


def test_brute_sims_match_high_precision():
    rng = np.random.default_rng(1)
    F = _rand_nonneg(rng, 40, 16, 0.2)
    Q = _rand_nonneg(rng, 3, 16, 0.2)
    res = ob.range_search(F, Q, -1.0)
    for j, (ids, sims) in enumerate(res):
        nz = [i for i in range(len(F)) if F[i].any()]
        assert list(ids) == nz
        for i, s in zip(ids, sims):
            c = float(exact.cos_decimal(Q[j], F[i]))
            assert abs(s - c) <= (16 + 4) * 2.0 ** -53 * abs(c) + 1e-300


# ------------------------------------------- the paper's algorithm, exactly
@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 8, 13, 16, 31])
def test_alg1_binary_splitting_equals_brute_force(n):
    """Sec. 2, binary splitting over the cumulative sums of Eq. 1 (Alg. 1 runs
    it with a stack), with the subtraction for the left half, returns exactly
    {i : q.f_i >= rho}; at most 2n - 1 dot products.  For a power-of-two n its
    tree is the level-wise walk's, which tests both children of every
    surviving pool: the splitting then takes one dot product for the root plus
    one per split, i.e. half the pools the level-wise walk tests below the root
    (Sec. 5: tests are half the pools)."""
    rng = np.random.default_rng(100 + n)
    for trial in range(6):
        d = 1 + trial % 4
        F = _rand_nonneg(rng, n, d, 0.25)
        q = _rand_nonneg(rng, 1, d, 0.1)[0]
        qf = [Fraction(float(x)) for x in q]
        for rho in (0.05, 0.2, 0.4, 0.8):
            want = [i for i in range(n)
                    if exact.dot(qf, [Fraction(float(x)) for x in F[i]]) >= Fraction(rho)]
            got, ndots = exact.binary_splitting(F, q, rho)
            assert got == want, (n, trial, rho)
            assert ndots <= 2 * n - 1
            lw, tests = exact.levelwise_walk(F, q, rho)
            assert lw == want, (n, trial, rho)
            if n & (n - 1) == 0:
                assert ndots == 1 + sum(tests[1:]) // 2, (n, trial, rho, ndots, tests)


def test_toy_pool_example():
    """Sec. 2 toy example: y = f1+f2+f3+f4; q.y < rho prunes every member, and
    the left half's score equals q.y - q.(right half)."""
    rng = np.random.default_rng(7)
    F = [[Fraction(float(x)) for x in row] for row in _rand_nonneg(rng, 4, 6, 0.0)]
    q = [Fraction(float(x)) for x in _rand_nonneg(rng, 1, 6, 0.0)[0]]
    y = [sum(c) for c in zip(*F)]
    qy = exact.dot(q, y)
    for i in range(4):
        assert exact.dot(q, F[i]) <= qy
    rho = qy + Fraction(1, 10**6)
    assert all(exact.dot(q, f) < rho for f in F)
    y1 = [a + b for a, b in zip(F[0], F[1])]
    y2 = [a + b for a, b in zip(F[2], F[3])]
    assert exact.dot(q, y1) == qy - exact.dot(q, y2)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13, 16])
def test_max_pool_walk_equals_brute_force_and_tests_no_more_than_sums(n):
    """Sec. 2, Our-Max: a pool is the element-wise maximum of its members; with
    non-negative vectors q.max >= q.f for every member, so the walk returns
    exactly {i : q.f_i >= rho}.  A max pool never scores above the sum pool of
    the same members, so at every level the max walk keeps a subset of the
    sum walk's pools and runs at most as many tests."""
    rng = np.random.default_rng(300 + n)
    for trial in range(5):
        d = 1 + trial % 4
        F = _rand_nonneg(rng, n, d, 0.25)
        q = _rand_nonneg(rng, 1, d, 0.1)[0]
        qf = [Fraction(float(x)) for x in q]
        for rho in (0.05, 0.2, 0.4, 0.8):
            want = [i for i in range(n)
                    if exact.dot(qf, [Fraction(float(x)) for x in F[i]]) >= Fraction(rho)]
            got, tmax = exact.levelwise_walk_max(F, q, rho)
            assert got == want, (n, trial, rho)
            _, tsum = exact.levelwise_walk(F, q, rho)
            assert len(tmax) == len(tsum)
            assert all(a <= b for a, b in zip(tmax, tsum)), (tmax, tsum)


def test_max_pool_worked_example():
    """A hand-worked case (unit vectors in R^2, sim = q.f, Sec. 2): f0 = (3/5,
    4/5), f1 = (4/5, 3/5), f2 = (1, 0), f3 = (0, 1), q = (0, 1), rho = 0.9.
    Member scores 0.8, 0.6, 0, 1: the only neighbour is f3.  Sum pools of the
    halves, (7/5, 7/5) and (1, 1), score 1.4 and 1 and both survive, so all
    four vectors are tested (tests per level 1, 2, 4).  Max pools, (4/5, 4/5)
    and (1, 1), score 0.8 and 1: the left half is pruned (tests 1, 2, 2)."""
    F = np.array([[0.6, 0.8], [0.8, 0.6], [1.0, 0.0], [0.0, 1.0]])
    q = np.array([0.0, 1.0])
    ids_s, t_s = exact.levelwise_walk(F, q, 0.9)
    ids_m, t_m = exact.levelwise_walk_max(F, q, 0.9)
    assert ids_s == ids_m == [3]
    assert t_s == [1, 2, 4] and t_m == [1, 2, 2]
    lv = pools.max_pool_tree(F)
    assert np.array_equal(lv[1], [[0.8, 0.8], [1.0, 1.0]])
    assert np.array_equal(lv[0], [[1.0, 1.0]])


def test_max_pool_tree_invariants_on_softmax_data():
    """Every Our-Max pool equals the element-wise maximum of its members taken
    directly, lies between each member and the sum pool, and scores at least
    the largest member score."""
    w = synth.workload_small(1000, 24, 4, seed_offset=4)
    F = np.asarray(w.feats, np.float64)
    mx = pools.max_pool_tree(F)
    sm = pools.pool_tree(F)
    D = len(mx) - 1
    for level in range(D + 1):
        span = 1 << (D - level)
        for j in range(0, 1 << level, max(1, (1 << level) // 7)):
            a, b = j * span, min(len(F), (j + 1) * span)
            direct = F[a:b].max(axis=0) if a < b else np.zeros(F.shape[1])
            assert np.array_equal(mx[level][j], direct)
            assert np.all(mx[level][j] <= sm[level][j] * (1 + 1e-12))
    for q in w.queries:
        leaf = mx[D] @ q
        for level in range(D):
            span = 1 << (D - level)
            assert np.all(mx[level] @ q >= leaf.reshape(-1, span).max(axis=1) * (1 - 1e-12))


def _rand_signed(rng, n, d, zero_frac=0.2):
    a = (rng.random((n, d)) * 2.0 - 1.0).astype(np.float32)
    a[rng.random((n, d)) < zero_frac] = 0.0
    return a


def _signed_brute(F, q, rho):
    qf = [Fraction(float(x)) for x in q]
    return [i for i in range(len(F))
            if exact.dot(qf, [Fraction(float(x)) for x in F[i]]) >= Fraction(float(rho))]


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13, 16])
def test_signed_walk_equals_brute_force(n):
    """Sec. 2, negative descriptors: with max/min pools scored by the maximum
    where q_k >= 0 and the minimum where q_k < 0, every member's q.f is at most
    its pool's score, so the walk returns exactly {i : q.f_i >= rho} for
    vectors and thresholds of any sign."""
    rng = np.random.default_rng(500 + n)
    for trial in range(5):
        d = 1 + trial % 4
        F = _rand_signed(rng, n, d)
        q = _rand_signed(rng, 1, d, 0.1)[0]
        for rho in (-0.3, 0.0, 0.1, 0.4, 0.8):
            got, tests = exact.levelwise_walk_signed(F, q, rho)
            assert got == _signed_brute(F, q, rho), (n, trial, rho)
            assert tests[0] == 1 and all(t % 2 == 0 for t in tests[1:])


@pytest.mark.parametrize("n", [2, 5, 8, 13])
def test_signed_walk_reduces_to_max_walk_on_nonnegative_data(n):
    """For non-negative vectors and queries the minimum is never used, so the
    signed walk is the Our-Max walk: same ids and the same tests per level
    (rho > 0, where a zero-padded max pool and a pool without members are both
    pruned)."""
    rng = np.random.default_rng(600 + n)
    for trial in range(4):
        d = 1 + trial % 3
        F = _rand_nonneg(rng, n, d, 0.25)
        q = _rand_nonneg(rng, 1, d, 0.1)[0]
        for rho in (0.05, 0.3, 0.7):
            assert exact.levelwise_walk_signed(F, q, rho) == exact.levelwise_walk_max(F, q, rho)


def test_signed_walk_worked_example():
    """A hand-worked case in R^2 (sim = q.f): f0 = (0, 1), f1 = (0, -1),
    f2 = (3/5, -4/5), f3 = (-4/5, 3/5), q = (3/5, -4/5).  Member scores -0.8,
    0.8, 1, -0.96.  Halves: {f0, f1} has max (0, 1) and min (0, -1), score
    (3/5) 0 + (-4/5)(-1) = 0.8; {f2, f3} has max (3/5, 3/5) and min (-4/5,
    -4/5), score 0.36 + 0.64 = 1.  At rho = 0.75 both halves survive and the
    neighbours are f1 and f2 (tests 1, 2, 4); at rho = 0.9 the first half is
    pruned (tests 1, 2, 2).  Scoring pools by their maxima alone would lose
    both neighbours: the root's maximum (3/5, 1) scores 0.36 - 0.8 < 0."""
    F = np.array([[0.0, 1.0], [0.0, -1.0], [0.6, -0.8], [-0.8, 0.6]])
    q = np.array([0.6, -0.8])
    assert exact.levelwise_walk_signed(F, q, 0.75) == ([1, 2], [1, 2, 4])
    assert exact.levelwise_walk_signed(F, q, 0.9) == ([2], [1, 2, 2])
    assert exact.levelwise_walk_max(F, q, 0.75) == ([], [1, 0, 0])
    mx, mn = pools.max_min_pool_tree(F)
    assert np.array_equal(mx[1], [[0.0, 1.0], [0.6, 0.6]])
    assert np.array_equal(mn[1], [[0.0, -1.0], [-0.8, -0.8]])
    sc = pools.signed_pool_scores(mx, mn, q)
    assert np.allclose(sc[1], [0.8, 1.0]) and np.allclose(sc[0], [0.36 + 0.8])


def test_signed_walk_without_the_minimum_is_caught(monkeypatch):
    """Planted mistake: scoring a pool by its maximum alone (dropping the
    minimum where q_k < 0) makes the brute-force pin fail."""
    def max_only(q, mx, mn):
        return exact.dot(q, mx)

    monkeypatch.setattr(exact, "signed_pool_score", max_only)
    with pytest.raises(AssertionError):
        for n in (5, 8, 13, 16):
            test_signed_walk_equals_brute_force(n)


def test_max_min_tree_invariants_on_signed_data():
    """Every max/min pool equals the element-wise maximum / minimum of its
    members taken directly; its score bounds the largest member score; on
    non-negative data the maxima of full nodes are the Our-Max pools."""
    rng = np.random.default_rng(41)
    F = _rand_signed(rng, 700, 12).astype(np.float64)
    mx, mn = pools.max_min_pool_tree(F)
    D = len(mx) - 1
    for level in range(D + 1):
        span = 1 << (D - level)
        for j in range(0, 1 << level, max(1, (1 << level) // 7)):
            a, b = j * span, min(len(F), (j + 1) * span)
            if a < b:
                assert np.array_equal(mx[level][j], F[a:b].max(axis=0))
                assert np.array_equal(mn[level][j], F[a:b].min(axis=0))
            else:
                assert np.all(np.isneginf(mx[level][j])) and np.all(np.isposinf(mn[level][j]))
    for q in _rand_signed(rng, 3, 12, 0.0).astype(np.float64):
        sc = pools.signed_pool_scores(mx, mn, q)
        leaf = np.full(1 << D, -np.inf)
        leaf[:len(F)] = F @ q
        for level in range(D):
            span = 1 << (D - level)
            assert np.all(sc[level] >= leaf.reshape(-1, span).max(axis=1) - 1e-12)
    P = np.abs(F[:512])
    mxp, _ = pools.max_min_pool_tree(P)
    ref = pools.max_pool_tree(P)
    for level in range(len(ref)):
        assert np.array_equal(mxp[level], ref[level])


def test_prefix_sum_pool_identity():
    """Sec. 2, Eq. 1: with cumulative sums C, the right half-pool of N rows is
    C_N - C_{floor(N/2)}; the explicit tree's node (level 1, index 1) equals it."""
    rng = np.random.default_rng(8)
    for N in (2, 4, 8, 16):
        F = _rand_nonneg(rng, N, 3, 0.0)
        C = exact.prefix_sums([[Fraction(float(x)) for x in r] for r in F])
        y12 = [a - b for a, b in zip(C[N], C[N // 2])]
        direct = [sum(Fraction(float(F[i, k])) for i in range(N // 2, N)) for k in range(3)]
        assert y12 == direct
        lv = pools.pool_tree(F)
        lo, hi = pools.exact_bounds(lv, 1)
        for k in range(3):
            assert lo[1, k] <= float(direct[k]) <= hi[1, k]


# ------------------------------------------------------------ pool invariants
def test_pool_tree_invariants_on_softmax_data():
    """Pool sums bracket the directly summed members; every pool's score is at
    least the largest member score (all terms non-negative, Sec. 2)."""
    w = synth.workload_small(1000, 24, 4, seed_offset=3)
    F = np.asarray(w.feats, np.float64)
    lv = pools.pool_tree(F)
    D = len(lv) - 1
    for level in range(D + 1):
        lo, hi = pools.exact_bounds(lv, level)
        span = 1 << (D - level)
        for j in range(0, 1 << level, max(1, (1 << level) // 7)):
            a, b = j * span, min(len(F), (j + 1) * span)
            direct = np.array([math.fsum(F[a:b, k]) for k in range(F.shape[1])]) if a < b else 0.0
            assert np.all(lo[j] <= direct) and np.all(direct <= hi[j])
    for q in w.queries:
        sc = pools.pool_scores(lv, q)
        leaf = sc[D]
        for level in range(D):
            span = 1 << (D - level)
            mx = leaf.reshape(-1, span).max(axis=1)
            assert np.all(sc[level] >= mx * (1 - 1e-12))


# -------------------------------------------------------------- special cases
def test_nonpositive_rho_returns_every_nonzero_row():
    rng = np.random.default_rng(9)
    F = _rand_nonneg(rng, 50, 7, 0.5)
    F[[3, 10]] = 0.0
    Q = _rand_nonneg(rng, 2, 7, 0.0)
    for rho in (0.0, -1e-300, -3.0):
        for ids, _ in ob.range_search(F, Q, rho):
            assert list(ids) == [i for i in range(50) if F[i].any()]


def test_zero_query_matches_nothing():
    F = _rand_nonneg(np.random.default_rng(10), 20, 5, 0.0)
    Q = np.zeros((1, 5), np.float32)
    for rho in (-1.0, 0.0, 0.5):
        assert len(ob.range_search(F, Q, rho)[0][0]) == 0


def test_self_similarity_is_one():
    w = synth.workload_small(64, 33, 8, seed_offset=4)
    F = np.asarray(w.feats)
    s = ob.pair_cos(F, F[:8], np.arange(8), np.arange(8))
    assert np.all(np.abs(s - 1.0) <= 33 * 2.0 ** -52)


# ------------------------------------------------ independent float64 BLAS path
def _blas_cos(F, Q):
    F = np.asarray(F, np.float64)
    Q = np.asarray(Q, np.float64)
    return (Q @ F.T) / np.linalg.norm(Q, axis=1)[:, None] / np.linalg.norm(F, axis=1)[None, :]


def _check_against_blas(F, Q, rho, lib_path=None):
    C = _blas_cos(F, Q)
    got = ob.range_search(F, Q, rho, lib_path=lib_path)
    fails = []
    for j, (ids, sims) in enumerate(got):
        want = np.nonzero(C[j] >= rho)[0]
        diff = set(want.tolist()) ^ set(ids.tolist())
        for i in diff:
            if abs(C[j, i] - rho) > 1e-12:
                fails.append(f"q{j} row{i} blas={C[j, i]}")
        if len(ids) and np.max(np.abs(sims - C[j, ids])) > 1e-13:
            fails.append(f"q{j} sims differ")
    return fails


@pytest.mark.parametrize("shape", [(16384, 128, 32), (999, 77, 9), (4097, 1000, 4)])
def test_brute_matches_blas(shape):
    n, d, nq = shape
    if (n, d) == (16384, 128):
        w = synth.workload0(nq)
    else:
        w = synth.workload_small(n, d, nq, temp=0.2, seed_offset=n)
    for rho in (0.8, 0.9, 0.95):
        assert _check_against_blas(np.asarray(w.feats), w.queries, rho) == []


def test_planted_neighbours_are_found():
    w = synth.workload0()
    C = _blas_cos(w.feats, w.queries)
    res = ob.range_search(w.feats, w.queries, w.rho)
    n_found = 0
    for j, (ids, _) in enumerate(res):
        for p in w.planted[j]:
            if C[j, p] >= w.rho[j] + 1e-9:
                assert p in set(ids.tolist())
                n_found += 1
    assert n_found >= 50


def test_row_permutation_permutes_results():
    w = synth.workload_small(3000, 40, 6, temp=0.2, seed_offset=11)
    F = np.asarray(w.feats)
    perm = np.random.default_rng(12).permutation(len(F))
    a = ob.range_search(F, w.queries, 0.8)
    b = ob.range_search(F[perm], w.queries, 0.8)
    for (ia, sa), (ib, sb) in zip(a, b):
        assert sorted(perm[ib].tolist()) == ia.tolist()
        np.testing.assert_array_equal(np.sort(sa), np.sort(sb))


def test_half_precision_storage_decodes_exactly():
    import torch

    w = synth.workload_small(500, 64, 5, temp=0.2, seed_offset=13)
    F32 = np.asarray(w.feats)
    for dt in ("f16", "bf16"):
        t = synth.to_storage(F32, dt)
        up = t.to(torch.float32).numpy()
        for (ia, sa), (ib, sb) in zip(ob.range_search(t, w.queries, 0.8),
                                      ob.range_search(up, w.queries, 0.8)):
            np.testing.assert_array_equal(ia, ib)
            np.testing.assert_array_equal(sa, sb)


# ------------------------------------------------------ planted mistakes caught
MUTANTS = {
    "drop_last_term": ("for (int32_t k = 0; k < d; ++k) {\n        double qk",
                       "for (int32_t k = 0; k < d - 1; ++k) {\n        double qk"),
    "strict_inequality": ("if (c >= J->rho[j])", "if (c > J->rho[j])"),
    "missing_sqrt": ("dot[r] / (nq_ * sqrt(ff[r]))", "dot[r] / (nq_ * ff[r])"),
    "shifted_operand": ("dot[r] = dot[r] + qk * rows[r * d + k];",
                        "dot[r] = dot[r] + qk * rows[r * d + (k + 1) % d];"),
    "off_by_one_id": ("vec_push(&J->out[j], i0 + r, c);", "vec_push(&J->out[j], i0 + r + 1, c);"),
}


def _pin_failures(lib_path):
    try:
        return _pin_failures_inner(lib_path)
    except Exception as e:  # a crash inside a pin is a caught mistake too
        return [repr(e)]


def _pin_failures_inner(lib_path):
    fails = []
    for F, Q, rho in _tiny_cases(5)[::3]:
        fails += _check_against_exact(F, Q, rho, lib_path)
    with open(os.path.join(GOLDEN, "closed_forms.json")) as fh:
        for c in json.load(fh)["cases"]:
            q = np.array([c["q"]], np.float32)
            f = np.array([c["f"]], np.float32)
            # rational cosines with integer norms are computed with one rounding,
            # so rho equal to the cosine is an exact tie that must be included
            rho = c["cos_num"] / c["cos_den"] if "cos_num" in c else \
                math.sqrt(c["cos_sq_num"] / c["cos_sq_den"]) - 1e-12
            if list(ob.range_search(f, q, rho, lib_path=lib_path)[0][0]) != [0]:
                fails.append(f"closed form {c['q']} {c['f']}")
    w = synth.workload_small(999, 77, 9, temp=0.2, seed_offset=999)
    fails += _check_against_blas(np.asarray(w.feats), w.queries, 0.8, lib_path)
    return fails


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_are_caught(name, tmp_path):
    src = open(os.path.join(os.path.dirname(ob.__file__), "range_oracle.c")).read()
    old, new = MUTANTS[name]
    assert old in src, name
    path = tmp_path / "range_oracle_mutant.c"
    path.write_text(src.replace(old, new))
    so = str(tmp_path / f"liboracle_{name}.so")
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-shared", "-fPIC", "-pthread",
                           "-o", so, str(path), "-lm"])
    assert _pin_failures(so), f"mutant {name} passed every pin"


def test_unmutated_oracle_passes_mutant_pins():
    assert _pin_failures(ob.build(force=False)) == []
