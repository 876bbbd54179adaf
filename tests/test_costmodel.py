"""The TNE cost model of paper Sec. 5 (Eq. 2, CLT / truncated-Erlang pool-score
laws, the Q_k recursion and Eq. 3), pinned to the paper's printed values and
to the mathematics (no GPU)."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from paper_2311_02573_amd import costmodel as cm

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_reproduces_table3_theoretical_sum():
    """Eq. 3 with the paper's lambda values gives Table 3's 'Theoretical (Sum)'
    column within 5% (the table does not state how pool sizes N / 2^k are
    rounded, nor how the Erlang law is normalised; integer sizes and the
    exact law for rho <= 1 land within 4%)."""
    with open(os.path.join(GOLDEN, "table3_theoretical_sum.json")) as fh:
        cases = json.load(fh)["cases"]
    for c in cases:
        for rho, want in zip(c["rho"], c["E"]):
            got = cm.expected_tests(c["N"], rho, c["lambda"])
            assert 0.95 <= got / want <= 1.05, (c["dataset"], rho, got, want)


def test_tne_moments_match_integration():
    for lam in (0.5, 3.0, 10.0, 34.0, 57.0):
        z = -math.expm1(-lam)
        p = lambda x: lam * math.exp(-lam * x) / z
        one = integrate.quad(p, 0, 1)[0]
        m = integrate.quad(lambda x: x * p(x), 0, 1)[0]
        v = integrate.quad(lambda x: (x - m) ** 2 * p(x), 0, 1)[0]
        assert abs(one - 1) < 1e-10
        assert abs(cm.tne_mean(lam) - m) < 1e-9 * max(1, m)
        assert abs(cm.tne_var(lam) - v) < 1e-9 * max(1e-3, v) + 1e-12


def _tne_samples(rng, lam, shape):
    u = rng.random(shape)
    return -np.log1p(-u * (-math.expm1(-lam))) / lam


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5])
def test_erlang_branch_is_the_exact_law(L):
    """For L < 6 and rho <= 1 the prune probability is exact: compare with a
    Monte Carlo estimate of P(sum of L TNE draws < rho) (10^6 draws; four
    standard errors)."""
    rng = np.random.default_rng(L)
    for lam in (10.0, 30.0):
        s = _tne_samples(rng, lam, (1_000_000, L)).sum(1)
        for rho in (0.05, 0.2, 0.5, 0.9):
            p = cm.prune_prob(L, rho, lam)
            mc = np.mean(s < rho)
            se = math.sqrt(max(p * (1 - p), 1e-12) / len(s))
            assert abs(mc - p) <= 4 * se + 1e-6, (L, lam, rho, p, mc)


@pytest.mark.parametrize("L,tol", [(8, 0.05), (16, 0.03), (32, 0.03)])
def test_clt_branch_approximates_the_law(L, tol):
    """For L >= 6 the Gaussian law is an approximation (the sum of L skewed
    draws); it is within a few hundredths of the exact probability."""
    rng = np.random.default_rng(100 + L)
    for lam in (10.0, 34.0):
        s = _tne_samples(rng, lam, (400_000, L)).sum(1)
        for rho in (0.3, 0.7, 0.9):
            assert abs(cm.prune_prob(L, rho, lam) - np.mean(s < rho)) < tol, (L, lam, rho)


def test_prune_probability_trends_stated_in_the_paper():
    """Sec. 5 (and the supplement's figure for rho = 0.7): p_L(rho) increases
    with lambda and decreases as L grows (up to 1e-6, the size of the step
    between the exact law below L = 6 and the Gaussian one above, far in the
    tail)."""
    for rho in (0.7, 0.8, 0.9):
        for L in (2, 8, 16, 32):
            ps = [cm.prune_prob(L, rho, lam) for lam in (5, 10, 20, 40, 80)]
            assert all(a <= b + 1e-15 for a, b in zip(ps, ps[1:])), (rho, L, ps)
        for lam in (10, 34, 57):
            ps = [cm.prune_prob(L, rho, lam) for L in (1, 2, 4, 8, 16, 32, 64)]
            assert all(a >= b - 1e-6 for a, b in zip(ps, ps[1:])), (rho, lam, ps)


def test_expected_tests_decrease_with_lambda_and_rho():
    for N in (1 << 16, 1_000_000):
        es = [cm.expected_tests(N, 0.8, lam) for lam in (10, 20, 40, 80)]
        assert all(a > b for a, b in zip(es, es[1:]))
        er = [cm.expected_tests(N, rho, 30) for rho in (0.7, 0.8, 0.9)]
        assert er[0] > er[1] > er[2]


def test_recursion_bounds_and_survivor_levels():
    """Q_k <= 2^(k-1) (at most every pool of round k), E(rho) >= 1, and the
    level survivors are Q_{l+2} / 2."""
    N = 1 << 20
    Q = cm.pools_per_round(N, 0.9, 30)
    assert len(Q) == 21 and Q[0] == 1.0
    assert all(q <= 2 ** k + 1e-9 for k, q in enumerate(Q))
    surv = cm.level_survivors(N, 0.9, 30, 20)
    for l in range(19):
        assert surv[l] == pytest.approx(Q[l + 1] / 2.0)
    assert cm.expected_tests(N, 0.9, 30) >= 1.0


def test_fit_lambda_recovers_the_parameter():
    rng = np.random.default_rng(5)
    for lam in (10.0, 34.0, 57.0):
        x = _tne_samples(rng, lam, 200_000)
        assert abs(cm.fit_lambda(x) / lam - 1) < 0.03


def test_loghist_fit_recovers_the_parameter():
    rng = np.random.default_rng(6)
    for lam in (5.0, 10.0, 20.0):
        x = _tne_samples(rng, lam, 400_000)
        assert abs(cm.fit_lambda_loghist(x, bins=25) / lam - 1) < 0.1



def test_sampled_model_reproduces_the_exact_walk():
    """With every pool of every level as the 'sample' and one query, the
    prune probabilities give exactly the surviving pools per level that the
    level-wise walk in rational arithmetic finds (tests at level l + 1 are
    twice the survivors of level l) at the threshold rho |q| m_min."""
    from oracle import exact, pools

    rng = np.random.default_rng(11)
    for trial in range(6):
        n, d = 64, 5
        F = rng.exponential(size=(n, d)) ** 3
        F /= np.linalg.norm(F, axis=1, keepdims=True)
        F = F.astype(np.float32).astype(np.float64)
        q = F[rng.integers(n)] + 0.05 * rng.random(d)
        q = q.astype(np.float32).astype(np.float64)
        rho = [0.5, 0.8, 0.9][trial % 3]
        m_min = float(np.min(np.linalg.norm(F, axis=1)))
        tau = rho * float(np.sqrt(q @ q)) * m_min
        lv = pools.pool_tree(F)
        D = len(lv) - 1
        p = cm.empirical_prune_probs({l: lv[l] for l in range(D + 1)}, q[None, :], rho, m_min)
        surv = cm.survivors_from_probs(p, D)
        _, tests = exact.levelwise_walk(F, q, tau)
        for l in range(D):
            want = tests[l + 1] / 2 if l + 1 < len(tests) else 0
            assert surv[l] == pytest.approx(want, abs=1e-9), (trial, l, surv[l], want)
        # leaves: members scoring at least tau
        assert surv[D] == pytest.approx(np.sum(F @ q >= tau), abs=1e-9)


def test_sampled_model_survivors_follow_any_probabilities():
    """The recursion with conditional prune probabilities returns 2^l (1 - p_l)
    for consecutive levels, whatever the probabilities."""
    p = {10: 0.2, 11: 0.6, 12: 0.95, 14: 0.99}
    s = cm.survivors_from_probs(p, 14)
    assert s[10] == pytest.approx(2 ** 10 * 0.8)
    assert s[11] == pytest.approx(2 ** 11 * 0.4)
    assert s[12] == pytest.approx(2 ** 12 * 0.05)
    assert s[14] == pytest.approx(2 ** 14 * 0.01)


def test_dense_level_from_model_picks_the_crossover():
    """The first level whose predicted entry density (no sharing within a
    tile) is at most 4.6e-4 x d_pad."""
    surv = {14: 400.0, 15: 380.0, 16: 345.0, 17: 299.0}
    # d_pad 1024: threshold 0.471; densities 1.0 (capped), 0.74, 0.337, 0.146
    assert cm.dense_level_from_model(surv, 20, 1024) == 16
    # half the tree populated: twice the density
    assert cm.dense_level_from_model(surv, 20, 1024, populated=0.5) == 17
    assert cm.dense_level_from_model(surv, 20, 128) is None
    # the largest tile frontier: level 15, 64 x 380 entries (level 14 is capped at 2^14)
    assert cm.entries_per_tile_from_model(surv) == pytest.approx(64 * 380)
