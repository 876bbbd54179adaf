"""Expected number of pool tests per query under the TNE similarity model
(paper Sec. 5: Eq. 2, the CLT and truncated-Erlang pool-score laws, the Q_k
recursion and Eq. 3).  Host-side arithmetic only: it predicts how many pools
per query survive each level of the walk, which the benchmark sets beside the
walk's own counts.  The walk itself never uses it.

Model (Sec. 5).  Each similarity x = q.f_i of a query with a database vector
is an independent draw from the truncated normalised exponential on [0, 1]
(Eq. 2): p(x) = lambda e^{-lambda x} / (1 - e^{-lambda}).  A pool of L
vectors scores the sum of L such draws, and is pruned when that sum is below
rho; p_L(rho) denotes that probability.
  * L >= 6: the sum is taken as Gaussian (central limit theorem) with mean
    L m and variance L v, m and v the TNE mean and variance.
  * L < 6: for rho <= 1 every draw of a sum below rho lies in [0, rho], where
    the truncated density is the exponential one divided by 1 - e^{-lambda};
    so p_L(rho) is the Erlang(L, lambda) distribution function at rho divided
    by (1 - e^{-lambda})^L (the truncated Erlang law of the text), exactly.
Round 1 tests the root (N vectors); a pool surviving round k-1 is split in two
for round k, so the expected number of pools in round k is
  Q_2 = 2 (1 - p_N),   Q_k = 2 (1 - p_{N / 2^{k-2}}) Q_{k-1},
and with one test per split (the other half by subtraction, Alg. 1) the
expected tests per query are E(rho) = 1 + (1/2) sum_{k=2}^{ceil(log2 N + 1)} Q_k
(Eq. 3).  Pool sizes N / 2^j are rounded to integers.
"""
from __future__ import annotations

import math

__all__ = ["tne_mean", "tne_var", "prune_prob", "pools_per_round", "expected_tests",
           "fit_lambda", "fit_lambda_loghist", "level_survivors"]


def tne_mean(lam: float) -> float:
    """Mean of the TNE law, 1/lambda - 1/(e^lambda - 1) (the text prints the
    second term as 1/(1 - e^lambda), the same value)."""
    return 1.0 / lam - 1.0 / math.expm1(lam)


def tne_var(lam: float) -> float:
    """Variance of the TNE law, 1/lambda^2 - e^lambda / (e^lambda - 1)^2."""
    e = math.expm1(lam)
    return 1.0 / (lam * lam) - (e + 1.0) / (e * e)


def _erlang_cdf(x: float, k: int, lam: float) -> float:
    """P(sum of k exponential(lambda) draws <= x) = 1 - e^{-lam x} sum_{n<k} (lam x)^n / n!"""
    if x <= 0.0:
        return 0.0
    t = lam * x
    term, acc = 1.0, 1.0
    for n in range(1, k):
        term *= t / n
        acc += term
    return -math.expm1(-t) if k == 1 else 1.0 - math.exp(-t) * acc


def _phi(z: float) -> float:
    return 0.5 * math.erfc(-z / math.sqrt(2.0))


def prune_prob(L: int, rho: float, lam: float) -> float:
    """p_L(rho): probability that a pool of L vectors scores below rho."""
    if L <= 0:
        return 1.0
    if L < 6:
        if rho >= L:
            return 1.0
        if rho > 1.0:
            # outside the exact region; the Gaussian law is used instead
            pass
        else:
            return min(1.0, _erlang_cdf(rho, L, lam) / (-math.expm1(-lam)) ** L)
    mu = L * tne_mean(lam)
    sd = math.sqrt(L * tne_var(lam))
    return _phi((rho - mu) / sd)


def _rounds(N: int) -> int:
    return math.ceil(math.log2(N) + 1)


def pools_per_round(N: int, rho: float, lam: float):
    """[Q_1, Q_2, ..., Q_K] with Q_1 = 1 (the root is always tested) and K =
    ceil(log2 N + 1); Q_k is the expected number of pools tested in round k."""
    K = _rounds(N)
    Q = [1.0]
    for k in range(2, K + 1):
        L = max(1, round(N / 2 ** (k - 2)))      # size of the round k-1 pools
        Q.append(2.0 * (1.0 - prune_prob(L, rho, lam)) * Q[-1])
    return Q


def expected_tests(N: int, rho: float, lam: float) -> float:
    """E(rho) of Eq. 3: 1 + (1/2) sum_{k >= 2} Q_k."""
    Q = pools_per_round(N, rho, lam)
    return 1.0 + 0.5 * sum(Q[1:])


def level_survivors(N: int, rho: float, lam: float, depth: int):
    """Expected pools per query that pass their test at each level of a
    complete tree of the given depth over N vectors (level l pools hold
    N / 2^l vectors): element l is Q_{l+2} / 2 = (1 - p_{N/2^l}) Q_{l+1}, the
    pools of level l that survive, i.e. half the tests of level l + 1."""
    Q = pools_per_round(N, rho, lam)
    out = []
    for l in range(depth + 1):
        k = l + 2
        out.append(Q[k - 1] / 2.0 if k - 1 < len(Q) else 0.0)
    return out


def fit_lambda(samples) -> float:
    """Moment fit of lambda to similarity samples in [0, 1]: the lambda whose
    TNE mean equals the sample mean (bisection; the mean decreases from 1/2
    at lambda -> 0 to 0 as lambda grows)."""
    xs = [min(1.0, max(0.0, float(x))) for x in samples]
    m = sum(xs) / len(xs)
    if not 0.0 < m < 0.5:
        raise ValueError("sample mean must lie in (0, 1/2) for a decaying TNE fit")
    lo, hi = 1e-6, 1e4
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if tne_mean(mid) > m:
            lo = mid
        else:
            hi = mid
    return math.sqrt(lo * hi)


def fit_lambda_loghist(samples, bins: int = 50) -> float:
    """Least-squares fit of the log of the TNE density to the log of the
    samples' histogram on [0, 1] (a straight line of slope -lambda through
    the non-empty bins), the way an exponential is fitted to a similarity
    histogram on a log scale."""
    import numpy as np

    x = np.clip(np.asarray(samples, np.float64), 0.0, 1.0)
    h, e = np.histogram(x, bins=bins, range=(0.0, 1.0))
    c = 0.5 * (e[1:] + e[:-1])
    ok = h > 0
    if ok.sum() < 2:
        raise ValueError("need at least two non-empty bins")
    dens = h[ok] / (h.sum() * (e[1] - e[0]))
    A = np.vstack([np.ones(ok.sum()), c[ok]]).T
    slope = np.linalg.lstsq(A, np.log(dens), rcond=None)[0][1]
    return float(max(1e-6, -slope))

