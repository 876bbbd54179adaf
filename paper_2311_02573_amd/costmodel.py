"""Expected number of pool tests per query under the TNE similarity model
(paper Sec. 5: Eq. 2, the CLT and truncated-Erlang pool-score laws, the Q_k
recursion and Eq. 3), and the same recursion fed with pool-score laws
sampled from an index.  Host-side arithmetic only: it predicts how many pools
per query survive each level of the walk; the sampled model's predictions
choose the first dense level of a call (gt option "dense_start") and the
serving loop's first memory estimates (frontier entries per query tile,
results per query).  Results never depend on it.

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
           "fit_lambda", "fit_lambda_loghist", "level_survivors", "empirical_prune_probs",
           "survivors_from_probs", "dense_level_from_model", "entries_per_tile_from_model",
           "sample_index", "plan"]


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



# --------------------------------------------------------------------------
# The same recursion fed with the index's own pool scores.
#
# The TNE law need not describe a database (a spike of near-zero similarities
# beside a flat tail holds for softmax features of few classes).  Eq. 3 only
# needs, per round, the probability that a pool of that round scores below
# the threshold; here it is read off the index: for a sample of queries and a
# sample of each level's stored pool sums, the fraction of (query, pool) pairs
# scoring below tau = rho |q| m_min is the level's prune probability p_l.  A
# pool never scores above its parent (non-negative members), so a pool of
# level l survives its test iff its score reaches tau, and the conditional
# probability that a child of a surviving pool is pruned is
#   1 - (1 - p_l) / (1 - p_{l-1}),
# which, put into Q_{l+1} = 2 (1 - p_{l+1 | l}) Q_l, gives 2^l (1 - p_l)
# surviving pools at level l.

def empirical_prune_probs(level_rows: dict, queries, rho, m_min: float):
    """p_l per level from sampled pool sums.  level_rows: {level: [m, d]
    float64 pool sums (a sample of the level's pools)}; queries: [s, d];
    rho: scalar or [s].  Returns {level: p_l} (the fraction of sampled
    (query, pool) pairs scoring below rho |q| m_min)."""
    import numpy as np

    q = np.asarray(queries, np.float64)
    r = np.broadcast_to(np.asarray(rho, np.float64), (q.shape[0],))
    tau = r * np.sqrt(np.einsum("ij,ij->i", q, q)) * m_min
    out = {}
    for l, rows in level_rows.items():
        S = np.asarray(rows, np.float64)
        scores = S[:, :q.shape[1]] @ q.T            # [m, s]
        out[l] = float(np.mean(scores < tau[None, :]))
    return out


def survivors_from_probs(p: dict, depth: int):
    """Expected surviving pools per query at each level in p (complete tree of
    the given depth) through the Q_k recursion with conditional prune
    probabilities: {level: 2^l (1 - p_l)}; levels absent from p are skipped."""
    out = {}
    prev_l, prev_p = None, None
    for l in sorted(p):
        if prev_l is None or l != prev_l + 1:
            surv = (2.0 ** l) * (1.0 - p[l])        # a fresh start: unconditional
        else:
            cond = 1.0 - (1.0 - p[l]) / max(1e-300, 1.0 - prev_p) if prev_p < 1.0 else 1.0
            q_tested = 2.0 * out[prev_l]           # Q of this round: children of survivors
            surv = q_tested * (1.0 - cond)
        out[l] = surv
        prev_l, prev_p = l, p[l]
    return out


def dense_level_from_model(survivors: dict, depth: int, d_pad: int, tile_queries: int = 64,
                           populated: float = 1.0, threshold_per_column: float = 4.6e-4):
    """First level whose predicted frontier density is at most the dense /
    sparse crossover: a dense step over level L costs in proportion to its
    pools x tiles x d_pad, a sparse step to the entries of level L; the dense
    step is cheaper while the entries fill more than threshold_per_column x
    d_pad of the (pool, tile) pairs of populated pools.  The entries of a
    tile at level L are taken as min(pools, tile_queries x survivors per
    query) (no two queries of a tile sharing a pool: an upper bound).
    Returns the level, or None."""
    thr = threshold_per_column * d_pad
    for L in sorted(survivors):
        pools = populated * 2.0 ** L
        entries = min(pools, tile_queries * survivors[L])
        if entries / pools <= thr:
            return L
    return None


def entries_per_tile_from_model(survivors: dict, tile_queries: int = 64, populated: float = 1.0):
    """Largest predicted frontier entries of one full query tile over the
    levels in survivors: min(pools, tile_queries x survivors per query)."""
    return max(min(populated * 2.0 ** L, tile_queries * s) for L, s in survivors.items())


def sample_index(index, queries, rho, levels, count: int = 16384, seed: int = 0):
    """Reads a contiguous block of `count` populated pools of each level from
    a GTIndex (float32 master sums, rounded up) and returns (p_l per level,
    survivors per query per level).  queries: [s, d] float32 host array."""
    import numpy as np

    st = index.stats()
    D, n = st["depth"], st["n"]
    g = np.random.default_rng(seed)
    rows = {}
    for l in levels:
        span = 1 << (D - l)
        pop = max(1, (n + span - 1) // span)        # pools holding a row
        c = min(count, pop)
        first = int(g.integers(0, pop - c + 1))
        rows[l] = index.read_pools(l, first, c, pool="f32").astype(np.float64)
    p = empirical_prune_probs(rows, queries, rho, st["m_min"])
    return p, survivors_from_probs(p, D)


def plan(index, queries, rho, levels=None, count: int = 16384, tile_queries: int = 64,
         seed: int = 0) -> dict:
    """Model of a workload from a sample of its queries: prune probabilities
    and surviving pools per query per level (sampled pool scores through the
    Eq. 3 recursion), the dense level it calls for (rows of 512 columns or
    more, where the dense / sparse crossover was measured; else None), the
    frontier entries of a full query tile at its largest sparse level, and
    the results per query (the leaves' survivors)."""
    st = index.stats()
    D, n, cap, dp = st["depth"], st["n"], st["capacity"], st["d_pad"]
    if levels is None:
        levels = list(range(max(1, D - 12), D + 1))
    p, surv = sample_index(index, queries, rho, levels, count=count, seed=seed)
    populated = min(1.0, n / cap)
    dense = None
    if dp >= 512:
        dense = dense_level_from_model({l: s for l, s in surv.items() if l < D}, D, dp,
                                       tile_queries, populated)
    start = dense if dense is not None else max(0, D - 4)
    sparse = {l: s for l, s in surv.items() if start <= l < D}
    return {"prune_probs": p, "survivors": surv, "dense_level": dense,
            "entries_per_tile": entries_per_tile_from_model(sparse or surv, tile_queries, populated),
            "results_per_query": surv.get(D, 0.0)}
