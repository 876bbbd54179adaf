"""Seeded synthetic workloads: softmax-shaped, non-negative, unit-norm feature vectors.

This module only draws inputs.  It holds none of the search method's arithmetic
(no pooling, no similarity, no thresholds); both the HIP path and the CPU oracle
consume what it returns.

The paper's features are VGG16 softmax outputs of dimension 1000, non-negative
and unit-normalised (Sec. 4, experimental setup).  The image datasets and the
network weights are not available here, so every workload is synthetic:

    z ~ N(0, I_d),  f = softmax(z / T),  f <- f / ||f||_2   (computed in float64)

then rounded (round-to-nearest-even) to float32, and from float32 to the storage
dtype (float16 / bfloat16) where a workload asks for one.  A *planted neighbour*
of a query with logits z_q is unit(softmax((z_q + eps) / T)) with
eps ~ N(0, sigma^2 I); it overwrites a database row at a position drawn
uniformly without replacement.

Random streams: numpy PCG64, seed = 2311_02573 + 100 * workload + stream, with
streams 0 = database, 1 = queries, 2 = planted neighbours, 3 = arrivals,
4 = inserted vectors.  Large draws are split into fixed-size row chunks, each
with its own SeedSequence([seed, chunk]) child, so the result does not depend on
the thread count.
"""
from __future__ import annotations

import dataclasses
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

SEED_BASE = 2311_02573
STREAM_DB, STREAM_QUERY, STREAM_PLANT, STREAM_ARRIVAL, STREAM_INSERT = 0, 1, 2, 3, 4
CHUNK_ROWS = 16384


def stream_seed(workload: int, stream: int) -> int:
    return SEED_BASE + 100 * workload + stream


def _rng(seed: int, chunk: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, chunk])))


def _softmax_unit_rows(z: np.ndarray, temp: float, centred: bool = False) -> np.ndarray:
    """float64 logits -> unit-norm softmax rows, rounded to float32.  With
    `centred`, the uniform mean 1/d is subtracted from the softmax before the
    normalisation (descriptors with negative values)."""
    x = z / temp
    x -= x.max(axis=1, keepdims=True)
    np.exp(x, out=x)
    x /= x.sum(axis=1, keepdims=True)
    if centred:
        x -= 1.0 / x.shape[1]
    x /= np.sqrt(np.einsum("ij,ij->i", x, x))[:, None]
    return x.astype(np.float32)


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def softmax_rows(seed: int, n: int, d: int, temp: float, return_logits: bool = False,
                 centred: bool = False):
    """n unit-norm softmax(z/T) rows in float32, z ~ N(0, I_d), chunked streams
    (centred: softmax(z/T) - 1/d, normalised)."""
    out = np.empty((n, d), dtype=np.float32)
    logits = np.empty((n, d), dtype=np.float64) if return_logits else None
    nchunks = (n + CHUNK_ROWS - 1) // CHUNK_ROWS

    def work(c):
        lo, hi = c * CHUNK_ROWS, min(n, (c + 1) * CHUNK_ROWS)
        z = _rng(seed, c).standard_normal((hi - lo, d))
        if logits is not None:
            logits[lo:hi] = z
        out[lo:hi] = _softmax_unit_rows(z, temp, centred)

    if nchunks == 1:
        work(0)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, range(nchunks)))
    return (out, logits) if return_logits else out


def to_storage(x32: np.ndarray, dtype: str):
    """Round float32 rows to the storage dtype.  Returns a torch CPU tensor for
    16-bit types (numpy has no bfloat16) and a numpy array for float32."""
    if dtype == "f32":
        return x32
    import torch

    t = torch.from_numpy(np.ascontiguousarray(x32))
    return t.to(torch.float16 if dtype == "f16" else torch.bfloat16)


@dataclasses.dataclass
class Workload:
    name: str
    index: int
    n: int
    d: int
    temp: float
    dtype: str                       # storage dtype of the database rows
    feats: object                    # [n, d] float32 numpy, or torch f16/bf16 CPU tensor
    queries: np.ndarray              # [nq, d] float32
    rho: np.ndarray                  # [nq] float64 thresholds
    planted: list                    # per query: np.ndarray of planted row ids
    capacity: int = 0
    extra: dict = dataclasses.field(default_factory=dict)


def _plant(feats32, q_logits, counts, temp, sigma, seed, centred=False):
    """Overwrite rows of feats32 with planted neighbours; returns ids per query."""
    n, d = feats32.shape
    total = int(counts.sum())
    g = _rng(seed, 0)
    pos = g.choice(n, size=total, replace=False)
    eps = g.standard_normal((total, d)) * sigma
    owner = np.repeat(np.arange(len(counts)), counts)
    rows = _softmax_unit_rows(q_logits[owner] + eps, temp, centred)
    feats32[pos] = rows
    planted, off = [], 0
    for c in counts:
        planted.append(np.sort(pos[off:off + c]))
        off += c
    return planted


def workload0(nq: int = 32, rho: float = 0.9) -> Workload:
    """N=16384, d=128, T=0.25, float32; 32 queries, 0..8 planted neighbours each
    (uniform), logit noise sigma=0.05; rho=0.9."""
    n, d, temp = 16384, 128, 0.25
    feats = softmax_rows(stream_seed(0, STREAM_DB), n, d, temp)
    queries, qz = softmax_rows(stream_seed(0, STREAM_QUERY), nq, d, temp, return_logits=True)
    counts = _rng(stream_seed(0, STREAM_PLANT), 1).integers(0, 9, size=nq)
    planted = _plant(feats, qz, counts, temp, 0.05, stream_seed(0, STREAM_PLANT))
    return Workload("softmax N=16384 d=128 T=0.25 f32", 0, n, d, temp, "f32", feats, queries,
                    np.full(nq, rho), planted, capacity=n)


def workload1(nq: int = 1024, rho: float = 0.9, n: int = 1 << 20, d: int = 1000,
              n_planted_queries: int = 4096) -> Workload:
    """N=2^20, d=1000, T=0.2, float32; queries drawn the same way, each with a
    geometric (mean 5, support 0,1,..) number of planted neighbours, logit noise
    sigma=0.05.  Planting is done for 4096 queries so that the 1024-query batch
    and the 4096-query batch share one database; a batch takes the first nq."""
    temp = 0.2
    feats = softmax_rows(stream_seed(1, STREAM_DB), n, d, temp)
    nqp = max(nq, n_planted_queries)
    queries, qz = softmax_rows(stream_seed(1, STREAM_QUERY), nqp, d, temp, return_logits=True)
    counts = _rng(stream_seed(1, STREAM_PLANT), 1).geometric(1.0 / 6.0, size=nqp) - 1
    planted = _plant(feats, qz, counts, temp, 0.05, stream_seed(1, STREAM_PLANT))
    return Workload(f"softmax N={n} d={d} T=0.2 f32", 1, n, d, temp, "f32", feats,
                    queries[:nq].copy(), np.full(nq, rho), planted[:nq], capacity=n)


def workload3(n0: int = 1 << 22, d: int = 512, capacity: int = 1 << 23, nq_pool: int = 8192,
              rho: float = 0.9) -> Workload:
    """Serving workload: N0=2^22 rows, d=512, T=0.2, stored float16, room for
    inserts up to `capacity`; a pool of queries drawn the same way from which
    requests take consecutive slices.  Arrivals: poisson_arrivals(3, ...);
    inserted rows: insert_rows(3, ...)."""
    temp = 0.2
    feats = softmax_rows(stream_seed(3, STREAM_DB), n0, d, temp)
    queries = softmax_rows(stream_seed(3, STREAM_QUERY), nq_pool, d, temp)
    return Workload(f"softmax N0={n0} d={d} T=0.2 f16", 3, n0, d, temp, "f16",
                    to_storage(feats, "f16"), queries, np.full(nq_pool, rho),
                    [np.zeros(0, np.int64)] * nq_pool, capacity=capacity)


def workload4(n: int = 1 << 17, d: int = 256, nq: int = 200, clusters: int = 8,
              per_cluster: int = 2000, sigma: float = 0.02, cluster_query_frac: float = 0.1,
              rho_lo: float = 0.75, rho_hi: float = 0.95) -> Workload:
    """Stress shape at a reduced size: rows softmax(z/0.3) stored as bfloat16;
    `clusters` centres each with `per_cluster` near-duplicates (logit noise
    sigma) written over uniformly chosen rows; a fraction of the queries are a
    centre plus the same noise (thousands of neighbours each); per-query
    thresholds uniform in [rho_lo, rho_hi]."""
    temp = 0.3
    feats = softmax_rows(stream_seed(4, STREAM_DB), n, d, temp)
    g = _rng(stream_seed(4, STREAM_PLANT), 0)
    centres = g.standard_normal((clusters, d))
    counts = np.full(clusters, per_cluster)
    members = _plant(feats, centres, counts, temp, sigma, stream_seed(4, STREAM_PLANT) + 1)
    queries, _ = softmax_rows(stream_seed(4, STREAM_QUERY), nq, d, temp, return_logits=True)
    nc = int(round(cluster_query_frac * nq))
    owner = g.integers(0, clusters, size=nc)
    queries[:nc] = _softmax_unit_rows(centres[owner] + g.standard_normal((nc, d)) * sigma,
                                      temp).astype(np.float32)
    rho = g.uniform(rho_lo, rho_hi, size=nq)
    planted = [members[o] for o in owner] + [np.zeros(0, np.int64)] * (nq - nc)
    return Workload(f"softmax N={n} d={d} T=0.3 bf16 clusters {clusters}x{per_cluster}", 4, n,
                    d, temp, "bf16", to_storage(feats, "bf16"), queries, rho, planted,
                    capacity=n)


def workload_small(n: int, d: int, nq: int, temp: float = 0.25, rho: float = 0.9,
                   max_planted: int = 8, seed_offset: int = 0, dtype: str = "f32",
                   capacity: int | None = None) -> Workload:
    """Same recipe at arbitrary small shapes (tests: ragged sizes, tails)."""
    wl = 50 + seed_offset
    feats = softmax_rows(stream_seed(wl, STREAM_DB), n, d, temp)
    queries, qz = softmax_rows(stream_seed(wl, STREAM_QUERY), nq, d, temp, return_logits=True)
    counts = _rng(stream_seed(wl, STREAM_PLANT), 1).integers(0, max_planted + 1, size=nq)
    counts = np.minimum(counts, max(0, n // max(1, nq)))
    planted = _plant(feats, qz, counts, temp, 0.05, stream_seed(wl, STREAM_PLANT)) if n else [np.zeros(0, np.int64)] * nq
    return Workload(f"softmax N={n} d={d} T={temp} {dtype}", wl, n, d, temp, dtype,
                    to_storage(feats, dtype), queries, np.full(nq, rho), planted,
                    capacity=capacity or n)


def workload_signed(n: int, d: int, nq: int, temp: float = 0.2, rho: float = 0.9,
                    max_planted: int = 8, seed_offset: int = 0, dtype: str = "f32",
                    capacity: int | None = None, geometric_planted: bool = False) -> Workload:
    """Descriptors with negative values (the paper's extension of max pooling
    to them has no experiment): centred softmax rows unit(softmax(z/T) - 1/d),
    queries and planted neighbours drawn the same way (uniform 0..max_planted
    neighbours per query, or geometric with mean 5)."""
    wl = 70 + seed_offset
    feats = softmax_rows(stream_seed(wl, STREAM_DB), n, d, temp, centred=True)
    queries, qz = softmax_rows(stream_seed(wl, STREAM_QUERY), nq, d, temp, return_logits=True,
                               centred=True)
    g = _rng(stream_seed(wl, STREAM_PLANT), 1)
    counts = g.geometric(1.0 / 6.0, size=nq) - 1 if geometric_planted else \
        g.integers(0, max_planted + 1, size=nq)
    counts = np.minimum(counts, max(0, n // max(1, nq)))
    planted = _plant(feats, qz, counts, temp, 0.05, stream_seed(wl, STREAM_PLANT), True) \
        if n else [np.zeros(0, np.int64)] * nq
    return Workload(f"centred softmax N={n} d={d} T={temp} {dtype}", wl, n, d, temp, dtype,
                    to_storage(feats, dtype), queries, np.full(nq, rho), planted,
                    capacity=capacity or n)


def insert_rows(workload: int, n_new: int, d: int, temp: float, offset: int = 0,
                centred: bool = False) -> np.ndarray:
    """Vectors to insert, from the insert stream; `offset` selects later chunks."""
    seed = stream_seed(workload, STREAM_INSERT) + 7919 * offset
    return softmax_rows(seed, n_new, d, temp, centred=centred)


def poisson_arrivals(workload: int, rate_per_s: float, duration_s: float,
                     max_batch: int, seed_offset: int = 0):
    """(arrival time in s, batch size) pairs: exponential gaps, sizes U{1..max_batch}."""
    g = _rng(stream_seed(workload, STREAM_ARRIVAL) + seed_offset, 0)
    t, out = 0.0, []
    while True:
        t += g.exponential(1.0 / rate_per_s)
        if t >= duration_s:
            return out
        out.append((t, int(g.integers(1, max_batch + 1))))
