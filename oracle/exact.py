"""Exact-arithmetic oracle pieces for tiny inputs -- test infrastructure only.

Everything here works on Python Fractions, so no rounding is involved:

* `exact_member` / `exact_range_search`: the membership decision cos(q,f) >= rho
  of the problem statement (Sec. 1; cosine of non-negative vectors, Sec. 2),
  decided without square roots: for rho >= 0 it is dot >= 0 and
  dot^2 >= rho^2 * qq * ff; for rho < 0 it is dot >= 0 or dot^2 <= rho^2 qq ff.
* `binary_splitting`: the paper's binary splitting (Sec. 2, Eq. 1; Alg. 1 is
  the same procedure run with a stack), as a recursion over index ranges whose
  pools are differences of cumulative sums, with the right half tested
  directly and the left half's score obtained by subtraction.  Similarity is
  the dot product q.f as in Sec. 2.
* `levelwise_walk`: the same implicit tree visited one level ("round") at a
  time (Sec. 4 analyses pruning per round), over a power-of-two capacity with
  zero padding, testing both children of every surviving pool directly.
* `levelwise_walk_max`: that walk with Our-Max pools (Sec. 2), each pool the
  element-wise maximum of its members.
* `levelwise_walk_signed`: the extension of Our-Max to descriptors with
  negative values (Sec. 2): a pool keeps the element-wise maximum and minimum
  of its members and is scored with the maximum where the query component is
  non-negative and the minimum where it is negative.

The binary-splitting and level-wise walks are the paper's method, kept here to
show that it returns exactly the brute-force set; the GPU path is compared with
the brute-force definition, not with these walks.
"""
from __future__ import annotations

from decimal import Decimal, getcontext
from fractions import Fraction


def to_frac_rows(a):
    """Exact Fractions of float values (float32/float64 are dyadic rationals)."""
    return [[Fraction(float(x)) for x in row] for row in a]


def dot(a, b):
    s = Fraction(0)
    for x, y in zip(a, b):
        s += x * y
    return s


def exact_member(q, f, rho) -> bool:
    """cos(q, f) >= rho in exact arithmetic; a zero vector is never a member
    (its cosine is undefined)."""
    qq, ff, dq = dot(q, q), dot(f, f), dot(q, f)
    if qq == 0 or ff == 0:
        return False
    r = Fraction(float(rho))
    rhs = r * r * qq * ff
    if r >= 0:
        return dq >= 0 and dq * dq >= rhs
    return dq >= 0 or dq * dq <= rhs


def exact_range_search(F, Q, rho):
    """List of sorted id lists, one per query."""
    Ff, Qf = to_frac_rows(F), to_frac_rows(Q)
    rhos = list(rho) if hasattr(rho, "__len__") else [rho] * len(Qf)
    return [[i for i, f in enumerate(Ff) if exact_member(q, f, r)] for q, r in zip(Qf, rhos)]


def cos_decimal(q, f, prec: int = 60) -> Decimal:
    """cos(q, f) to `prec` significant digits (NaN for a zero vector)."""
    getcontext().prec = prec
    qf, ff_ = [Fraction(float(x)) for x in q], [Fraction(float(x)) for x in f]
    qq, ff, dq = dot(qf, qf), dot(ff_, ff_), dot(qf, ff_)
    if qq == 0 or ff == 0:
        return Decimal("NaN")
    num = Decimal(dq.numerator) / Decimal(dq.denominator)
    den = (Decimal(qq.numerator) / Decimal(qq.denominator) *
           Decimal(ff.numerator) / Decimal(ff.denominator)).sqrt()
    return num / den


def prefix_sums(F):
    """Cumulative sums of Eq. 1, with a leading zero row so that the sum of rows
    a..b (0-based, inclusive) is C[b+1] - C[a]."""
    d = len(F[0]) if F else 0
    C = [[Fraction(0)] * d]
    for f in F:
        C.append([c + x for c, x in zip(C[-1], f)])
    return C


def binary_splitting(F, q, rho):
    """Binary splitting over cumulative sums (Sec. 2 and Eq. 1), in exact
    arithmetic with sim = q.f.  Returns the sorted 0-based neighbour ids and
    the number of dot products taken.

    Definition followed: the pool of all N vectors is tested first; a pool
    scoring below rho holds no neighbour and is dropped; a pool that reaches
    rho and has more than one member is split into its first floor(n/2)
    members and the rest, and both halves are treated the same way; a
    single-member pool is a neighbour iff its own score reaches rho.  A pool
    of rows [a, b) is C[b] - C[a] with the cumulative sums C of Eq. 1, so only
    the right half of a split costs a dot product; the left half's score is
    the parent's minus the right half's (pools are sums, so scores add).
    """
    N = len(F)
    if N == 0:
        return [], 0
    qf = [Fraction(float(x)) for x in q]
    C = prefix_sums([[Fraction(float(x)) for x in f] for f in F])
    r = Fraction(float(rho))

    def score(a, b):  # q . (f_a + ... + f_{b-1})
        return dot(qf, [hi - lo for hi, lo in zip(C[b], C[a])])

    def neighbours(a, b, s):
        """(ids of neighbours among rows [a, b), dot products spent below)."""
        if s < r:
            return set(), 0
        if b - a == 1:
            return {a}, 0
        m = a + (b - a) // 2
        s_right = score(m, b)
        left, n_left = neighbours(a, m, s - s_right)
        right, n_right = neighbours(m, b, s_right)
        return left | right, 1 + n_left + n_right

    ids, spent = neighbours(0, N, score(0, N))
    return sorted(ids), 1 + spent


def levelwise_walk(F, q, rho, capacity: int | None = None):
    """Level-by-level walk of an explicit pool-sum tree (Sec. 2 pools, visited
    per round as in Sec. 4) over a power-of-two capacity, zero-padded; both
    children of each surviving pool are tested directly, and a leaf is a
    member iff its own score reaches rho.  Returns (ids, tests per level)."""
    N = len(F)
    if N == 0:
        return [], []
    cap = capacity or 1 << max(0, (N - 1).bit_length())
    assert cap >= N and cap & (cap - 1) == 0
    d = len(F[0])
    qf = [Fraction(float(x)) for x in q]
    leaves = [[Fraction(float(x)) for x in f] for f in F] + [[Fraction(0)] * d] * (cap - N)
    levels = [leaves]
    while len(levels[0]) > 1:
        below = levels[0]
        levels.insert(0, [[a + b for a, b in zip(below[2 * j], below[2 * j + 1])]
                          for j in range(len(below) // 2)])
    r = Fraction(float(rho))
    frontier = [0] if dot(qf, levels[0][0]) >= r else []
    tests = [1]
    for lvl in range(1, len(levels)):
        nxt = []
        for p in frontier:
            for c in (2 * p, 2 * p + 1):
                if dot(qf, levels[lvl][c]) >= r:
                    nxt.append(c)
        tests.append(2 * len(frontier))
        frontier = nxt
    return sorted(i for i in frontier if i < N), tests


def levelwise_walk_max(F, q, rho, capacity: int | None = None):
    """The same level-by-level walk with Our-Max pools (Sec. 2): a pool is the
    element-wise maximum of its members.  For non-negative q and members,
    q.max >= q.f_i for every member i, so a pool scoring below rho holds no
    neighbour.  Both children of each surviving pool are tested directly; a
    leaf (a single vector, its own maximum) is a member iff q.f >= rho.
    Returns (ids, tests per level)."""
    N = len(F)
    if N == 0:
        return [], []
    cap = capacity or 1 << max(0, (N - 1).bit_length())
    assert cap >= N and cap & (cap - 1) == 0
    d = len(F[0])
    qf = [Fraction(float(x)) for x in q]
    leaves = [[Fraction(float(x)) for x in f] for f in F] + [[Fraction(0)] * d] * (cap - N)
    levels = [leaves]
    while len(levels[0]) > 1:
        below = levels[0]
        levels.insert(0, [[max(a, b) for a, b in zip(below[2 * j], below[2 * j + 1])]
                          for j in range(len(below) // 2)])
    r = Fraction(float(rho))
    frontier = [0] if dot(qf, levels[0][0]) >= r else []
    tests = [1]
    for lvl in range(1, len(levels)):
        nxt = []
        for p in frontier:
            for c in (2 * p, 2 * p + 1):
                if dot(qf, levels[lvl][c]) >= r:
                    nxt.append(c)
        tests.append(2 * len(frontier))
        frontier = nxt
    return sorted(i for i in frontier if i < N), tests



def signed_pool_score(q, mx, mn):
    """Score of a max/min pool (Sec. 2, negative descriptors): sum over k of
    q_k * max_k where q_k >= 0 and q_k * min_k where q_k < 0.  Each term is the
    largest value q_k * f_k takes over the members, so the score bounds every
    member's q.f from above."""
    s = Fraction(0)
    for x, hi, lo in zip(q, mx, mn):
        s += x * (hi if x >= 0 else lo)
    return s


def levelwise_walk_signed(F, q, rho, capacity: int | None = None):
    """The level-by-level walk over max/min pools of vectors of any sign (Sec.
    3, negative descriptors), over a power-of-two capacity.  A pool holds the
    element-wise maximum and minimum over its members; padding slots past N
    are not members, and a pool with no member is never tested positive.  Both
    children of each surviving pool are tested with `signed_pool_score`; a leaf
    (one vector: its own maximum and minimum) is a member iff q.f >= rho.
    Returns (ids, tests per level)."""
    N = len(F)
    if N == 0:
        return [], []
    cap = capacity or 1 << max(0, (N - 1).bit_length())
    assert cap >= N and cap & (cap - 1) == 0
    qf = [Fraction(float(x)) for x in q]
    rows = [[Fraction(float(x)) for x in f] for f in F]
    # each level: list of (max, min) per node, None for a node with no member
    levels = [[(r, r) for r in rows] + [None] * (cap - N)]
    while len(levels[0]) > 1:
        below = levels[0]
        up = []
        for j in range(len(below) // 2):
            a, b = below[2 * j], below[2 * j + 1]
            if a is None or b is None:
                up.append(a if b is None else b)
            else:
                up.append(([max(x, y) for x, y in zip(a[0], b[0])],
                           [min(x, y) for x, y in zip(a[1], b[1])]))
        levels.insert(0, up)
    r = Fraction(float(rho))

    def live(node):
        return node is not None and signed_pool_score(qf, node[0], node[1]) >= r

    frontier = [0] if live(levels[0][0]) else []
    tests = [1]
    for lvl in range(1, len(levels)):
        nxt = []
        for p in frontier:
            for c in (2 * p, 2 * p + 1):
                if live(levels[lvl][c]):
                    nxt.append(c)
        tests.append(2 * len(frontier))
        frontier = nxt
    return sorted(frontier), tests
