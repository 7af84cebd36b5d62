"""Ordinary double-double and quad-double arithmetic with operation counters.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper's operation-count table (Section 1, Table 1) lists how many
double operations an m-double addition, multiplication and division costs
for m = 2, 4, 8, 16, without naming the algorithms.  This module builds
"ordinary" double-double addition and multiplication from published
error-free transformations and counts every double operation, so that the
table's double-double addition entry (20) can be reproduced and the
multiplication entry compared:

* TwoSum (Knuth): s = a + b and its exact error, 6 operations;
* Fast2Sum (Dekker, |a| >= |b|): 3 operations;
* Veltkamp split into 26- and 27-bit halves: 4 operations;
* TwoProd without a fused multiply-add (Dekker): 17 operations;
* accurate double-double addition (Hida, Li, Bailey): TwoSum of the high
  parts, TwoSum of the low parts, two Fast2Sum renormalisations and two
  plain additions: 20 operations;
* double-double multiplication: TwoProd of the high parts, the two cross
  products added to its error, one Fast2Sum: 24 operations (the table says
  23; the paper does not name its variant, so this entry stays unpinned).

The counters are the ordinary method's cost model: an ordinary m-double
product of an M x K by a K x N matrix costs M N K (add_m + mul_m) double
operations.
"""
from __future__ import annotations

# Table 1 of the paper: double operations per m-double add, mul, div and the
# average of the three.
TABLE1 = {
    2: (20, 23, 70, 37.7),
    4: (89, 336, 893, 439.3),
    8: (269, 1742, 5126, 2379.0),
    16: (925, 11499, 33041, 15155.0),
}


class Counter:
    """Counts double operations (+, -, *) routed through it."""

    def __init__(self):
        self.n = 0

    def add(self, a: float, b: float) -> float:
        self.n += 1
        return a + b

    def sub(self, a: float, b: float) -> float:
        self.n += 1
        return a - b

    def mul(self, a: float, b: float) -> float:
        self.n += 1
        return a * b


def two_sum(c: Counter, a: float, b: float):
    s = c.add(a, b)
    bb = c.sub(s, a)
    e = c.add(c.sub(a, c.sub(s, bb)), c.sub(b, bb))
    return s, e


def fast_two_sum(c: Counter, a: float, b: float):
    s = c.add(a, b)
    e = c.sub(b, c.sub(s, a))
    return s, e


_SPLITTER = 134217729.0  # 2^27 + 1


def split(c: Counter, a: float):
    t = c.mul(_SPLITTER, a)
    hi = c.sub(t, c.sub(t, a))
    lo = c.sub(a, hi)
    return hi, lo


def two_prod(c: Counter, a: float, b: float):
    p = c.mul(a, b)
    ah, al = split(c, a)
    bh, bl = split(c, b)
    e = c.sub(c.mul(ah, bh), p)
    e = c.add(e, c.mul(ah, bl))
    e = c.add(e, c.mul(al, bh))
    e = c.add(e, c.mul(al, bl))
    return p, e


def dd_add(c: Counter, x, y):
    """Accurate double-double addition (x, y are (hi, lo) pairs)."""
    s1, s2 = two_sum(c, x[0], y[0])
    t1, t2 = two_sum(c, x[1], y[1])
    s2 = c.add(s2, t1)
    s1, s2 = fast_two_sum(c, s1, s2)
    s2 = c.add(s2, t2)
    return fast_two_sum(c, s1, s2)


def dd_mul(c: Counter, x, y):
    """Double-double multiplication without a fused multiply-add."""
    p1, p2 = two_prod(c, x[0], y[0])
    cross = c.add(c.mul(x[0], y[1]), c.mul(x[1], y[0]))
    p2 = c.add(p2, cross)
    return fast_two_sum(c, p1, p2)


# ---------------------------------------------------------------------------
# quad-double operations (m = 4): terms grouped by order (order k is about
# 2^(-53 k) of the leading word), error-free transformations up to the order
# a quad-double keeps, plain sums beyond, then one renormalisation.  The
# style of Hida, Li and Bailey's quad-double algorithms, written here with a
# branch-free renormalisation so that a GPU kernel can repeat it operation
# for operation.
# ---------------------------------------------------------------------------

def three_sum(c: Counter, a: float, b: float, d: float):
    """(s, e1, e2) with s + e1 + e2 = a + b + d exactly: three TwoSums."""
    u, v = two_sum(c, a, b)
    s, w = two_sum(c, u, d)
    e1, e2 = two_sum(c, v, w)
    return s, e1, e2


def renorm5(c: Counter, x0: float, x1: float, x2: float, x3: float, x4: float):
    """Five terms of decreasing order to four words: Fast2Sums bottom-up,
    then top-down (no data-dependent branches)."""
    s, t4 = fast_two_sum(c, x3, x4)
    s, t3 = fast_two_sum(c, x2, s)
    s, t2 = fast_two_sum(c, x1, s)
    t0, t1 = fast_two_sum(c, x0, s)
    y0, e = fast_two_sum(c, t0, t1)
    y1, e = fast_two_sum(c, e, t2)
    y2, e = fast_two_sum(c, e, t3)
    y3 = c.add(e, t4)
    return y0, y1, y2, y3


def qd_add(c: Counter, x, y):
    """Quad-double addition: TwoSum word by word, the errors folded in by
    order (TwoSums through order 3, a plain sum at order 4), renormalised."""
    s0, e0 = two_sum(c, x[0], y[0])
    s1, e1 = two_sum(c, x[1], y[1])
    s2, e2 = two_sum(c, x[2], y[2])
    s3, e3 = two_sum(c, x[3], y[3])
    s1, e0 = two_sum(c, s1, e0)                 # order 1; e0 now order 2
    s2, e0, e1 = three_sum(c, s2, e0, e1)       # order 2; e0 order 3, e1 order 4
    s3, u = two_sum(c, s3, e0)                  # order 3
    s3, v = two_sum(c, s3, e2)
    t = c.add(c.add(c.add(e1, e3), u), v)       # order 4
    return renorm5(c, s0, s1, s2, s3, t)


def qd_mul(c: Counter, x, y):
    """Quad-double multiplication: exact products (TwoProd) through order
    2, plain products at order 3, the orders summed with TwoSums through
    order 2 and plainly at order 3, renormalised."""
    p0, q0 = two_prod(c, x[0], y[0])            # order 0
    p1, q1 = two_prod(c, x[0], y[1])            # order 1
    p2, q2 = two_prod(c, x[1], y[0])
    p3, q3 = two_prod(c, x[0], y[2])            # order 2
    p4, q4 = two_prod(c, x[1], y[1])
    p5, q5 = two_prod(c, x[2], y[0])
    p6 = c.add(c.add(c.add(c.mul(x[0], y[3]), c.mul(x[1], y[2])), c.mul(x[2], y[1])),
               c.mul(x[3], y[0]))               # order 3
    r1, u1, v1 = three_sum(c, p1, p2, q0)       # order 1; u1 order 2, v1 order 3
    r2, w1, w2 = three_sum(c, p3, p4, p5)       # order 2; w1, w2 order 3
    r2, z1 = two_sum(c, r2, q1)
    r2, z2 = two_sum(c, r2, q2)
    r2, z3 = two_sum(c, r2, u1)
    r3 = p6
    for t in (q3, q4, q5, v1, w1, w2, z1, z2, z3):
        r3 = c.add(r3, t)                       # order 3
    return renorm5(c, p0, r1, r2, r3, 0.0)


def d_add(c: Counter, x, y):
    """Ordinary 1-double addition: one IEEE rounding."""
    return (c.add(x[0], y[0]),)


def d_mul(c: Counter, x, y):
    """Ordinary 1-double multiplication: one IEEE rounding."""
    return (c.mul(x[0], y[0]),)


ORDINARY = {1: (d_add, d_mul), 2: (dd_add, dd_mul), 4: (qd_add, qd_mul)}


def ordinary_dot(c: Counter, xs, ys, m: int):
    """sum_k x_k * y_k in ordinary m-double arithmetic (m = 1, 2, 4): the
    accumulator starts at zero and takes add(acc, mul(x_k, y_k)) for k in
    increasing order, each operation renormalised."""
    add, mul = ORDINARY[m]
    acc = (0.0,) * m
    for x, y in zip(xs, ys):
        acc = add(c, acc, mul(c, x, y))
    return acc


def ordinary_gemm(A, B, rows=None, cols=None):
    """C = A B in ordinary m-double arithmetic for the entries rows x cols:
    entry (i, j) is ``ordinary_dot`` over k of the words of A[:, i, k] and
    B[:, k, j].  A is (m, M, K), B is (m, K, N) float64 planes; returns
    planes (m, len(rows), len(cols))."""
    import numpy as np
    m, M, K = A.shape
    N = B.shape[2]
    rows = range(M) if rows is None else rows
    cols = range(N) if cols is None else cols
    c = Counter()
    out = np.zeros((m, len(rows), len(cols)))
    for a, i in enumerate(rows):
        xs = [tuple(float(v) for v in A[:, i, k]) for k in range(K)]
        for b, j in enumerate(cols):
            ys = [tuple(float(v) for v in B[:, k, j]) for k in range(K)]
            out[:, a, b] = ordinary_dot(c, xs, ys, m)
    return out


def op_count(fn, m: int = 2) -> int:
    """Double operations one call of an m-double ``fn`` (m = 2, 4) costs."""
    c = Counter()
    x = (1.0, 2.0 ** -60, 2.0 ** -115, -(2.0 ** -170))[:m]
    y = (3.0, -(2.0 ** -58), 2.0 ** -112, 2.0 ** -166)[:m]
    fn(c, x, y)
    return c.n


def ordinary_gemm_ops(m: int, M: int, N: int, K: int) -> int:
    """Double operations of an ordinary m-double matrix product (Table 1)."""
    add, mul, _, _ = TABLE1[m]
    return M * N * K * (add + mul)
