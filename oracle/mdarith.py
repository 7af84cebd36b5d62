"""Ordinary double-double arithmetic with operation counters.

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


def op_count(fn) -> int:
    """Double operations one call of a double-double ``fn`` costs."""
    c = Counter()
    fn(c, (1.0, 2.0 ** -60), (3.0, -(2.0 ** -58)))
    return c.n


def ordinary_gemm_ops(m: int, M: int, N: int, K: int) -> int:
    """Double operations of an ordinary m-double matrix product (Table 1)."""
    add, mul, _, _ = TABLE1[m]
    return M * N * K * (add + mul)
