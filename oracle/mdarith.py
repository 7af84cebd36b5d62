"""Ordinary double-, quad- and octo-double arithmetic with operation counters.

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

Octo-double addition and multiplication follow floating-point expansion
arithmetic (CAMPARY's VecSum, VecSumErrBranch, merge-based addition and the
truncated product of expansions), see the section that defines them; their
counts (135 and 1769) stand beside the table's 269 and 1742, unpinned.

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


# ---------------------------------------------------------------------------
# octo-double operations (m = 8, and hexa-double, m = 16, the same algorithms
# on 16 words): floating-point expansion arithmetic in the
# manner of CAMPARY (Joldes, Muller, Popescu and Tucker; the paper's
# reference for multiple double arithmetic of any length), built from the
# same error-free transformations:
#
# * VecSum: from the last term up, TwoSum of each term with the running sum;
#   the exact sum is kept, the first output is the rounded sum;
# * VecSumErrBranch: Fast2Sum down the terms, starting a new output word
#   whenever the error is nonzero, until m words are out;
# * renormalisation to m words: VecSumErrBranch of VecSum;
# * addition: the 2m words of both operands merged by decreasing magnitude
#   (here with Batcher's odd-even merge network, a fixed order of
#   compare-exchanges, so that a GPU thread runs it without branches), then
#   renormalised;
# * multiplication (Joldes, Muller and Popescu's product of expansions
#   truncated at order m): for order n = 0 .. m-1 the n+1 products
#   x_i y_(n-i) by TwoProd; their high parts and the errors carried from the
#   orders below pass through VecSum, whose first word is the result's word
#   of order n and whose other words are carried on with the new TwoProd
#   errors; at order m the products x_i y_(m-i) and every carried error are
#   added plainly; the m+1 words are renormalised.
# ---------------------------------------------------------------------------

def vec_sum(c: Counter, x):
    """VecSum: (s_0, e_1, .., e_(n-1)) with s_0 + sum e_i = sum x_i exactly."""
    n = len(x)
    out = [0.0] * n
    s = x[n - 1]
    for i in range(n - 2, -1, -1):
        s, out[i + 1] = two_sum(c, x[i], s)
    out[0] = s
    return out


def vec_sum_err_branch(c: Counter, e, m: int):
    """VecSumErrBranch: m words from a VecSum output, a new word started
    only where the Fast2Sum error is nonzero (zeros pad the tail)."""
    r = [0.0] * m
    j = 0
    eps = e[0]
    for i in range(len(e) - 1):
        rj, nxt = fast_two_sum(c, eps, e[i + 1])
        r[j] = rj
        if nxt != 0.0:
            if j >= m - 1:
                return r
            j += 1
            eps = nxt
        else:
            eps = rj
    r[j] = eps
    return r


def renormalize(c: Counter, x, m: int):
    """The terms x (roughly decreasing) as m nonoverlapping words."""
    return vec_sum_err_branch(c, vec_sum(c, x), m)


def odd_even_merge(n: int):
    """Batcher's odd-even merge of two sorted runs of n = 2^k terms: the
    compare-exchange pairs (i, j), i < j, in order."""
    pairs = []

    def merge(lo, hi, r):
        step = 2 * r
        if step < hi - lo:
            merge(lo, hi, step)
            merge(lo + r, hi, step)
            pairs.extend((i, i + r) for i in range(lo + r, hi - r, step))
        else:
            pairs.append((lo, lo + r))

    merge(0, 2 * n - 1, 1)
    return pairs


def merge_by_magnitude(x, y):
    """The words of x and y (each by decreasing magnitude) in one list by
    decreasing magnitude: the merge network, exchanging where the earlier
    word is strictly smaller in magnitude."""
    z = list(x) + list(y)
    for i, j in odd_even_merge(len(x)):
        if abs(z[i]) < abs(z[j]):
            z[i], z[j] = z[j], z[i]
    return z


def od_add(c: Counter, x, y):
    """Octo-double addition: merge, then renormalise 16 words to 8."""
    return renormalize(c, merge_by_magnitude(x, y), 8)


def md_mul_expansion(c: Counter, x, y, m: int):
    """The product of two m-word expansions truncated at order m (see the
    section comment), renormalised to m words."""
    p, e = two_prod(c, x[0], y[0])
    r = [p]
    errs = [e]
    for n in range(1, m):
        P, Eh = [], []
        for i in range(n + 1):
            pi, ei = two_prod(c, x[i], y[n - i])
            P.append(pi)
            Eh.append(ei)
        s = vec_sum(c, P + errs)
        r.append(s[0])
        errs = s[1:] + Eh
    t = c.mul(x[1], y[m - 1])
    for i in range(2, m):
        t = c.add(t, c.mul(x[i], y[m - i]))
    for e in errs:
        t = c.add(t, e)
    r.append(t)
    return renormalize(c, r, m)


def od_mul(c: Counter, x, y):
    """Octo-double multiplication."""
    return md_mul_expansion(c, x, y, 8)


def hd_add(c: Counter, x, y):
    """Hexa-double addition (m = 16): the octo-double algorithm on 16 words,
    merge of 32 words, then renormalise to 16."""
    return renormalize(c, merge_by_magnitude(x, y), 16)


def hd_mul(c: Counter, x, y):
    """Hexa-double multiplication: the expansion product truncated at order 16."""
    return md_mul_expansion(c, x, y, 16)


def d_add(c: Counter, x, y):
    """Ordinary 1-double addition: one IEEE rounding."""
    return (c.add(x[0], y[0]),)


def d_mul(c: Counter, x, y):
    """Ordinary 1-double multiplication: one IEEE rounding."""
    return (c.mul(x[0], y[0]),)


ORDINARY = {1: (d_add, d_mul), 2: (dd_add, dd_mul), 4: (qd_add, qd_mul), 8: (od_add, od_mul),
            16: (hd_add, hd_mul)}


def ordinary_dot(c: Counter, xs, ys, m: int):
    """sum_k x_k * y_k in ordinary m-double arithmetic (m = 1, 2, 4, 8, 16): the
    accumulator starts at zero and takes add(acc, mul(x_k, y_k)) for k in
    increasing order, each operation renormalised."""
    add, mul = ORDINARY[m]
    acc = (0.0,) * m
    for x, y in zip(xs, ys):
        acc = add(c, acc, mul(c, x, y))
    return acc


def ordinary_dot_lanes(c: Counter, xs, ys, m: int, lanes: int = 64):
    """sum_k x_k * y_k in ordinary m-double arithmetic, in the order of a
    batched kernel that gives one vector pair to ``lanes`` threads: thread l
    accumulates add(acc, mul(x_k, y_k)) over k = l, l + lanes, l + 2 lanes,
    .. from zero (as ``ordinary_dot``), then the partial sums meet pairwise:
    for h = lanes/2, lanes/4, .., 1, thread l < h takes add(acc_l, acc_(l+h)).
    ``lanes`` = 1 is ``ordinary_dot``."""
    add, _ = ORDINARY[m]
    acc = [ordinary_dot(c, xs[l::lanes], ys[l::lanes], m) for l in range(lanes)]
    h = lanes // 2
    while h >= 1:
        for l in range(h):
            acc[l] = add(c, acc[l], acc[l + h])
        h //= 2
    return acc[0]


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
    """Double operations one call of an m-double ``fn`` (m = 2, 4, 8) costs
    on full-length operands (the octo-double renormalisation stops early on
    short ones)."""
    c = Counter()
    x = tuple((-1.0) ** (w // 3) * (1.0 + w / 16) * 2.0 ** (-57 * w) for w in range(m))
    y = tuple((-1.0) ** (w // 2) * (3.0 - w / 16) * 2.0 ** (-55 * w) for w in range(m))
    fn(c, x, y)
    return c.n


def ordinary_gemm_ops(m: int, M: int, N: int, K: int) -> int:
    """Double operations of an ordinary m-double matrix product (Table 1)."""
    add, mul, _, _ = TABLE1[m]
    return M * N * K * (add + mul)
