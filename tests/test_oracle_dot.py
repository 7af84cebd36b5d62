"""Oracle pins for the batched inner products (the paper's experiment,
Section 3: 1,024 sums of 6,144 products in m-double precision, m = 1..16).

The oracle computes pair b as the 1 x 1 product of the row x_b and the
column y_b, so its arithmetic is the matrix product's (pinned in
test_oracle.py).  Pinned here, against facts the paper and the mathematics
fix:

* exact dot products against a Fraction brute force;
* the paper's own parameters on the paper's bit pattern (Section 2: 13-bit
  quarters, S = 4m): all S^2 digit pairs reproduce the exact dot product
  (lossless split), and the kept triangle s + u <= S - 1 errs by at most
  (4m - 1) 2^(2 - 52 m) of sum_k |x_k||y_k| (each dropped digit product is
  below 2^(2 - 13 t) for t >= S, and |x_k|, |y_k| >= 1), plus the final
  rounding;
* the magnitude certificate is the minimum over the pairs of a brute-force
  integer sum;
* the slice-count rule meets 2^-T on random batches, and a forced smaller S
  does not.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import mdinputs
from oracle import exact as ox


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def batch(m, nb, n, seed, lead=("uniform",)):
    r = rng(seed)
    return mdinputs.mdouble(r, m, (nb, n), lead), mdinputs.mdouble(r, m, (nb, n), lead)


@pytest.mark.parametrize("m", [1, 2, 16])
def test_exact_dots_brute_force(m):
    X, Y = batch(m, 3, 5, 10 + m)
    X[:, 1, 2] = 0.0
    vals, absvals = ox.exact_dots(X, Y)
    for b in range(3):
        ref = sum(ox.entry_value(X[:, b, k]) * ox.entry_value(Y[:, b, k]) for k in range(5))
        aref = sum(abs(ox.entry_value(X[:, b, k])) * abs(ox.entry_value(Y[:, b, k])) for k in range(5))
        assert vals[b] == ref and absvals[b] == aref


def paper_batch(m, nb, n, seed):
    r = rng(seed)
    X, _, _ = mdinputs.paper_pattern(r, m, (nb, n))
    Y, _, _ = mdinputs.paper_pattern(r, m, (nb, n))
    return X, Y


@pytest.mark.parametrize("m", [1, 2, 4, 8, 16])
def test_paper_parameters_all_pairs_lossless(m):
    """beta = 13, S = 4m on the bit pattern: summing every digit pair folds
    to the exact dot product."""
    X, Y = paper_batch(m, 3, 7, 20 + m)
    vals, _ = ox.exact_dots(X, Y)
    S = 4 * m
    for b in range(3):
        x, y = ox.pair_operands(X, Y, b)
        E, _ = ox.row_exponents(x[0])
        F, _ = ox.row_exponents(y[0].T)
        assert E == [1] and F == [1]          # leading words in [1, 2)
        dA = ox.split_planes(x, E, 13, S, by_columns=False)
        dB = ox.split_planes(y, F, 13, S, by_columns=True)
        assert np.abs(dA).max() < (1 << 13) and np.abs(dA).min() >= (1 << 12)
        D = ox.diagonal_sums(dA, dB, S, all_pairs=True)
        assert ox.fold(D[:, 0, 0], E[0], F[0], 13) == vals[b]


@pytest.mark.parametrize("m", [1, 2, 4, 8, 16])
def test_paper_parameters_triangle_bound(m):
    """The kept triangle with the paper's parameters errs by at most
    (4m - 1) 2^(2 - 52m) of sum_k |x_k||y_k|, plus the final rounding of
    the m words (2^(1 - 53m) relative); and the bound is not vacuous: the
    dropped pairs do contribute for m >= 1."""
    X, Y = paper_batch(m, 4, 9, 30 + m)
    vals, absvals = ox.exact_dots(X, Y)
    _, out = ox.method_dot(X, Y, 13, 4 * m)
    bound = Fraction(4 * m - 1) * Fraction(2) ** (2 - 52 * m) * Fraction(1001, 1000) \
        + Fraction(2) ** (1 - 53 * m)
    worst = Fraction(0)
    for b in range(4):
        err = abs(ox.entry_value(out[:, b]) - vals[b])
        assert err <= bound * absvals[b], (b, float(err / absvals[b]))
        worst = max(worst, err / absvals[b])
    assert worst > Fraction(2) ** (-52 * m - 40)


def test_rho_certificate_is_min_over_pairs():
    X, Y = batch(2, 5, 11, 40, lead=("log2uniform", 6.0))
    n = X.shape[2]
    P = []
    for b in range(5):
        ex = max(ox.frexp_exponent(float(v)) for v in X[0, b] if v != 0.0)
        ey = max(ox.frexp_exponent(float(v)) for v in Y[0, b] if v != 0.0)
        qx = [math.floor(abs(Fraction(float(v))) * Fraction(2) ** (7 - ex)) for v in X[0, b]]
        qy = [math.floor(abs(Fraction(float(v))) * Fraction(2) ** (7 - ey)) for v in Y[0, b]]
        P.append(sum(a * c for a, c in zip(qx, qy)))
    minP, g = ox.rho_G_dot(X, Y)
    assert minP == min(P)
    assert (minP << g) >= n * (1 << 14) + 1 and (g == 0 or (minP << (g - 1)) < n * (1 << 14) + 1)


@pytest.mark.parametrize("m,form", [(1, "int8"), (2, "fp64"), (4, "int8"), (16, "fp64")])
def test_rule_meets_target_and_small_S_fails(m, form):
    T = ox.TARGET_BITS[m]
    X, Y = batch(m, 3, 40, 50 + m, lead=("log2uniform", 8.0))
    vals, absvals = ox.exact_dots(X, Y)
    beta, S, _ = ox.budget_params(form, X.shape[2], ox.TARGET_BITS[X.shape[0]], ox.dot_G(X, Y))
    _, out = ox.method_dot(X, Y, beta, S)
    for b in range(3):
        err = abs(ox.entry_value(out[:, b]) - vals[b])
        assert err <= Fraction(2) ** -T * absvals[b]
    # far fewer slices: the bound must fail somewhere
    Ssmall = max(1, S - 6)
    _, bad = ox.method_dot(X, Y, beta, Ssmall)
    errs = [abs(ox.entry_value(bad[:, b]) - vals[b]) / absvals[b] for b in range(3)]
    assert max(errs) > Fraction(2) ** -T
