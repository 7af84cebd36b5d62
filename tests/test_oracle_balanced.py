"""Pins of the oracle's balanced INT8 digits (the second INT8 encoding:
8-bit digits in [-128, 127] on the grid 2^(E+2)) against what the
arithmetic fixes.

* ``balanced_digits`` against brute force: for S = 1, 2 every integer in
  the reachable range has exactly one digit string, round trips, and
  everything outside raises;
* the truncated integer two ways: exact Fractions (``truncated_integer``)
  and the sign-magnitude 8-bit fields of ``split_entry`` on the same grid;
* the vectorised split (sign-magnitude fields, then carries) against the
  scalar one (exact integer, then centred remainders), entry by entry,
  mixed-sign words and zeros included;
* the truncation error (below one unit of the last digit) and the
  headroom: for S >= 2, 2^(8S-1) - 1 needs more than S balanced digits,
  2^(8S-2) - 1 does not;
* all pairs kept, the fold is exactly the product of the truncated
  entries; the per-term budget (S+3) 2^(E+F+2-8S) of
  ``slice_count_balanced`` holds on adversarial single terms;
* the whole method with the rule's S stays within 2^-T of the exact
  product, and at the quad-double benchmark's K = 4096, G = 3 the rule
  takes S = 27 against the sign-magnitude form's 30;
* the exactness chunk for digits up to 128.
"""
from fractions import Fraction

import numpy as np
import pytest

import mdinputs
from oracle import exact as ox


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def value(d):
    v = 0
    for x in d:
        v = 256 * v + int(x)
    return v


@pytest.mark.parametrize("S", [1, 2])
def test_balanced_digits_brute_force(S):
    lo = -128 * (256 ** S - 1) // 255
    hi = 127 * (256 ** S - 1) // 255
    seen = set()
    for X in range(lo - 300, hi + 301):
        if lo <= X <= hi:
            d = ox.balanced_digits(X, S)
            assert all(-128 <= x <= 127 for x in d)
            assert value(d) == X
            seen.add(tuple(d))
        else:
            with pytest.raises(ValueError):
                ox.balanced_digits(X, S)
    # one digit string per integer: the strings cover the 256^S
    assert len(seen) == 256 ** S


def test_balanced_digits_examples():
    assert ox.balanced_digits(0, 3) == [0, 0, 0]
    assert ox.balanced_digits(127, 3) == [0, 0, 127]
    assert ox.balanced_digits(128, 3) == [0, 1, -128]
    assert ox.balanced_digits(-128, 3) == [0, 0, -128]
    assert ox.balanced_digits(255, 3) == [0, 1, -1]
    assert ox.balanced_digits(-129, 3) == [0, -1, 127]
    assert ox.balanced_digits(65535, 3) == [1, 0, -1]


def adversarial_entries(r, m, n):
    """Entries near 2^E (all-ones leading mantissas), mixed word signs,
    zero trailing words, and ordinary ones."""
    X = mdinputs.mdouble(r, m, (1, n), ("log2uniform", 4.0))[:, 0, :]
    for k in range(0, n, 3):
        X[0, k] = np.copysign(np.nextafter(2.0, 0.0), X[0, k])   # (2 - 2^-52), E = 1
        X[1:, k] = 0.0
        if m > 1:
            X[1, k] = -np.copysign(2.0 ** -54, X[0, k])           # half an ulp, other sign
    for k in range(1, n, 5):
        X[1:, k] = 0.0
    assert all(ox.is_nonoverlapping(X[:, k], strong=True) for k in range(n))
    return X


@pytest.mark.parametrize("m", [1, 2, 4, 8])
def test_truncated_integer_two_ways(m):
    r = rng(10 + m)
    X = adversarial_entries(r, m, 60)
    for k in range(X.shape[1]):
        words = X[:, k]
        E = max(ox.frexp_exponent(w) for w in words[:1] if w != 0.0)
        for S in (1, 5, 27, 53):
            t = ox.truncated_integer(words, E + 2, 8 * S)
            sm = ox.split_entry(words, E + 2, 8, S)        # fields in [-255, 255]
            assert value(sm) == t
            bal = ox.split_entry_balanced(words, E, S)
            assert value(bal) == t
            assert all(-128 <= x <= 127 for x in bal)
            # below one unit of the last digit
            err = ox.entry_value(words) - Fraction(t) * Fraction(2) ** (E + 2 - 8 * S)
            assert abs(err) < Fraction(2) ** (E + 2 - 8 * S)


def test_headroom():
    for S in (2, 3, 27):
        with pytest.raises(ValueError):
            ox.balanced_digits(2 ** (8 * S - 1) - 1, S)
        for X in (2 ** (8 * S - 2) - 1, -(2 ** (8 * S - 2) - 1)):
            assert value(ox.balanced_digits(X, S)) == X


@pytest.mark.parametrize("m,by_columns", [(1, False), (2, True), (4, False), (8, True)])
def test_split_planes_balanced_matches_scalar(m, by_columns):
    r = rng(20 + m)
    P = mdinputs.mdouble(r, m, (6, 9), ("log2uniform", 12.0))
    P[:, 2, 3] = 0.0
    P[1:, 4, :] = 0.0
    P[0, 5, 0] = np.nextafter(1.0, 0.0)
    lead = P[0].T if by_columns else P[0]
    E, _ = ox.row_exponents(lead)
    S = 19
    d = ox.split_planes_balanced(P, E, S, by_columns)
    assert d.min() >= -128 and d.max() <= 127
    for i in range(6):
        for k in range(9):
            e = E[k] if by_columns else E[i]
            assert list(d[:, i, k]) == ox.split_entry_balanced(P[:, i, k], e, S)


def test_all_pairs_fold_is_truncated_product():
    A, B = mdinputs.workload("qd1024", M=3, N=2, K=7)
    S = 9
    E, _ = ox.row_exponents(A[0])
    F, _ = ox.row_exponents(B[0].T)
    dA = ox.split_planes_balanced(A, E, S, False)
    dB = ox.split_planes_balanced(B, F, S, True)
    D = ox.diagonal_sums(dA, dB, S, all_pairs=True)
    for i in range(3):
        for j in range(2):
            got = ox.fold(D[:, i, j], E[i] + 2, F[j] + 2, 8)
            want = sum(Fraction(ox.truncated_integer(A[:, i, k], E[i] + 2, 8 * S)) *
                       Fraction(ox.truncated_integer(B[:, k, j], F[j] + 2, 8 * S))
                       for k in range(7)) * Fraction(2) ** (E[i] + F[j] + 4 - 16 * S)
            assert got == want


@pytest.mark.parametrize("S", [1, 2, 3, 8, 27, 40])
def test_per_term_budget(S):
    """One product term a b, K = 1: the kept triangle errs by less than
    (S+3) 2^(E+F+2-8S), on adversarial entries."""
    r = rng(30 + S)
    X = adversarial_entries(r, 4, 24)
    Y = adversarial_entries(r, 4, 24)
    for k in range(24):
        a = X[:, k:k + 1][:, None, :]            # (m, 1, 1)
        b = Y[:, k:k + 1][:, :, None]
        res = ox.method_product(a, b, 8, S, balanced=True)
        E, F = res["E"][0], res["F"][0]
        kept = ox.fold(res["D"][:, 0, 0], E + 2, F + 2, 8)
        exact = ox.entry_value(X[:, k]) * ox.entry_value(Y[:, k])
        assert abs(kept - exact) < (S + 3) * Fraction(2) ** (E + F + 2 - 8 * S)


def test_rule_and_headline_slice_count():
    assert ox.slice_count_balanced(200, 3) == 27
    assert ox.slice_count(7, 200, 3) == 30
    # the rule's inequality at the result and its failure one below
    for T, G in [(50, 0), (100, 3), (200, 3), (400, 12), (800, 5)]:
        S = ox.slice_count_balanced(T, G)
        assert 8 * S >= T + G + ox.ceil_log2(S + 3) + 3
        assert 8 * (S - 1) < T + G + ox.ceil_log2(S + 2) + 3
    assert ox.budget_params("int8bal", 4096, 200, 3) == (8, 27, 4096)


def test_exact_depth_balanced():
    """The largest exact depth: S kc dmax^2 < 2^31 <= S (kc + 1) dmax^2,
    dmax = 128 for the balanced digits and 2^beta - 1 otherwise."""
    kc = ox.exact_depth("int8bal", 8, 27)
    assert 27 * kc * 128 * 128 < 2 ** 31 <= 27 * (kc + 1) * 128 * 128
    kc = ox.exact_depth("int8", 7, 30)
    assert 30 * kc * 127 * 127 < 2 ** 31 <= 30 * (kc + 1) * 127 * 127
    kc = ox.exact_depth("fp64", 21, 10)
    assert 10 * kc * (2 ** 21 - 1) ** 2 < 2 ** 53 <= 10 * (kc + 1) * (2 ** 21 - 1) ** 2


@pytest.mark.parametrize("m,lead", [(2, ("uniform",)), (4, ("log2uniform", 8.0)), (8, ("log2uniform", 16.0))])
def test_method_within_target(m, lead):
    r = rng(40 + m)
    M, N, K = 5, 4, 37
    A = mdinputs.mdouble(r, m, (M, K), lead)
    B = mdinputs.mdouble(r, m, (K, N), lead)
    A[:, 1, :] = 0.0                                   # an all-zero row
    _, G = ox.rho_G(A[:, [0, 2, 3, 4]], B)
    _, sa = ox.row_exponents(A[0])
    _, sb = ox.row_exponents(B[0].T)
    G = min(ox.span_G(max(sa), max(sb)), G if G is not None else 10 ** 6)
    T = ox.TARGET_BITS[m]
    beta, S, _ = ox.budget_params("int8bal", K, T, G)
    res = ox.method_product(A, B, beta, S, balanced=True)
    num, L = ox.exact_product(A, B)
    anum, _ = ox.abs_product(A, B)
    rep = ox.error_report(res["C"], num, anum, L)
    assert max(rep.values()) <= -T
    assert np.all(res["C"][:, 1, :] == 0.0)
    for i in range(M):
        for j in range(N):
            assert ox.is_nonoverlapping(res["C"][:, i, j], strong=True)
