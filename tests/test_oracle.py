"""Pins of the exact oracle against facts that do not come from the oracle.

Each test names what fixes the expected value: the paper (its bit-pattern
construction, its tables), a closed form, an invariant, a library routine
with a known contract, or brute force on tiny inputs.
"""
import json
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest

import mdinputs
from oracle import exact as ox
from oracle import mdarith

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _lossless_S(planes, E, beta, rows_axis):
    """Digits needed so that the grid from 2^E reaches every set bit of
    every word (rows_axis 1: E per row, 2: E per column)."""
    need = 1
    m = planes.shape[0]
    for idx in np.ndindex(planes.shape[1:]):
        e_row = E[idx[0]] if rows_axis == 1 else E[idx[1]]
        for w in range(m):
            x = float(planes[(w,) + idx])
            if x != 0.0:
                num, den = Fraction(abs(x)).as_integer_ratio()
                low = (num & -num).bit_length() - 1 - (den.bit_length() - 1)
                need = max(need, e_row - low)
    return -(-need // beta)


# --------------------------------------------------------------------------
# rounding: the integer round-to-nearest against Python's correctly rounded
# int/int true division (its documented contract), ties and subnormals
# --------------------------------------------------------------------------

def test_round_nearest_matches_correctly_rounded_division():
    rnd = random.Random(1)
    cases = []
    for _ in range(3000):
        p = rnd.getrandbits(rnd.randint(1, 300)) + 1
        q = rnd.getrandbits(rnd.randint(1, 300)) + 1
        cases.append(Fraction(p, q) * rnd.choice([1, -1]))
    # exact ties between two doubles, both parities of the last bit
    for k in range(200):
        base = rnd.getrandbits(52) | (1 << 52)
        e = rnd.randint(-1000, 900)
        cases.append(Fraction(2 * base + 1, 2) * Fraction(2) ** e)
    # subnormal range, the smallest subnormal and halfway below it
    for k in range(200):
        cases.append(Fraction(rnd.getrandbits(60) + 1, 1 << (1074 + rnd.randint(0, 60))))
    cases.append(Fraction(1, 1 << 1075))
    cases.append(Fraction(3, 1 << 1076))
    for x in cases:
        assert ox.round_nearest(x) == float(x), x


def test_renorm_rn_properties():
    rnd = random.Random(2)
    for m in (1, 2, 4, 8):
        for _ in range(300):
            x = Fraction(rnd.getrandbits(600) - (1 << 599), 1 << rnd.randint(0, 700))
            w = ox.renorm_rn(x, m)
            assert w[0] == float(x)
            assert ox.is_nonoverlapping(w, strong=True)
            rem = x - ox.entry_value(w)
            # greedy rounding: the remainder is below half an ulp of the last
            # nonzero word, i.e. below 2^(-53 m) |x| up to the first word's scale
            if x != 0:
                assert abs(rem) <= abs(x) * Fraction(1, 1 << (53 * m)) * 2


def test_nonoverlap_predicate_edges():
    assert ox.is_nonoverlapping([1.0, 2.0 ** -54, 0.0, 0.0])
    assert ox.is_nonoverlapping([1.0, 2.0 ** -53])            # exactly ulp/2
    assert not ox.is_nonoverlapping([1.0, 2.0 ** -52])        # a whole ulp
    assert not ox.is_nonoverlapping([0.0, 1.0])               # zero not trailing
    assert ox.is_nonoverlapping([-0.0, 0.0])
    assert ox.is_nonoverlapping([1.5, -(2.0 ** -54)])         # mixed signs
    # weak form: bit-disjoint but not within half an ulp
    assert ox.is_nonoverlapping([1.0, 2.0 ** -52], strong=False)
    assert not ox.is_nonoverlapping([1.0 + 2.0 ** -52, 2.0 ** -52], strong=False)


# --------------------------------------------------------------------------
# exact layer: brute force with Fractions on tiny inputs; m = 1 reduces to an
# integer matrix product (numpy int64 matmul, exact for these sizes)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m", [1, 2, 4, 8])
def test_exact_product_brute_force(m):
    rng = _rng(10 + m)
    for (M, N, K) in [(1, 1, 1), (2, 3, 4), (4, 4, 4), (3, 1, 2)]:
        A = mdinputs.mdouble(rng, m, (M, K), ("log2uniform", 30.0))
        B = mdinputs.mdouble(rng, m, (K, N), ("uniform",))
        A[:, 0, 0] = 0.0                      # a zero entry
        num, L = ox.exact_product(A, B)
        anum, _ = ox.abs_product(A, B)
        for i in range(M):
            for j in range(N):
                ref = sum(ox.entry_value(A[:, i, k]) * ox.entry_value(B[:, k, j]) for k in range(K))
                aref = sum(abs(ox.entry_value(A[:, i, k])) * abs(ox.entry_value(B[:, k, j])) for k in range(K))
                assert Fraction(int(num[i, j]), 1 << L) == ref
                assert Fraction(int(anum[i, j]), 1 << L) == aref


def test_exact_product_m1_integer_matmul():
    rng = _rng(3)
    A = rng.integers(-2 ** 20, 2 ** 20, size=(1, 7, 9)).astype(np.float64)
    B = rng.integers(-2 ** 20, 2 ** 20, size=(1, 9, 5)).astype(np.float64)
    num, L = ox.exact_product(A, B)
    ref = A[0].astype(np.int64) @ B[0].astype(np.int64)
    assert L == 0
    assert all(int(num[i, j]) == int(ref[i, j]) for i in range(7) for j in range(5))


# --------------------------------------------------------------------------
# exponents
# --------------------------------------------------------------------------

def test_row_exponents_frexp_contract():
    rng = _rng(4)
    lead = mdinputs.mdouble(rng, 1, (6, 50), ("log2uniform", 40.0))[0]
    lead[2, :] = 0.0
    lead[3, 5:] = 0.0
    E, span = ox.row_exponents(lead)
    for r in range(6):
        nz = [abs(x) for x in lead[r] if x != 0.0]
        if not nz:
            assert E[r] == 0 and span[r] == 0
            continue
        # every entry below 2^E, some entry at least 2^(E-1)
        assert all(x < 2.0 ** E[r] for x in nz)
        assert any(x >= 2.0 ** (E[r] - 1) for x in nz)
        assert min(nz) >= 2.0 ** (E[r] - span[r] - 1)
        assert min(nz) < 2.0 ** (E[r] - span[r])


# --------------------------------------------------------------------------
# split: the paper's bit pattern (Section 2) fixes the quarters by
# construction; invariants for general data
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m", [1, 2, 4, 8])
def test_split_paper_pattern_quarters(m):
    rng = _rng(20 + m)
    planes, groups, signs = mdinputs.paper_pattern(rng, m, (5, 6))
    # the leading words lie in [1, 2): frexp exponent 1 for every row
    E, _ = ox.row_exponents(planes[0])
    assert E == [1] * 5
    d = ox.split_planes(planes, E, 13, 4 * m, by_columns=False)
    for w in range(m):
        for q in range(4):
            np.testing.assert_array_equal(d[4 * w + q], signs[w] * groups[w, q])
    # the per-entry definition agrees
    for i in range(5):
        for k in range(6):
            assert ox.split_entry(planes[:, i, k], 1, 13, 4 * m) == [int(v) for v in d[:, i, k]]


@pytest.mark.parametrize("beta", [7, 13, 18, 22])
def test_split_digit_bound_and_lossless_reconstruction(beta):
    rng = _rng(30 + beta)
    for m in (2, 4, 8):
        A = mdinputs.mdouble(rng, m, (4, 16), ("log2uniform", 12.0))
        E, span = ox.row_exponents(A[0])
        S = _lossless_S(A, E, beta, 1)
        d = ox.split_planes(A, E, beta, S, by_columns=False)
        assert np.abs(d).max() <= (1 << beta) - 1
        for i in range(4):
            for k in range(16):
                rec = sum(Fraction(int(d[s, i, k])) * Fraction(2) ** (E[i] - beta * (s + 1)) for s in range(S))
                assert rec == ox.entry_value(A[:, i, k])


def test_split_truncation_error_bound():
    rng = _rng(5)
    beta, m = 7, 4
    A = mdinputs.mdouble(rng, m, (8, 32), ("uniform",))
    E, _ = ox.row_exponents(A[0])
    for S in (3, 10, 25):
        d = ox.split_planes(A, E, beta, S, by_columns=False)
        for i in range(8):
            for k in range(32):
                a = ox.entry_value(A[:, i, k])
                rec = sum(Fraction(int(d[s, i, k])) * Fraction(2) ** (E[i] - beta * (s + 1)) for s in range(S))
                err = abs(a - rec)
                assert err < Fraction(2) ** (E[i] - beta * S)
                # truncation toward zero, word by word: the reconstruction
                # never exceeds the entry in magnitude for single-signed words
                if all(x >= 0 for x in A[:, i, k]) or all(x <= 0 for x in A[:, i, k]):
                    assert abs(rec) <= abs(a)


# --------------------------------------------------------------------------
# diagonal sums: the convolution formula as literal loops vs int64 matmul;
# all pairs of digits reproduce the exact product (closed form)
# --------------------------------------------------------------------------

def test_diagonal_sums_loop_vs_matmul():
    rng = _rng(6)
    S = 5
    dA = rng.integers(-127, 128, size=(S, 3, 4))
    dB = rng.integers(-127, 128, size=(S, 4, 2))
    D = ox.diagonal_sums(dA, dB, S)
    Dl = ox.diagonal_sums_loop([[list(dA[:, i, k]) for k in range(4)] for i in range(3)],
                               [[list(dB[:, k, j]) for j in range(2)] for k in range(4)], S)
    for t in range(S):
        for i in range(3):
            for j in range(2):
                assert D[t, i, j] == Dl[t][i][j]


@pytest.mark.parametrize("m,beta", [(2, 13), (2, 22), (4, 7), (4, 18)])
def test_all_pairs_lossless_equals_exact_product(m, beta):
    rng = _rng(40 + m + beta)
    M, N, K = 3, 4, 5
    A = mdinputs.mdouble(rng, m, (M, K), ("log2uniform", 6.0))
    B = mdinputs.mdouble(rng, m, (K, N), ("uniform",))
    E, sA = ox.row_exponents(A[0])
    F, sB = ox.row_exponents(B[0].T)
    S = max(_lossless_S(A, E, beta, 1), _lossless_S(B, F, beta, 2))
    dA = ox.split_planes(A, E, beta, S, by_columns=False)
    dB = ox.split_planes(B, F, beta, S, by_columns=True)
    D = ox.diagonal_sums(dA, dB, S, all_pairs=True)
    num, L = ox.exact_product(A, B)
    for i in range(M):
        for j in range(N):
            x = ox.fold(D[:, i, j], E[i], F[j], beta)
            assert x == Fraction(int(num[i, j]), 1 << L)


def test_identity_right_factor_returns_left_factor():
    rng = _rng(7)
    m, beta = 4, 7
    A = mdinputs.mdouble(rng, m, (5, 6), ("log2uniform", 3.0))
    B = np.zeros((m, 6, 6))
    B[0] = np.eye(6)
    E, sA = ox.row_exponents(A[0])
    S = _lossless_S(A, E, beta, 1)
    res = ox.method_product(A, B, beta, S)
    np.testing.assert_array_equal(res["C"], A)


# --------------------------------------------------------------------------
# the error budget: rule-chosen S meets 2^-T of |A||B| entry by entry; a
# forced too-small S must violate it (the checker is not vacuous)
# --------------------------------------------------------------------------

def _max_err(A, B, beta, S):
    res = ox.method_product(A, B, beta, S)
    num, L = ox.exact_product(A, B)
    anum, _ = ox.abs_product(A, B)
    rep = ox.error_report(res["C"], num, anum, L)
    return max(rep.values()), res


@pytest.mark.parametrize("name,form", [("dd64", "fp64"), ("dd64", "int8"), ("qd1024", "fp64"),
                                       ("qd1024", "int8"), ("od1024", "int8")])
def test_budget_rule_meets_target(name, form):
    _, m, _, _, _, _, _ = mdinputs.WORKLOADS[name]
    A, B = mdinputs.workload(name, M=6, N=5, K=24)
    T = ox.TARGET_BITS[m]
    _, sA = ox.row_exponents(A[0])
    _, sB = ox.row_exponents(B[0].T)
    G = ox.span_G(max(sA), max(sB))
    beta, S, kc = ox.budget_params(form, 24, T, G)
    worst, res = _max_err(A, B, beta, S)
    assert worst <= -T
    for i in range(6):
        for j in range(5):
            assert ox.is_nonoverlapping(res["C"][:, i, j], strong=True)
    # exactness of the accumulations the rule promises
    limit = 2 ** 31 if form == "int8" else 2 ** 53
    assert np.abs(res["D"]).max() < limit


def test_too_few_slices_violate_target():
    A, B = mdinputs.workload("qd1024", M=4, N=4, K=16)
    worst, _ = _max_err(A, B, 7, 20)
    assert worst > -200


def test_paper_parameters_triangle_bound():
    """beta = 13, S = 4m on the paper's pattern (Section 2): the split is
    lossless, so only the dropped triangle errs; per term it is below
    (S-1) 2^(E+F-13 S) with E = F = 1."""
    rng = _rng(8)
    for m in (2, 4):
        A, _, _ = mdinputs.paper_pattern(rng, m, (3, 7))
        Bt, _, _ = mdinputs.paper_pattern(rng, m, (4, 7))
        B = np.ascontiguousarray(np.transpose(Bt, (0, 2, 1)))
        S = 4 * m
        res = ox.method_product(A, B, 13, S)
        num, L = ox.exact_product(A, B)
        for i in range(3):
            for j in range(4):
                ctil = ox.fold(res["D"][:, i, j], 1, 1, 13)
                err = abs(ctil - Fraction(int(num[i, j]), 1 << L))
                assert err < 7 * (S - 1) * Fraction(2) ** (2 - 13 * S)


# --------------------------------------------------------------------------
# gradients: the loss sum(W * C) is bilinear, so a central difference with
# step 2^-40 is exact and must equal the closed form W B^T
# --------------------------------------------------------------------------

def test_exact_gradient_equals_exact_central_difference():
    rng = _rng(9)
    m = 2
    A = mdinputs.mdouble(rng, m, (3, 4), ("uniform",))
    B = mdinputs.mdouble(rng, m, (4, 2), ("uniform",))
    W = mdinputs.mdouble(rng, m, (3, 2), ("uniform",))
    (ga, La), (gb, Lb) = ox.exact_gradients(A, B, W)
    h = Fraction(1, 1 << 40)
    val = lambda P, idx: ox.entry_value(P[(slice(None),) + idx])

    def loss(Av, Bv):
        return sum(val(W, (i, j)) * sum(Av[i][k] * Bv[k][j] for k in range(4))
                   for i in range(3) for j in range(2))
    Av = [[val(A, (i, k)) for k in range(4)] for i in range(3)]
    Bv = [[val(B, (k, j)) for j in range(2)] for k in range(4)]
    for (i, k) in [(0, 0), (2, 3), (1, 2)]:
        Ap = [row[:] for row in Av]
        Am = [row[:] for row in Av]
        Ap[i][k] += h
        Am[i][k] -= h
        fd = (loss(Ap, Bv) - loss(Am, Bv)) / (2 * h)
        assert fd == Fraction(int(ga[i, k]), 1 << La)
    for (k, j) in [(0, 0), (3, 1)]:
        Bp = [row[:] for row in Bv]
        Bm = [row[:] for row in Bv]
        Bp[k][j] += h
        Bm[k][j] -= h
        fd = (loss(Av, Bp) - loss(Av, Bm)) / (2 * h)
        assert fd == Fraction(int(gb[k, j]), 1 << Lb)


# --------------------------------------------------------------------------
# the paper's tables
# --------------------------------------------------------------------------

def test_table1_counts_and_average_column():
    tab = json.load(open(os.path.join(GOLDEN, "table1.json")))["rows"]
    for m, (add, mul, div, avg) in tab.items():
        assert round((add + mul + div) / 3, 1) == avg
        assert tuple(mdarith.TABLE1[int(m)]) == (add, mul, div, avg)
    # the accurate double-double addition costs exactly the table's 20
    assert mdarith.op_count(mdarith.dd_add) == tab["2"][0]
    # multiplication: Dekker's product without FMA costs 24 against the
    # table's 23 (the paper's variant is unnamed: unpinned)
    assert mdarith.op_count(mdarith.dd_mul) == 24


def test_double_double_ops_accuracy():
    rnd = random.Random(11)
    for _ in range(500):
        hx = rnd.uniform(-1, 1)
        hy = rnd.uniform(-1, 1)
        x = (hx, math.ulp(hx) * rnd.uniform(-0.5, 0.5))
        y = (hy, math.ulp(hy) * rnd.uniform(-0.5, 0.5))
        c = mdarith.Counter()
        s = mdarith.dd_add(c, x, y)
        p = mdarith.dd_mul(c, x, y)
        xs, ys = Fraction(x[0]) + Fraction(x[1]), Fraction(y[0]) + Fraction(y[1])
        exact_s = xs + ys
        exact_p = xs * ys
        assert abs(Fraction(s[0]) + Fraction(s[1]) - exact_s) <= (abs(xs) + abs(ys)) * Fraction(1, 1 << 103)
        assert abs(Fraction(p[0]) + Fraction(p[1]) - exact_p) <= abs(exact_p) * Fraction(1, 1 << 100)


def test_table2_ratio_columns():
    tab = json.load(open(os.path.join(GOLDEN, "table2.json")))["rows"]
    order = ["1d", "2d", "4d", "8d", "16d"]
    for a, b in zip(order[1:], order[:-1]):
        o = tab[a]["ordinary_ms"] / tab[b]["ordinary_ms"]
        v = tab[a]["vectorized_ms"] / tab[b]["vectorized_ms"]
        if tab[a]["ordinary_ratio"] is not None:
            assert round(o, 1) == tab[a]["ordinary_ratio"]
        # both ratio columns sit on the higher-precision row
        assert round(v, 1) == tab[a]["vectorized_ratio"]
    for r in order:
        assert round(tab[r]["ordinary_ms"] / tab[r]["vectorized_ms"], 1) == tab[r]["speedup"]
    # the garbled "12.x" and "13.x" entries read as 12.5 and 13.2
    assert round(tab["4d"]["ordinary_ms"] / tab["2d"]["ordinary_ms"], 1) == 12.5
    assert round(tab["2d"]["ordinary_ms"] / tab["1d"]["ordinary_ms"], 1) == 13.2


# --------------------------------------------------------------------------
# inputs
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", list(mdinputs.WORKLOADS))
def test_generated_inputs_strongly_nonoverlapping(name):
    A, B, W = mdinputs.workload(name, M=16, N=12, K=20, with_w=True)
    for P in (A, B, W):
        assert mdinputs.strongly_nonoverlapping(P)
        for idx in [(0, 0), (3, 5), (7, 11)]:
            assert ox.is_nonoverlapping(P[(slice(None),) + idx], strong=True)
    A2, _ = mdinputs.workload(name, M=16, N=12, K=20)
    np.testing.assert_array_equal(A, A2)


def test_precondition_flags():
    """The input preconditions on hand-made entries: finite words, weak
    nonoverlap (disjoint bit ranges, decreasing, zeros only at the tail) and
    the range of the leading word."""
    pf = ox.precondition_flags
    ok = [1.5, 2.0 ** -60, -(2.0 ** -120), 0.0]
    assert pf(ok) == 0
    assert pf([0.0, 0.0]) == 0
    # weak but not strong: the second word touches the first's last bit range
    w = [1.0 + 2.0 ** -40, 2.0 ** -41]
    assert pf(w) == 0 and not ox.is_nonoverlapping(w, strong=True)
    assert pf([1.0 + 2.0 ** -40, 2.0 ** -40]) == ox.PRE_OVERLAP       # same bit
    assert pf([1.0, 3.0]) == ox.PRE_OVERLAP                          # increasing
    assert pf([1.0, 0.0, 2.0 ** -80]) == ox.PRE_OVERLAP              # zero gap
    assert pf([float("nan"), 0.0]) == ox.PRE_NONFINITE
    assert pf([1.0, float("inf")]) == ox.PRE_NONFINITE
    assert pf([2.0 ** 900, 0.0]) == ox.PRE_RANGE
    assert pf([2.0 ** 899 * 1.5, 0.0]) == 0
    assert pf([2.0 ** -900, 0.0]) == 0
    assert pf([2.0 ** -901, 0.0]) == ox.PRE_RANGE
    assert pf([-(2.0 ** -1070), 0.0]) == ox.PRE_RANGE                 # subnormal lead
    assert pf([2.0 ** 950, 2.0 ** 950]) == ox.PRE_OVERLAP | ox.PRE_RANGE


@pytest.mark.parametrize("balanced", [False, True])
def test_fixed_product_rounds_to_the_method_and_splits_over_depth(balanced):
    """The exact fixed-point sum rounds (greedy, to nearest) to the method's
    output; over a depth split with the full rows' and columns' exponents
    the two partial integers add up exactly to the whole product's (the
    diagonal sums are sums over k), and the scales agree."""
    A, B = mdinputs.workload("qd1024", M=5, N=4, K=40)
    beta, S = (8, 27) if balanced else (7, 30)
    X, sc = ox.fixed_product(A, B, beta, S, balanced=balanced)
    ref = ox.method_product(A, B, beta, S, balanced=balanced)
    for i in range(5):
        for j in range(4):
            x = Fraction(X[i, j]) * Fraction(2) ** int(sc[i, j])
            assert tuple(ox.renorm_rn(x, 4)) == tuple(ref["C"][:, i, j])
    E, _ = ox.row_exponents(A[0])
    F, _ = ox.row_exponents(B[0].T)
    X1, s1 = ox.fixed_product(A[:, :, :17], B[:, :17, :], beta, S, E, F, balanced)
    X2, s2 = ox.fixed_product(A[:, :, 17:], B[:, 17:, :], beta, S, E, F, balanced)
    assert np.array_equal(s1, sc) and np.array_equal(s2, sc)
    assert all(X1[i, j] + X2[i, j] == X[i, j] for i in range(5) for j in range(4))


def test_fixed_limbs():
    assert ox.fixed_limbs(0, 2) == [0, 0]
    assert ox.fixed_limbs(-1, 2) == [0xffffffff, 0xffffffff]
    assert ox.fixed_limbs((1 << 40) + 5, 2) == [5, 256]
    with pytest.raises(ValueError):
        ox.fixed_limbs(1 << 63, 2)


@pytest.mark.parametrize("form,beta,shift", [("int8", 7, 7), ("int8bal", 8, 6), ("fp64", 20, 20)])
def test_fixed_product_one_slice_closed_form(form, beta, shift):
    """With one word and one slice the integer is a plain truncated
    product: X_ij = sum_k t(a_ik) t(b_kj), t(x) = sgn(x) floor(|x|
    2^(shift - E)) with shift = beta (balanced: 8 - 2, the grid starting
    2^2 above E), and scale = E_i + F_j - 2 shift."""
    r = np.random.Generator(np.random.PCG64(77))
    A = np.ldexp(r.uniform(-1, 1, (1, 4, 9)), r.integers(-8, 9, (1, 4, 9)))
    B = np.ldexp(r.uniform(-1, 1, (1, 9, 3)), r.integers(-8, 9, (1, 9, 3)))
    A[0, 1, :] = 0.0
    X, sc = ox.fixed_product(A, B, beta, 1, balanced=form == "int8bal")
    for i in range(4):
        nz = [abs(v) for v in A[0, i] if v != 0]
        Ei = int(max(np.frexp(v)[1] for v in nz)) if nz else 0
        for j in range(3):
            Fj = int(max(np.frexp(abs(v))[1] for v in B[0, :, j] if v != 0))

            def t(x, e):
                q = Fraction(abs(float(x))) * Fraction(2) ** (shift - e)
                return (1 if x >= 0 else -1) * (q.numerator // q.denominator)

            want = sum(t(A[0, i, k], Ei) * t(B[0, k, j], Fj) for k in range(9))
            assert X[i, j] == want, (i, j)
            assert sc[i, j] == Ei + Fj - 2 * shift


def test_log2_fraction_pinned():
    """log2_fraction against exact Fraction arithmetic, not against itself:
    powers of two give their exponent exactly; for any x, writing the
    result as n + f (n an integer) the exact quotient x / 2^n, rounded once
    to a double, has log2 within 1e-12 of f; and 2^(n-1) <= x < 2^(n+2)
    holds exactly, for magnitudes from 2^-3000 to 2^3000."""
    import math
    r = np.random.Generator(np.random.PCG64(4161))
    for k in (-3000, -1075, -1, 0, 1, 52, 53, 1024, 3000):
        assert ox.log2_fraction(Fraction(2) ** k) == k
    for _ in range(400):
        bits_p = int(r.integers(1, 3000))
        bits_q = int(r.integers(1, 3000))
        p = int(r.integers(1, 1 << 62)) << max(bits_p - 62, 0) | int(r.integers(0, 1 << 30))
        q = int(r.integers(1, 1 << 62)) << max(bits_q - 62, 0) | 1
        x = Fraction(p, q)
        v = ox.log2_fraction(x)
        n = math.floor(v)
        f = v - n
        y = x / Fraction(2) ** n                    # exact
        assert abs(math.log2(float(y)) - f) < 1e-12, (v, float(y))
        assert Fraction(2) ** (n - 1) <= x < Fraction(2) ** (n + 2)
    # a planted mistake of one bit in the scaling would be seen
    x = Fraction(3, 1 << 2000)
    assert abs(ox.log2_fraction(x) - (math.log2(3) - 2000)) < 1e-12


@pytest.mark.parametrize("balanced", [False, True])
def test_depth_split_with_rows_zero_in_one_block(balanced):
    """A row of A zero in the first depth block and a column of B zero in
    the second, both with negative whole-depth exponents: on the whole
    depth's grid the blocks' integers are zero there and still add up to
    the whole product's, which rounds to the method's output."""
    m, M, N, K, k0 = 4, 5, 4, 30, 12
    r = np.random.Generator(np.random.PCG64(516))
    A = mdinputs.mdouble(r, m, (M, K), ("log2uniform", 8.0))
    B = mdinputs.mdouble(r, m, (K, N), ("log2uniform", 8.0))
    A[:, 1, :] *= 2.0 ** -20
    B[:, :, 3] *= 2.0 ** -20
    A[:, 1, :k0] = 0.0
    B[:, k0:, 3] = 0.0
    beta, S = (8, 14) if balanced else (7, 16)
    E, _ = ox.row_exponents(A[0])
    F, _ = ox.row_exponents(B[0].T)
    assert E[1] < 0 and F[3] < 0
    # the block's own exponents differ: all-zero (0 by convention)
    Eb, _ = ox.row_exponents(A[0, :, :k0])
    assert Eb[1] == 0 != E[1]
    X, sc = ox.fixed_product(A, B, beta, S, balanced=balanced)
    X1, s1 = ox.fixed_product(A[:, :, :k0], B[:, :k0, :], beta, S, E, F, balanced)
    X2, s2 = ox.fixed_product(A[:, :, k0:], B[:, k0:, :], beta, S, E, F, balanced)
    assert all(X1[1, j] == 0 for j in range(N)) and all(X2[i, 3] == 0 for i in range(M))
    assert np.array_equal(s1, sc) and np.array_equal(s2, sc)
    assert all(X1[i, j] + X2[i, j] == X[i, j] for i in range(M) for j in range(N))
    ref = ox.method_product(A, B, beta, S, balanced=balanced)
    for i in range(M):
        for j in range(N):
            x = Fraction(X[i, j]) * Fraction(2) ** int(sc[i, j])
            assert tuple(ox.renorm_rn(x, m)) == tuple(ref["C"][:, i, j])
