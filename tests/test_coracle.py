"""The C oracle against the pinned Python oracle (same definitions, written
independently), on inputs small enough for exact Python arithmetic."""
from fractions import Fraction

import numpy as np
import pytest

import mdinputs
from oracle import coracle
from oracle import exact as ox


@pytest.mark.parametrize("name", ["dd64", "qd1024", "od1024"])
def test_exact_entries_match_python(name):
    A, B = mdinputs.workload(name, M=5, N=4, K=9)
    m = A.shape[0]
    A[:, 1, :] = 0.0                        # an all-zero row
    num, L = ox.exact_product(A, B)
    anum, _ = ox.abs_product(A, B)
    ii, jj = np.meshgrid(np.arange(5), np.arange(4), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    # a perturbed result to measure: the exact product rounded, last word off
    Crn, absab, _ = coracle.exact_entries(A, B, ii, jj)
    Cq = Crn.copy()
    Cq[:, m - 1] *= 1.5
    _, _, err = coracle.exact_entries(A, B, ii, jj, Cq)
    for e, (i, j) in enumerate(zip(ii, jj)):
        x = Fraction(int(num[i, j]), 1 << L)
        assert list(Crn[e]) == ox.renorm_rn(x, m)
        assert absab[e] == ox.round_nearest(Fraction(int(anum[i, j]), 1 << L))
        assert err[e] == ox.round_nearest(x - ox.entry_value(Cq[e]))


@pytest.mark.parametrize("name,beta,S", [("dd64", 22, 5), ("dd64", 7, 16), ("qd1024", 7, 33),
                                         ("qd1024", 19, 12), ("od1024", 7, 64)])
def test_method_entries_match_python(name, beta, S):
    A, B = mdinputs.workload(name, M=6, N=7, K=40)
    rows, cols = [0, 3, 5], [1, 2, 6]
    E, F, D, C = coracle.method_entries(A, B, beta, S, rows, cols)
    ref = ox.method_product(A, B, beta, S, rows=rows, cols=cols)
    assert list(E) == ref["E"] and list(F) == ref["F"]
    np.testing.assert_array_equal(np.transpose(D, (2, 0, 1)), ref["D"])
    np.testing.assert_array_equal(C, ref["C"])


def test_exponents_match_python():
    A, B = mdinputs.workload("od1024", M=9, N=11, K=30)
    A[0, 4, :] = 0.0
    E, span = coracle.exponents(A[0], by_columns=False)
    Er, sr = ox.row_exponents(A[0])
    assert list(E) == Er and list(span) == sr
    F, spanF = coracle.exponents(B[0], by_columns=True)
    Fr, sfr = ox.row_exponents(B[0].T)
    assert list(F) == Fr and list(spanF) == sfr


@pytest.mark.parametrize("name,S", [("dd64", 5), ("dd64", 14), ("qd1024", 27), ("qd1024", 33),
                                    ("od1024", 52), ("od1024", 70)])
def test_method_entries_balanced_match_python(name, S):
    """The C oracle's balanced 8-bit digits (recoding of the truncated
    integer, grids at 2^(E+2)) against the Python oracle's, on ragged
    shapes, with leading words just below 2^E (the largest digit the
    headroom admits) and an all-zero row and column."""
    A, B = mdinputs.workload(name, M=7, N=6, K=45)
    A[:, 2, :] = 0.0
    B[:, :, 4] = 0.0
    E, _ = ox.row_exponents(A[0])
    F, _ = ox.row_exponents(B[0].T)
    for i, k in ((0, 3), (5, 44), (6, 0)):
        A[:, i, k] = 0.0
        A[0, i, k] = np.nextafter(2.0 ** E[i], 0.0) * (-1) ** k
    for k, j in ((7, 1), (44, 5)):
        B[:, k, j] = 0.0
        B[0, k, j] = -np.nextafter(2.0 ** F[j], 0.0)
    rows, cols = [0, 2, 5, 6], [1, 3, 4, 5]
    E, F, D, C = coracle.method_entries(A, B, 8, S, rows, cols, balanced=True)
    ref = ox.method_product(A, B, 8, S, rows=rows, cols=cols, balanced=True)
    assert list(E) == ref["E"] and list(F) == ref["F"]
    assert np.abs(ref["dA"]).max() == 128 or S == 5       # the digit range is reached
    np.testing.assert_array_equal(np.transpose(D, (2, 0, 1)), ref["D"])
    np.testing.assert_array_equal(C, ref["C"])
