"""The m-double adjoint behind torch.autograd.Function (needs an MI355X).

The loss is sum(W * C) with C = A B, so the exact gradients are
dA* = W B^T and dB* = A^T W (bilinear).  Checks:

* small shapes: both gradients bit-exact against the oracle's method layer
  on (W, B^T) and (A^T, W) at the library's parameters (checked against
  the budget);
* double-double 2048^3 (FP64 form): 64 sampled entries of dA and of dB
  within 2^-100 of (|W||B^T|) and (|A^T||W|) of the exact gradient, and
  against quad-double central differences with step 2^-40 (the perturbed
  row or column of C recomputed as a quad-double product; the loss sums
  exact);
* octo-double 1024^3 (both INT8 forms): 64 sampled entries of each gradient
  within 2^-400 of the exact gradient (central differences cannot resolve
  2^-400).
"""
from fractions import Fraction

import numpy as np
import pytest
import torch

import mdinputs
import paper_2606_20863_amd as md
from oracle import coracle
from oracle import exact as ox

import rulecheck

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rule_G(X, Y):
    """The ratio exponent G the rule certifies for X Y (the oracle's span
    and magnitude certificates)."""
    _, sx = ox.row_exponents(X[0])
    _, sy = ox.row_exponents(Y[0].T)
    G = ox.span_G(max(sx), max(sy))
    _, g_rho = ox.rho_G(X, Y)
    if g_rho is not None:
        G = min(G, g_rho)
    return G


def tr(X):
    return np.ascontiguousarray(np.transpose(X, (0, 2, 1)))


@pytest.mark.parametrize("form,name", [("fp64", "dd64"), ("int8", "dd64"), ("int8", "qd1024"),
                                       ("fp64", "od1024"), ("int8bal", "qd1024"),
                                       ("int8bal", "od1024")])
def test_adjoint_small_bitexact(form, name):
    A, B, W = mdinputs.workload(name, M=23, N=31, K=40, with_w=True)
    m = A.shape[0]
    T = ox.TARGET_BITS[m]
    tA = dev(A).requires_grad_(True)
    tB = dev(B).requires_grad_(True)
    C = md.MDGemm.apply(tA, tB, form)
    C.backward(dev(W))
    dA, dB = host(tA.grad), host(tB.grad)
    bal = form == "int8bal"
    # the library's parameters for each backward product (its host rule on
    # the oracle's certified G), checked against the budget
    for X, Y, got in ((W, tr(B), dA), (tr(A), W, dB)):
        G = rule_G(X, Y)
        beta, S, kc, band = md.choose_params(form, X.shape[2], T, G)
        rulecheck.check_params(form, X.shape[2], T, G, beta, S, kc, band)
        np.testing.assert_array_equal(got, ox.method_product(X, Y, beta, S, balanced=bal)["C"])
    # and within 2^-T of the exact gradients
    (ga, La), (gb, Lb) = ox.exact_gradients(A, B, W)
    ab, _ = ox.abs_product(W, tr(B))
    assert max(ox.error_report(dA, ga, ab, La).values()) <= -T
    ab, _ = ox.abs_product(tr(A), W)
    assert max(ox.error_report(dB, gb, ab, Lb).values()) <= -T


def sample(n, hi, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, hi, size=n)


def grad_errors(X, Y, G, ii, jj):
    """log2(|G_ij - (X Y)_ij| / (|X||Y|)_ij) for the sampled entries."""
    Gq = np.ascontiguousarray(G[:, ii, jj].T)
    _, absab, err = coracle.exact_entries(X, Y, ii, jj, Gq)
    return np.log2(np.maximum(np.abs(err), 2.0 ** -1074) / absab)


def as_qd(X):
    out = np.zeros((4,) + X.shape[1:])
    out[:X.shape[0]] = X
    return out


def test_dd2048_forward_adjoint_fp64():
    A, B, W = mdinputs.workload("dd2048", with_w=True)
    M, K = A.shape[1], A.shape[2]
    N = B.shape[2]
    tA = dev(A).requires_grad_(True)
    tB = dev(B).requires_grad_(True)
    C = md.MDGemm.apply(tA, tB, "fp64")
    C.backward(dev(W))
    Ch, dA, dB = host(C), host(tA.grad), host(tB.grad)
    # forward, 64 sampled entries
    ii, jj = sample(64, M, 1), sample(64, N, 2)
    assert np.max(grad_errors(A, B, Ch, ii, jj)) <= -100
    # gradients against the exact ones
    ia, ka = sample(64, M, 3), sample(64, K, 4)
    kb, jb = sample(64, K, 5), sample(64, N, 6)
    ea = grad_errors(W, tr(B), dA, ia, ka)
    eb = grad_errors(tr(A), W, dB, kb, jb)
    assert np.max(ea) <= -100 and np.max(eb) <= -100
    # quad-double central differences, step 2^-40, on all 64 sampled
    # entries of dA and of dB.  A perturbed row of A changes one row of C
    # (its own exponent, its own products), so the 128 perturbed rows go
    # through one quad-double product; likewise the perturbed columns of B.
    h = Fraction(1, 1 << 40)
    Wv = [[None] * N for _ in range(M)]

    def w(i, j):
        if Wv[i][j] is None:
            Wv[i][j] = ox.entry_value(W[:, i, j])
        return Wv[i][j]

    rows = np.zeros((4, 128, K))
    for e, (i, k) in enumerate(zip(ia, ka)):
        for q, sgn in enumerate((1, -1)):
            rows[:2, 2 * e + q] = A[:, i]
            rows[:, 2 * e + q, k] = ox.renorm_rn(ox.entry_value(A[:, i, k]) + sgn * h, 4)
    Cr = host(md.gemm_ex(dev(rows), dev(as_qd(B)), form="fp64")[0])
    _, abs_a, _ = coracle.exact_entries(W, tr(B), ia, ka)
    for e, (i, k) in enumerate(zip(ia, ka)):
        Lp = sum(w(i, j) * ox.entry_value(Cr[:, 2 * e, j]) for j in range(N))
        Lm = sum(w(i, j) * ox.entry_value(Cr[:, 2 * e + 1, j]) for j in range(N))
        fd = (Lp - Lm) / (2 * h)
        diff = abs(fd - ox.entry_value(dA[:, i, k]))
        assert diff <= Fraction(abs_a[e]) * Fraction(1, 1 << 99), (i, k)
    cols = np.zeros((4, K, 128))
    for e, (k, j) in enumerate(zip(kb, jb)):
        for q, sgn in enumerate((1, -1)):
            cols[:2, :, 2 * e + q] = B[:, :, j]
            cols[:, k, 2 * e + q] = ox.renorm_rn(ox.entry_value(B[:, k, j]) + sgn * h, 4)
    Cc = host(md.gemm_ex(dev(as_qd(A)), dev(cols), form="fp64")[0])
    _, abs_b, _ = coracle.exact_entries(tr(A), W, kb, jb)
    for e, (k, j) in enumerate(zip(kb, jb)):
        Lp = sum(w(i, j) * ox.entry_value(Cc[:, i, 2 * e]) for i in range(M))
        Lm = sum(w(i, j) * ox.entry_value(Cc[:, i, 2 * e + 1]) for i in range(M))
        fd = (Lp - Lm) / (2 * h)
        diff = abs(fd - ox.entry_value(dB[:, k, j]))
        assert diff <= Fraction(abs_b[e]) * Fraction(1, 1 << 99), (k, j)


@pytest.mark.parametrize("form", ["int8", "int8bal"])
def test_od1024_forward_adjoint_int8(form):
    A, B, W = mdinputs.workload("od1024", with_w=True)
    M, K = A.shape[1], A.shape[2]
    N = B.shape[2]
    tA = dev(A).requires_grad_(True)
    tB = dev(B).requires_grad_(True)
    C = md.MDGemm.apply(tA, tB, form)
    C.backward(dev(W))
    Ch, dA, dB = host(C), host(tA.grad), host(tB.grad)
    ii, jj = sample(64, M, 7), sample(64, N, 8)
    assert np.max(grad_errors(A, B, Ch, ii, jj)) <= -400
    ia, ka = sample(64, M, 9), sample(64, K, 10)
    kb, jb = sample(64, K, 11), sample(64, N, 12)
    assert np.max(grad_errors(W, tr(B), dA, ia, ka)) <= -400
    assert np.max(grad_errors(tr(A), W, dB, kb, jb)) <= -400
    for i, j in zip(ii[:8], jj[:8]):
        assert ox.is_nonoverlapping(Ch[:, i, j], strong=True)
