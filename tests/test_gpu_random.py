"""Seeded random parity sweep of the matrix product (needs an MI355X).

48 cases drawn from one seeded generator: slice form (FP64, INT8
sign-magnitude, INT8 balanced), word count m = 1, 2, 4, 8, 16, ragged sizes
(M, N up to 80, K up to 300; smaller for m = 8, 16), transposed operands,
leading words U(-1,1) or 2^U(-r,r) with random signs and r up to 20, the
rho or span rule, and now and then a forced slice count that the form
accepts (the whole-triangle kernels, the banded kernels with the sum
buffer).  Every output word equals the oracle's method layer; under the
library's own rule every entry is also within 2^-T of the exact product.
24 more cases of batched inner products (up to 70 pairs of length up to
400), compared pair by pair with the oracle's method.
"""
import numpy as np
import pytest
import torch

import mdinputs
import paper_2606_20863_amd as md
from oracle import exact as ox

import rulecheck

pytestmark = pytest.mark.gpu

FORMS = ("fp64", "int8", "int8bal")
MS = (1, 2, 4, 8, 16)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def draw_cases(n=48, seed=20863):
    r = np.random.Generator(np.random.PCG64(seed))
    cases = []
    for c in range(n):
        form = FORMS[c % 3]
        m = int(r.choice(MS))
        hi_mn, hi_k = {16: (12, 40), 8: (40, 160)}.get(m, (80, 300))
        M, N = int(r.integers(1, hi_mn + 1)), int(r.integers(1, hi_mn + 1))
        K = int(r.integers(1, hi_k + 1))
        lead = ("uniform",) if r.random() < 0.4 else ("log2uniform", float(r.integers(1, 21)))
        tA, tB = bool(r.random() < 0.3), bool(r.random() < 0.3)
        rule = "span" if r.random() < 0.25 else "rho"
        force = None
        if r.random() < 0.3:
            if form == "fp64":
                beta = int(r.integers(12, 23))
                force = (int(r.integers(2, 12)), beta)
            else:
                beta = 7 if form == "int8" else 8
                S = int(r.integers(1, 33)) if r.random() < 0.7 else int(r.choice([36, 48, 64]))
                force = (S, beta)
        cases.append((c, form, m, M, N, K, lead, tA, tB, rule, force, int(r.integers(0, 2 ** 31))))
    return cases


@pytest.mark.parametrize("case", draw_cases(), ids=lambda c: f"case{c[0]}-{c[1]}-m{c[2]}")
def test_random_case(case):
    _, form, m, M, N, K, lead, tA, tB, rule, force, seed = case
    r = np.random.Generator(np.random.PCG64(seed))
    A = mdinputs.mdouble(r, m, (M, K), lead)
    B = mdinputs.mdouble(r, m, (K, N), lead)
    if M > 2 and r.random() < 0.5:
        A[:, int(r.integers(0, M)), :] = 0.0          # an all-zero row
    Ain = np.ascontiguousarray(np.transpose(A, (0, 2, 1))) if tA else A
    Bin = np.ascontiguousarray(np.transpose(B, (0, 2, 1))) if tB else B
    kw = dict(transA=tA, transB=tB, form=form, rule=rule)
    if force is not None:
        kw.update(force_S=force[0], force_beta=force[1])
    C, info = md.gemm_ex(dev(Ain), dev(Bin), **kw)
    torch.cuda.synchronize()
    C = C.cpu().numpy()
    ref = ox.method_product(A, B, info["beta"], info["S"], balanced=form == "int8bal")
    np.testing.assert_array_equal(C, ref["C"])
    if force is None:
        num, L = ox.exact_product(A, B)
        anum, _ = ox.abs_product(A, B)
        assert max(ox.error_report(C, num, anum, L).values()) <= -ox.TARGET_BITS[m]


def draw_dot_cases(n=24, seed=6144):
    r = np.random.Generator(np.random.PCG64(seed))
    cases = []
    for c in range(n):
        form = FORMS[c % 3]
        m = int(r.choice(MS))
        batch = int(r.integers(1, 71))
        length = int(r.integers(1, 401))
        lead = ("uniform",) if r.random() < 0.4 else ("log2uniform", float(r.integers(1, 17)))
        force = None
        if r.random() < 0.3:
            if form == "fp64":
                force = (int(r.integers(2, 12)), int(r.integers(12, 23)))
            else:
                force = (int(r.integers(1, 33)), 7 if form == "int8" else 8)
        cases.append((c, form, m, batch, length, lead, force, int(r.integers(0, 2 ** 31))))
    return cases


@pytest.mark.parametrize("case", draw_dot_cases(), ids=lambda c: f"dot{c[0]}-{c[1]}-m{c[2]}")
def test_random_dot_case(case):
    """Batched inner products: every output word equals the oracle's method
    on each pair (and the rule's parameters sit within the oracle's budget)."""
    _, form, m, batch, length, lead, force, seed = case
    r = np.random.Generator(np.random.PCG64(seed))
    X = mdinputs.mdouble(r, m, (batch, length), lead)
    Y = mdinputs.mdouble(r, m, (batch, length), lead)
    kw = dict(form=form)
    if force is not None:
        kw.update(force_S=force[0], force_beta=force[1])
    out, info = md.dot_ex(dev(X), dev(Y), **kw)
    torch.cuda.synchronize()
    if force is None:
        rulecheck.check_info(info, form, length, ox.TARGET_BITS[m], ox.dot_G(X, Y))
    _, ref = ox.method_dot(X, Y, info["beta"], info["S"], balanced=form == "int8bal")
    np.testing.assert_array_equal(out.cpu().numpy(), ref)
