"""Seeded sweep of the production path (no debug buffers, the slice rule
chooses S) over ragged shapes, word counts, the three slice forms, all four
operand orientations, wide exponent ranges and rows or columns that are all
zero.  Every output word equals the oracle's method layer at the (beta, S)
the call reports (the C oracle, bit for bit: greedy round-to-nearest of the
exact truncated sum is unique, Section 2), and sampled entries meet the
call's certified bound against the exact product.
"""
import numpy as np
import pytest
import torch

import mdinputs
import paper_2606_20863_amd as md
from oracle import coracle
from oracle import exact as ox

pytestmark = pytest.mark.gpu

FORMS = ("int8bal", "int8", "fp64")


def case(seed, deep=False):
    """(rng, m, form, M, N, K, transA, transB, lead, zero rows of A, zero
    columns of B); deep: few outputs over a depth of several exactness
    chunks of the INT8 forms."""
    rng = np.random.Generator(np.random.PCG64((7000 if deep else 5000) + seed))
    m = int(rng.choice([2, 4] if deep else [1, 2, 4, 8, 16]))
    form = FORMS[seed % 3]
    hi = 25 if deep else (41 if m == 16 else 97)
    M, N = (int(x) for x in rng.integers(1, hi, size=2))
    K = int(rng.integers(4500, 9000) if deep else rng.integers(1, 420))
    transA, transB = bool(rng.integers(2)), bool(rng.integers(2))
    lead = ("uniform",) if rng.integers(2) else ("log2uniform", float(rng.integers(4, 30)))
    zr = rng.choice(M, size=min(M, int(rng.integers(0, 3))), replace=False)
    zc = rng.choice(N, size=min(N, int(rng.integers(0, 3))), replace=False)
    return rng, m, form, M, N, K, transA, transB, lead, zr, zc


def run_case(seed, deep):
    rng, m, form, M, N, K, transA, transB, lead, zr, zc = case(seed, deep)
    print(f"[sweep] seed {seed} deep={deep}: m={m} {form} M={M} N={N} K={K} transA={transA} "
          f"transB={transB} lead={lead}", flush=True)
    A = mdinputs.mdouble(rng, m, (M, K), lead)
    B = mdinputs.mdouble(rng, m, (K, N), lead)
    A[:, zr, :] = 0.0
    B[:, :, zc] = 0.0
    Ap = np.ascontiguousarray(np.transpose(A, (0, 2, 1))) if transA else A
    Bp = np.ascontiguousarray(np.transpose(B, (0, 2, 1))) if transB else B
    C, info = md.gemm_ex(torch.from_numpy(Ap).cuda(), torch.from_numpy(Bp).cuda(), transA=transA,
                         transB=transB, form=form)
    torch.cuda.synchronize()
    C = C.cpu().numpy()
    assert C.shape == (m, M, N)
    beta, S = info["beta"], info["S"]
    print(f"[sweep]   S={S} beta={beta} kc={info['kc']}", flush=True)
    _, _, _, ref = coracle.method_entries(A, B, beta, S, np.arange(M), np.arange(N),
                                          balanced=(form == "int8bal"))
    np.testing.assert_array_equal(C, ref)
    assert not C[:, zr, :].any() and not C[:, :, zc].any()
    # the certified bound on sampled entries against the exact product
    n = min(M * N, 200)
    flat = rng.choice(M * N, size=n, replace=False)
    ii, jj = flat // N, flat % N
    Cq = np.transpose(C[:, ii, jj])
    _, absab, err = coracle.exact_entries(A, B, ii, jj, Cq)
    nz = absab > 0
    assert not err[~nz].any()
    if nz.any():
        worst = float(np.max(np.log2(np.maximum(np.abs(err[nz]), 2.0 ** -1074) / absab[nz])))
        assert worst <= info["log2_bound"] + 1e-9
        assert worst <= -ox.TARGET_BITS[m]


@pytest.mark.parametrize("seed", range(90))
def test_rule_path_sweep(seed):
    run_case(seed, False)


@pytest.mark.parametrize("seed", range(12))
def test_rule_path_sweep_deep(seed):
    """Depths of 4,500-9,000: beyond one exactness chunk of the quad-double
    INT8 forms (S K 127^2 < 2^31 holds to K = 4416 at S = 30), where the
    kernels carry their fold between chunks."""
    run_case(seed, True)
