"""The ordinary m-double matrix product on the GPU (the paper's comparison
baseline) against the oracle's ordinary arithmetic, through the C ABI
(needs an MI355X).  Both perform the same IEEE operations in the same
order, so every output word must agree; the result is also checked against
the exact product within the ordinary method's own error growth,
K 2^-(52 m - 3) of (|A||B|)_ij.
"""
from fractions import Fraction

import numpy as np
import pytest
import torch

import mdinputs
import paper_2606_20863_amd as md
from oracle import exact as ox
from oracle import mdarith as ma

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("m,name,shape", [(m, name, shape) for m, name in ((1, "dd64"), (2, "dd64"), (4, "qd1024"))
                                          for shape in ((19, 21, 70), (16, 16, 32), (1, 1, 1), (33, 5, 97))]
                         + [(8, "od1024", shape) for shape in ((7, 5, 33), (1, 1, 1), (4, 3, 70))])
def test_ordinary_bitexact(m, name, shape):
    M, N, K = shape
    A, B = mdinputs.workload(name, M=M, N=N, K=K)
    A, B = np.ascontiguousarray(A[:m]), np.ascontiguousarray(B[:m])
    C = host(md.gemm_ordinary(dev(A), dev(B)))
    np.testing.assert_array_equal(C, ma.ordinary_gemm(A, B))
    num, L = ox.exact_product(A, B)
    anum, _ = ox.abs_product(A, B)
    rep = ox.error_report(C, num, anum, L)
    assert max(rep.values()) <= np.log2(K) - (52 * m - 3)


def test_ordinary_qd_sampled_256():
    A, B = mdinputs.workload("qd4096", M=256, N=256, K=256)
    C = host(md.gemm_ordinary(dev(A), dev(B)))
    rows = [0, 77, 255]
    cols = [3, 128, 250]
    np.testing.assert_array_equal(C[:, rows][:, :, cols], ma.ordinary_gemm(A, B, rows, cols))


def test_ordinary_degenerate():
    Z = torch.full((4, 3, 5), 2.0, dtype=torch.float64, device="cuda")
    C = md.gemm_ordinary(torch.zeros((4, 3, 0), dtype=torch.float64, device="cuda"),
                         torch.zeros((4, 0, 5), dtype=torch.float64, device="cuda"))
    assert np.all(host(C) == 0.0)
    L = md.lib()
    assert L.md_gemm_ordinary(16, 4, 4, 4, None, None, None, None) == 1
    assert L.md_dot_ordinary(32, 4, 4, None, None, None, None) == 1
    assert L.md_dot_ordinary(3, 4, 4, None, None, None, None) == 1
    del Z


@pytest.mark.parametrize("m", [1, 2, 4, 8, 16])
def test_ordinary_dot_bitexact_ragged(m):
    """Batched ordinary inner products against the oracle's lane-order
    definition, every output word; lengths below, at and above one word per
    lane, a zero vector, and the exact value within K 2^-(52m-3) (smaller
    batches for the hexa-doubles, whose oracle runs in Python)."""
    r = np.random.Generator(np.random.PCG64(800 + m))
    for batch, n in (((3, 1), (4, 64), (3, 150)) if m == 16 else ((5, 1), (9, 64), (7, 333))):
        X = mdinputs.mdouble(r, m, (batch, n), ("log2uniform", 8.0))
        Y = mdinputs.mdouble(r, m, (batch, n), ("log2uniform", 8.0))
        X[:, 1, :] = 0.0
        out = host(md.dot_ordinary(dev(X), dev(Y)))
        for b in range(batch):
            xs = [tuple(X[:, b, k]) for k in range(n)]
            ys = [tuple(Y[:, b, k]) for k in range(n)]
            ref = ma.ordinary_dot_lanes(ma.Counter(), xs, ys, m)
            assert tuple(out[:, b]) == tuple(ref), (batch, n, b)
            exact = sum(ox.entry_value(x) * ox.entry_value(y) for x, y in zip(xs, ys))
            absum = sum(abs(ox.entry_value(x) * ox.entry_value(y)) for x, y in zip(xs, ys))
            assert abs(ox.entry_value(out[:, b]) - exact) <= n * Fraction(2) ** -(52 * m - 3) * absum
        assert np.all(out[:, 1] == 0.0)


@pytest.mark.parametrize("m", [1, 2, 4, 8])
def test_ordinary_dot_paper_workload_sampled(m):
    """The paper's experiment in ordinary arithmetic: 1,024 pairs of length
    6,144 on its bit pattern; 4 sampled pairs bit-exact against the oracle's
    lane order."""
    X, Y = mdinputs.paper_dot_workload(m)
    out = host(md.dot_ordinary(dev(X), dev(Y)))
    for b in ((0, 401, 1023) if m < 8 else (777,)):
        xs = [tuple(X[:, b, k]) for k in range(X.shape[2])]
        ys = [tuple(Y[:, b, k]) for k in range(X.shape[2])]
        assert tuple(out[:, b]) == tuple(ma.ordinary_dot_lanes(ma.Counter(), xs, ys, m)), b
