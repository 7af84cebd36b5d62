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


@pytest.mark.parametrize("m,name", [(1, "dd64"), (2, "dd64"), (4, "qd1024")])
@pytest.mark.parametrize("shape", [(19, 21, 70), (16, 16, 32), (1, 1, 1), (33, 5, 97)])
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
    assert L.md_gemm_ordinary(8, 4, 4, 4, None, None, None, None) == 1
    del Z
