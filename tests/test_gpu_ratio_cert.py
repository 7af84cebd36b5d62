"""The ratio certificate's magnitude product, min_ij P_ij with P = q_A q_B
(q the 7-bit magnitude digit of each leading word on its row's or column's
exponent), for products of 4096^2 outputs and more (256 x 256 outputs per
workgroup) and below (128 x 128), ragged edges included (needs an MI355X).

The library's G_rho equals the oracle's, and a single pair with P_ij = 0
planted anywhere (corners, tile edges, the ragged last row and column)
makes the certificate unavailable (G_rho = -1): every output is examined.
Leading words within a factor of two of each other keep every other P_ij
positive.
"""
import numpy as np
import pytest
import torch

import mdinputs
import paper_2606_20863_amd as md
from oracle import exact as ox

pytestmark = pytest.mark.gpu

K = 64
SHAPES = [(4096, 4096), (4100, 4097), (1000, 700)]


def operands(M, N, seed, K=K):
    r = np.random.Generator(np.random.PCG64(seed))
    A = mdinputs.mdouble(r, 2, (M, K), ("log2uniform", 0.5))
    B = mdinputs.mdouble(r, 2, (K, N), ("log2uniform", 0.5))
    return A, B


def g_rho(A, B):
    _, info = md.gemm_ex(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), form="int8bal", rule="rho")
    return info["G_rho"]


@pytest.mark.parametrize("M,N", SHAPES)
def test_ratio_certificate_equals_oracle(M, N):
    print(f"[ratio cert] {M} x {N} x {K}", flush=True)
    A, B = operands(M, N, 31 + M + N)
    _, G = ox.rho_G(A, B)
    assert G is not None
    assert g_rho(A, B) == G


@pytest.mark.parametrize("M,N,K", [(M, N, K) for M, N in SHAPES] + [(4096, 4096, 576), (1000, 700, 576)])
def test_ratio_certificate_sees_a_zero_pair_anywhere(M, N, K):
    """Depth 64 (one depth step) and 576 (nine, an odd count against the
    wide tile's two steps in flight)."""
    A, B = operands(M, N, 57 + M + N, K)
    assert g_rho(A, B) >= 0
    k0, k1 = 3, 40
    spots = [(0, 0), (M - 1, N - 1), (0, N - 1), (M - 1, 0), (255, 256), (256, 255), (M // 2 + 3, N // 3 + 5)]
    for i, j in spots:
        print(f"[ratio cert] {M} x {N} x {K}: zero pair at ({i}, {j})", flush=True)
        A2, B2 = A.copy(), B.copy()
        # row i keeps a nonzero magnitude digit at depth k0 only, column j at
        # k1 only, so P_ij = 0 (scaling by 2^-20 keeps the words valid)
        A2[:, i, np.arange(K) != k0] *= 2.0 ** -20
        B2[:, np.arange(K) != k1, j] *= 2.0 ** -20
        assert g_rho(A2, B2) == -1, (i, j)
