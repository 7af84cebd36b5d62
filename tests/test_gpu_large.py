"""Shapes past one launch's second grid dimension (needs an MI355X).

The splits, the magnitude product and the inner-product contraction put
row (or pair) blocks of 16 on the grid's second dimension, at most 65535
per launch; beyond 1,048,560 rows the launchers issue several launches.
A product with 1,050,000 rows and a batch of 1,100,000 inner products,
both with the rule choosing S (so the magnitude certificate runs over every
row) and with S forced: rows or pairs are independent once S is fixed, so
sampled ones, including the last, equal the oracle's method on those rows
or pairs alone.
"""
import numpy as np
import pytest
import torch

import paper_2606_20863_amd as md
from oracle import exact as ox

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("form", ["int8bal", "fp64"])
def test_product_with_more_row_blocks_than_one_launch(form):
    r = np.random.Generator(np.random.PCG64(1))
    M, N, K = 1_050_000, 3, 64
    A = r.uniform(-1, 1, (1, M, K))
    B = r.uniform(-1, 1, (1, K, N))
    Ad, Bd = dev(A), dev(B)
    C, info = md.gemm_ex(Ad, Bd, form=form)
    Cf, _ = md.gemm_ex(Ad, Bd, form=form, force_S=info["S"], force_beta=info["beta"])
    torch.cuda.synchronize()
    assert torch.equal(C, Cf)
    rows = np.array([0, 1, 524_287, 1_048_559, 1_048_560, 1_048_575, 1_048_576, M - 1], dtype=np.int64)
    ref = ox.method_product(A[:, rows, :], B, info["beta"], info["S"], balanced=form == "int8bal")
    np.testing.assert_array_equal(C[:, torch.from_numpy(rows).cuda(), :].cpu().numpy(), ref["C"])


@pytest.mark.parametrize("form", ["int8bal", "fp64"])
def test_inner_products_with_more_pair_blocks_than_one_launch(form):
    r = np.random.Generator(np.random.PCG64(2))
    batch, n = 1_100_000, 64
    X = r.uniform(-1, 1, (1, batch, n))
    Y = r.uniform(-1, 1, (1, batch, n))
    out, info = md.dot_ex(dev(X), dev(Y), form=form)
    torch.cuda.synchronize()
    pairs = np.array([0, 7, 1_048_559, 1_048_560, 1_048_576, batch - 1], dtype=np.int64)
    _, ref = ox.method_dot(X[:, pairs, :], Y[:, pairs, :], info["beta"], info["S"],
                           balanced=form == "int8bal")
    np.testing.assert_array_equal(out[:, torch.from_numpy(pairs).cuda()].cpu().numpy(), ref)
