"""Run-to-run bit identity and failure without side effects (needs an
MI355X).

The same product, repeated, on another stream, and with a caller workspace
instead of the library's pool, gives bit-identical words in every form and
through every kernel family (whole triangle, bands with the sum buffer,
FP64 LDS fold; the batched inner products, whose partial sums meet in
integer atomics).  A workspace too small for the digit planes (but large
enough for the first scratch blocks) fails with MD_ENOMEM and leaves C as
it was.
"""
import numpy as np
import pytest
import torch

import mdinputs
import paper_2606_20863_amd as md

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("form,m", [("int8bal", 4), ("int8", 4), ("fp64", 4), ("int8bal", 8), ("fp64", 16)])
def test_repeated_products_are_bit_identical(form, m):
    r = np.random.Generator(np.random.PCG64(31 + m))
    M, N, K = 150, 140, 520
    A = dev(mdinputs.mdouble(r, m, (M, K), ("log2uniform", 6.0)))
    B = dev(mdinputs.mdouble(r, m, (K, N), ("log2uniform", 6.0)))
    C0, info = md.gemm_ex(A, B, form=form)
    runs = [md.gemm_ex(A, B, form=form)[0] for _ in range(3)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        runs.append(md.gemm_ex(A, B, form=form, stream=side)[0])
    torch.cuda.current_stream().wait_stream(side)
    ws = torch.empty(md.lib().md_gemm_workspace_size(md._FORMS[form], M, N, K, info["S"]), dtype=torch.uint8,
                     device="cuda")
    runs.append(md.gemm_ex(A, B, form=form, workspace=ws)[0])
    torch.cuda.synchronize()
    for C in runs:
        assert torch.equal(C, C0)


@pytest.mark.parametrize("form", ["int8bal", "int8", "fp64"])
def test_repeated_inner_products_are_bit_identical(form):
    X, Y = mdinputs.paper_dot_workload(4, batch=300, n=2000)
    Xd, Yd = dev(X), dev(Y)
    out0, _ = md.dot_ex(Xd, Yd, form=form)
    for _ in range(3):
        out, _ = md.dot_ex(Xd, Yd, form=form)
        torch.cuda.synchronize()
        assert torch.equal(out, out0)


@pytest.mark.parametrize("form", ["int8bal", "fp64"])
def test_too_small_workspace_leaves_C_untouched(form):
    r = np.random.Generator(np.random.PCG64(5))
    M, N, K, m = 64, 48, 200, 2
    A = dev(mdinputs.mdouble(r, m, (M, K)))
    B = dev(mdinputs.mdouble(r, m, (K, N)))
    C = torch.full((m, M, N), 7.0, dtype=torch.float64, device="cuda")
    small = torch.empty(64 * 1024, dtype=torch.uint8, device="cuda")   # the exponent scratch fits, digits do not
    with pytest.raises(md.MDError) as e:
        md.gemm_ex(A, B, C, form=form, workspace=small)
    assert e.value.code == 5
    torch.cuda.synchronize()
    assert bool((C == 7.0).all())
