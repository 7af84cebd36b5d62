"""md_gemm_ex_noalloc, the entry point for callers that cannot allocate
(needs an MI355X).

Through the C ABI, against md_gemm_ex on the same inputs, word for word:
two (or three) calls in a row on one device, the later ones smaller, in the
three slice forms, through the whole-triangle, banded (sum buffer) and FP64
kernels, with the slice rule, a forced S and a hint; a product whose scratch
exceeds the library's array is refused with MD_ENOMEM and C untouched.
"""
import numpy as np
import pytest
import torch

import mdinputs
import paper_2606_20863_amd as md

pytestmark = pytest.mark.gpu


def operands(seed, m, M, N, K):
    r = np.random.Generator(np.random.PCG64(seed))
    lead = ("log2uniform", 8.0) if m >= 8 else ("uniform",)
    A = mdinputs.mdouble(r, m, (M, K), lead)
    B = mdinputs.mdouble(r, m, (K, N), lead)
    return torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()


def both(A, B, **kw):
    """(noalloc C, md_gemm_ex C, noalloc info, md_gemm_ex info)."""
    m, M, N = A.shape[0], A.shape[1], B.shape[2]
    C = torch.full((m, M, N), 3.0, dtype=torch.float64, device="cuda")
    C, i1 = md.gemm_ex(A, B, C, noalloc=True, **kw)
    C2, i2 = md.gemm_ex(A, B, **kw)
    torch.cuda.synchronize()
    return C, C2, i1, i2


@pytest.mark.parametrize("form", ["int8bal", "int8", "fp64"])
def test_noalloc_equals_gemm_ex_two_calls(form):
    # first call: quad-double 200 x 180 x 300 with the slice rule
    A, B = operands(1, 4, 200, 180, 300)
    C, Cr, i1, i2 = both(A, B, form=form)
    assert i1["S"] == i2["S"] and torch.equal(C, Cr)
    # second call, smaller: double-double 40 x 30 x 70 with a forced S
    A, B = operands(2, 2, 40, 30, 70)
    S, beta = {"int8bal": (14, 8), "int8": (16, 7), "fp64": (5, 22)}[form]
    C, Cr, _, _ = both(A, B, form=form, force_S=S, force_beta=beta)
    assert torch.equal(C, Cr)
    # third call, smaller still, on a slice-count hint
    A, B = operands(3, 2, 17, 9, 33)
    _, info = md.gemm_ex(A, B, form=form)
    cert = md.new_cert()
    C, Cr, _, _ = both(A, B, form=form, s_hint=info["S"], force_beta=info["beta"] if form == "fp64" else 0,
                       cert=cert)
    assert torch.equal(C, Cr)
    assert md.read_cert(cert)["flags"] == 0


def test_noalloc_banded_then_smaller_triangle():
    """Octo-doubles through the banded kernels and their sum buffer (in the
    array), then a smaller whole-triangle product: the buffer's old
    contents do not leak into either."""
    A, B = operands(4, 8, 100, 90, 130)
    C, Cr, i1, _ = both(A, B, form="int8bal")
    assert i1["S"] > 32 and torch.equal(C, Cr)
    A, B = operands(5, 4, 60, 50, 64)
    C, Cr, i1, _ = both(A, B, form="int8bal")
    assert i1["S"] <= 32 and torch.equal(C, Cr)


def test_noalloc_refuses_products_beyond_the_array():
    """Quad-double 1536^3 in the balanced form needs about 130 MB of digit
    scratch, above the 64 MiB array: MD_ENOMEM, C untouched; a call after
    it still works."""
    A, B = operands(6, 4, 1536, 1536, 1536)
    need = md.lib().md_gemm_workspace_size(md._FORMS["int8bal"], 1536, 1536, 1536, 27)
    assert need > 64 << 20
    C = torch.full((4, 1536, 1536), 3.0, dtype=torch.float64, device="cuda")
    with pytest.raises(md.MDError) as err:
        md.gemm_ex(A, B, C, form="int8bal", force_S=27, force_beta=8, noalloc=True)
    assert err.value.code == 5
    with pytest.raises(md.MDError) as err:
        md.gemm_ex(A, B, C, form="int8bal", noalloc=True)
    assert err.value.code == 5
    torch.cuda.synchronize()
    assert bool((C == 3.0).all())
    A, B = operands(7, 4, 64, 64, 64)
    C, Cr, _, _ = both(A, B, form="int8bal")
    assert torch.equal(C, Cr)
