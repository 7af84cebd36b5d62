"""Validation mode (md_opts.validate) on the GPU: the library's check of the
input preconditions against the oracle's ``precondition_flags`` (needs an
MI355X).

* valid inputs (the generated workloads, including weakly but not strongly
  nonoverlapping entries): MD_OK, flags 0, outputs equal to a call without
  validation;
* one planted violation at a time, in A or in B (transposed or not), and in
  the inner products' X or Y: MD_EINPUT, the flags equal the OR of the
  oracle's flags over all entries, and the output is left untouched.
"""
import numpy as np
import pytest
import torch

import mdinputs
import paper_2606_20863_amd as md
from oracle import exact as ox

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def oracle_flags(*mats):
    f = 0
    for X in mats:
        m, R, K = X.shape
        for i in range(R):
            for k in range(K):
                f |= ox.precondition_flags(X[:, i, k])
    return f


PLANTS = {
    "nan": lambda X: X.__setitem__((0, 2, 3), np.nan),
    "inf": lambda X: X.__setitem__((1, 0, 0), np.inf),
    "overlap": lambda X: X.__setitem__((1, 4, 5), X[0, 4, 5]),
    "zero_gap": lambda X: (X.__setitem__((1, 3, 1), 0.0), X.__setitem__((2, 3, 1), 2.0 ** -200)),
    "range": lambda X: X.__setitem__((slice(None), 1, 2), np.array([2.0 ** 950, 0.0, 0.0, 0.0])),
    "subnormal": lambda X: X.__setitem__((slice(None), 5, 0), np.array([2.0 ** -1060, 0.0, 0.0, 0.0])),
}


@pytest.mark.parametrize("form", ["fp64", "int8", "int8bal"])
def test_valid_inputs_pass(form):
    A, B = mdinputs.workload("qd1024", M=37, N=29, K=70)
    # weakly but not strongly nonoverlapping entry: still valid
    A[:, 0, 0] = [1.0 + 2.0 ** -40, 2.0 ** -41, 0.0, 0.0]
    ref, _ = md.gemm_ex(dev(A), dev(B), form=form)
    C, info = md.gemm_ex(dev(A), dev(B), form=form, validate=True)
    torch.cuda.synchronize()
    assert info["input_flags"] == 0
    np.testing.assert_array_equal(C.cpu().numpy(), ref.cpu().numpy())


@pytest.mark.parametrize("where", ["A", "B", "Bt"])
@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_planted_violation(plant, where):
    A, B = mdinputs.workload("qd1024", M=12, N=10, K=9)
    PLANTS[plant](A if where == "A" else B)
    want = oracle_flags(A, B)
    assert want != 0
    Bin = np.ascontiguousarray(np.transpose(B, (0, 2, 1))) if where == "Bt" else B
    C = torch.full((4, 12, 10), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(md.MDError) as e:
        md.gemm_ex(dev(A), dev(Bin), C, transB=where == "Bt", form="int8bal", validate=True)
    assert e.value.code == 9
    assert e.value.input_flags == want
    torch.cuda.synchronize()
    assert np.all(C.cpu().numpy() == 7.0)


@pytest.mark.parametrize("plant", ["nan", "overlap", "range"])
def test_dot_validation(plant):
    r = np.random.Generator(np.random.PCG64(3))
    X = mdinputs.mdouble(r, 4, (8, 12), ("log2uniform", 4.0))
    Y = mdinputs.mdouble(r, 4, (8, 12), ("log2uniform", 4.0))
    _, info = md.dot_ex(dev(X), dev(Y), validate=True)
    assert info["input_flags"] == 0
    PLANTS[plant](Y)
    want = oracle_flags(X, Y)
    out = torch.full((4, 8), 5.0, dtype=torch.float64, device="cuda")
    with pytest.raises(md.MDError) as e:
        md.dot_ex(dev(X), dev(Y), out, validate=True)
    assert e.value.code == 9 and e.value.input_flags == want
    torch.cuda.synchronize()
    assert np.all(out.cpu().numpy() == 5.0)
