"""API behaviour on the GPU: caller workspace, streams, concurrency
(needs an MI355X)."""
import numpy as np
import pytest
import torch

import mdinputs
import paper_2606_20863_amd as md

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("form", ["int8", "int8bal", "fp64"])
def test_caller_workspace(form):
    """With a workspace of md_gemm_workspace_size bytes the library allocates
    nothing and gives the same words; a workspace too small is MD_ENOMEM."""
    A, B = mdinputs.workload("qd1024", M=40, N=56, K=130)
    ref, info = md.gemm_ex(dev(A), dev(B), form=form)
    ref = host(ref)
    nbytes = md.lib().md_gemm_workspace_size(md._FORMS[form], 40, 56, 130, info["S"])
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    C, info2 = md.gemm_ex(dev(A), dev(B), form=form, workspace=ws)
    np.testing.assert_array_equal(host(C), ref)
    assert info2["S"] == info["S"]
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(md.MDError) as e:
        md.gemm_ex(dev(A), dev(B), form=form, workspace=small)
    assert e.value.code == 5


def test_workspace_covers_the_global_fold():
    """Hexa-double FP64: the [S][M][N] diagonal-sum buffer is part of
    md_gemm_workspace_size."""
    r = np.random.Generator(np.random.PCG64(9))
    A = mdinputs.mdouble(r, 16, (24, 40))
    B = mdinputs.mdouble(r, 16, (40, 20))
    ref, info = md.gemm_ex(dev(A), dev(B), form="fp64")
    nbytes = md.lib().md_gemm_workspace_size(0, 24, 20, 40, info["S"])
    assert nbytes >= info["S"] * 24 * 20 * 8
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    C, _ = md.gemm_ex(dev(A), dev(B), form="fp64", workspace=ws)
    np.testing.assert_array_equal(host(C), host(ref))


def test_workspace_covers_the_int8_sum_buffer():
    """Octo-double balanced INT8 (S > 32, bands): the diagonal-sum buffer of
    the banded kernels is part of md_gemm_workspace_size."""
    A, B = mdinputs.workload("od1024", M=70, N=36, K=90)
    ref, info = md.gemm_ex(dev(A), dev(B), form="int8bal")
    assert info["S"] > 32
    nbytes = md.lib().md_gemm_workspace_size(md._FORMS["int8bal"], 70, 36, 90, info["S"])
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    C, _ = md.gemm_ex(dev(A), dev(B), form="int8bal", workspace=ws)
    np.testing.assert_array_equal(host(C), host(ref))


def test_streams_and_concurrency():
    """Products queued on two non-default streams at once give the words of
    the same products on the default stream."""
    A1, B1 = mdinputs.workload("qd1024", M=64, N=64, K=256)
    A2, B2 = mdinputs.workload("od1024", M=48, N=80, K=200)
    r1 = host(md.gemm_ex(dev(A1), dev(B1), form="int8")[0])
    r2 = host(md.gemm_ex(dev(A2), dev(B2), form="fp64")[0])
    dA1, dB1, dA2, dB2 = dev(A1), dev(B1), dev(A2), dev(B2)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for _ in range(3):
        with torch.cuda.stream(s1):
            c1 = md.gemm_ex(dA1, dB1, form="int8", stream=s1)[0]
        with torch.cuda.stream(s2):
            c2 = md.gemm_ex(dA2, dB2, form="fp64", stream=s2)[0]
        outs.append((c1, c2))
    torch.cuda.synchronize()
    for c1, c2 in outs:
        np.testing.assert_array_equal(c1.cpu().numpy(), r1)
        np.testing.assert_array_equal(c2.cpu().numpy(), r2)


@pytest.mark.parametrize("form", ["int8bal", "fp64"])
def test_dot_caller_workspace(form):
    """md_dot_ex with a workspace of md_dot_workspace_size bytes (the slice
    rule's magnitude slices included) gives the same words; a workspace too
    small is MD_ENOMEM and leaves the output as it was."""
    r = np.random.Generator(np.random.PCG64(12))
    X = dev(mdinputs.mdouble(r, 4, (70, 900)))
    Y = dev(mdinputs.mdouble(r, 4, (70, 900)))
    ref, info = md.dot_ex(X, Y, form=form)
    nbytes = md.lib().md_dot_workspace_size(md._FORMS[form], 70, 900, info["S"])
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out, info2 = md.dot_ex(X, Y, form=form, workspace=ws)
    np.testing.assert_array_equal(host(out), host(ref))
    assert info2["S"] == info["S"]
    keep = torch.full_like(ref, 3.0)
    with pytest.raises(md.MDError) as e:
        md.dot_ex(X, Y, keep, form=form, workspace=torch.empty(2048, dtype=torch.uint8, device="cuda"))
    assert e.value.code == 5
    torch.cuda.synchronize()
    assert bool((keep == 3.0).all())


@pytest.mark.parametrize("form", ["int8bal", "fp64"])
def test_scratch_from_torch_equals_pool(form):
    """Calls without a workspace take their scratch from torch's caching
    allocator once the shape's S is known (a hint, or the S the same shape
    and options took last time): the same words as calls on the library's
    pool, for products and inner products, with the rule and on a hint.
    When the rule then picks a larger S on the same shape (wider exponent
    spans), the workspace sized for the last S is too small: the call stops
    with MD_ENOMEM before writing an output and runs again on the pool, with
    the pool's words."""
    A, B = mdinputs.workload("qd1024", M=40, N=56, K=130)
    ref, i1 = md.gemm_ex(dev(A), dev(B), form=form, pool=True)
    ref = host(ref)
    for _ in range(2):   # the first call records S, the second runs on torch's scratch
        C, i2 = md.gemm_ex(dev(A), dev(B), form=form)
        np.testing.assert_array_equal(host(C), ref)
        assert i2["S"] == i1["S"]
    cert = md.new_cert()
    fb = i1["beta"] if form == "fp64" else 0   # the FP64 form's hint names its beta
    Ch, _ = md.gemm_ex(dev(A), dev(B), form=form, s_hint=i1["S"], force_beta=fb, cert=cert)
    np.testing.assert_array_equal(host(Ch), ref)
    assert md.read_cert(cert)["flags"] == 0
    # the span rule (S follows the exponent spans) on the same shape: the
    # last S recorded, then wider spans in the rows of A
    _, i1s = md.gemm_ex(dev(A), dev(B), form=form, rule="span")
    A2 = A.copy()
    A2[:, :, ::5] *= 2.0 ** -90
    ref2, i3 = md.gemm_ex(dev(A2), dev(B), form=form, rule="span", pool=True)
    assert i3["S"] > i1s["S"]
    size = lambda S: md.lib().md_gemm_workspace_size(md._FORMS[form], 40, 56, 130, S)
    assert size(i3["S"]) > size(i1s["S"])
    C2, i4 = md.gemm_ex(dev(A2), dev(B), form=form, rule="span")
    np.testing.assert_array_equal(host(C2), host(ref2))
    assert i4["S"] == i3["S"]

    r = np.random.Generator(np.random.PCG64(77))
    X = mdinputs.mdouble(r, 4, (33, 700), ("log2uniform", 6.0))
    Y = mdinputs.mdouble(r, 4, (33, 700), ("log2uniform", 6.0))
    oref, j1 = md.dot_ex(dev(X), dev(Y), form=form, pool=True)
    oref = host(oref)
    for _ in range(2):
        o, j2 = md.dot_ex(dev(X), dev(Y), form=form)
        np.testing.assert_array_equal(host(o), oref)
        assert j2["S"] == j1["S"]
    oh, _ = md.dot_ex(dev(X), dev(Y), form=form, s_hint=j1["S"], force_beta=j1["beta"] if form == "fp64" else 0,
                      cert=cert)
    np.testing.assert_array_equal(host(oh), oref)
    _, j1s = md.dot_ex(dev(X), dev(Y), form=form, rule="span")
    X2 = X.copy()
    X2[:, :, ::5] *= 2.0 ** -90
    oref2, j3 = md.dot_ex(dev(X2), dev(Y), form=form, rule="span", pool=True)
    assert j3["S"] > j1s["S"]
    size = lambda S: md.lib().md_dot_workspace_size(md._FORMS[form], 33, 700, S)
    assert size(j3["S"]) > size(j1s["S"])
    o2, j4 = md.dot_ex(dev(X2), dev(Y), form=form, rule="span")
    np.testing.assert_array_equal(host(o2), host(oref2))
    assert j4["S"] == j3["S"]
