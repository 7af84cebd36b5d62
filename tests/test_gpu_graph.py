"""HIP graph capture of the matrix product (needs an MI355X).

With a forced slice count and a caller workspace, md_gemm_ex only launches
kernels, so a torch CUDA/HIP graph can hold it.  Each graph is replayed
several times with new inputs copied in eagerly between the replays (and a
synchronisation after each); every replay must equal an eager call on the
same inputs word for word, and the first one the oracle's method.  Cases:
the launch-bound double-double 64^3 product in the three forms, ragged
quad-double sizes (whole-triangle INT8 kernels, FP64 LDS fold), octo-double
balanced INT8 (banded kernels and their sum buffer), hexa-double FP64 (the
buffer fold), a forward + adjoint step (three products in one graph), and
batched inner products (md_dot_ex with md_dot_workspace_size bytes).
"""
import numpy as np
import pytest
import torch

import mdinputs
import paper_2606_20863_amd as md
from oracle import exact as ox

pytestmark = pytest.mark.gpu

CASES = [(2, 64, 64, 64, "fp64"), (2, 64, 64, 64, "int8"), (2, 64, 64, 64, "int8bal"),
         (4, 70, 45, 130, "int8"), (4, 70, 45, 130, "int8bal"), (4, 70, 45, 130, "fp64"),
         (8, 40, 36, 90, "int8bal"), (16, 24, 20, 40, "fp64")]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def workspace(form, M, N, K, S):
    n = md.lib().md_gemm_workspace_size(md._FORMS[form], M, N, K, S)
    return torch.empty(n, dtype=torch.uint8, device="cuda")


def warm_and_capture(fn):
    """One eager call on a side stream (as torch asks before capture), then
    the capture."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


@pytest.mark.parametrize("m,M,N,K,form", CASES, ids=lambda v: str(v))
def test_graph_replays_equal_eager_calls(m, M, N, K, form):
    r = np.random.Generator(np.random.PCG64(1000 * m + K))
    lead = ("log2uniform", 8.0) if m >= 8 else ("uniform",)
    A = dev(mdinputs.mdouble(r, m, (M, K), lead))
    B = dev(mdinputs.mdouble(r, m, (K, N), lead))
    _, info = md.gemm_ex(A, B, form=form)
    S, beta = info["S"], info["beta"]
    ws = workspace(form, M, N, K, S)
    C = torch.empty((m, M, N), dtype=torch.float64, device="cuda")
    kw = dict(form=form, force_S=S, force_beta=beta)
    g = warm_and_capture(lambda: md.gemm_ex(A, B, C, workspace=ws, **kw))
    for rep in range(4):
        Ah = mdinputs.mdouble(r, m, (M, K), lead)
        Bh = mdinputs.mdouble(r, m, (K, N), lead)
        A.copy_(torch.from_numpy(Ah))
        B.copy_(torch.from_numpy(Bh))
        C.fill_(np.nan)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = C.cpu().numpy()
        ref, _ = md.gemm_ex(A, B, **kw)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got, ref.cpu().numpy())
        if rep == 0:
            want = ox.method_product(Ah, Bh, beta, S, balanced=form == "int8bal")["C"]
            np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("form", ["fp64", "int8bal"])
def test_graph_of_forward_and_adjoint(form):
    """C = A B, dA = W B^T, dB = A^T W captured as one graph."""
    m, M, N, K = 2, 48, 40, 56
    r = np.random.Generator(np.random.PCG64(77))
    A = dev(mdinputs.mdouble(r, m, (M, K)))
    B = dev(mdinputs.mdouble(r, m, (K, N)))
    W = dev(mdinputs.mdouble(r, m, (M, N)))
    shapes = [(A, B, False, False, M, N, K), (W, B, False, True, M, K, N), (A, W, True, False, K, N, M)]
    outs, wss, kws = [], [], []
    for a, b, ta, tb, Mo, No, Ko in shapes:
        _, info = md.gemm_ex(a, b, transA=ta, transB=tb, form=form)
        kws.append(dict(transA=ta, transB=tb, form=form, force_S=info["S"], force_beta=info["beta"]))
        wss.append(workspace(form, Mo, No, Ko, info["S"]))
        outs.append(torch.empty((m, Mo, No), dtype=torch.float64, device="cuda"))

    def step():
        for (a, b, *_), C, ws, kw in zip(shapes, outs, wss, kws):
            md.gemm_ex(a, b, C, workspace=ws, **kw)

    g = warm_and_capture(step)
    for rep in range(3):
        for T, shp in ((A, (M, K)), (B, (K, N)), (W, (M, N))):
            T.copy_(torch.from_numpy(mdinputs.mdouble(r, m, shp)))
        for C in outs:
            C.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (a, b, *_), C, kw in zip(shapes, outs, kws):
            ref, _ = md.gemm_ex(a, b, **kw)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(C.cpu().numpy(), ref.cpu().numpy())


@pytest.mark.parametrize("form", ["int8bal", "int8", "fp64"])
def test_graph_of_inner_products(form):
    """Batched inner products with a forced S and a workspace of
    md_dot_workspace_size bytes, captured and replayed with new inputs: every
    replay equals an eager call (and the first the oracle's method)."""
    m, batch, n = 4, 90, 700
    r = np.random.Generator(np.random.PCG64(404))
    X = dev(mdinputs.mdouble(r, m, (batch, n)))
    Y = dev(mdinputs.mdouble(r, m, (batch, n)))
    _, info = md.dot_ex(X, Y, form=form)
    kw = dict(form=form, force_S=info["S"], force_beta=info["beta"])
    ws = torch.empty(md.lib().md_dot_workspace_size(md._FORMS[form], batch, n, info["S"]), dtype=torch.uint8,
                     device="cuda")
    out = torch.empty((m, batch), dtype=torch.float64, device="cuda")
    g = warm_and_capture(lambda: md.dot_ex(X, Y, out, workspace=ws, **kw))
    for rep in range(3):
        Xh = mdinputs.mdouble(r, m, (batch, n))
        Yh = mdinputs.mdouble(r, m, (batch, n))
        X.copy_(torch.from_numpy(Xh))
        Y.copy_(torch.from_numpy(Yh))
        out.fill_(np.nan)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref, _ = md.dot_ex(X, Y, **kw)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got, ref.cpu().numpy())
        if rep == 0:
            _, want = ox.method_dot(Xh, Yh, info["beta"], info["S"], balanced=form == "int8bal")
            np.testing.assert_array_equal(got, want)
