"""Calls that run on a slice-count hint, and the double-range certificate
(needs an MI355X).

With ``s_hint`` a call takes the given S at once and the device checks the
data's certificate into an md_cert record, so the call queues its kernels
without waiting (it can be captured into a HIP graph).  A hint that meets
the rule gives the rule's output word for word; a hint below it is flagged
and the output still meets the bound the record certifies for the S used,
against the exact product.  Entries whose products leave the double range
are flagged, with no bound.
"""
import math

import numpy as np
import pytest
import torch

import mdinputs
import paper_2606_20863_amd as md
from oracle import exact as ox

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("form", ["int8bal", "int8", "fp64"])
@pytest.mark.parametrize("name", ["dd64", "qd1024", "od1024"])
def test_hint_equal_to_the_rule(name, form):
    """The rule's own S as the hint: the same words as the rule's call, the
    record's certificates equal md_info's, no flag."""
    A, B = mdinputs.workload(name, M=48, N=40, K=72)
    dA, dB = dev(A), dev(B)
    C, info = md.gemm_ex(dA, dB, form=form)
    cert = md.new_cert()
    Ch, hi = md.gemm_ex(dA, dB, form=form, s_hint=info["S"], force_beta=info["beta"] if form == "fp64" else 0,
                        cert=cert)
    np.testing.assert_array_equal(host(Ch), host(C))
    c = md.read_cert(cert)
    assert c["flags"] == 0
    assert (c["S_min"], c["S"], c["G"], c["G_span"], c["G_rho"]) == \
        (info["S"], info["S"], info["G"], info["G_span"], info["G_rho"])
    assert abs(c["log2_bound"] - info["log2_bound"]) < 1e-9
    assert hi["S"] == info["S"] and math.isnan(hi["log2_bound"])


@pytest.mark.parametrize("form,m", [("int8bal", 4), ("int8", 2), ("fp64", 4)])
def test_hint_too_small_is_flagged_and_bounded(form, m):
    """A hint well below the rule's S: MD_CERT_SMALL, and every entry's
    error against the exact product within the record's bound for the S
    used (which is above 2^-T)."""
    name = {2: "dd64", 4: "qd1024"}[m]
    A, B = mdinputs.workload(name, M=24, N=20, K=40)
    dA, dB = dev(A), dev(B)
    _, info = md.gemm_ex(dA, dB, form=form)
    S = info["S"] - 5 if form != "fp64" else info["S"] - 2
    cert = md.new_cert()
    C, _ = md.gemm_ex(dA, dB, form=form, s_hint=S, force_beta=info["beta"] if form == "fp64" else 0, cert=cert)
    C = host(C)
    c = md.read_cert(cert)
    assert c["flags"] & md.CERT_SMALL and not c["flags"] & md.CERT_RANGE
    assert c["S"] == S and c["S_min"] == info["S"]
    assert c["log2_bound"] > -ox.TARGET_BITS[m]
    ref = ox.method_product(A, B, info["beta"], S, balanced=form == "int8bal")
    np.testing.assert_array_equal(C, ref["C"])
    num, L = ox.exact_product(A, B)
    anum, _ = ox.abs_product(A, B)
    assert max(ox.error_report(C, num, anum, L).values()) <= c["log2_bound"]


def test_hinted_call_is_captured_in_a_graph():
    """A hinted call with a workspace only launches kernels: a graph holds
    it, and every replay (new inputs copied in between) equals an eager
    call, its certificate record rewritten by each replay."""
    m, M, N, K, form = 4, 70, 45, 130, "int8bal"
    r = np.random.Generator(np.random.PCG64(77))
    A = dev(mdinputs.mdouble(r, m, (M, K), ("uniform",)))
    B = dev(mdinputs.mdouble(r, m, (K, N), ("uniform",)))
    _, info = md.gemm_ex(A, B, form=form)
    S = info["S"]
    ws = torch.empty(md.lib().md_gemm_workspace_size(md._FORMS[form], M, N, K, S), dtype=torch.uint8,
                     device="cuda")
    cert = md.new_cert()
    C = torch.empty((m, M, N), dtype=torch.float64, device="cuda")

    def call():
        md.gemm_ex(A, B, C, form=form, s_hint=S, cert=cert, workspace=ws)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        call()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    torch.cuda.synchronize()
    for rep in range(3):
        A.copy_(dev(mdinputs.mdouble(r, m, (M, K), ("uniform",))))
        B.copy_(dev(mdinputs.mdouble(r, m, (K, N), ("uniform",))))
        cert.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        Cg = C.clone()
        c = md.read_cert(cert)
        Ce, ie = md.gemm_ex(A, B, form=form, force_S=S, force_beta=8)
        assert torch.equal(Cg, Ce), rep
        assert c["S"] == S and c["S_min"] > 0
        _, ir = md.gemm_ex(A, B, form=form)
        assert c["S_min"] == ir["S"] and c["G"] == ir["G"]


@pytest.mark.parametrize("scale,form", [(-540, "int8bal"), (-540, "fp64"), (500, "int8"), (-300, "int8bal")])
def test_range_flag(scale, form):
    """Leading words near 2^-540 (products near 2^-1080, below the normal
    range) or 2^500 (products near 2^1000, K of them near 2^1006: in
    range) inside the documented input range.  Out of range: md_info flags
    bit 16, no bound (+inf), and a hinted call's record MD_CERT_RANGE; in
    range: no flag, and the output within the bound of the exact product."""
    A, B = mdinputs.workload("dd64", M=16, N=12, K=40)
    A = A * 2.0 ** scale
    B = B * 2.0 ** scale
    dA, dB = dev(A), dev(B)
    C, info = md.gemm_ex(dA, dB, form=form)
    C = host(C)
    cert = md.new_cert()
    md.gemm_ex(dA, dB, form=form, s_hint=info["S"], force_beta=info["beta"] if form == "fp64" else 0, cert=cert)
    c = md.read_cert(cert)
    out = scale <= -540
    assert bool(info["input_flags"] & 16) == out
    assert bool(c["flags"] & md.CERT_RANGE) == out
    if out:
        assert info["log2_bound"] == math.inf and c["log2_bound"] == math.inf
    else:
        num, L = ox.exact_product(A, B)
        anum, _ = ox.abs_product(A, B)
        assert max(ox.error_report(C, num, anum, L).values()) <= info["log2_bound"] <= -100
        assert np.all(np.isfinite(C))


@pytest.mark.parametrize("form", ["int8bal", "fp64"])
def test_dot_hint(form):
    """Batched inner products on a hint: equal to the rule's call, the
    record equal to md_info's certificate."""
    r = np.random.Generator(np.random.PCG64(31))
    X = dev(mdinputs.mdouble(r, 4, (40, 300), ("log2uniform", 8.0)))
    Y = dev(mdinputs.mdouble(r, 4, (40, 300), ("log2uniform", 8.0)))
    out, info = md.dot_ex(X, Y, form=form)
    cert = md.new_cert()
    oh, _ = md.dot_ex(X, Y, form=form, s_hint=info["S"], force_beta=info["beta"] if form == "fp64" else 0,
                      cert=cert)
    assert torch.equal(out, oh)
    c = md.read_cert(cert)
    assert c["flags"] == 0 and c["S_min"] == info["S"] and c["G"] == info["G"]
