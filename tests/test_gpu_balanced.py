"""The balanced INT8 slice form (8-bit digits in [-128, 127] on the grid
2^(E+2)) against the oracle, through the C ABI (needs an MI355X).

* every step bit-exact on ragged shapes (exponents, digits, diagonal sums,
  output words), transposed operands, m = 1 .. 16, the banded kernels with
  the diagonal-sum buffer (S > 32), and entries whose leading words sit just
  below a power of two (the truncated integers close to the headroom);
* every whole-triangle instantiation (S = 1..32), with the whole depth in
  one exactness chunk and with several chunks;
* the library's rule equals the oracle's (fewer slices than the
  sign-magnitude form), outputs bit-exact and within 2^-T of the exact
  product, the reported bound above the measured error;
* the quad-double 4096^3 benchmark workload: sampled entries bit-exact
  against the C oracle and within 2^-200 of the exact product;
* batched inner products (the paper's experiment) in this form;
* degenerate sizes.
"""
import numpy as np
import pytest
import torch

import mdinputs
import paper_2606_20863_amd as md
from oracle import coracle
from oracle import exact as ox

import rulecheck

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def run_debug(A, B, S, transA=False, transB=False):
    m = A.shape[0]
    M, K = (A.shape[2], A.shape[1]) if transA else (A.shape[1], A.shape[2])
    N = B.shape[1] if transB else B.shape[2]
    dbg = {
        "E": torch.zeros(M, dtype=torch.int32, device="cuda"),
        "F": torch.zeros(N, dtype=torch.int32, device="cuda"),
        "digits_A": torch.zeros((S, M, K), dtype=torch.int32, device="cuda"),
        "digits_B": torch.zeros((S, N, K), dtype=torch.int32, device="cuda"),
        "D": torch.zeros((S, M, N), dtype=torch.int64, device="cuda"),
    }
    C, info = md.gemm_ex(dev(A), dev(B), transA=transA, transB=transB, form="int8bal", force_S=S,
                         force_beta=8, debug=dbg)
    out = {k: host(v) for k, v in dbg.items()}
    out["C"] = host(C)
    return out, info


def check_steps(A, B, got, S):
    ref = ox.method_product(A, B, 8, S, balanced=True)
    np.testing.assert_array_equal(got["E"], np.array(ref["E"], dtype=np.int32))
    np.testing.assert_array_equal(got["F"], np.array(ref["F"], dtype=np.int32))
    np.testing.assert_array_equal(got["digits_A"], ref["dA"])
    np.testing.assert_array_equal(got["digits_B"], np.transpose(ref["dB"], (0, 2, 1)))
    np.testing.assert_array_equal(got["D"], ref["D"])
    np.testing.assert_array_equal(got["C"], ref["C"])


RAGGED = [(37, 45, 130), (16, 16, 64), (1, 1, 1), (33, 7, 65), (50, 64, 17)]


@pytest.mark.parametrize("shape", RAGGED)
@pytest.mark.parametrize("S", [5, 27])
def test_bitexact_steps_ragged(shape, S):
    M, N, K = shape
    A, B = mdinputs.workload("qd1024", M=M, N=N, K=K)
    A[:, min(3, M - 1), :] = 0.0        # an all-zero row
    got, info = run_debug(A, B, S)
    assert (info["S"], info["beta"]) == (S, 8)
    check_steps(A, B, got, S)


@pytest.mark.parametrize("m,S", [(1, 9), (2, 16), (4, 32), (8, 52), (16, 105)])
def test_bitexact_word_counts(m, S):
    """S > 32 runs the banded kernels (bands of at most 16 diagonals, the
    sums through the buffer and the fold-and-round kernel)."""
    r = rng(100 + m)
    A = mdinputs.mdouble(r, m, (40, 96), ("log2uniform", 10.0))
    B = mdinputs.mdouble(r, m, (96, 24), ("log2uniform", 10.0))
    got, info = run_debug(A, B, S)
    assert info["S"] == S
    check_steps(A, B, got, S)


@pytest.mark.parametrize("transA,transB", [(False, True), (True, False), (True, True)])
def test_bitexact_transposed_operands(transA, transB):
    A, B = mdinputs.workload("dd64", M=29, N=35, K=77)
    Ain = np.ascontiguousarray(np.transpose(A, (0, 2, 1))) if transA else A
    Bin = np.ascontiguousarray(np.transpose(B, (0, 2, 1))) if transB else B
    got, _ = run_debug(Ain, Bin, 15, transA=transA, transB=transB)
    check_steps(A, B, got, 15)


def test_leading_words_below_a_power_of_two():
    """Leading words (2 - 2^-52) 2^e with trailing words of both signs: the
    truncated integers come within a factor of two of 2^(8S-2)."""
    r = rng(7)
    A = mdinputs.mdouble(r, 4, (33, 70), ("log2uniform", 3.0))
    B = mdinputs.mdouble(r, 4, (70, 20), ("log2uniform", 3.0))
    # A: (2 - 2^-52) 2^e, then a word of the other sign a quarter ulp
    # below it (nonoverlapping), then zeros
    A[0] = np.copysign(np.ldexp(np.nextafter(2.0, 0.0), np.frexp(A[0])[1]), A[0])
    A[1] = -np.copysign(np.ldexp(1.0, np.frexp(A[0])[1] - 55), A[0])
    A[2:] = 0.0
    # B: every other row 1 - 2^-53 with a trailing word of the other sign
    B[0, ::2] = np.copysign(np.nextafter(1.0, 0.0), B[0, ::2])
    B[1, ::2] = -np.copysign(2.0 ** -55, B[0, ::2])
    B[2:, ::2] = 0.0
    for X in (A, B):
        for i in range(0, X.shape[1], 5):
            for k in range(0, X.shape[2], 3):
                assert ox.is_nonoverlapping(X[:, i, k], strong=True)
    for S in (27, 30):
        got, _ = run_debug(A, B, S)
        check_steps(A, B, got, S)


@pytest.mark.parametrize("S", range(1, 33))
def test_triangle_every_S_one_chunk(S):
    """The two-row-block triangle kernels of the 8-bit digits (no debug
    dump, depth within one exactness chunk); M = 70 leaves a row block past
    the padded digit array."""
    A, B = mdinputs.workload("qd1024", M=70, N=33, K=100)
    C, info = md.gemm_ex(dev(A), dev(B), form="int8bal", force_S=S, force_beta=8)
    assert info["kc"] >= 100
    np.testing.assert_array_equal(host(C), ox.method_product(A, B, 8, S, balanced=True)["C"])


@pytest.mark.parametrize("S", range(1, 33))
def test_triangle_every_S_several_chunks(S):
    """The one-row-block triangle kernels: the depth exceeds one exactness
    chunk (S K 128^2 >= 2^31), so the 32-bit fold columns carry between
    chunks."""
    kc = rulecheck.library_chunk("int8bal", 8, S)
    K = kc + 81
    A, B = mdinputs.workload("dd64", M=17, N=19, K=K)
    C, info = md.gemm_ex(dev(A), dev(B), form="int8bal", force_S=S, force_beta=8)
    assert info["kc"] == kc < K
    np.testing.assert_array_equal(host(C), ox.method_product(A, B, 8, S, balanced=True)["C"])


@pytest.mark.parametrize("rule", ["rho", "span"])
@pytest.mark.parametrize("name", ["dd64", "qd1024", "od1024"])
def test_rule_and_bound_small(name, rule):
    _, m, _, _, _, _, _ = mdinputs.WORKLOADS[name]
    A, B = mdinputs.workload(name, M=48, N=40, K=72)
    C, info = md.gemm_ex(dev(A), dev(B), form="int8bal", rule=rule)
    C = host(C)
    T = ox.TARGET_BITS[m]
    _, sA = ox.row_exponents(A[0])
    _, sB = ox.row_exponents(B[0].T)
    G = ox.span_G(max(sA), max(sB))
    if rule == "rho":
        _, G_rho = ox.rho_G(A, B)
        assert info["G_rho"] == (-1 if G_rho is None else G_rho)
        if G_rho is not None:
            G = min(G, G_rho)
    assert info["G"] == G
    rulecheck.check_info(info, "int8bal", 72, T, G)
    beta, S = info["beta"], info["S"]
    assert S < ox.min_slices("int8", T, G)
    np.testing.assert_array_equal(C, ox.method_product(A, B, beta, S, balanced=True)["C"])
    num, L = ox.exact_product(A, B)
    anum, _ = ox.abs_product(A, B)
    rep = ox.error_report(C, num, anum, L)
    assert max(rep.values()) <= -T
    assert max(rep.values()) <= info["log2_bound"] + 1e-9
    for i in range(0, 48, 7):
        for j in range(0, 40, 5):
            assert ox.is_nonoverlapping(C[:, i, j], strong=True)


@pytest.mark.parametrize("m", [1, 16])
def test_word_counts_one_and_sixteen_rule(m):
    r = rng(700 + m)
    A = mdinputs.mdouble(r, m, (20, 50), ("log2uniform", 6.0))
    B = mdinputs.mdouble(r, m, (50, 24), ("log2uniform", 6.0))
    C, info = md.gemm_ex(dev(A), dev(B), form="int8bal")
    C = host(C)
    beta, S = info["beta"], info["S"]
    np.testing.assert_array_equal(C, ox.method_product(A, B, beta, S, balanced=True)["C"])
    num, L = ox.exact_product(A, B)
    anum, _ = ox.abs_product(A, B)
    assert max(ox.error_report(C, num, anum, L).values()) <= -ox.TARGET_BITS[m]


@pytest.mark.parametrize("m", [1, 2, 4, 8, 16])
def test_dot_rule_bitexact(m):
    r = rng(900 + m)
    X = mdinputs.mdouble(r, m, (37, 130), ("log2uniform", 8.0))
    Y = mdinputs.mdouble(r, m, (37, 130), ("log2uniform", 8.0))
    X[:, 5, :] = 0.0
    out, info = md.dot_ex(dev(X), dev(Y), form="int8bal")
    out = host(out)
    rulecheck.check_info(info, "int8bal", 130, ox.TARGET_BITS[m], ox.dot_G(X, Y))
    beta, S = info["beta"], info["S"]
    _, ref = ox.method_dot(X, Y, beta, S, balanced=True)
    np.testing.assert_array_equal(out, ref)
    assert np.all(out[:, 5] == 0.0)


def test_dot_equals_gemm_diagonal():
    r = rng(950)
    X = mdinputs.mdouble(r, 4, (40, 200), ("log2uniform", 8.0))
    Y = mdinputs.mdouble(r, 4, (40, 200), ("log2uniform", 8.0))
    for S in (27, 48):
        out, _ = md.dot_ex(dev(X), dev(Y), form="int8bal", force_S=S, force_beta=8)
        C, _ = md.gemm_ex(dev(X), dev(Y), transB=True, form="int8bal", force_S=S, force_beta=8)
        np.testing.assert_array_equal(host(out), host(C)[:, np.arange(40), np.arange(40)])


def test_degenerate_sizes():
    Z = torch.full((2, 5, 6), 7.0, dtype=torch.float64, device="cuda")
    C, _ = md.gemm_ex(torch.zeros((2, 5, 0), dtype=torch.float64, device="cuda"),
                      torch.zeros((2, 0, 6), dtype=torch.float64, device="cuda"), Z, form="int8bal")
    assert np.all(host(C) == 0.0)
    A, B = mdinputs.workload("dd64", M=5, N=6, K=7)
    C, _ = md.gemm_ex(dev(np.zeros_like(A)), dev(B), form="int8bal")
    assert np.all(host(C) == 0.0) and not np.any(np.signbit(host(C)))
    a, b = A[:, :1, :1], B[:, :1, :1]
    C, info = md.gemm_ex(dev(a), dev(b), form="int8bal")
    np.testing.assert_array_equal(host(C), ox.method_product(a, b, 8, info["S"], balanced=True)["C"])
    # a forced width other than 8 is refused
    with pytest.raises(md.MDError):
        md.gemm_ex(dev(a), dev(b), form="int8bal", force_S=10, force_beta=7)
