"""HIP path against the oracle, through the C ABI (needs an MI355X).

Bit-exact: exponents, digits, diagonal sums and (greedy round-to-nearest
being unique) the output words, against the oracle's method layer on the
same seeded inputs.  Within bound: the output against the exact product,
2^-T of (|A||B|)_ij for every checked entry, T = 50 m.
"""
import functools

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


def run_debug(A, B, form, S, beta, transA=False, transB=False):
    """Forced (S, beta) with every debug buffer; A, B as passed to gemm_ex."""
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
    C, info = md.gemm_ex(dev(A), dev(B), transA=transA, transB=transB, form=form, force_S=S,
                         force_beta=beta, debug=dbg)
    out = {k: host(v) for k, v in dbg.items()}
    out["C"] = host(C)
    return out, info


def check_against_oracle(A, B, got, beta, S):
    """A (m, M, K), B (m, K, N) in plain orientation."""
    ref = ox.method_product(A, B, beta, S)
    np.testing.assert_array_equal(got["E"], np.array(ref["E"], dtype=np.int32))
    np.testing.assert_array_equal(got["F"], np.array(ref["F"], dtype=np.int32))
    np.testing.assert_array_equal(got["digits_A"], ref["dA"])
    np.testing.assert_array_equal(got["digits_B"], np.transpose(ref["dB"], (0, 2, 1)))
    np.testing.assert_array_equal(got["D"], ref["D"])
    np.testing.assert_array_equal(got["C"], ref["C"])


RAGGED = [(37, 45, 130), (16, 16, 64), (1, 1, 1), (33, 7, 65), (50, 64, 17)]


@pytest.mark.parametrize("shape", RAGGED)
@pytest.mark.parametrize("form,S,beta", [("int8", 12, 7), ("int8", 30, 7), ("fp64", 6, 20),
                                         ("fp64", 11, 18)])
def test_bitexact_steps_ragged(shape, form, S, beta):
    M, N, K = shape
    A, B = mdinputs.workload("qd1024", M=M, N=N, K=K)
    A[:, min(3, M - 1), :] = 0.0        # an all-zero row
    got, info = run_debug(A, B, form, S, beta)
    assert info["S"] == S and info["beta"] == beta
    check_against_oracle(A, B, got, beta, S)


@pytest.mark.parametrize("m", [2, 4, 8])
@pytest.mark.parametrize("form", ["int8", "fp64"])
def test_bitexact_word_counts(m, form):
    name = {2: "dd64", 4: "qd1024", 8: "od1024"}[m]
    A, B = mdinputs.workload(name, M=40, N=24, K=96)
    S, beta = (32, 7) if form == "int8" else (16, 16)
    got, _ = run_debug(A, B, form, S, beta)
    check_against_oracle(A, B, got, beta, S)


@pytest.mark.parametrize("transA,transB", [(False, True), (True, False), (True, True)])
@pytest.mark.parametrize("form,S,beta", [("int8", 16, 7), ("fp64", 8, 19)])
def test_bitexact_transposed_operands(transA, transB, form, S, beta):
    A, B = mdinputs.workload("dd64", M=29, N=35, K=77)
    Ain = np.ascontiguousarray(np.transpose(A, (0, 2, 1))) if transA else A
    Bin = np.ascontiguousarray(np.transpose(B, (0, 2, 1))) if transB else B
    got, _ = run_debug(Ain, Bin, form, S, beta, transA=transA, transB=transB)
    check_against_oracle(A, B, got, beta, S)


@pytest.mark.parametrize("rule", ["rho", "span"])
@pytest.mark.parametrize("form", ["int8", "fp64"])
@pytest.mark.parametrize("name", ["dd64", "qd1024", "od1024"])
def test_rule_and_bound_small(form, name, rule):
    """Default parameters: the library's certificates equal the oracle's,
    its slice count sits within the budget (at least the minimal S, less
    than one band more), the output equals the oracle's method layer at the
    library's S bit for bit, and every entry is within 2^-T of
    (|A||B|)_ij of the exact product."""
    _, m, _, _, _, _, _ = mdinputs.WORKLOADS[name]
    A, B = mdinputs.workload(name, M=48, N=40, K=72)
    C, info = md.gemm_ex(dev(A), dev(B), form=form, rule=rule)
    C = host(C)
    T = ox.TARGET_BITS[m]
    E, sA = ox.row_exponents(A[0])
    F, sB = ox.row_exponents(B[0].T)
    G_span = ox.span_G(max(sA), max(sB))
    assert (info["span_A"], info["span_B"], info["G_span"]) == (max(sA), max(sB), G_span)
    G = G_span
    if rule == "rho":
        _, G_rho = ox.rho_G(A, B)
        assert info["G_rho"] == (-1 if G_rho is None else G_rho)
        if G_rho is not None:
            G = min(G_span, G_rho)
    assert info["G"] == G
    rulecheck.check_info(info, form, 72, T, G)
    beta, S = info["beta"], info["S"]
    ref = ox.method_product(A, B, beta, S)
    np.testing.assert_array_equal(C, ref["C"])
    num, L = ox.exact_product(A, B)
    anum, _ = ox.abs_product(A, B)
    rep = ox.error_report(C, num, anum, L)
    assert max(rep.values()) <= -T
    assert max(rep.values()) <= info["log2_bound"] + 1e-9
    for i in range(0, 48, 7):
        for j in range(0, 40, 5):
            assert ox.is_nonoverlapping(C[:, i, j], strong=True)


@pytest.mark.parametrize("S", range(1, 33))
def test_triangle_kernel_every_S_one_chunk(S):
    """Every whole-triangle instantiation with two row blocks per wave
    (forced S, beta = 7, no debug dump, depth within one exactness chunk);
    M = 70 leaves a row block past the padded digit array."""
    A, B = mdinputs.workload("qd1024", M=70, N=33, K=100)
    C, info = md.gemm_ex(dev(A), dev(B), form="int8", force_S=S, force_beta=7)
    assert info["kc"] >= 100
    np.testing.assert_array_equal(host(C), ox.method_product(A, B, 7, S)["C"])


@pytest.mark.parametrize("S", range(1, 33))
def test_triangle_kernel_every_S_several_chunks(S):
    """Every one-row-block triangle instantiation without the debug dump:
    the depth exceeds one exactness chunk (S K 127^2 >= 2^31), so the
    register fold carries between chunks."""
    kc = rulecheck.library_chunk("int8", 7, S)
    K = kc + 81
    A, B = mdinputs.workload("dd64", M=17, N=19, K=K)
    C, info = md.gemm_ex(dev(A), dev(B), form="int8", force_S=S, force_beta=7)
    assert info["kc"] == kc < K
    np.testing.assert_array_equal(host(C), ox.method_product(A, B, 7, S)["C"])


@pytest.mark.parametrize("beta", [7, 8])
@pytest.mark.parametrize("S", range(36, 65, 4))
def test_two_band_kernel_every_S(S, beta):
    """Every two-band instantiation (S = 36 .. 64, both digit widths): two
    bands of S/2 diagonals over the whole depth, folded in registers and
    LDS, bit-exact against the oracle; M = 70 leaves a row block past the
    padded digit array, N and K are ragged."""
    form = "int8" if beta == 7 else "int8bal"
    A, B = mdinputs.workload("od1024", M=70, N=33, K=100)
    A[:, 5, :] = 0.0
    C, info = md.gemm_ex(dev(A), dev(B), form=form, force_S=S, force_beta=beta)
    assert info["band"] == S // 2 and info["kc"] >= 100
    np.testing.assert_array_equal(host(C), ox.method_product(A, B, beta, S, balanced=beta == 8)["C"])


def test_two_bands_need_one_exactness_chunk():
    """A depth beyond one exactness chunk at S = 56 runs in bands of 14
    (the sum buffer); S = 40, which splits into neither, is refused; the
    debug dump of the diagonal sums also takes the bands."""
    kc = rulecheck.library_chunk("int8bal", 8, 56)
    A, B = mdinputs.workload("od1024", M=20, N=18, K=kc + 70)
    C, info = md.gemm_ex(dev(A), dev(B), form="int8bal", force_S=56, force_beta=8)
    assert info["band"] == 14 and info["kc"] == kc
    np.testing.assert_array_equal(host(C), ox.method_product(A, B, 8, 56, balanced=True)["C"])
    kc40 = rulecheck.library_chunk("int8bal", 8, 40)
    A, B = mdinputs.workload("od1024", M=4, N=4, K=kc40 + 70)
    with pytest.raises(md.MDError) as err:
        md.gemm_ex(dev(A), dev(B), form="int8bal", force_S=40, force_beta=8)
    assert err.value.code == 7
    A, B = mdinputs.workload("od1024", M=21, N=19, K=70)
    got, info = run_debug(A, B, "int8", 56, 7)
    assert info["band"] == 14
    check_against_oracle(A, B, got, 7, 56)


@pytest.mark.parametrize("m", [1, 16])
@pytest.mark.parametrize("form", ["int8", "fp64"])
def test_word_counts_one_and_sixteen(m, form):
    """Doubles and hexa-doubles: the rule's parameters sit within the
    oracle's budget, the output equals the oracle's method at the library's
    S bit for bit and is within 2^-T.
    At m = 16 the banded kernels' LDS fold does not fit (S = 120 INT8,
    about 40 FP64), so their diagonal sums go through the [S][M][N] buffer
    and the separate fold-and-round kernel."""
    r = np.random.Generator(np.random.PCG64(700 + m))
    A = mdinputs.mdouble(r, m, (20, 50), ("log2uniform", 6.0))
    B = mdinputs.mdouble(r, m, (50, 24), ("log2uniform", 6.0))
    C, info = md.gemm_ex(dev(A), dev(B), form=form)
    C = host(C)
    T = ox.TARGET_BITS[m]
    _, sA = ox.row_exponents(A[0])
    _, sB = ox.row_exponents(B[0].T)
    G = ox.span_G(max(sA), max(sB))
    _, G_rho = ox.rho_G(A, B)
    if G_rho is not None:
        G = min(G, G_rho)
    rulecheck.check_info(info, form, 50, T, G)
    beta, S = info["beta"], info["S"]
    np.testing.assert_array_equal(C, ox.method_product(A, B, beta, S)["C"])
    num, L = ox.exact_product(A, B)
    anum, _ = ox.abs_product(A, B)
    assert max(ox.error_report(C, num, anum, L).values()) <= -T


def test_global_fold_debug_dump():
    """Forced S = 80 (five bands of 16): the LDS fold would need 172 KB, so
    the banded kernel adds its diagonal sums into the caller's debug buffer,
    which the fold-and-round kernel then reads; every step bit-exact."""
    A, B = mdinputs.workload("od1024", M=37, N=45, K=130)
    got, info = run_debug(A, B, "int8", 80, 7)
    assert info["S"] == 80 and info["band"] == 16
    check_against_oracle(A, B, got, 7, 80)


def test_rho_certificate_falls_back_to_span():
    """A zero magnitude product (disjoint supports) leaves only the span
    certificate; the product is then exactly zero where it must be."""
    A, B = mdinputs.workload("dd64", M=16, N=16, K=64)
    A[:, :, 32:] = 0.0
    B[:, :32, :] = 0.0
    C, info = md.gemm_ex(dev(A), dev(B), form="int8")
    assert info["G_rho"] == -1 and info["G"] == info["G_span"]
    assert np.all(host(C) == 0.0)


def test_dd64_workload_both_forms_full():
    """The double-double 64^3 workload, every entry."""
    A, B = mdinputs.workload("dd64")
    num, L = ox.exact_product(A, B)
    anum, _ = ox.abs_product(A, B)
    for form in ("fp64", "int8"):
        C, info = md.gemm_ex(dev(A), dev(B), form=form)
        C = host(C)
        ref = ox.method_product(A, B, info["beta"], info["S"])
        np.testing.assert_array_equal(C, ref["C"])
        assert max(ox.error_report(C, num, anum, L).values()) <= -100


def test_degenerate_sizes():
    A, B = mdinputs.workload("dd64", M=5, N=6, K=7)
    # K = 0: exact zeros
    Z = torch.full((2, 5, 6), 7.0, dtype=torch.float64, device="cuda")
    C, _ = md.gemm_ex(torch.zeros((2, 5, 0), dtype=torch.float64, device="cuda"),
                      torch.zeros((2, 0, 6), dtype=torch.float64, device="cuda"), Z)
    assert np.all(host(C) == 0.0)
    # M = 0: nothing happens
    C0, _ = md.gemm_ex(torch.zeros((2, 0, 7), dtype=torch.float64, device="cuda"), dev(B))
    assert C0.shape == (2, 0, 6)
    # all-zero inputs
    C, _ = md.gemm_ex(dev(np.zeros_like(A)), dev(B), form="int8")
    assert np.all(host(C) == 0.0) and not np.any(np.signbit(host(C)))
    # a single entry: the m-double product of two m-doubles
    a, b = A[:, :1, :1], B[:, :1, :1]
    for form in ("int8", "fp64"):
        C, info = md.gemm_ex(dev(a), dev(b), form=form)
        ref = ox.method_product(a, b, info["beta"], info["S"])
        np.testing.assert_array_equal(host(C), ref["C"])


def test_run_to_run_bit_identity():
    A, B = mdinputs.workload("qd1024", M=96, N=80, K=300)
    dA, dB = dev(A), dev(B)
    for form in ("int8", "fp64"):
        C1 = host(md.gemm_ex(dA, dB, form=form)[0])
        C2 = host(md.gemm_ex(dA, dB, form=form)[0])
        np.testing.assert_array_equal(C1, C2)


def test_forced_too_few_slices_fail_the_bound():
    """The bound check is not vacuous: too few slices must violate it."""
    A, B = mdinputs.workload("qd1024", M=16, N=16, K=64)
    C, _ = md.gemm_ex(dev(A), dev(B), form="int8", force_S=16, force_beta=7)
    num, L = ox.exact_product(A, B)
    anum, _ = ox.abs_product(A, B)
    assert max(ox.error_report(host(C), num, anum, L).values()) > -200


@pytest.mark.parametrize("form", ["int8", "fp64"])
def test_qd1024_workload_sampled(form):
    """Quad-double 1024^3 (leading words +-2^U(-8,8)): a 48 x 48 grid of
    entries bit-exact against the C oracle's method layer and within 2^-200
    of the exact product."""
    A, B = mdinputs.workload("qd1024")
    C, info = md.gemm_ex(dev(A), dev(B), form=form)
    C = host(C)
    rows = np.linspace(0, 1023, 48).astype(np.int64)
    cols = np.linspace(0, 1023, 48).astype(np.int64)
    E, F, D, Cref = coracle.method_entries(A, B, info["beta"], info["S"], rows, cols)
    np.testing.assert_array_equal(C[:, rows][:, :, cols], Cref)
    ii, jj = np.meshgrid(rows, cols, indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    Cq = np.ascontiguousarray(np.transpose(C[:, ii, jj], (1, 0)))
    _, absab, err = coracle.exact_entries(A, B, ii, jj, Cq)
    rel = np.abs(err) / absab
    assert np.all(rel <= 2.0 ** -200), np.log2(rel.max())


@functools.lru_cache(maxsize=1)
def qd4096():
    return mdinputs.workload("qd4096")


GRID64 = np.linspace(0, 4095, 64).astype(np.int64)


@pytest.mark.parametrize("form", ["int8bal", "int8", "fp64"])
def test_qd4096_benchmark_workload_grid64(form):
    """The quad-double 4096^3 benchmark product in the launch configuration
    the benchmark times, in its three forms: a 64 x 64 grid of entries
    (4,096, every 65th row and column from 0 to 4095) bit-exact against the
    C oracle's method layer at the library's S, within 2^-200 of the exact
    product, and within the certified bound; S within the budget."""
    A, B = qd4096()
    C, info = md.gemm_ex(dev(A), dev(B), form=form)
    C = host(C)
    assert info["S"] == {"int8bal": 27, "int8": 30, "fp64": 10}[form]
    rulecheck.check_info(info, form, 4096, 200, info["G"])
    rows = cols = GRID64
    _, _, _, Cref = coracle.method_entries(A, B, info["beta"], info["S"], rows, cols,
                                           balanced=form == "int8bal")
    np.testing.assert_array_equal(C[:, rows][:, :, cols], Cref)
    ii, jj = np.meshgrid(rows, cols, indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    Cq = np.ascontiguousarray(np.transpose(C[:, ii, jj], (1, 0)))
    _, absab, err = coracle.exact_entries(A, B, ii, jj, Cq)
    rel = np.abs(err) / absab
    assert np.all(rel <= 2.0 ** -200), np.log2(rel.max())
    assert np.log2(rel.max()) <= info["log2_bound"]
