"""Exact fixed-point results on the GPU (needs an MI355X).

md_gemm_fixed returns the product's exact sum before rounding as 32-bit
limb planes and a scale.  Checks, on ragged sizes (several tiles and a
tail) for the three slice forms, the whole-triangle and banded INT8
kernels (S up to 32 and beyond) and m = 1, 2, 4, 8:

* every limb and scale equals the oracle's fixed_product / fixed_limbs,
  also where the depth spans several exactness chunks;
* md_fixed_round of it equals md_gemm_ex with the same S and beta (and
  the oracle's method) word for word;
* a depth-split product: md_exponents of the full matrices equals the
  oracle's row exponents; the blocks' integers on those exponents (each
  computed on its own stream) equal the oracle's per block, md_fixed_add
  sums them to the whole product's integer bit for bit, and that rounds
  to md_gemm_ex's result for the whole product;
* an exponent below the data's own is refused (MD_EINPUT, flag 8), or reported in a
  device flag word without waiting;
* a seeded sweep of depth splits over forms, word counts, sizes, forced S
  and one to three random cuts.
"""
import numpy as np
import pytest
import torch

import mdinputs
import paper_2606_20863_amd as md
from oracle import exact as ox

import rulecheck

pytestmark = pytest.mark.gpu

# (form, beta, S): FP64 slices folded in LDS (sums captured, folded after)
# and through the sum buffer (beta (S+1) > 230 bits: the buffer fold writes
# the integers); INT8 whole triangle (7-bit, 8-bit: the fixed-point triangle
# kernels); INT8 bands with the diagonal-sum buffer (S > 32, equal bands of
# at most 16: the buffer fold)
CASES = [("fp64", 16, 7), ("fp64", 20, 12), ("int8", 7, 12), ("int8bal", 8, 9), ("int8bal", 8, 27),
         ("int8", 7, 42), ("int8bal", 8, 48)]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def operands(seed, m, M, N, K, zero_row=True):
    r = np.random.Generator(np.random.PCG64(seed))
    A = mdinputs.mdouble(r, m, (M, K), ("log2uniform", 6.0))
    B = mdinputs.mdouble(r, m, (K, N), ("uniform",))
    if zero_row:
        A[:, 3, :] = 0.0
        B[:, :, 5] = 0.0
    return A, B


def limbs_of(X, nlimb):
    """(nlimb, M, N) int32 array of the oracle's integers."""
    M, N = X.shape
    out = np.zeros((nlimb, M, N), dtype=np.uint32)
    for i in range(M):
        for j in range(N):
            out[:, i, j] = ox.fixed_limbs(int(X[i, j]), nlimb)
    return out.view(np.int32)


@pytest.mark.parametrize("form,beta,S", CASES)
@pytest.mark.parametrize("m", [2, 4])
def test_fixed_product_matches_oracle_and_rounds_to_the_product(form, beta, S, m):
    M, N, K = 37, 45, 150
    A, B = operands(100 * S + m, m, M, N, K)
    X, scale, info = md.gemm_fixed(dev(A), dev(B), S=S, beta=beta, form=form)
    torch.cuda.synchronize()
    assert (info["S"], info["beta"]) == (S, beta)
    nlimb = X.shape[0]
    assert nlimb == md.fixed_limbs(beta, S, K)
    Xo, so = ox.fixed_product(A, B, beta, S, balanced=form == "int8bal")
    np.testing.assert_array_equal(X.cpu().numpy(), limbs_of(Xo, nlimb))
    np.testing.assert_array_equal(scale.cpu().numpy(), so.astype(np.int32))
    C = md.fixed_round(X, scale, m)
    Cg, _ = md.gemm_ex(dev(A), dev(B), form=form, force_S=S, force_beta=beta)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(C.cpu().numpy(), Cg.cpu().numpy())
    ref = ox.method_product(A, B, beta, S, balanced=form == "int8bal")
    np.testing.assert_array_equal(C.cpu().numpy(), ref["C"])


@pytest.mark.parametrize("form,beta,S,K,kc", [("int8bal", 8, 27, 5000, 4800), ("int8", 7, 30, 4500, 4416),
                                               ("int8bal", 8, 36, 3700, 3584), ("fp64", 20, 10, 900, 816)])
def test_fixed_product_over_several_exactness_chunks(form, beta, S, K, kc):
    """Depths beyond one exactness chunk (kc: the oracle's exact depth for
    this S and beta, rounded down to whole fragments): the captured diagonal
    sums accumulate over the chunks (whole-triangle, banded and FP64
    kernels), the integer equals the oracle's and rounds to md_gemm_ex's
    output."""
    assert rulecheck.library_chunk(form, beta, S) == kc < K
    m, M, N = 2, 20, 24
    A, B = operands(K + S, m, M, N, K)
    X, scale, info = md.gemm_fixed(dev(A), dev(B), S=S, beta=beta, form=form)
    torch.cuda.synchronize()
    assert info["kc"] == kc
    Xo, so = ox.fixed_product(A, B, beta, S, balanced=form == "int8bal")
    np.testing.assert_array_equal(X.cpu().numpy(), limbs_of(Xo, X.shape[0]))
    np.testing.assert_array_equal(scale.cpu().numpy(), so.astype(np.int32))
    C = md.fixed_round(X, scale, m)
    Cg, _ = md.gemm_ex(dev(A), dev(B), form=form, force_S=S, force_beta=beta)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(C.cpu().numpy(), Cg.cpu().numpy())


@pytest.mark.parametrize("form,beta,S", [("fp64", 20, 6), ("int8", 7, 16), ("int8bal", 8, 13),
                                         ("int8bal", 8, 36)])
@pytest.mark.parametrize("m", [1, 8])
def test_depth_split_sums_exactly(form, beta, S, m):
    M, N, K, k0 = 33, 70, 200, 77
    A, B = operands(7000 + S + m, m, M, N, K)
    # the second block's rows of A are scaled down so that its own
    # exponents differ from the full rows'
    A[:, :, k0:] *= 2.0 ** -5
    Ad, Bd = dev(A), dev(B)
    E, F = md.exponents(Ad, Bd)
    torch.cuda.synchronize()
    Eo, _ = ox.row_exponents(A[0])
    Fo, _ = ox.row_exponents(B[0].T)
    np.testing.assert_array_equal(E.cpu().numpy(), Eo)
    np.testing.assert_array_equal(F.cpu().numpy(), Fo)
    nlimb = md.fixed_limbs(beta, S, K)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    cur = torch.cuda.current_stream()
    s1.wait_stream(cur)
    s2.wait_stream(cur)
    with torch.cuda.stream(s1):
        X1, sc1, _ = md.gemm_fixed(Ad[:, :, :k0], Bd[:, :k0, :], E, F, S=S, beta=beta, form=form,
                                   nlimb=nlimb, stream=s1)
    with torch.cuda.stream(s2):
        X2, sc2, _ = md.gemm_fixed(Ad[:, :, k0:], Bd[:, k0:, :], E, F, S=S, beta=beta, form=form,
                                   nlimb=nlimb, stream=s2)
    cur.wait_stream(s1)
    cur.wait_stream(s2)
    Xs = md.fixed_add(X1, X2)
    Xw, scw, _ = md.gemm_fixed(Ad, Bd, S=S, beta=beta, form=form)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(sc1.cpu().numpy(), scw.cpu().numpy())
    np.testing.assert_array_equal(sc2.cpu().numpy(), scw.cpu().numpy())
    np.testing.assert_array_equal(Xs.cpu().numpy(), Xw.cpu().numpy())
    bal = form == "int8bal"
    for Xb, sl in ((X1, slice(0, k0)), (X2, slice(k0, K))):
        Xo, _ = ox.fixed_product(A[:, :, sl], B[:, sl, :], beta, S, E=Eo, F=Fo, balanced=bal)
        np.testing.assert_array_equal(Xb.cpu().numpy(), limbs_of(Xo, nlimb))
    C = md.fixed_round(Xs, scw, m)
    Cg, _ = md.gemm_ex(Ad, Bd, form=form, force_S=S, force_beta=beta)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(C.cpu().numpy(), Cg.cpu().numpy())


def test_depth_split_in_four_blocks_with_coarser_exponents():
    """Exponents above the data's own (a coarser grid) are taken as given:
    four blocks add up to the whole product on that grid."""
    m, M, N, K, S, beta = 4, 20, 24, 260, 14, 8
    A, B = operands(42, m, M, N, K, zero_row=False)
    Ad, Bd = dev(A), dev(B)
    E, F = md.exponents(Ad, Bd)
    E = (E + 1).contiguous()
    F = (F + 2).contiguous()
    nlimb = md.fixed_limbs(beta, S, K)
    cuts = [0, 64, 65, 200, K]
    acc = None
    for a, b in zip(cuts[:-1], cuts[1:]):
        Xb, sc, _ = md.gemm_fixed(Ad[:, :, a:b], Bd[:, a:b, :], E, F, S=S, beta=beta, form="int8bal",
                                  nlimb=nlimb)
        acc = Xb if acc is None else md.fixed_add(acc, Xb)
    Xw, scw, _ = md.gemm_fixed(Ad, Bd, E, F, S=S, beta=beta, form="int8bal")
    torch.cuda.synchronize()
    np.testing.assert_array_equal(acc.cpu().numpy(), Xw.cpu().numpy())
    np.testing.assert_array_equal(sc.cpu().numpy(), scw.cpu().numpy())
    Eo = [int(v) for v in E.cpu().numpy()]
    Fo = [int(v) for v in F.cpu().numpy()]
    Xo, so = ox.fixed_product(A, B, beta, S, E=Eo, F=Fo, balanced=True)
    np.testing.assert_array_equal(Xw.cpu().numpy(), limbs_of(Xo, nlimb))
    np.testing.assert_array_equal(scw.cpu().numpy(), so.astype(np.int32))


def test_fixed_add_wraps_and_carries():
    """Limb addition with carries across every limb, and two's complement
    wrap-around, against Python integers."""
    r = np.random.Generator(np.random.PCG64(5))
    nlimb, count = 6, 1000
    vals = []
    for _ in range(count):
        k = int(r.integers(0, 4))
        if k == 0:
            a, b = (1 << 191) - 1, 1                                   # wraps to -2^191
        elif k == 1:
            a, b = -1, 1                                               # carries through all limbs
        else:
            a = int.from_bytes(r.bytes(23), "little") - (1 << 183)
            b = int.from_bytes(r.bytes(23), "little") - (1 << 183)
        vals.append((a, b))
    X = np.array([ox.fixed_limbs(a, nlimb) for a, _ in vals], dtype=np.uint32).T.copy().view(np.int32)
    Y = np.array([ox.fixed_limbs(b, nlimb) for _, b in vals], dtype=np.uint32).T.copy().view(np.int32)
    Z = md.fixed_add(dev(X), dev(Y)).cpu().numpy().view(np.uint32)
    for e, (a, b) in enumerate(vals):
        s = (a + b) % (1 << 192)
        assert [int(v) for v in Z[:, e]] == [(s >> (32 * k)) & 0xffffffff for k in range(nlimb)]


def test_fixed_round_matches_oracle_on_sparse_integers():
    """Rounding alone: exact ties, runs of ones, negative values, zero."""
    r = np.random.Generator(np.random.PCG64(11))
    nlimb, count, m = 8, 400, 4
    ints, scales = [], []
    for e in range(count):
        if e == 0:
            v = 0
        elif e % 3 == 0:
            v = ((1 << 53) + 1) << int(r.integers(0, 150))
        elif e % 3 == 1:
            v = ((1 << int(r.integers(60, 200))) - 1) * int(r.choice([1, -1]))
        else:
            v = int.from_bytes(r.bytes(31), "little") - (1 << 247)
        ints.append(v)
        scales.append(int(r.integers(-400, 100)))
    X = np.array([ox.fixed_limbs(v, nlimb) for v in ints], dtype=np.uint32).T.copy().view(np.int32)
    C = md.fixed_round(dev(X), dev(np.array(scales, dtype=np.int32)), m).cpu().numpy()
    from fractions import Fraction
    for e, (v, s) in enumerate(zip(ints, scales)):
        ref = ox.renorm_rn(Fraction(v) * Fraction(2) ** s, m)
        got = list(C[:, e])
        assert all(a == b and np.signbit(a) == np.signbit(b) for a, b in zip(got, ref)), (e, got, ref)


def test_exponent_below_the_data_is_refused():
    m, M, N, K = 2, 16, 16, 64
    A, B = operands(3, m, M, N, K, zero_row=False)
    Ad, Bd = dev(A), dev(B)
    E, F = md.exponents(Ad, Bd)
    E[4] -= 1
    with pytest.raises(md.MDError) as ei:
        md.gemm_fixed(Ad, Bd, E, F, S=6, beta=8, form="int8bal")
    assert ei.value.code == 9 and ei.value.input_flags == 8
    F[0] = 1101
    E[4] += 1
    with pytest.raises(md.MDError) as ei:
        md.gemm_fixed(Ad, Bd, E, F, S=6, beta=8, form="int8bal")
    assert ei.value.input_flags == 8


def test_depth_split_at_the_benchmark_size():
    """The quad-double 4096^3 benchmark product in the balanced INT8 form
    (S = 27, the rule's choice) cut into four uneven depth blocks: the
    blocks' integers on the full matrices' exponents add up to the whole
    product's integer in every entry, that rounds to md_gemm_ex's output in
    every entry, and an 8 x 8 grid of the integers equals the oracle's
    fixed product of those rows and columns."""
    A, B = mdinputs.workload("qd4096")
    Ad, Bd = dev(A), dev(B)
    Cg, info = md.gemm_ex(Ad, Bd, form="int8bal")
    S, beta, K = info["S"], info["beta"], 4096
    assert (S, beta) == (27, 8)
    E, F = md.exponents(Ad, Bd)
    nlimb = md.fixed_limbs(beta, S, K)
    cuts = [0, 1000, 2048, 3001, K]
    acc = sc = None
    for a, b in zip(cuts[:-1], cuts[1:]):
        Xb, sc, _ = md.gemm_fixed(Ad[:, :, a:b], Bd[:, a:b, :], E, F, S=S, beta=beta, form="int8bal",
                                  nlimb=nlimb)
        acc = Xb if acc is None else md.fixed_add(acc, Xb)
        del Xb
    Xw, scw, _ = md.gemm_fixed(Ad, Bd, S=S, beta=beta, form="int8bal")
    assert torch.equal(acc, Xw) and torch.equal(sc, scw)
    del acc
    assert torch.equal(md.fixed_round(Xw, scw, 4), Cg)
    rows = np.linspace(0, 4095, 8).astype(np.int64)
    cols = np.linspace(0, 4095, 8).astype(np.int64)
    Eh, Fh = E.cpu().numpy(), F.cpu().numpy()
    assert list(Eh[rows]) == ox.row_exponents(A[0][rows])[0]
    assert list(Fh[cols]) == ox.row_exponents(B[0][:, cols].T)[0]
    Xo, so = ox.fixed_product(np.ascontiguousarray(A[:, rows, :]), np.ascontiguousarray(B[:, :, cols]),
                              beta, S, E=list(Eh[rows]), F=list(Fh[cols]), balanced=True)
    ti, tj = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()
    np.testing.assert_array_equal(Xw[:, ti][:, :, tj].cpu().numpy(), limbs_of(Xo, nlimb))
    np.testing.assert_array_equal(scw[ti][:, tj].cpu().numpy(), so.astype(np.int32))


@pytest.mark.parametrize("S", range(1, 33))
@pytest.mark.parametrize("form", ["int8", "int8bal"])
def test_fixed_triangle_kernel_every_S(form, S):
    """Every instantiated fixed-point triangle kernel (S = 1..32, 7- and
    8-bit digits) on ragged sizes (row and column tiles past M and N): the
    integers equal the oracle's, and rounding them gives md_gemm_ex's
    output."""
    m, M, N, K = 2, 40, 36, 70
    beta = 8 if form == "int8bal" else 7
    A, B = operands(500 + S, m, M, N, K)
    X, scale, info = md.gemm_fixed(dev(A), dev(B), S=S, beta=beta, form=form)
    Cg, _ = md.gemm_ex(dev(A), dev(B), form=form, force_S=S, force_beta=beta)
    torch.cuda.synchronize()
    assert info["band"] == S
    Xo, so = ox.fixed_product(A, B, beta, S, balanced=form == "int8bal")
    np.testing.assert_array_equal(X.cpu().numpy(), limbs_of(Xo, X.shape[0]))
    np.testing.assert_array_equal(scale.cpu().numpy(), so.astype(np.int32))
    np.testing.assert_array_equal(md.fixed_round(X, scale, m).cpu().numpy(), Cg.cpu().numpy())


def test_broadcast_views_are_refused():
    """A broadcast view would be read past its storage if taken as dense
    planes: the binding refuses it before any call."""
    A = torch.zeros(64, dtype=torch.float64, device="cuda").expand(2, 16, 64)
    B = torch.zeros(2, 64, 8, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        md.gemm_fixed(A, B, S=4, beta=8, form="int8bal")
    with pytest.raises(ValueError):
        md.exponents(A, B)


def test_exponent_flags_without_waiting():
    """With a device flag word the fixed-point calls do not synchronise: two
    depth blocks on two streams with one shared flag word sum to the whole
    product, the word stays 0; an exponent below the data's own sets bit 8
    in it instead of raising."""
    m, M, N, K, k0, S, beta = 2, 30, 26, 140, 61, 10, 8
    A, B = operands(8080, m, M, N, K)
    Ad, Bd = dev(A), dev(B)
    E, F = md.exponents(Ad, Bd)
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    nlimb = md.fixed_limbs(beta, S, K)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    cur = torch.cuda.current_stream()
    s1.wait_stream(cur)
    s2.wait_stream(cur)
    with torch.cuda.stream(s1):
        X1, sc, _ = md.gemm_fixed(Ad[:, :, :k0], Bd[:, :k0, :], E, F, S=S, beta=beta, form="int8bal",
                                  nlimb=nlimb, flags=flags, stream=s1)
    with torch.cuda.stream(s2):
        X2, _, _ = md.gemm_fixed(Ad[:, :, k0:], Bd[:, k0:, :], E, F, S=S, beta=beta, form="int8bal",
                                 nlimb=nlimb, flags=flags, stream=s2)
    cur.wait_stream(s1)
    cur.wait_stream(s2)
    Xs = md.fixed_add(X1, X2)
    Xw, scw, _ = md.gemm_fixed(Ad, Bd, S=S, beta=beta, form="int8bal")
    torch.cuda.synchronize()
    assert int(flags.item()) == 0
    assert torch.equal(Xs, Xw) and torch.equal(sc, scw)
    E[2] -= 1
    md.gemm_fixed(Ad, Bd, E, F, S=S, beta=beta, form="int8bal", flags=flags)
    torch.cuda.synchronize()
    assert int(flags.item()) == 8


def draw_split_cases(n=24, seed=4096):
    r = np.random.Generator(np.random.PCG64(seed))
    cases = []
    for c in range(n):
        form = ("fp64", "int8", "int8bal")[c % 3]
        m = int(r.choice([1, 2, 4, 8, 16]))
        M, N = int(r.integers(1, 71)), int(r.integers(1, 71))
        K = int(r.integers(2, 301))
        if form == "fp64":
            beta = int(r.integers(12, 23))
            S = int(r.integers(2, 15))
        else:
            beta = 7 if form == "int8" else 8
            S = int(r.integers(1, 33)) if r.random() < 0.7 else int(r.choice([36, 42, 48, 52, 60, 64]))
        ncut = int(r.integers(1, 4))
        cuts = sorted(set(int(v) for v in r.integers(1, K, ncut)))
        cases.append((c, form, m, M, N, K, beta, S, cuts, int(r.integers(0, 2 ** 31))))
    return cases


@pytest.mark.parametrize("case", draw_split_cases(), ids=lambda c: f"split{c[0]}-{c[1]}-m{c[2]}-S{c[7]}")
def test_random_depth_split(case):
    """Seeded sweep: slice form, word count, ragged sizes, forced S (whole
    triangles, bands, FP64 LDS and buffer folds), one to three random depth
    cuts.  The blocks' integers on the full exponents sum to the whole
    product's, which equals the oracle's; rounding the sum gives
    md_gemm_ex's output."""
    _, form, m, M, N, K, beta, S, cuts, seed = case
    r = np.random.Generator(np.random.PCG64(seed))
    lead = ("uniform",) if r.random() < 0.5 else ("log2uniform", float(r.integers(1, 12)))
    A = mdinputs.mdouble(r, m, (M, K), lead)
    B = mdinputs.mdouble(r, m, (K, N), lead)
    Ad, Bd = dev(A), dev(B)
    E, F = md.exponents(Ad, Bd)
    nlimb = md.fixed_limbs(beta, S, K)
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    acc = sc = None
    for a, b in zip([0] + cuts, cuts + [K]):
        Xb, sc, _ = md.gemm_fixed(Ad[:, :, a:b], Bd[:, a:b, :], E, F, S=S, beta=beta, form=form, nlimb=nlimb,
                                  flags=flags)
        acc = Xb if acc is None else md.fixed_add(acc, Xb)
    Xw, scw, _ = md.gemm_fixed(Ad, Bd, S=S, beta=beta, form=form)
    Cg, _ = md.gemm_ex(Ad, Bd, form=form, force_S=S, force_beta=beta)
    C = md.fixed_round(acc, sc, m)
    torch.cuda.synchronize()
    assert int(flags.item()) == 0
    assert torch.equal(acc, Xw) and torch.equal(sc, scw)
    assert torch.equal(C, Cg)
    Xo, so = ox.fixed_product(A, B, beta, S, balanced=form == "int8bal")
    np.testing.assert_array_equal(Xw.cpu().numpy(), limbs_of(Xo, nlimb))
    np.testing.assert_array_equal(scw.cpu().numpy(), so.astype(np.int32))


def test_exponents_of_a_very_deep_product():
    """Depth 20,000,000 (beyond 65535 blocks of 256 in the exponent pass's
    second grid dimension, so its blocks deepen): the shared exponents of
    both operands equal the oracle's."""
    r = np.random.Generator(np.random.PCG64(77))
    K = 20_000_000
    A = np.ldexp(r.uniform(-1, 1, (1, 2, K)), r.integers(-30, 30, (1, 2, K)))
    B = np.ldexp(r.uniform(-1, 1, (1, K, 3)), r.integers(-30, 30, (1, K, 3)))
    A[0, 1, K - 1] = 2.0 ** 40           # the maximum sits in the last block
    B[0, 0, 2] = 2.0 ** 41
    E, F = md.exponents(dev(A), dev(B))
    torch.cuda.synchronize()
    assert list(E.cpu().numpy()) == ox.row_exponents(A[0])[0]
    assert list(F.cpu().numpy()) == ox.row_exponents(B[0].T)[0]


@pytest.mark.parametrize("form,beta,S", [("int8bal", 8, 14), ("int8", 7, 16), ("fp64", 20, 6)])
def test_depth_split_with_rows_zero_in_one_block(form, beta, S):
    """A row of A and a column of B that are zero in one depth block only,
    with negative whole-depth exponents (leading words below 1/2): the
    block's integers on the whole-depth grid are zero there, the call takes
    the given exponents (no flag), and the blocks sum and round to the
    whole product's output."""
    m, M, N, K, k0 = 4, 12, 10, 90, 40
    r = np.random.Generator(np.random.PCG64(515))
    A = mdinputs.mdouble(r, m, (M, K), ("log2uniform", 8.0))
    B = mdinputs.mdouble(r, m, (K, N), ("log2uniform", 8.0))
    A[:, 2, :] *= 2.0 ** -20            # whole-depth exponents well below 0
    B[:, :, 7] *= 2.0 ** -20
    A[:, 2, :k0] = 0.0                  # zero in the first block only
    B[:, k0:, 7] = 0.0                  # zero in the second block only
    Eo, _ = ox.row_exponents(A[0])
    Fo, _ = ox.row_exponents(B[0].T)
    assert Eo[2] < 0 and Fo[7] < 0
    Ad, Bd = dev(A), dev(B)
    E, F = md.exponents(Ad, Bd)
    nlimb = md.fixed_limbs(beta, S, K)
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    X1, sc, _ = md.gemm_fixed(Ad[:, :, :k0], Bd[:, :k0, :], E, F, S=S, beta=beta, form=form, nlimb=nlimb,
                              flags=flags)
    X2, sc2, _ = md.gemm_fixed(Ad[:, :, k0:], Bd[:, k0:, :], E, F, S=S, beta=beta, form=form, nlimb=nlimb,
                               flags=flags)
    Xs = md.fixed_add(X1, X2)
    C = md.fixed_round(Xs, sc, m)
    Cg, _ = md.gemm_ex(Ad, Bd, form=form, force_S=S, force_beta=beta)
    torch.cuda.synchronize()
    assert int(flags.item()) == 0
    np.testing.assert_array_equal(sc.cpu().numpy(), sc2.cpu().numpy())
    bal = form == "int8bal"
    for Xb, sl in ((X1, slice(0, k0)), (X2, slice(k0, K))):
        Xo, so = ox.fixed_product(A[:, :, sl], B[:, sl, :], beta, S, E=Eo, F=Fo, balanced=bal)
        np.testing.assert_array_equal(Xb.cpu().numpy(), limbs_of(Xo, nlimb))
        np.testing.assert_array_equal(sc.cpu().numpy(), so.astype(np.int32))
    np.testing.assert_array_equal(C.cpu().numpy(), Cg.cpu().numpy())
