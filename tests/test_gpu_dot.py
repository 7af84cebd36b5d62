"""Batched m-double inner products on the GPU (the paper's experiment,
Section 3) against the oracle, through the C ABI (needs an MI355X).

* small ragged batches, m = 1, 2, 4, 8, 16, all three slice forms, the
  library's own rule: parameters within the oracle's budget, every output
  word equal to the oracle's method (greedy rounding makes the output
  unique), and every product within 2^-T of sum_k |x_k||y_k| of the exact
  one;
* the lane-wise INT8 kernels (digits cut in registers, m <= 4) and the
  matrix-core kernel (digits through LDS, m = 8 and 16) where each pair's depth
  is split over several workgroups, and where one workgroup takes a whole
  pair and finds its exponents and certificate statistics itself (hinted
  calls equal to the rule's, forced S equal to the oracle);
* the paper's parameters (FP64 form, beta = 13, S = 4m) on the paper's bit
  pattern, m = 1..16: bit-exact against the oracle;
* the inner products against the diagonal of the matrix product (a separate
  GPU path) with the same forced parameters: bit-identical;
* the paper's workload size (1,024 pairs of length 6,144, bit pattern):
  sampled pairs bit-exact against the C oracle's method and within 2^-T of
  the exact products;
* degenerate sizes.
"""
from fractions import Fraction

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


def random_batch(m, nb, n, seed, lead=("log2uniform", 8.0)):
    r = rng(seed)
    return mdinputs.mdouble(r, m, (nb, n), lead), mdinputs.mdouble(r, m, (nb, n), lead)


def check_bound(X, Y, out, T):
    vals, absvals = ox.exact_dots(X, Y)
    for b in range(X.shape[1]):
        err = abs(ox.entry_value(out[:, b]) - vals[b])
        assert err <= Fraction(2) ** -T * absvals[b], b
        assert ox.is_nonoverlapping(out[:, b], strong=True), b


@pytest.mark.parametrize("m", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("form", ["int8bal", "int8", "fp64"])
def test_dot_small_rule_bitexact(m, form):
    X, Y = random_batch(m, 37, 130, 100 + m)
    X[:, 5, :] = 0.0                      # an all-zero vector: its product is 0
    out, info = md.dot_ex(dev(X), dev(Y), form=form)
    out = host(out)
    rulecheck.check_info(info, form, 130, ox.TARGET_BITS[m], ox.dot_G(X, Y))
    beta, S = info["beta"], info["S"]
    _, ref = ox.method_dot(X, Y, beta, S, balanced=form == "int8bal")
    np.testing.assert_array_equal(out, ref)
    assert np.all(out[:, 5] == 0.0)
    check_bound(X, Y, out, ox.TARGET_BITS[m])


@pytest.mark.parametrize("m", [1, 2, 4, 8, 16])
def test_dot_paper_parameters_on_paper_pattern(m):
    r = rng(200 + m)
    X, _, _ = mdinputs.paper_pattern(r, m, (20, 100))
    Y, _, _ = mdinputs.paper_pattern(r, m, (20, 100))
    out, info = md.dot_ex(dev(X), dev(Y), form="fp64", force_S=4 * m, force_beta=13)
    assert (info["S"], info["beta"]) == (4 * m, 13)
    _, ref = ox.method_dot(X, Y, 13, 4 * m)
    np.testing.assert_array_equal(host(out), ref)


@pytest.mark.parametrize("form,S,beta", [("int8", 30, 7), ("int8", 48, 7), ("fp64", 12, 18)])
def test_dot_equals_gemm_diagonal(form, S, beta):
    """Pair b's product is entry (b, b) of X Y^T: the matrix-product kernels
    with the same forced parameters must give the same words."""
    X, Y = random_batch(4, 40, 200, 300)
    out, _ = md.dot_ex(dev(X), dev(Y), form=form, force_S=S, force_beta=beta)
    C, _ = md.gemm_ex(dev(X), dev(Y), transB=True, form=form, force_S=S, force_beta=beta)
    C = host(C)
    np.testing.assert_array_equal(host(out), C[:, np.arange(40), np.arange(40)])


@pytest.mark.parametrize("form", ["int8", "int8bal"])
@pytest.mark.parametrize("m,nb", [(4, 1024), (16, 256)])
def test_dot_paper_workload_sampled(m, nb, form):
    """Inner products of length 6,144 on the bit pattern (the paper's Table 2
    workload: 1,024 pairs; 256 at m = 16 to bound the generator's host
    memory), both INT8 forms: 16 sampled pairs bit-exact against the C
    oracle's method and within 2^-T of the exact products."""
    r = rng(400 + m)
    X, _, _ = mdinputs.paper_pattern(r, m, (nb, 6144))
    Y, _, _ = mdinputs.paper_pattern(r, m, (nb, 6144))
    out, info = md.dot_ex(dev(X), dev(Y), form=form)
    out = host(out)
    pairs = np.linspace(0, nb - 1, 16).astype(np.int64)
    Xs = np.ascontiguousarray(X[:, pairs, :])
    Ys = np.ascontiguousarray(np.transpose(Y[:, pairs, :], (0, 2, 1)))
    idx = np.arange(len(pairs), dtype=np.int64)
    for a in idx:
        _, _, _, Cref = coracle.method_entries(Xs, Ys, info["beta"], info["S"], idx[a:a + 1],
                                               idx[a:a + 1], balanced=form == "int8bal")
        np.testing.assert_array_equal(out[:, pairs[a]], Cref[:, 0, 0])
    Cq = np.ascontiguousarray(out[:, pairs].T)
    _, absab, err = coracle.exact_entries(Xs, Ys, idx, idx, Cq)
    assert np.all(np.abs(err) / absab <= 2.0 ** -ox.TARGET_BITS[m])


@pytest.mark.parametrize("form", ["int8bal", "int8"])
@pytest.mark.parametrize("m", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("nb,n", [(3, 9037), (2, 20011)])
def test_dot_lane_depth_ranges(nb, n, m, form):
    """A few long pairs: the lane-wise INT8 kernels (m <= 4) and the
    matrix-core kernel (m = 8, 16) split each pair's depth over several
    workgroups (64-bit atomic adds into the diagonal sums, then the separate
    rounding kernel); the statistics from the per-pair pass (3 pairs) or from
    the exponent and magnitude kernels over the whole depth (2 pairs of
    20,011).  Ragged lengths; bit-exact against the oracle's method at the
    library's S."""
    X, Y = random_batch(m, nb, n, 700 + m + n)
    X[:, 1, 4000:4100] = 0.0
    out, info = md.dot_ex(dev(X), dev(Y), form=form)
    _, ref = ox.method_dot(X, Y, info["beta"], info["S"], balanced=form == "int8bal")
    np.testing.assert_array_equal(host(out), ref)


@pytest.mark.parametrize("form", ["int8bal", "int8"])
@pytest.mark.parametrize("rule", ["span", "rho"])
@pytest.mark.parametrize("m", [2, 4, 8, 16])
def test_dot_whole_pair_calls(m, rule, form):
    """Calls with a given S take each pair in one workgroup that finds the
    exponents, the statistics and (ratio rule) the magnitude product itself
    and rounds the pair's product: a hinted call equals the rule's call word
    for word and certifies what the rule chose (S_min, G, G_span, G_rho); a
    forced S equals the oracle's method at that S.  A zero vector and a run
    of zero entries included."""
    X, Y = random_batch(m, 70, 530, 800 + m)
    X[:, 3, :] = 0.0
    Y[:, 7, 100:200] = 0.0
    out, info = md.dot_ex(dev(X), dev(Y), form=form, rule=rule)
    cert = md.new_cert()
    oh, _ = md.dot_ex(dev(X), dev(Y), form=form, rule=rule, s_hint=info["S"], cert=cert)
    np.testing.assert_array_equal(host(oh), host(out))
    c = md.read_cert(cert)
    assert c["flags"] == 0 and c["S_min"] == info["S"]
    assert (c["G"], c["G_span"], c["G_rho"]) == (info["G"], info["G_span"], info["G_rho"])
    # a forced S above the rule's: one band up to 32, else the fewest bands
    # of at most 16 that split it equally
    S2 = next(c for c in range(info["S"] + 1, info["S"] + 17)
              if c <= 32 or c % -(-c // 16) == 0)
    of, i2 = md.dot_ex(dev(X), dev(Y), form=form, force_S=S2, force_beta=info["beta"])
    assert i2["S"] == S2
    _, ref = ox.method_dot(X, Y, info["beta"], S2, balanced=form == "int8bal")
    np.testing.assert_array_equal(host(of), ref)
    assert np.all(host(out)[:, 3] == 0.0)


def test_dot_degenerate_sizes():
    # n = 0: exact zeros
    X = torch.zeros((4, 6, 0), dtype=torch.float64, device="cuda")
    out = torch.full((4, 6), 3.0, dtype=torch.float64, device="cuda")
    md.dot_ex(X, X, out)
    assert np.all(host(out) == 0.0)
    # batch = 0: nothing happens
    E = torch.zeros((2, 0, 5), dtype=torch.float64, device="cuda")
    assert md.dot_ex(E, E)[0].shape == (2, 0)
    # one pair of length one: the m-double product of two m-doubles
    for m in (1, 8, 16):
        X, Y = random_batch(m, 1, 1, 500 + m)
        for form in ("int8", "fp64"):
            out, info = md.dot_ex(dev(X), dev(Y), form=form)
            _, ref = ox.method_dot(X, Y, info["beta"], info["S"])
            np.testing.assert_array_equal(host(out), ref)


@pytest.mark.parametrize("form", ["int8bal", "int8"])
@pytest.mark.parametrize("m,S", [(8, 20), (8, 36), (8, 48), (8, 64), (16, 70), (16, 90), (16, 112), (16, 128)])
def test_dot_matrix_core_containers(m, S, form):
    """The matrix-core inner-product kernel in every container it is built
    for (m = 8: 32, 48, 64 digits; m = 16: 80, 96, 112, 128), both digit
    forms (the sign-magnitude limb store sits beside the digit rows in the
    containers of 32 and 48), with S forced (one band up to 32, else equal
    bands of at most 16), a ragged depth over several rounds and a zero
    vector: every word equal to the oracle's method at that S."""
    X, Y = random_batch(m, 5, 301, 900 + m + S)
    X[:, 2, :] = 0.0
    beta = 8 if form == "int8bal" else 7
    out, info = md.dot_ex(dev(X), dev(Y), form=form, force_S=S, force_beta=beta)
    assert info["S"] == S
    _, ref = ox.method_dot(X, Y, beta, S, balanced=form == "int8bal")
    np.testing.assert_array_equal(host(out), ref)
    assert np.all(host(out)[:, 2] == 0.0)
