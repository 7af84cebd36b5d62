"""Seeded sweep of batched inner products (``md_dot_ex``) over ragged batch
sizes and lengths, m = 1, 2, 4, 8, 16, the three slice forms, wide exponent
ranges, zero vectors and runs of zero entries.  The slice rule picks S; every
output word equals the oracle's method layer at the call's (beta, S) (the C
oracle, one pair at a time: a 1 x 1 product whose exponents are the pair's),
sampled pairs meet the call's certified bound against the exact inner
product, and in the INT8 forms a call hinted with the rule's S returns the
same words and certifies that S (Section 3, Table 2's inner products).
"""
import numpy as np
import pytest
import torch

import mdinputs
import paper_2606_20863_amd as md
from oracle import coracle
from oracle import exact as ox

pytestmark = pytest.mark.gpu

FORMS = ("int8bal", "int8", "fp64")


def case(seed):
    rng = np.random.Generator(np.random.PCG64(9000 + seed))
    m = int(rng.choice([1, 2, 4, 8, 16]))
    form = FORMS[seed % 3]
    nb = int(rng.integers(1, 61 if m == 16 else 301))
    n = int(rng.integers(1, 801 if m == 16 else 3001))
    lead = ("uniform",) if rng.integers(2) else ("log2uniform", float(rng.integers(4, 30)))
    return rng, m, form, nb, n, lead


def oracle_pairs(X, Y, beta, S, balanced):
    m, nb, _ = X.shape
    out = np.zeros((m, nb))
    z = np.zeros(1, dtype=np.int64)
    for b in range(nb):
        _, _, _, C = coracle.method_entries(np.ascontiguousarray(X[:, b:b + 1, :]),
                                            np.ascontiguousarray(np.transpose(Y[:, b:b + 1, :], (0, 2, 1))),
                                            beta, S, z, z, balanced=balanced)
        out[:, b] = C[:, 0, 0]
    return out


@pytest.mark.parametrize("seed", range(60))
def test_dot_rule_path_sweep(seed):
    rng, m, form, nb, n, lead = case(seed)
    print(f"[dot sweep] seed {seed}: m={m} {form} batch={nb} n={n} lead={lead}", flush=True)
    X = mdinputs.mdouble(rng, m, (nb, n), lead)
    Y = mdinputs.mdouble(rng, m, (nb, n), lead)
    zb = rng.choice(nb, size=min(nb, int(rng.integers(0, 3))), replace=False)
    X[:, zb, :] = 0.0
    if n > 8:
        b, k0 = int(rng.integers(nb)), int(rng.integers(n - 8))
        Y[:, b, k0:k0 + int(rng.integers(1, 9))] = 0.0
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.from_numpy(Y).cuda()
    out, info = md.dot_ex(Xd, Yd, form=form)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    beta, S = info["beta"], info["S"]
    print(f"[dot sweep]   S={S} beta={beta}", flush=True)
    np.testing.assert_array_equal(out, oracle_pairs(X, Y, beta, S, form == "int8bal"))
    assert not out[:, zb].any()
    # the certified bound on sampled pairs against the exact inner products
    idx = rng.choice(nb, size=min(nb, 48), replace=False).astype(np.int64)
    Xs = np.ascontiguousarray(X[:, idx, :])
    Ys = np.ascontiguousarray(np.transpose(Y[:, idx, :], (0, 2, 1)))
    e = np.arange(len(idx), dtype=np.int64)
    _, absab, err = coracle.exact_entries(Xs, Ys, e, e, np.ascontiguousarray(out[:, idx].T))
    nz = absab > 0
    assert not err[~nz].any()
    if nz.any():
        worst = float(np.max(np.log2(np.maximum(np.abs(err[nz]), 2.0 ** -1074) / absab[nz])))
        assert worst <= info["log2_bound"] + 1e-9
        assert worst <= -ox.TARGET_BITS[m]
    if form != "fp64":
        cert = md.new_cert()
        oh, _ = md.dot_ex(Xd, Yd, form=form, s_hint=S, cert=cert)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(oh.cpu().numpy(), out)
        c = md.read_cert(cert)
        assert c["flags"] == 0 and c["S_min"] == S
