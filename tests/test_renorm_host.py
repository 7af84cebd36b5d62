"""Host build of the kernels' renormalisation header against the oracle.

``paper_2606_20863_amd/csrc/renorm.h`` holds the exact greedy
round-to-nearest that the INT8 triangle kernels run in registers: carry the
28-bit fold columns, take the magnitude in 32-bit limbs, then one rounding
step per word (left-aligned limbs with fixed-place significand, round and
sticky bits; the general step where a word would be subnormal).  Compiled
for the host with g++ (the two device annotations defined away), it must
reproduce the oracle's ``renorm_rn`` word for word, the sign of zero
included, on random multiword integers, sparse bit patterns with exact ties
and long runs of ones, small integers, and scales that make the words
subnormal or round them to zero.  The GPU parity tests cover the same code
inside the kernels on the generated workloads, whose outputs are never
subnormal.
"""
import ctypes
import os
import random
import subprocess
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact as ox

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_20863_amd", "csrc")

# S values whose register layouts differ: (columns, limbs) = (2, 3), (5, 6), (9, 9)
S_VALUES = (4, 16, 30)

DRIVER = r"""
#define __device__
#define __forceinline__ inline
#include "renorm.h"
using namespace mdg;

template <int S>
static void run(const int64_t* cols, int scale, int m, double* out)
{
    int64_t x[Tri<S>::kCols];
    for (int j = 0; j < Tri<S>::kCols; ++j)
        x[j] = cols[j];
    carry28(x);
    uint32_t L[Tri<S>::kLimbs];
    double sgn = to_limbs(x, L) ? -1.0 : 1.0;
    for (int t = 0; t < m; ++t)
        out[t] = rn_next(L, sgn, scale);
}

extern "C" int layout(int S, int which)
{
    switch (S) {
    case 4: return which ? Tri<4>::kLimbs : Tri<4>::kCols;
    case 16: return which ? Tri<16>::kLimbs : Tri<16>::kCols;
    case 30: return which ? Tri<30>::kLimbs : Tri<30>::kCols;
    }
    return -1;
}

extern "C" void renorm(int S, const int64_t* cols, int scale, int m, double* out)
{
    switch (S) {
    case 4: run<4>(cols, scale, m, out); break;
    case 16: run<16>(cols, scale, m, out); break;
    case 30: run<30>(cols, scale, m, out); break;
    }
}
"""


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    d = tmp_path_factory.mktemp("renorm")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    so = d / "librenorm_host.so"
    subprocess.run(["g++", "-std=c++17", "-O1", "-shared", "-fPIC", "-I", CSRC, str(src), "-o",
                    str(so)], check=True)
    L = ctypes.CDLL(str(so))
    L.layout.argtypes = [ctypes.c_int, ctypes.c_int]
    L.renorm.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_int,
                         ctypes.POINTER(ctypes.c_double)]
    return L


def columns_of(X: int, nc: int):
    """28-bit columns of X (sign on every column), the top one taking the rest."""
    s = -1 if X < 0 else 1
    a = abs(X)
    cols = [(a >> (28 * j)) & ((1 << 28) - 1) for j in range(nc - 1)] + [a >> (28 * (nc - 1))]
    return [s * c for c in cols]


def value_of(cols):
    return sum(c * (1 << (28 * j)) for j, c in enumerate(cols))


def cases(rng: random.Random, nc: int, n: int):
    """(columns, scale, m): the integer stays within what the layout holds
    (top column below 2^62)."""
    width = 28 * (nc - 1) + 62
    for it in range(n):
        kind = it % 5
        if kind == 0:       # carried columns, random top
            cols = [rng.randrange(0, 1 << 28) for _ in range(nc - 1)] + [rng.randrange(-(1 << 40), 1 << 40)]
        elif kind == 1:     # uncarried column sums as a depth chunk leaves them
            cols = [rng.randrange(-(1 << 52), 1 << 52) for _ in range(nc - 1)] + [0]
        elif kind == 2:     # sparse bits: exact ties, runs of ones
            X = 0
            for _ in range(rng.randrange(1, 6)):
                X += rng.choice([1, -1]) * (1 << rng.randrange(0, width - 60))
            if rng.random() < 0.5:
                X *= (1 << rng.randrange(1, 58)) - 1
            cols = columns_of(X, nc)
        elif kind == 3:     # small integers (fewer than 53 bits)
            cols = [rng.randrange(-(1 << 60), 1 << 60)] + [0] * (nc - 1)
        else:               # a random prefix of columns
            k = rng.randrange(1, nc)
            cols = [rng.randrange(-(1 << 52), 1 << 52) for _ in range(k)] + [0] * (nc - k)
        X = value_of(cols)
        r = rng.random()
        if r < 0.6:
            scale = rng.randrange(-300, 10)
        elif r < 0.9:       # words near and below the subnormal threshold
            scale = -1074 - max(abs(X).bit_length(), 1) + rng.randrange(-5, 120)
        else:
            scale = rng.randrange(-1400, -900)
        yield cols, scale, rng.choice([1, 2, 4, 8])


def same_words(got, ref):
    return all(a == b and np.signbit(a) == np.signbit(b) for a, b in zip(got, ref))


@pytest.mark.parametrize("S", S_VALUES)
def test_renorm_header_matches_oracle(lib, S):
    nc, nl = lib.layout(S, 0), lib.layout(S, 1)
    assert nc == (S + 3) // 4 + 1 and nl * 32 >= 28 * (nc - 1) + 64
    rng = random.Random(1000 + S)
    out = (ctypes.c_double * 8)()
    bad = []
    for cols, scale, m in cases(rng, nc, 2500):
        arr = (ctypes.c_int64 * nc)(*cols)
        lib.renorm(S, arr, scale, m, out)
        got = list(out)[:m]
        ref = ox.renorm_rn(Fraction(value_of(cols)) * Fraction(2) ** scale, m)
        if not same_words(got, ref):
            bad.append((cols, scale, m, got, ref))
    assert not bad, bad[:3]


def test_renorm_header_zero_and_exact_halves(lib):
    """X = 0 gives +0 words; X = 2^53 + 1 (a tie) rounds to even, leaving +-1."""
    nc = lib.layout(30, 0)
    out = (ctypes.c_double * 4)()
    for X, scale in ((0, 0), ((1 << 53) + 1, 0), (-((1 << 53) + 3), -10), ((1 << 200) - 1, -200)):
        lib.renorm(30, (ctypes.c_int64 * nc)(*columns_of(X, nc)), scale, 4, out)
        ref = ox.renorm_rn(Fraction(X) * Fraction(2) ** scale, 4)
        assert same_words(list(out), ref), (X, list(out), ref)
