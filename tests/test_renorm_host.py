"""Host build of the kernels' renormalisation header against the oracle.

``paper_2606_20863_amd/csrc/renorm.h`` holds the exact greedy
round-to-nearest that the INT8 triangle kernels run in registers: carry the
fold columns (28 bits for 7-bit digits, 32 for the balanced 8-bit ones),
take the magnitude in 32-bit limbs, then one rounding
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

# (S, digit bits) whose register layouts differ: (columns, limbs) =
# (2, 3), (5, 6), (9, 9), (16, 16) for 28-bit columns, (3, 4), (8, 9),
# (15, 17) for 32-bit ones (the last two of each: octo-double widths, where
# seven of eight words take the fixed-place alignment of a remainder)
LAYOUTS = ((4, 7), (16, 7), (30, 7), (60, 7), (5, 8), (27, 8), (56, 8))

DRIVER = r"""
#define __device__
#define __forceinline__ inline
#include "renorm.h"
using namespace mdg;

template <int S, int B>
static void run(const int64_t* cols, int scale, int m, double* out)
{
    typedef Tri<S, B> T;
    int64_t x[T::kCols];
    for (int j = 0; j < T::kCols; ++j)
        x[j] = cols[j];
    carry_cols<T::kCW>(x);
    uint32_t L[T::kLimbs];
    double sgn = to_limbs<T::kCW>(x, L) ? -1.0 : 1.0;
    for (int t = 0; t < m; ++t)
        out[t] = rn_next(L, sgn, scale);
}

template <int S, int B>
static int lay(int which)
{
    return which == 2 ? Tri<S, B>::kCW : (which ? Tri<S, B>::kLimbs : Tri<S, B>::kCols);
}

extern "C" int layout(int S, int B, int which)
{
    if (B == 7)
        switch (S) {
        case 4: return lay<4, 7>(which);
        case 16: return lay<16, 7>(which);
        case 30: return lay<30, 7>(which);
        case 60: return lay<60, 7>(which);
        }
    if (B == 8)
        switch (S) {
        case 5: return lay<5, 8>(which);
        case 27: return lay<27, 8>(which);
        case 56: return lay<56, 8>(which);
        }
    return -1;
}

extern "C" void renorm(int S, int B, const int64_t* cols, int scale, int m, double* out)
{
    if (B == 7)
        switch (S) {
        case 4: run<4, 7>(cols, scale, m, out); break;
        case 16: run<16, 7>(cols, scale, m, out); break;
        case 30: run<30, 7>(cols, scale, m, out); break;
        case 60: run<60, 7>(cols, scale, m, out); break;
        }
    if (B == 8)
        switch (S) {
        case 5: run<5, 8>(cols, scale, m, out); break;
        case 27: run<27, 8>(cols, scale, m, out); break;
        case 56: run<56, 8>(cols, scale, m, out); break;
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
    L.layout.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.renorm.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                         ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    return L


def columns_of(X: int, nc: int, cw: int = 28):
    """cw-bit columns of X (sign on every column), the top one taking the rest."""
    s = -1 if X < 0 else 1
    a = abs(X)
    cols = [(a >> (cw * j)) & ((1 << cw) - 1) for j in range(nc - 1)] + [a >> (cw * (nc - 1))]
    return [s * c for c in cols]


def value_of(cols, cw: int = 28):
    return sum(c * (1 << (cw * j)) for j, c in enumerate(cols))


def cases(rng: random.Random, nc: int, n: int, cw: int = 28):
    """(columns, scale, m): the integer stays within what the layout holds
    (top column below 2^62)."""
    width = cw * (nc - 1) + 62
    for it in range(n):
        kind = it % 5
        if kind == 0:       # carried columns, random top
            cols = [rng.randrange(0, 1 << cw) for _ in range(nc - 1)] + [rng.randrange(-(1 << 40), 1 << 40)]
        elif kind == 1:     # uncarried column sums as a depth chunk leaves them
            cols = [rng.randrange(-(1 << 52), 1 << 52) for _ in range(nc - 1)] + [0]
        elif kind == 2:     # sparse bits: exact ties, runs of ones
            X = 0
            for _ in range(rng.randrange(1, 6)):
                X += rng.choice([1, -1]) * (1 << rng.randrange(0, width - 60))
            if rng.random() < 0.5:
                X *= (1 << rng.randrange(1, 58)) - 1
            cols = columns_of(X, nc, cw)
        elif kind == 3:     # small integers (fewer than 53 bits)
            cols = [rng.randrange(-(1 << 60), 1 << 60)] + [0] * (nc - 1)
        else:               # a random prefix of columns
            k = rng.randrange(1, nc)
            cols = [rng.randrange(-(1 << 52), 1 << 52) for _ in range(k)] + [0] * (nc - k)
        X = value_of(cols, cw)
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


@pytest.mark.parametrize("S,B", LAYOUTS)
def test_renorm_header_matches_oracle(lib, S, B):
    nc, nl, cw = lib.layout(S, B, 0), lib.layout(S, B, 1), lib.layout(S, B, 2)
    assert cw == 4 * B and nc == (S + 3) // 4 + 1 and nl * 32 >= cw * (nc - 1) + 64
    rng = random.Random(1000 + S)
    out = (ctypes.c_double * 8)()
    bad = []
    for cols, scale, m in cases(rng, nc, 2500, cw):
        arr = (ctypes.c_int64 * nc)(*cols)
        lib.renorm(S, B, arr, scale, m, out)
        got = list(out)[:m]
        ref = ox.renorm_rn(Fraction(value_of(cols, cw)) * Fraction(2) ** scale, m)
        if not same_words(got, ref):
            bad.append((cols, scale, m, got, ref))
    assert not bad, bad[:3]


def test_renorm_header_zero_and_exact_halves(lib):
    """X = 0 gives +0 words; X = 2^53 + 1 (a tie) rounds to even, leaving +-1."""
    for S, B in ((30, 7), (27, 8)):
        nc, cw = lib.layout(S, B, 0), lib.layout(S, B, 2)
        out = (ctypes.c_double * 4)()
        for X, scale in ((0, 0), ((1 << 53) + 1, 0), (-((1 << 53) + 3), -10), ((1 << 200) - 1, -200)):
            lib.renorm(S, B, (ctypes.c_int64 * nc)(*columns_of(X, nc, cw)), scale, 4, out)
            ref = ox.renorm_rn(Fraction(X) * Fraction(2) ** scale, 4)
            assert same_words(list(out), ref), (S, X, list(out), ref)
