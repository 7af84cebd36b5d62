"""Host build of the word-placement digit split against the oracle.

``paper_2606_20863_amd/csrc/split.h`` cuts an m-double entry into digits by
placing each word's truncated significand into at most two limbs of the
entry's integer (56-bit limbs with a carry for the balanced 8-bit digits,
63-bit positive and negative limbs for the 7-bit sign-magnitude digits),
four entries at a time, one per byte of each output word.  The limbs live
in a store indexed at run time (LDS in the kernels, a plain array here,
which also checks that every index stays inside the store and that the
limbs read back are left zero).  Built for the host with g++ (the
byte-permute builtin emulated from its definition: byte i of the result is
byte sel_i of the 64-bit value src:dst), it must give
the oracle's digits (``split_entry_balanced``, ``split_entry``) for every
slice count, in containers of more digits than the entry has (the extra
low digits zero), on entries far below their row's exponent, entries whose
trailing words are cut by the grid or lie wholly below it, zero and
subnormal words, negative words, and leading words just below 2^E.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import mdinputs
from oracle import exact as ox

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_20863_amd", "csrc")

# (words, container digits) pairs built by the driver
SHAPES = [(1, 8), (1, 16), (1, 24), (2, 8), (2, 16), (2, 24), (2, 32), (4, 16), (4, 24),
          (4, 32), (4, 40), (4, 48), (8, 32), (8, 40), (8, 48), (8, 56), (8, 64)]

DRIVER = r"""
#include <cstdint>
static inline uint32_t host_perm(uint32_t s0, uint32_t s1, uint32_t sel)
{
    const uint64_t d = ((uint64_t)s0 << 32) | s1;
    uint32_t r = 0;
    for (int i = 0; i < 4; ++i) {
        const uint32_t b = (sel >> (8 * i)) & 0xff;
        const uint32_t v = b < 8 ? (uint32_t)(d >> (8 * b)) & 0xff : (b == 12 ? 0u : 0xffu);
        r |= v << (8 * i);
    }
    return r;
}
#define __builtin_amdgcn_perm(a, b, c) host_perm(a, b, c)
#define __umul24(a, b) (((a) & 0xffffffu) * ((b) & 0xffffffu))
#include "split.h"
using namespace mdg;

// the limb store as a plain array, checked to start and end at zero and to
// be indexed inside its limbs
template <int NS>
struct HostLimbs {
    uint64_t v[NS] = {};
    bool bad = false;
    void add(int i, uint64_t x)
    {
        if (i < 0 || i >= NS)
            bad = true;
        else
            v[i] += x;
    }
    uint64_t take(int i)
    {
        const uint64_t x = v[i];
        v[i] = 0;
        return x;
    }
};

template <int MW, int SC, bool BAL>
static int run(const double* words, const int* kn, int pad, uint32_t* xs_out)
{
    constexpr int NS = store_limbs<SC, BAL>();
    constexpr int NL = BAL ? bal_limbs<SC>() : sm_limbs<SC>();
    HostLimbs<NS> L;
    uint32_t xs[SC];
    for (int s = 0; s < SC; ++s)
        xs[s] = 0;
    double x[4][MW];
    for (int q = 0; q < 4; ++q)
        for (int w = 0; w < MW; ++w)
            x[q][w] = words[q * MW + w];
    int rc = 0;
    auto spare_clear = [&]() {
        // every limb read back is zero again; clear the spare ones
        for (int i = 0; i < NS; ++i) {
            const bool spare = i == NL || (!BAL && i == 2 * NL + 1);
            if (!spare && L.v[i])
                rc = 2;
            if (spare)
                L.v[i] = 0;
        }
    };
    if (BAL) {
        digits_bal<0, MW, SC>(x[0], kn[0], pad, xs, L);
        spare_clear();
        digits_bal<1, MW, SC>(x[1], kn[1], pad, xs, L);
        spare_clear();
        digits_bal<2, MW, SC>(x[2], kn[2], pad, xs, L);
        spare_clear();
        digits_bal<3, MW, SC>(x[3], kn[3], pad, xs, L);
        spare_clear();
        for (int s = 0; s < SC; ++s)
            xs[s] ^= 0x80808080u;
    } else {
        digits_sm<0, MW, SC>(x[0], kn[0], pad, xs, L);
        spare_clear();
        digits_sm<1, MW, SC>(x[1], kn[1], pad, xs, L);
        spare_clear();
        digits_sm<2, MW, SC>(x[2], kn[2], pad, xs, L);
        spare_clear();
        digits_sm<3, MW, SC>(x[3], kn[3], pad, xs, L);
        spare_clear();
    }
    for (int s = 0; s < SC; ++s)
        xs_out[s] = xs[s];
    return L.bad ? 3 : rc;
}

extern "C" int host_digits(int bal, int m, int SC, const double* words, const int* kn, int pad,
                           uint32_t* xs)
{
#define CASE(MW, C)                                                   \
    if (m == MW && SC == C)                                           \
        return bal ? run<MW, C, true>(words, kn, pad, xs) : run<MW, C, false>(words, kn, pad, xs);
    CASES
    return 1;
}
"""


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    d = tmp_path_factory.mktemp("splithost")
    src = d / "split_host.cpp"
    cases = " ".join(f"CASE({m}, {sc})" for m, sc in SHAPES)
    src.write_text(DRIVER.replace("CASES", cases))
    so = d / "libsplit_host.so"
    subprocess.run(["g++", "-std=c++17", "-O1", "-shared", "-fPIC", "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", "-I" + CSRC, str(src), "-o", str(so)], check=True)
    L = ctypes.CDLL(str(so))
    L.host_digits.restype = ctypes.c_int
    L.host_digits.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                              ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    return L


def library_digits(lib, bal, words4, Es, S, SC):
    """Digits (4, SC) of four entries (words4: (4, m)), shared exponents Es."""
    m = words4.shape[1]
    bits = 8 if bal else 7
    Eg = [E + (ox.BAL_HEADROOM if bal else 0) for E in Es]
    kn = np.array([g + 1075 - bits * S for g in Eg], dtype=np.int32)
    w = np.ascontiguousarray(words4, dtype=np.float64)
    xs = np.zeros(SC, dtype=np.uint32)
    rc = lib.host_digits(int(bal), m, SC, w.ctypes.data, kn.ctypes.data, bits * (SC - S), xs.ctypes.data)
    assert rc == 0, rc   # 1 no such shape, 2 a limb left nonzero, 3 a limb index outside the store
    by = xs.view(np.uint8).reshape(SC, 4).T.astype(np.int8).astype(np.int64)
    return by


def oracle_digits(bal, words, E, S):
    if bal:
        return ox.split_entry_balanced(words, E, S)
    return ox.split_entry(words, E, 7, S)


def entries(m, seed, n):
    """n entries of m words with their shared exponents: the row's exponent
    at or above the entry's own, by up to 80 bits."""
    r = np.random.Generator(np.random.PCG64(seed))
    planes = mdinputs.mdouble(r, m, (n,), ("log2uniform", 20.0))
    words = planes.T.copy()                       # (n, m)
    Es = []
    for i in range(n):
        e = ox.frexp_exponent(words[i, 0]) if words[i, 0] != 0.0 else 0
        Es.append(e + int(r.integers(0, 4)) + (int(r.integers(0, 80)) if i % 5 == 0 else 0))
    return words, Es


def check(lib, bal, words, Es, S, SC):
    n = words.shape[0]
    for i in range(0, n - 3, 4):
        got = library_digits(lib, bal, words[i:i + 4], Es[i:i + 4], S, SC)
        for q in range(4):
            want = oracle_digits(bal, words[i + q], Es[i + q], S)
            assert list(got[q, :S]) == want, (bal, S, SC, words[i + q], Es[i + q])
            assert not np.any(got[q, S:]), (bal, S, SC)


@pytest.mark.parametrize("bal", [True, False])
@pytest.mark.parametrize("m,SC", SHAPES)
def test_placement_digits_equal_oracle(lib, bal, m, SC):
    words, Es = entries(m, 1000 + 10 * m + SC + bal, 48)
    bits = 8 if bal else 7
    # every S that fits the container, down to where most words are cut
    smin = max(1, SC - 7)
    for S in range(smin, SC + 1):
        if bal and bits * S < 4:
            continue
        check(lib, bal, words, Es, S, SC)


@pytest.mark.parametrize("bal", [True, False])
def test_placement_edge_entries(lib, bal):
    """Zero and subnormal words, leading words just below 2^E, negative
    trailing words, and entries wholly below the grid."""
    m, SC, S = 4, 32, 27 if bal else 30
    tiny = np.nextafter(0.0, 1.0)
    cases = [
        ([np.nextafter(1.0, 0.0), 2.0 ** -54, -2.0 ** -108, 2.0 ** -163], 0),
        ([-np.nextafter(1.0, 0.0), -2.0 ** -54, 2.0 ** -108, -2.0 ** -163], 0),
        ([0.75, -2.0 ** -55, 0.0, 0.0], 0),
        ([0.0, 0.0, 0.0, 0.0], 5),
        ([2.0 ** -1000, 2.0 ** -1060, 4 * tiny, tiny], -999),
        ([-2.0 ** -1020, tiny * 3, 0.0, 0.0], -1019),
        ([1.5 * 2.0 ** 600, -2.0 ** 548, 2.0 ** 494, -2.0 ** 440], 601),
        ([2.0 ** -300, 2.0 ** -354, 2.0 ** -408, 2.0 ** -462], -100),   # far below the row
        ([0.5, 2.0 ** -300, 0.0, 0.0], 0),                              # second word below the grid
        ([-0.5 - 2.0 ** -53, -2.0 ** -107, -2.0 ** -161, -2.0 ** -215], 0),
    ]
    words = np.array([c[0] for c in cases] + [[0.0] * 4] * 2)
    Es = [c[1] for c in cases] + [0, 0]
    check(lib, bal, words, Es, S, SC)
