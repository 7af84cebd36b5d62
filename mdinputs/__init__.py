"""Seeded synthetic m-double matrices for the m-double matrix product.

This module is shared by the oracle and by the HIP path (tests and bench).
It only draws words; it holds none of the method's arithmetic (no exponent
alignment, no split, no slice products, no fold, no renormalisation).

Layout: an m-double matrix of shape (R, C) is a float64 array of shape
(m, R, C), one plane per word, word 0 the leading one.

Workloads (the five product configurations of the method):

* ``dd64``    m=2, 64^3, leading words U(-1,1).
* ``qd1024``  m=4, 1024^3, leading words +-2^U(-8,8) (random sign).
* ``qd4096``  m=4, 4096^3, leading words U(-1,1).
* ``dd2048``  m=2, 2048^3, forward plus adjoint; W drawn like A and B.
* ``od1024``  m=8, 1024^3, leading words +-2^U(-16,16); W with U(-1,1)
  leading words (the workload does not say how W is drawn).

Trailing words follow w_{t+1} = w_t * 2^-53 * U(-1,1).  Where that draw
exceeds ulp(w_t)/2 in magnitude, one ulp(w_t) moves from w_{t+1} into w_t
(the sum is unchanged and both moves are exact), so every generated entry is
nonoverlapping in the strong sense |w_{t+1}| <= ulp(w_t)/2.

Seeds: workload index c uses ``np.random.SeedSequence(20863 + c).spawn(3)``,
one PCG64 stream each for A, B and W.

``paper_pattern`` draws the bit pattern of the paper's timing experiment
(Section 2): every word's 52 fraction bits are four groups of a leading one
followed by twelve random bits, so the four 13-bit quarters of a word have
fixed exponents.  It returns the drawn groups too, so that a split can be
checked against them.
"""
from __future__ import annotations

import numpy as np

WORKLOADS = {
    # name: (index, m, M, N, K, lead distribution for A and B, lead for W)
    "dd64": (0, 2, 64, 64, 64, ("uniform",), ("uniform",)),
    "qd1024": (1, 4, 1024, 1024, 1024, ("log2uniform", 8.0), ("uniform",)),
    "qd4096": (2, 4, 4096, 4096, 4096, ("uniform",), ("uniform",)),
    "dd2048": (3, 2, 2048, 2048, 2048, ("uniform",), ("uniform",)),
    "od1024": (4, 8, 1024, 1024, 1024, ("log2uniform", 16.0), ("uniform",)),
}


def _lead(rng: np.random.Generator, shape, dist) -> np.ndarray:
    if dist[0] == "uniform":
        return rng.uniform(-1.0, 1.0, size=shape)
    if dist[0] == "log2uniform":
        r = dist[1]
        mag = np.exp2(rng.uniform(-r, r, size=shape))
        sign = np.where(rng.integers(0, 2, size=shape) == 0, -1.0, 1.0)
        return sign * mag
    raise ValueError(f"unknown lead distribution {dist!r}")


def mdouble(rng: np.random.Generator, m: int, shape, lead=("uniform",)) -> np.ndarray:
    """Draw an m-double array of the given shape (returned as (m, *shape))."""
    shape = tuple(int(s) for s in shape)
    out = np.zeros((m,) + shape, dtype=np.float64)
    out[0] = _lead(rng, shape, lead)
    for t in range(m - 1):
        w = out[t]
        u = rng.uniform(-1.0, 1.0, size=shape)
        raw = (w * u) * 2.0 ** -53
        ulp = np.spacing(np.abs(w))
        ulp = np.where(w == 0.0, 0.0, ulp)
        fix = np.abs(raw) > 0.5 * ulp
        step = np.where(fix, np.sign(raw) * ulp, 0.0)
        out[t] = w + step
        out[t + 1] = raw - step
    if not strongly_nonoverlapping(out):
        raise RuntimeError("generated words overlap; choose another seed")
    return out


def strongly_nonoverlapping(planes: np.ndarray) -> bool:
    """|w_{t+1}| <= ulp(w_t)/2 for every entry, zero words only trailing."""
    m = planes.shape[0]
    for t in range(m - 1):
        a = np.abs(planes[t])
        b = np.abs(planes[t + 1])
        ulp = np.where(a == 0.0, 0.0, np.spacing(a))
        if np.any(b > 0.5 * ulp):
            return False
    return True


def seeds(index: int):
    """(rng_A, rng_B, rng_W) for workload index ``index``."""
    ss = np.random.SeedSequence(20863 + index).spawn(3)
    return tuple(np.random.Generator(np.random.PCG64(s)) for s in ss)


def workload(name: str, M=None, N=None, K=None, with_w: bool = False):
    """Planes (A, B[, W]) for a named workload, optionally at other sizes.

    A is (m, M, K), B is (m, K, N), W is (m, M, N).  Sizes default to the
    workload's own; smaller sizes draw from the same seeded streams.
    """
    idx, m, M0, N0, K0, lead, wlead = WORKLOADS[name]
    M = M0 if M is None else M
    N = N0 if N is None else N
    K = K0 if K is None else K
    ra, rb, rw = seeds(idx)
    A = mdouble(ra, m, (M, K), lead)
    B = mdouble(rb, m, (K, N), lead)
    if not with_w:
        return A, B
    W = mdouble(rw, m, (M, N), wlead)
    return A, B, W


def paper_pattern(rng: np.random.Generator, m: int, shape):
    """Words in the bit pattern of the paper's experiment (Section 2).

    Each word is +-(1 g_0 1 g_1 1 g_2 1 g_3) read as a binary fraction whose
    first one is the leading (hidden) bit at 2^0, scaled by 2^(-52 w) for word
    w, with g_q twelve random bits.  Word w's quarter q then holds exactly
    the 13 bits ``(1 << 12) | g_q`` at weights 2^(-13(4w+q))..2^(-13(4w+q)-12),
    so all quarters of all words tile one 13-bit grid.

    Returns (planes, groups, signs): planes (m, *shape) float64, groups
    (m, 4, *shape) int64 holding the 13-bit quarter values, signs (m, *shape)
    in {-1, +1}.
    """
    shape = tuple(int(s) for s in shape)
    groups = rng.integers(0, 1 << 12, size=(m, 4) + shape, dtype=np.int64)
    groups = groups | (1 << 12)
    signs = np.where(rng.integers(0, 2, size=(m,) + shape) == 0, -1, 1)
    planes = np.zeros((m,) + shape, dtype=np.float64)
    for w in range(m):
        mant = np.zeros(shape, dtype=np.int64)
        for q in range(4):
            mant = (mant << 13) | groups[w, q]
        # mant has 52 significant bits: its top bit is 2^0 of the word, so
        # the word is mant * 2^-51 * 2^(-52 w).
        planes[w] = signs[w] * np.ldexp(mant.astype(np.float64), -51 - 52 * w)
    return planes, groups, signs


# The paper's experiment (Section 3, Table 2): 1,024 inner products of
# vectors of length 6,144 in the bit pattern, m = 1, 2, 4, 8, 16.
PAPER_DOT = {"index": 5, "batch": 1024, "n": 6144, "m": (1, 2, 4, 8, 16)}


def paper_dot_workload(m: int = 16, batch=None, n=None):
    """(X, Y), each (m, batch, n) planes in the paper's bit pattern, from
    the seeded streams of the inner-product workload.  The first w words of
    an m-word pattern entry are a w-word pattern entry, so one draw at
    m = 16 serves every smaller m by slicing."""
    batch = PAPER_DOT["batch"] if batch is None else batch
    n = PAPER_DOT["n"] if n is None else n
    rx, ry, _ = seeds(PAPER_DOT["index"])
    X, _, _ = paper_pattern(rx, m, (batch, n))
    Y, _, _ = paper_pattern(ry, m, (batch, n))
    return X, Y
