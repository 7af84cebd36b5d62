"""Exact oracle for the m-double matrix product by error-free summation.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU leg of ``bench.py`` (``cpu_baseline`` and the sampled error
check); never by the product path.

Notation (paper Section 2, generalised from the double-double inner product
to a matrix product):

* A is M x K and B is K x N; each entry is an m-double, an unevaluated sum of
  nonoverlapping doubles (paper Section 1).  Planes: ``A[w, i, k]``.
* E_i is the shared exponent of row i of A, F_j that of column j of B.
* beta is the slice (digit) width, S the number of slices per entry.  The
  paper cuts each double into four 13-bit quarters, i.e. beta = 13 and
  S = 4m (Section 2).
* The diagonal sums D_t = sum_{s+u=t} sum_k d^A_{ik,s} d^B_{kj,u} for
  t = 0..S-1 are the paper's convolution sums s_i (Section 2, and the
  convolutions of the Conclusions), with S in place of 8.

Three layers:

1. exact:  C* = A B and |A||B| with every word decoded exactly;
2. method: exponents, digits, diagonal sums and their exact fold C~;
3. rounding: greedy round-to-nearest renormalisation into m words, the
   nonoverlap predicate and the error report.

Readings of the paper used here (the paper states none of these rules):

* shared exponent: E_i = max over k of the frexp exponent of the leading
  word a_ik^(0), zero words skipped, E_i = 0 for an all-zero row;
* split: per-word truncation toward zero, sign-magnitude digits,
  d_s = sum_w sgn(w) (floor(|w| 2^(beta(s+1)-E)) mod 2^beta);
* balanced INT8 digits (a second INT8 encoding, not in the paper): the same
  per-word truncation on the 8-bit grid that starts at 2^(E+2), the
  truncated integer written in base 256 with digits in [-128, 127];
* kept products: the triangle s + u <= S-1, as the paper keeps s_0..s_7;
* fusion: the diagonal sums are folded exactly and rounded once, greedily
  to nearest (ties to even) word by word.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

# Target relative accuracy 2^-T of each m-double output entry, measured
# against (|A||B|)_ij.
TARGET_BITS = {1: 50, 2: 100, 4: 200, 8: 400, 16: 800}


# ---------------------------------------------------------------------------
# exact decoding
# ---------------------------------------------------------------------------

def frexp_exponent(x: float):
    """The integer e with 2^(e-1) <= |x| < 2^e (frexp's exponent), None for 0."""
    if x == 0.0:
        return None
    return math.frexp(x)[1]


def entry_value(words) -> Fraction:
    """Exact value of an m-double given as a sequence of floats."""
    return sum((Fraction(float(w)) for w in words), Fraction(0))


def _to_scaled_ints(planes: np.ndarray):
    """Exact integer image of an m-double matrix: value = X[r, c] / 2^L.

    Returns (X, L) with X a numpy object array of Python ints.
    """
    m = planes.shape[0]
    L = 0
    for w in range(m):
        for x in planes[w].ravel():
            if x != 0.0:
                den = Fraction(float(x)).denominator
                L = max(L, den.bit_length() - 1)
    X = np.empty(planes.shape[1:], dtype=object)
    flat = X.reshape(-1)
    src = planes.reshape(m, -1)
    for idx in range(flat.shape[0]):
        v = Fraction(0)
        for w in range(m):
            v += Fraction(float(src[w, idx]))
        flat[idx] = v.numerator * (1 << L) // v.denominator
    return X, L


def exact_product(A: np.ndarray, B: np.ndarray):
    """C* = A B exactly (paper Section 2: sum_k x_k * y_k without rounding).

    A is (m, M, K), B is (m, K, N) float64 planes.  Returns (Cnum, L): an
    (M, N) object array of Python ints with C*_ij = Cnum[i, j] / 2^L.
    """
    XA, LA = _to_scaled_ints(A)
    XB, LB = _to_scaled_ints(B)
    return XA.dot(XB), LA + LB


def abs_product(A: np.ndarray, B: np.ndarray):
    """(|A||B|)_ij = sum_k |a_ik| |b_kj| exactly; same (num, L) form."""
    XA, LA = _to_scaled_ints(A)
    XB, LB = _to_scaled_ints(B)
    absf = np.vectorize(abs, otypes=[object])
    return absf(XA).dot(absf(XB)), LA + LB


# ---------------------------------------------------------------------------
# method layer: exponent alignment, split, diagonal sums, fold
# ---------------------------------------------------------------------------

def row_exponents(lead: np.ndarray):
    """Shared exponent and span of each row of a leading-word matrix (R, K).

    E_r = max_k frexp_exponent(lead[r, k]) over nonzero entries (0 if none);
    span_r = E_r - min_k frexp_exponent(lead[r, k]) (0 if none).
    For the columns of B pass ``B[0].T``.  Returns two lists of ints.
    """
    lead = np.asarray(lead, dtype=np.float64)
    _, ex = np.frexp(lead)
    nz = lead != 0.0
    any_nz = nz.any(axis=1)
    hi = np.where(nz, ex, np.iinfo(np.int32).min).max(axis=1, initial=np.iinfo(np.int32).min)
    lo = np.where(nz, ex, np.iinfo(np.int32).max).min(axis=1, initial=np.iinfo(np.int32).max)
    E = np.where(any_nz, hi, 0)
    span = np.where(any_nz, hi - lo, 0)
    return [int(v) for v in E], [int(v) for v in span]


def split_entry(words, E: int, beta: int, S: int):
    """Digits d_0..d_{S-1} of one m-double entry aligned to exponent E.

    d_s = sum_w sgn(w) * (floor(|w| * 2^(beta(s+1) - E)) mod 2^beta):
    each word is cut into beta-bit fields of the grid that starts at 2^E, as
    the paper cuts each double into quarters (Section 2, Figure 1), and the
    fields are truncated toward zero below 2^(E - beta S).
    """
    mask = (1 << beta) - 1
    d = [0] * S
    for w in words:
        w = float(w)
        if w == 0.0:
            continue
        num, den = Fraction(abs(w)).as_integer_ratio()
        e = -(den.bit_length() - 1)  # |w| = num * 2^e
        sgn = -1 if w < 0 else 1
        for s in range(S):
            sh = e + beta * (s + 1) - E
            field = (num << sh) if sh >= 0 else (num >> -sh)
            d[s] += sgn * (field & mask)
    return d


def split_planes(planes: np.ndarray, E, beta: int, S: int, by_columns: bool) -> np.ndarray:
    """Digits of every entry of an m-double matrix, as an int64 array.

    Rows of A (``by_columns=False``): planes (m, M, K), E per row, result
    (S, M, K).  Columns of B (``by_columns=True``): planes (m, K, N), E per
    column, result (S, K, N).  Same rule as ``split_entry``; vectorised with
    numpy integer shifts for speed.
    """
    m = planes.shape[0]
    E = np.asarray(E, dtype=np.int64)
    Ebc = E[None, :] if by_columns else E[:, None]
    mask = (1 << beta) - 1
    out = np.zeros((S,) + planes.shape[1:], dtype=np.int64)
    for w in range(m):
        x = planes[w]
        f, ex = np.frexp(np.abs(x))           # |x| = f 2^ex, f in [0.5, 1)
        num = np.ldexp(f, 53).astype(np.int64)  # exact: 53-bit integer
        e = ex.astype(np.int64) - 53            # |x| = num 2^e
        sgn = np.where(x < 0, -1, 1).astype(np.int64)
        for s in range(S):
            sh = e + beta * (s + 1) - Ebc
            left = np.clip(sh, 0, 62)
            right = np.clip(-sh, 0, 63)
            field = np.where(sh >= 0,
                             np.where(sh >= beta, 0, num << left),
                             np.where(-sh >= 63, 0, num >> right))
            out[s] += sgn * (field & mask)
    return out


# Balanced INT8 digits.  The sign-magnitude digits above leave the int8
# value -128 unused and spend a bit of every digit on the sign; the INT8
# matrix cores take any value in [-128, 127].  Here the digit grid starts at
# 2^(E+2), each word is truncated toward zero on it 8 S bits down, exactly
# as the sign-magnitude split truncates, and the truncated integer X is
# written in base 256 with balanced digits:
#   X = sum_s d_s 256^(S-1-s),  d_s in [-128, 127].
# |X| < 2^(8S-2) (the words' bits are disjoint and below 2^E), inside the
# range S balanced digits reach.  The entry is X 2^(E + 2 - 8 S).
BAL_BETA = 8        # digit width of the balanced form
BAL_HEADROOM = 2    # its grid starts at 2^(E + BAL_HEADROOM)
BAL_DMAX = 128      # largest digit magnitude


def truncated_integer(words, Eg: int, bits: int) -> int:
    """X = sum_w sgn(w) floor(|w| 2^(bits - Eg)): every word truncated toward
    zero on the grid of unit 2^(Eg - bits)."""
    X = 0
    for w in words:
        w = float(w)
        if w == 0.0:
            continue
        x = Fraction(abs(w)) * Fraction(2) ** (bits - Eg)
        v = x.numerator // x.denominator
        X += v if w > 0 else -v
    return X


def balanced_digits(X: int, S: int):
    """The digits d_0..d_{S-1} in [-128, 127] (d_0 most significant) with
    X = sum_s d_s 256^(S-1-s): centred remainders from the least
    significant digit up.  ValueError if S digits do not reach X."""
    d = [0] * S
    for s in range(S - 1, -1, -1):
        r = X % 256
        if r >= 128:
            r -= 256
        d[s] = r
        X = (X - r) // 256
    if X != 0:
        raise ValueError("no balanced representation in S digits")
    return d


def split_entry_balanced(words, E: int, S: int):
    """Balanced digits of one m-double entry whose shared exponent is E."""
    return balanced_digits(truncated_integer(words, E + BAL_HEADROOM, BAL_BETA * S), S)


def recode_balanced(d: np.ndarray) -> np.ndarray:
    """Base-256 digits (S, ...) of any sign, d_0 most significant, rewritten
    as balanced digits of the same integers: each digit plus the carry from
    below is replaced by its centred remainder mod 256, the rest carried up.
    ValueError if a carry leaves the top digit."""
    out = np.empty_like(d)
    carry = np.zeros(d.shape[1:], dtype=np.int64)
    for s in range(d.shape[0] - 1, -1, -1):
        v = d[s] + carry
        r = (v + 128) % 256 - 128
        out[s] = r
        carry = (v - r) // 256
    if np.any(carry != 0):
        raise ValueError("no balanced representation in S digits")
    return out


def split_planes_balanced(planes: np.ndarray, E, S: int, by_columns: bool) -> np.ndarray:
    """Balanced digits of every entry (layout as ``split_planes``): the
    sign-magnitude 8-bit digits on the grid 2^(E+2) hold the truncated
    integer with digits in [-255, 255]; ``recode_balanced`` carries them
    into [-128, 127]."""
    Eg = np.asarray(E, dtype=np.int64) + BAL_HEADROOM
    return recode_balanced(split_planes(planes, Eg, BAL_BETA, S, by_columns))


def diagonal_sums_loop(dA, dB, S: int):
    """D_t[i][j] = sum_k sum_{s=0..t} dA[i][k][s] dB[k][j][t-s], t < S.

    The convolution sums of the paper (Section 2) written out with Python
    loops, for tiny inputs: dA[i][k] and dB[k][j] are digit lists.
    """
    M, K = len(dA), len(dA[0]) if dA else 0
    N = len(dB[0]) if dB else 0
    D = [[[0] * N for _ in range(M)] for _ in range(S)]
    for t in range(S):
        for i in range(M):
            for j in range(N):
                acc = 0
                for k in range(K):
                    for s in range(t + 1):
                        acc += dA[i][k][s] * dB[k][j][t - s]
                D[t][i][j] = acc
    return D


def diagonal_sums(dA: np.ndarray, dB: np.ndarray, S: int, all_pairs: bool = False) -> np.ndarray:
    """D_t = sum_{s+u=t} dA_s @ dB_u with int64 matrix products.

    dA is (S, M, K) and dB is (S, K, N) (from ``split_planes``).  The
    triangle s + u <= S-1 gives t = 0..S-1; ``all_pairs`` keeps every pair
    (t = 0..2S-2), which reproduces the product of the truncated inputs.
    The digit bound keeps every partial sum far below 2^63.
    """
    Smax = 2 * S - 1 if all_pairs else S
    K = dA.shape[2]
    dmax = int(max(np.abs(dA).max(initial=0), np.abs(dB).max(initial=0)))
    assert S * max(K, 1) * dmax * dmax < 2 ** 62, "int64 diagonal sums could overflow"
    D = np.zeros((Smax, dA.shape[1], dB.shape[2]), dtype=np.int64)
    for t in range(Smax):
        for s in range(max(0, t - S + 1), min(t, S - 1) + 1):
            D[t] += dA[s] @ dB[t - s]
    return D


def fold(D, Ei: int, Fj: int, beta: int):
    """C~_ij = sum_t D_t 2^(E_i + F_j - beta (t + 2)) as an exact Fraction.

    D is the list of diagonal sums of one output entry.  The paper adds
    s_0 + ... + s_7 in double-double arithmetic; here the sum is exact and is
    rounded once afterwards (postponed renormalisation, Conclusions).
    """
    x = Fraction(0)
    for t, v in enumerate(D):
        x += Fraction(int(v)) * Fraction(2) ** (Ei + Fj - beta * (t + 2))
    return x


# ---------------------------------------------------------------------------
# rounding layer
# ---------------------------------------------------------------------------

def round_nearest(x: Fraction) -> float:
    """Round a rational to the nearest binary64, ties to even.

    Integer arithmetic only: 53 significant bits, the unit clamped at
    2^-1074 for subnormal results, +-inf past the largest finite double.
    """
    if x == 0:
        return 0.0
    sign = -1.0 if x < 0 else 1.0
    p, q = abs(x.numerator), x.denominator
    e = p.bit_length() - q.bit_length()        # 2^e <= p/q < 2^(e+1) ?
    if (p << max(-e, 0)) < (q << max(e, 0)):
        e -= 1
    unit = max(e - 52, -1074)
    if unit >= 0:
        n, r = divmod(p, q << unit)
        den = q << unit
    else:
        n, r = divmod(p << -unit, q)
        den = q
    if 2 * r > den or (2 * r == den and (n & 1)):
        n += 1
    try:
        return sign * math.ldexp(float(n), unit)
    except OverflowError:
        return sign * math.inf


def renorm_rn(x: Fraction, m: int):
    """Greedy m-word renormalisation: w_t = RN(x - sum_{u<t} w_u)."""
    words = []
    r = Fraction(x)
    for _ in range(m):
        w = round_nearest(r)
        words.append(w)
        r -= Fraction(w)
    return words


def ulp(w: float) -> Fraction:
    """Unit in the last place of a nonzero double (2^-1074 for subnormals)."""
    e = frexp_exponent(w)
    return Fraction(2) ** max(e - 53, -1074)


def is_nonoverlapping(words, strong: bool = True) -> bool:
    """Nonoverlap of an m-double.

    strong: |w_{t+1}| <= ulp(w_t)/2 for every t, and once a word is zero all
    later words are zero (-0 counts as 0).
    weak:   words decreasing with disjoint bit ranges: the lowest set bit of
    w_t lies above the highest set bit of w_{t+1}.
    """
    words = [float(w) for w in words]
    for t in range(len(words) - 1):
        a, b = words[t], words[t + 1]
        if a == 0.0:
            if b != 0.0:
                return False
            continue
        if b == 0.0:
            continue
        if strong:
            if Fraction(abs(b)) > ulp(a) / 2:
                return False
        else:
            na, da = Fraction(abs(a)).as_integer_ratio()
            nb, db = Fraction(abs(b)).as_integer_ratio()
            low_a = (na & -na).bit_length() - 1 - (da.bit_length() - 1)
            high_b = nb.bit_length() - 1 - (db.bit_length() - 1)
            if not high_b < low_a:
                return False
    return True


# Preconditions of the method's inputs, as flags (0: all hold).
PRE_NONFINITE = 1   # a word is an infinity or a NaN
PRE_OVERLAP = 2     # not weakly nonoverlapping (a zero word before a nonzero one included)
PRE_RANGE = 4       # a nonzero leading word outside [2^-900, 2^900)


def precondition_flags(words) -> int:
    """The preconditions an m-double entry must meet: finite words, weakly
    nonoverlapping (``is_nonoverlapping(strong=False)``), and a leading word
    that is zero or has 2^-900 <= |w_0| < 2^900 (so that the digit grids and
    the fold scale stay inside the double range).  Returns the OR of the
    PRE_* flags that fail."""
    words = [float(w) for w in words]
    if any(math.isinf(w) or math.isnan(w) for w in words):
        return PRE_NONFINITE
    f = 0
    if not is_nonoverlapping(words, strong=False):
        f |= PRE_OVERLAP
    w0 = words[0]
    if w0 != 0.0 and not (Fraction(2) ** -900 <= Fraction(abs(w0)) < Fraction(2) ** 900):
        f |= PRE_RANGE
    return f


def log2_fraction(x: Fraction) -> float:
    """log2 of a positive Fraction, accurate to a few ulps, any magnitude."""
    p, q = x.numerator, x.denominator
    sp = max(p.bit_length() - 60, 0)
    sq = max(q.bit_length() - 60, 0)
    return math.log2(p >> sp) + sp - math.log2(q >> sq) - sq


def error_report(C: np.ndarray, Cnum, Canum, L: int, entries=None):
    """log2(|sum_w C_ij^(w) - C*_ij| / (|A||B|)_ij) for each checked entry.

    C is (m, M, N) planes; Cnum / Canum are the exact C* and |A||B| numerators
    over 2^L (``exact_product``, ``abs_product``).  An entry with
    (|A||B|)_ij = 0 reports -inf when C_ij is exactly zero and +inf otherwise;
    an exact entry reports -inf.  Returns a dict (i, j) -> float.
    """
    m, M, N = C.shape
    if entries is None:
        entries = [(i, j) for i in range(M) for j in range(N)]
    scale = Fraction(1, 1 << L)
    out = {}
    for (i, j) in entries:
        err = abs(entry_value(C[:, i, j]) - Fraction(int(Cnum[i, j])) * scale)
        den = Fraction(int(Canum[i, j])) * scale
        if den == 0:
            out[(i, j)] = -math.inf if err == 0 else math.inf
        elif err == 0:
            out[(i, j)] = -math.inf
        else:
            out[(i, j)] = log2_fraction(err / den)
    return out


# ---------------------------------------------------------------------------
# the slice-count rule (error budget) and parameter choice
# ---------------------------------------------------------------------------

def ceil_log2(n: int) -> int:
    return (n - 1).bit_length()


def slice_count(beta: int, T: int, G: int) -> int:
    """Smallest S with beta*S >= T + G + ceil(log2(S+2)) + 1.

    Budget: per product term the truncated split and the dropped triangle
    err by less than (S + 1 + 2^-(beta S)) 2^(E_i + F_j - beta S); with
    2^G >= max_ij N_ij 2^(E_i+F_j) / (|A||B|)_ij this is < 2^-(T+1) of
    (|A||B|)_ij, and the final rounding adds at most 2^-(53m) < 2^-(T+5).
    """
    S = 1
    while beta * S < T + G + ceil_log2(S + 2) + 1:
        S += 1
    return S


def slice_count_balanced(T: int, G: int) -> int:
    """Smallest S with 8 S >= T + G + ceil(log2(S+3)) + 3 (balanced form).

    Budget per product term a b (|a| < 2^E_i, |b| < 2^F_j, grids 2^(E_i+2)
    and 2^(F_j+2)): truncation errs by less than 2^(E_i+2-8S) on a (the
    dropped bits of the words are disjoint) and |a^| < 2^E_i, so the
    truncated product errs by less than 2^(E_i+F_j+3-8S); the dropped pairs
    s + u >= S, with |d| <= 128, add less than
    (S-1) (256/255) 2^(E_i+F_j+2-8S).  Together less than
    (S+3) 2^(E_i+F_j+2-8S) for S <= 511, which the rule keeps below
    2^-(T+1) of (|A||B|)_ij as for the sign-magnitude form.
    """
    S = 1
    while BAL_BETA * S < T + G + ceil_log2(S + 3) + 3:
        S += 1
    return S


def span_G(span_A: int, span_B: int) -> int:
    """G from exponent spans: every nonzero |a_ik| >= 2^(E_i - span_A - 1)
    (strongly nonoverlapping words), likewise b, so the ratio
    N_ij 2^(E_i+F_j) / (|A||B|)_ij is below 2^(span_A + span_B + 2)."""
    return span_A + span_B + 2


def rho_G(A: np.ndarray, B: np.ndarray):
    """Magnitude certificate for the ratio N_ij 2^(E_i+F_j) / (|A||B|)_ij.

    q_ik = floor(|a_ik^(0)| 2^(7 - E_i)) and likewise for the columns of B;
    strongly nonoverlapping words give |a_ik| >= (1 - 2^-52) q_ik 2^(E_i-7),
    hence the ratio is at most K 2^14 / ((1 - 2^-51) min_ij P_ij) with
    P = q_A q_B.  Returns (min P, G): G the smallest g >= 0 with
    min P * 2^g >= K 2^14 + 1, or None when min P = 0.
    """
    K = A.shape[2]
    E, _ = row_exponents(A[0])
    F, _ = row_exponents(B[0].T)
    qa = np.zeros(A.shape[1:], dtype=np.int64)
    qb = np.zeros(B.shape[1:], dtype=np.int64)
    for i in range(A.shape[1]):
        for k in range(K):
            x = Fraction(abs(float(A[0, i, k]))) * Fraction(2) ** (7 - E[i])
            qa[i, k] = x.numerator // x.denominator
    for k in range(K):
        for j in range(B.shape[2]):
            x = Fraction(abs(float(B[0, k, j]))) * Fraction(2) ** (7 - F[j])
            qb[k, j] = x.numerator // x.denominator
    P = qa @ qb
    minP = int(P.min())
    if minP == 0:
        return 0, None
    target = K * (1 << 14) + 1
    g = 0
    while (minP << g) < target:
        g += 1
    return minP, g


# Exactness ranges of the accumulators (Section 2: the partial sums of the
# slice products must stay below a threshold for the summation to be exact).
INT32_LIMIT = 1 << 31   # INT8 slices, INT32 accumulation
FP64_LIMIT = 1 << 53    # FP64 slices: every integer below 2^53 is a double
FP64_BETAS = range(8, 25)   # FP64 digit widths considered


def digit_max(form: str, beta: int) -> int:
    """Largest digit magnitude: 2^beta - 1 for sign-magnitude digits, 128 for
    the balanced 8-bit digits."""
    return BAL_DMAX if form == "int8bal" else (1 << beta) - 1


def min_slices(form: str, T: int, G: int, beta: int = 0) -> int:
    """The budget's smallest slice count for target 2^-T and ratio exponent
    G: ``slice_count`` with beta = 7 (int8) or the given beta (fp64), or
    ``slice_count_balanced`` (int8bal)."""
    if form == "int8":
        return slice_count(7, T, G)
    if form == "int8bal":
        return slice_count_balanced(T, G)
    if form == "fp64":
        if not 1 <= beta <= 53:
            raise ValueError("fp64 needs a digit width")
        return slice_count(beta, T, G)
    raise ValueError(form)


def exact_depth(form: str, beta: int, S: int) -> int:
    """Largest depth Kc over which every diagonal sum stays exact: a
    diagonal of S slices holds at most S digit pairs per depth step, each
    product at most dmax^2 in magnitude, so |partial sum| <= S Kc dmax^2,
    which must stay below 2^31 (INT32) or 2^53 (FP64)."""
    limit = FP64_LIMIT if form == "fp64" else INT32_LIMIT
    d = digit_max(form, beta)
    return (limit - 1) // (S * d * d)


def budget_params(form: str, K: int, T: int, G: int):
    """(beta, S, Kc) from the error budget and the exactness range alone:
    S the smallest slice count meeting 2^-T, Kc the largest exact depth
    capped at K.  int8: beta = 7; int8bal: beta = 8; fp64: the beta in
    [8, 24] with the fewest slices, ties to the larger exact depth."""
    if form in ("int8", "int8bal"):
        beta = 7 if form == "int8" else BAL_BETA
        S = min_slices(form, T, G)
        return beta, S, min(exact_depth(form, beta, S), max(K, 1))
    if form == "fp64":
        best = None
        for beta in FP64_BETAS:
            S = min_slices(form, T, G, beta)
            kc = min(exact_depth(form, beta, S), max(K, 1))
            if kc < 1:
                continue
            if best is None or (S, -kc) < (best[1], -best[2]):
                best = (beta, S, kc)
        if best is None:
            raise ValueError("no exact FP64 parameters")
        return best
    raise ValueError(form)


# ---------------------------------------------------------------------------
# whole method on (small or sampled) inputs
# ---------------------------------------------------------------------------

def method_product(A: np.ndarray, B: np.ndarray, beta: int, S: int,
                   rows=None, cols=None, balanced: bool = False):
    """The method end to end for the entries rows x cols.

    Exponents come from the full rows of A and columns of B; only the
    sampled rows and columns are split.  Returns a dict with E, F (full),
    the digits of the sampled rows/columns, D (S, len(rows), len(cols)) and
    the renormalised output C (m, len(rows), len(cols)).  ``balanced``: the
    balanced 8-bit digits (beta must be 8); the fold then takes the grids
    2^(E_i+2) and 2^(F_j+2).
    """
    if balanced and beta != BAL_BETA:
        raise ValueError("balanced digits are 8 bits wide")
    m = A.shape[0]
    M, K = A.shape[1], A.shape[2]
    N = B.shape[2]
    rows = list(range(M)) if rows is None else list(rows)
    cols = list(range(N)) if cols is None else list(cols)
    E, spanA = row_exponents(A[0])
    F, spanB = row_exponents(B[0].T)
    As = A[:, rows, :]
    Bs = B[:, :, cols]
    Er = [E[i] for i in rows]
    Fc = [F[j] for j in cols]
    if balanced:
        dA = split_planes_balanced(As, Er, S, by_columns=False)
        dB = split_planes_balanced(Bs, Fc, S, by_columns=True)
    else:
        dA = split_planes(As, Er, beta, S, by_columns=False)
        dB = split_planes(Bs, Fc, beta, S, by_columns=True)
    h = BAL_HEADROOM if balanced else 0
    D = diagonal_sums(dA, dB, S)
    C = np.zeros((m, len(rows), len(cols)))
    for a, i in enumerate(rows):
        for b, j in enumerate(cols):
            x = fold(D[:, a, b], E[i] + h, F[j] + h, beta)
            C[:, a, b] = renorm_rn(x, m)
    return {"E": E, "F": F, "spanA": spanA, "spanB": spanB,
            "dA": dA, "dB": dB, "D": D, "C": C}


# ---------------------------------------------------------------------------
# exact fixed-point results ("multiple integers", Section 1)
# ---------------------------------------------------------------------------

def fixed_product(A: np.ndarray, B: np.ndarray, beta: int, S: int, E=None, F=None,
                  balanced: bool = False):
    """The method's exact sum before rounding, as integers: for every entry
    X_ij = sum_t D_t 2^(beta (S-1-t)) and scale_ij = E_i + F_j + 2h -
    beta (S+1) (h = 2 for the balanced digits, else 0), so that the fold
    is C~_ij = X_ij 2^scale_ij.  E, F: shared exponents to use instead of
    those of A's rows and B's columns (a product over part of the depth
    then uses the full rows' and columns' grids).  Returns (X, scale) as
    object and int64 arrays of shape (M, N)."""
    M, K = A.shape[1], A.shape[2]
    N = B.shape[2]
    if E is None:
        E, _ = row_exponents(A[0])
    if F is None:
        F, _ = row_exponents(B[0].T)
    E = [int(e) for e in E]
    F = [int(f) for f in F]
    h = BAL_HEADROOM if balanced else 0
    if balanced:
        dA = split_planes_balanced(A, E, S, by_columns=False)
        dB = split_planes_balanced(B, F, S, by_columns=True)
    else:
        dA = split_planes(A, E, beta, S, by_columns=False)
        dB = split_planes(B, F, beta, S, by_columns=True)
    D = diagonal_sums(dA, dB, S)
    X = np.zeros((M, N), dtype=object)
    scale = np.zeros((M, N), dtype=np.int64)
    for i in range(M):
        for j in range(N):
            X[i, j] = sum(int(D[t, i, j]) << (beta * (S - 1 - t)) for t in range(S))
            scale[i, j] = E[i] + F[j] + 2 * h - beta * (S + 1)
    return X, scale


def fixed_limbs(X: int, nlimb: int):
    """Two's complement 32-bit limbs of X, least significant first
    (ValueError if X does not fit in 32 nlimb bits)."""
    if not -(1 << (32 * nlimb - 1)) <= X < (1 << (32 * nlimb - 1)):
        raise ValueError("does not fit")
    u = X % (1 << (32 * nlimb))
    return [(u >> (32 * k)) & 0xffffffff for k in range(nlimb)]


# ---------------------------------------------------------------------------
# batched inner products (the paper's experiment, Section 3)
# ---------------------------------------------------------------------------

def pair_operands(X: np.ndarray, Y: np.ndarray, b: int):
    """Pair b of a batch as a 1 x 1 product: x_b as a row (m, 1, n), y_b as
    a column (m, n, 1).  Every step of the method then is the matrix
    product's: E is the row exponent of x_b, F the column exponent of y_b."""
    return X[:, b:b + 1, :], np.ascontiguousarray(Y[:, b, :][:, :, None])


def exact_dots(X: np.ndarray, Y: np.ndarray):
    """Exact sum_k x_bk y_bk and sum_k |x_bk| |y_bk| for every pair b, as
    lists of Fractions.  X and Y are (m, batch, n) planes."""
    vals, absvals = [], []
    for b in range(X.shape[1]):
        x, y = pair_operands(X, Y, b)
        num, L = exact_product(x, y)
        anum, _ = abs_product(x, y)
        vals.append(Fraction(int(num[0, 0]), 1 << L))
        absvals.append(Fraction(int(anum[0, 0]), 1 << L))
    return vals, absvals


def rho_G_dot(X: np.ndarray, Y: np.ndarray):
    """The magnitude certificate of ``rho_G`` over the pairs of a batch:
    min P is the smallest pair's sum_k qx_bk qy_bk.  Returns (min P, G), G
    None when min P = 0."""
    n = X.shape[2]
    minP = min(rho_G(*pair_operands(X, Y, b))[0] for b in range(X.shape[1]))
    if minP == 0:
        return 0, None
    target = n * (1 << 14) + 1
    g = 0
    while (minP << g) < target:
        g += 1
    return minP, g


def dot_G(X: np.ndarray, Y: np.ndarray, rule: str = "rho") -> int:
    """The ratio exponent G of a batch of inner products: the span bound
    over all vectors and, for the rho rule, the smallest pair's magnitude
    certificate when it is smaller."""
    _, sx = row_exponents(X[0])
    _, sy = row_exponents(Y[0])
    G = span_G(max(sx), max(sy))
    if rule == "rho":
        _, g = rho_G_dot(X, Y)
        if g is not None:
            G = min(G, g)
    return G


def method_dot(X: np.ndarray, Y: np.ndarray, beta: int, S: int, balanced: bool = False):
    """The method on every pair of a batch (``method_product`` on the 1 x 1
    product of pair b).  Returns D (S, batch) and out (m, batch)."""
    m, batch, _ = X.shape
    D = np.zeros((S, batch), dtype=object)
    out = np.zeros((m, batch))
    for b in range(batch):
        r = method_product(*pair_operands(X, Y, b), beta, S, balanced=balanced)
        D[:, b] = r["D"][:, 0, 0]
        out[:, b] = r["C"][:, 0, 0]
    return D, out


def exact_gradients(A: np.ndarray, B: np.ndarray, W: np.ndarray):
    """Exact gradients of the loss sum(W * C) with C = A B.

    The loss is bilinear, so dA* = W B^T and dB* = A^T W exactly.  Returns
    ((num, L) of dA*, (num, L) of dB*) as from ``exact_product``.
    """
    Bt = np.ascontiguousarray(np.transpose(B, (0, 2, 1)))
    At = np.ascontiguousarray(np.transpose(A, (0, 2, 1)))
    return exact_product(W, Bt), exact_product(At, W)
