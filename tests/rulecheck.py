"""The library's slice parameters against the oracle's error budget.

The oracle gives only what the error analysis fixes: the smallest slice
count that meets 2^-T (``min_slices``) and the largest depth over which
every accumulation stays exact (``exact_depth``).  The library rounds both
to what its kernels take; the constants below are those kernel facts, so
the checks say how far the library may sit from the budget, not what it
must choose.
"""
from oracle import exact as ox

GRAN = {"int8": 64, "int8bal": 64, "fp64": 16}    # depth granule of a fragment
ONE_BAND = {"int8": 32, "int8bal": 32, "fp64": 0}  # whole-triangle kernels: S up to this
WIDEST_BAND = 16                                   # diagonals per band otherwise
TWO_BANDS = (36, 64)   # INT8: S a multiple of 4 in this range may run as two bands of S/2


def two_bands(form, S, band):
    return form != "fp64" and S % 4 == 0 and TWO_BANDS[0] <= S <= TWO_BANDS[1] and 2 * band == S


def check_params(form, K, T, G, beta, S, kc, band):
    """The library's (beta, S, kc, band) for a call of depth K, target T and
    ratio exponent G: at least the budget's slices, fewer than one band
    more; every accumulation exact; the chunk as deep as the exact range
    and the depth allow, to within one granule."""
    if form == "int8":
        assert beta == 7
    elif form == "int8bal":
        assert beta == 8
    else:
        assert beta in ox.FP64_BETAS
    smin = ox.min_slices(form, T, G, beta)
    assert S >= smin, (S, smin)
    assert band >= 1 and S % band == 0
    assert S - smin < band, (S, smin, band)
    if smin <= ONE_BAND[form]:
        assert S == smin == band
    elif two_bands(form, S, band):
        # two bands over the whole depth: one exactness chunk
        assert kc >= K and (S - smin < 4 or S == TWO_BANDS[0])
    else:
        assert band <= WIDEST_BAND
    if form == "fp64":
        best = min(ox.min_slices(form, T, G, b) for b in ox.FP64_BETAS)
        assert S - best < WIDEST_BAND
    kmax = ox.exact_depth(form, beta, S)
    assert 1 <= kc <= kmax, (kc, kmax)
    assert kc % GRAN[form] == 0
    assert kc >= min(K, kmax - GRAN[form] + 1), (kc, K, kmax)


def check_info(info, form, K, T, G):
    check_params(form, K, T, G, info["beta"], info["S"], info["kc"], info["band"])


def library_chunk(form, beta, S):
    """The chunk depth the library takes for a deep contraction: the exact
    range rounded down to whole fragments."""
    return ox.exact_depth(form, beta, S) // GRAN[form] * GRAN[form]
