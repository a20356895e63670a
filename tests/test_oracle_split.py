"""Pins for oracle.ozaki: split width alpha and the binary64 split (CPU only)."""

from fractions import Fraction
import json
import math
import os

import numpy as np
import pytest

from oracle import ozaki as oz

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_alpha_printed_values():
    for n, L, a in GOLDEN["alpha_two_prime"]["cases"]:
        assert oz.alpha_crt(n, L) == a
    g = GOLDEN["alpha_original_single"]
    assert oz.alpha_original(g["n"], g["u_bits"]) == g["alpha"]
    # single-prime alpha is only slightly larger than the original (Sec. 4.2)
    assert g["alpha"] < oz.alpha_single_prime(g["n"], 2130706433) < oz.alpha_crt(g["n"], 1)


def test_alpha_integer_form_equals_formula():
    for L in (1, 2, 3, 4, 8):
        for n in list(range(1, 4097)) + [10007, 16384, 65536, 65521, 1 << 17, 1 << 18, 1 << 20, (1 << 23) + 1]:
            assert oz.alpha_crt(n, L) == oz.alpha_crt_float(n, L), (n, L)


def test_alpha_guarantees_crt_range():
    # L * n * 4^alpha <= (P-1)/2, and alpha+1 violates it
    from oracle.ntt import PP_HALF
    for n in (1, 3, 1024, 10007, 1 << 18, 1 << 23):
        for L in (1, 3):
            a = oz.alpha_crt(n, L)
            assert L * n * 4 ** a <= PP_HALF < L * n * 4 ** (a + 1)


def test_ceil_log2_exact():
    assert oz.ceil_log2(1.0) == 0
    assert oz.ceil_log2(0.5) == -1
    assert oz.ceil_log2(np.nextafter(1.0, 2.0)) == 1
    assert oz.ceil_log2(0.75) == 0
    assert oz.ceil_log2(5e-324) == -1074
    assert oz.ceil_log2(2.0 ** -1030 * 3) == -1028
    assert oz.ceil_log2(1.7976931348623157e308) == 1024


def _grid_round(r: Fraction, E: int, alpha: int) -> Fraction:
    """Closed form of fl(fl(r + sigma) - sigma) with sigma = 2^(E+53-alpha):
    r + sigma lies in [sigma, 2 sigma) for r >= 0 (grid 2^(E-alpha+1)) and
    in [sigma/2, sigma) for r < 0 (grid 2^(E-alpha)); round to nearest, ties
    to the even multiple (sigma is an even multiple of either grid)."""
    g = Fraction(2) ** (E - alpha + (1 if r >= 0 else 0))
    q = r / g
    fl = math.floor(q)
    rem = q - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return fl * g


def _check_split(v, alpha, K):
    slices, resid, st = oz.split(v, alpha, K)
    assert st == oz.STATUS_OK
    r = [Fraction(float(t)) for t in v]
    prevE = None
    for a, E in slices:
        mu = max(abs(t) for t in r)
        assert mu > 0
        assert Fraction(2) ** (E - 1) < mu <= Fraction(2) ** E      # E = ceil(log2 mu)
        if prevE is not None:
            assert E <= prevE - alpha                                 # gaps only widen
        prevE = E
        assert np.all(np.abs(a) <= 2 ** alpha)                        # |a_k| <= 2^alpha
        for j in range(len(r)):
            x = _grid_round(r[j], E, alpha)
            assert x == Fraction(int(a[j])) * Fraction(2) ** (E - alpha), (j, E)
            r[j] -= x
    assert [Fraction(float(t)) for t in resid] == r                  # exact remainder
    return slices


@pytest.mark.parametrize("alpha", [20, 21, 25, 29])
def test_split_closed_form_uniform(alpha):
    rng = np.random.default_rng(alpha)
    v = rng.uniform(-1, 1, 300)
    sl = _check_split(v, alpha, None)
    assert len(sl) <= oz.split_count_bound(v, alpha)
    _check_split(v, alpha, 3)


def test_split_closed_form_wide_and_ties():
    rng = np.random.default_rng(7)
    alpha = 21
    v = np.exp2(rng.uniform(-30, 30, 200)) * rng.choice([-1.0, 1.0], 200)
    sl = _check_split(v, alpha, None)
    assert len(sl) <= oz.split_count_bound(v, alpha)
    # ties: with max 1 (E = 0) the grids are 2^-alpha (r<0) and 2^(1-alpha) (r>=0)
    g = 2.0 ** -alpha
    ties = np.array([1.0, 0.5 * g, 1.5 * g, -0.5 * g, -1.5 * g, 2.5 * g, 3 * g, -2.5 * g, 0.0, -0.0])
    _check_split(ties, alpha, None)


def test_split_zero_and_special():
    sl, r, st = oz.split(np.zeros(5), 21, 3)
    assert sl == [] and st == oz.STATUS_OK
    sl, r, st = oz.split(np.array([1.0, np.nan]), 21, 3)
    assert st == oz.STATUS_NONFINITE
    sl, r, st = oz.split(np.array([2.0 ** 1000, 1.0]), 21, 3)
    assert st == oz.STATUS_RANGE
    sl, r, st = oz.split(np.array([2.0 ** -1010, 0.0]), 21, 3)
    assert st == oz.STATUS_RANGE
    # a tiny remainder after the first slice ends the split instead
    sl, r, st = oz.split(np.array([1.0, 2.0 ** -1040]), 21, None)
    assert st == oz.STATUS_OK and len(sl) == 1 and r[1] == 2.0 ** -1040


def test_split_cap():
    v = np.random.default_rng(3).uniform(-1, 1, 100)
    for K in (1, 2, 3):
        sl, _, _ = oz.split(v, 21, K)
        assert len(sl) == K
