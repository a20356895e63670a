"""Oracle: split width and the Ozaki splitting procedure in binary64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper splits triple-single vectors with single-precision arithmetic
(Alg. 6).  Here the same procedure is carried out on binary64 vectors
(unit roundoff u = 2^-53), which is the form Alg. 3 takes for double
precision: rho = log2(u^{-1}) - alpha = 53 - alpha, sigma =
2^(ceil(log2 mu) + rho), slice = fl(fl(r + sigma) - sigma), integer slice =
slice * (u*sigma)^{-1} = slice * 2^(alpha - E).  FastTwoSum (Alg. 7) is not
needed: in binary64 the remainder r - slice is exact.
"""

from __future__ import annotations

import math

import numpy as np

from .ntt import PP

# Status bits reported per transform (shared convention with the library).
STATUS_OK = 0
STATUS_NONFINITE = 1      # a premultiplied input value is NaN or infinite
STATUS_RANGE = 2          # the first slice would leave the binary64 range

MANTISSA_BITS = 53        # log2(u^{-1}) for binary64
EMIN_GRID = -1022         # smallest slice grid exponent E - alpha allowed


def alpha_crt(n: int, L: int = 1, modulus_product: int = PP) -> int:
    """Split width for the two-prime CRT with NTT-domain accumulation bound L
    (Sec. 4.2, two-prime alpha; Sec. 4.4, alpha with L):

        alpha = floor( (log2(p0*p1/2) - log2(L*n)) / 2 ).

    Evaluated exactly: alpha is the largest integer a with
    2*a <= log2(P / (2*L*n)), i.e. 2*L*n*4^a <= P.
    """
    if n < 1 or L < 1:
        raise ValueError("n and L must be positive")
    a = 0
    while 2 * L * n * 4 ** (a + 1) <= modulus_product:
        a += 1
    if 2 * L * n * 4 ** a > modulus_product:
        raise ValueError("no non-negative alpha for this n, L")
    return a


def alpha_crt_float(n: int, L: int = 1) -> int:
    """The same formula evaluated literally in floating point (for tests)."""
    return math.floor((math.log2(PP / 2) - math.log2(L * n)) / 2)


def alpha_single_prime(n: int, p: int) -> int:
    """Single-modulus alpha, floor((log2(p/2) - log2 n)/2) (Sec. 4.2)."""
    return math.floor((math.log2(p / 2) - math.log2(n)) / 2)


def alpha_original(n: int, u_bits: int) -> int:
    """Original Ozaki alpha, floor((log2 u^{-1} - log2 n)/2) (Sec. 3.4)."""
    return math.floor((u_bits - math.log2(n)) / 2)


def ceil_log2(mu: float) -> int:
    """ceil(log2(mu)) for a positive binary64 value, exactly (frexp gives
    mu = m * 2^e with m in [0.5, 1); mu is a power of two iff m == 0.5)."""
    m, e = math.frexp(mu)
    return e - 1 if m == 0.5 else e


def split(v, alpha: int, K: int | None):
    """Split a real binary64 vector into at most K integer slices.

    Alg. 3 (Sec. 3.4) with the cap K on the number of splits (Sec. 4.4) and
    the integer scaling c = (u*sigma)^{-1} of Alg. 6, in binary64:

        mu_k    = max |r_k|                      (stop when mu_k == 0)
        E_k     = ceil(log2 mu_k)
        sigma_k = 2^(E_k + 53 - alpha)
        x_k     = fl(fl(r_k + sigma_k) - sigma_k)
        a_k     = x_k * 2^(alpha - E_k)          (an integer, |a_k| <= 2^alpha)
        r_{k+1} = r_k - x_k                      (exact)

    The slice value is a_k * 2^(E_k - alpha).  Range rules (the paper works
    far from the binary64 limits and is silent here): the split also stops
    before a slice k > 0 whose grid exponent E_k - alpha would be below -1022;
    for k == 0 the same condition, or sigma_0 overflowing, returns
    STATUS_RANGE.  A non-finite value returns STATUS_NONFINITE.

    Returns (slices, residual, status) where slices is a list of
    (int64 array a_k, int E_k).
    """
    r = np.array(v, dtype=np.float64, copy=True)
    rho = MANTISSA_BITS - alpha
    if r.size and not np.all(np.isfinite(r)):
        return [], r, STATUS_NONFINITE
    slices = []
    k = 0
    while K is None or k < K:
        mu = float(np.max(np.abs(r))) if r.size else 0.0
        if mu == 0.0:
            break
        E = ceil_log2(mu)
        if E - alpha < EMIN_GRID:
            if k == 0:
                return [], r, STATUS_RANGE
            break
        if E + rho > 1023:
            return [], r, STATUS_RANGE
        sigma = math.ldexp(1.0, E + rho)
        x = (r + sigma) - sigma
        a = x * math.ldexp(1.0, alpha - E)
        ai = a.astype(np.int64)
        assert np.all(ai == a), "slice is not an integer"
        r = r - x
        slices.append((ai, E))
        k += 1
    return slices, r, STATUS_OK


def split_count_bound(v, alpha: int) -> int:
    """Upper bound on the number of splits (Sec. 3.4, Eq. k-upper-limit):
    ceil((log2 max|x| - log2 min|x| + log2 u^{-1} - 1) / (alpha - 1)), with
    min over the non-zero entries."""
    a = np.abs(np.asarray(v, dtype=np.float64))
    a = a[a > 0]
    if a.size == 0:
        return 0
    num = math.log2(float(a.max())) - math.log2(float(a.min())) + MANTISSA_BITS - 1
    return math.ceil(num / (alpha - 1))
