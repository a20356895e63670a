"""Oracle: arithmetic modulo the 32-bit primes, NTT and CRT (two primes, and
three for the d = 3 variant).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Everything here is exact integer arithmetic: numpy uint64/int64 where every
intermediate provably fits (residues < 2^31, so products < 2^62), Python ints
elsewhere.
"""

from __future__ import annotations

import numpy as np

# The two primes of the paper's experiments (Sec. 5.1; also used for Fig. 1
# in Sec. 4.2).  p0 - 1 = 127 * 2^24, p1 - 1 = 63 * 2^25.
P0 = 2130706433
P1 = 2113929217
PRIMES = (P0, P1)
# Smallest primitive roots (checked by tests against the factorisation of p-1).
GENERATORS = {P0: 3, P1: 5}
# Product of the moduli and the bound of the symmetric CRT range.
PP = P0 * P1
PP_HALF = (PP - 1) // 2
# Garner's constant: p0^{-1} mod p1 (Sec. 3.3, Garner's algorithm with d = 2).
P0_INV_MOD_P1 = pow(P0, -1, P1)
# Largest power-of-two NTT length supported by both primes: gcd(p0-1, p1-1).
MAX_LOG2_N = 24

# Third modulus for the d = 3 CRT (Sec. 3.3 with d moduli; Sec. 4.2's alpha
# formula with the product of all moduli): p2 = 15 * 2^27 + 1 < 2^31, its
# 2-power part 2^27 covers every NTT length above.
P2 = 2013265921
GENERATORS[P2] = 31
PRIMES3 = (P0, P1, P2)
PPP = P0 * P1 * P2
PPP_HALF = (PPP - 1) // 2


def smod(a: int, m: int) -> int:
    """Symmetric remainder a mod m in [-m/2, m/2) (Sec. 3.1, Notation)."""
    # a - m*floor(a/m + 1/2), computed exactly with integers.
    return a - m * ((2 * a + m) // (2 * m))


def root_of_unity(p: int, N: int) -> int:
    """A primitive N-th root of unity mod p: g^((p-1)/N) with g the smallest
    primitive root (the paper leaves the root unspecified, Sec. 3.3)."""
    if N < 1 or (p - 1) % N:
        raise ValueError(f"N={N} does not divide p-1 for p={p}")
    return pow(GENERATORS[p], (p - 1) // N, p)


def ntt_direct(x, p: int, inverse: bool = False):
    """O(N^2) evaluation of the NTT definition (Sec. 3.3, Eq. ntt / intt).

    Python ints only; used to pin :func:`ntt` on small lengths.
    """
    x = [int(v) % p for v in x]
    N = len(x)
    w = root_of_unity(p, N)
    if inverse:
        w = pow(w, -1, p)
    out = []
    for k in range(N):
        s = 0
        for j in range(N):
            s += x[j] * pow(w, j * k, p)
        out.append(s % p)
    if inverse:
        ninv = pow(N, -1, p)
        out = [(v * ninv) % p for v in out]
    return out


_TW_CACHE: dict = {}


def _powers(w: int, count: int, p: int) -> np.ndarray:
    """[w^0, w^1, ..., w^(count-1)] mod p as uint64 (by repeated doubling)."""
    out = np.ones(1, dtype=np.uint64)
    wp = w % p
    while out.size < count:
        out = np.concatenate([out, (out * np.uint64(wp)) % np.uint64(p)])
        wp = (wp * wp) % p
    return out[:count]


def _twiddles(p: int, N: int, inverse: bool) -> np.ndarray:
    key = (p, N, inverse)
    t = _TW_CACHE.get(key)
    if t is None:
        w = root_of_unity(p, N)
        if inverse:
            w = pow(w, -1, p)
        t = _powers(w, max(N // 2, 1), p)
        _TW_CACHE[key] = t
    return t


def _bitrev(N: int) -> np.ndarray:
    logn = N.bit_length() - 1
    idx = np.arange(N, dtype=np.int64)
    rev = np.zeros(N, dtype=np.int64)
    for b in range(logn):
        rev |= ((idx >> b) & 1) << (logn - 1 - b)
    return rev


def ntt(x, p: int, inverse: bool = False) -> np.ndarray:
    """NTT / inverse NTT of a power-of-two length vector, natural order in and
    out (Sec. 3.3, Eq. ntt / intt), by the textbook iterative radix-2
    Cooley-Tukey recursion (bit-reversal permutation followed by butterflies).

    The inverse multiplies by N^{-1} mod p.  Input may be any integers; they
    are reduced mod p first.  Returns uint64 residues in [0, p).
    """
    a = np.asarray(x)
    if a.dtype != np.uint64:
        a = np.mod(a.astype(np.int64), p).astype(np.uint64)
    else:
        a = a % np.uint64(p)
    N = a.size
    if N & (N - 1) or N == 0:
        raise ValueError("length must be a power of two")
    if N == 1:
        return a.copy()
    pp = np.uint64(p)
    tw_all = _twiddles(p, N, inverse)
    a = a[_bitrev(N)]
    h = 1
    while h < N:
        tw = tw_all[:: N // (2 * h)][:h]
        blk = a.reshape(-1, 2 * h)
        u = blk[:, :h]
        v = (blk[:, h:] * tw) % pp
        a = np.concatenate([(u + v) % pp, (u + (pp - v)) % pp], axis=1).reshape(-1)
        h *= 2
    if inverse:
        a = (a * np.uint64(pow(N, -1, p))) % pp
    return a


def cyclic_convolution_direct(a, b):
    """Exact integer cyclic convolution by its definition (Python ints)."""
    a = [int(v) for v in a]
    b = [int(v) for v in b]
    N = len(a)
    return [sum(a[j] * b[(k - j) % N] for j in range(N)) for k in range(N)]


def garner_crt(z0, z1) -> np.ndarray:
    """Two-prime CRT in Garner's incremental form (Sec. 3.3; the
    reconstruction line of Alg. 5 / Alg. 8):
        z = z0 + ((z1 - z0) * p0^{-1} mod p1) * p0,
    then mapped to the symmetric range [-(P-1)/2, (P-1)/2] with P = p0*p1
    (Sec. 3.1 symmetric remainder).  Inputs are residues in [0, p0), [0, p1);
    returns int64 (|z| < 2^61).
    """
    z0 = np.asarray(z0, dtype=np.uint64)
    z1 = np.asarray(z1, dtype=np.uint64)
    p1 = np.uint64(P1)
    d = (z1 + p1 - (z0 % p1)) % p1
    h = (d * np.uint64(P0_INV_MOD_P1)) % p1
    z = z0.astype(np.int64) + h.astype(np.int64) * np.int64(P0)  # in [0, P) < 2^62
    return np.where(z > PP_HALF, z - np.int64(PP), z)


def garner_crt3(z0, z1, z2) -> np.ndarray:
    """Three-prime CRT in Garner's mixed-radix form (Sec. 3.3, Garner's
    algorithm with d = 3):
        h1 = (z1 - z0) p0^{-1} mod p1,
        h2 = (z2 - z0 - p0 h1) (p0 p1)^{-1} mod p2,
        z  = z0 + p0 h1 + p0 p1 h2,
    then mapped to the symmetric range [-(M-1)/2, (M-1)/2], M = p0 p1 p2.
    Returns an object array of Python ints (|z| < 2^92)."""
    out = []
    for a, b, c in zip(np.asarray(z0).tolist(), np.asarray(z1).tolist(), np.asarray(z2).tolist()):
        h1 = ((b - a) * pow(P0, -1, P1)) % P1
        t = a + P0 * h1
        h2 = ((c - t) * pow(P0 * P1, -1, P2)) % P2
        z = t + P0 * P1 * h2
        out.append(z - PPP if z > PPP_HALF else z)
    return np.array(out, dtype=object)


def crt_explicit(residues, moduli) -> int:
    """CRT by the explicit formula a = sum a_j M_j (M_j^{-1} mod m_j) mod M
    (Sec. 3.3, Eq. crt), then the symmetric remainder.  Python ints; used to
    pin :func:`garner_crt`."""
    M = 1
    for m in moduli:
        M *= m
    acc = 0
    for a, m in zip(residues, moduli):
        Mj = M // m
        acc += int(a) * Mj * pow(Mj, -1, m)
    return smod(acc % M, M)
