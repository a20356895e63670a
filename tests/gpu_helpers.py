"""Helpers shared by the GPU parity tests (no method arithmetic here)."""

import numpy as np


def ordered(a):
    """Map binary64 values to integers whose differences count ulps
    (+0 and -0 both map to 0)."""
    i = np.ascontiguousarray(a, dtype=np.float64).view(np.int64)
    mag = i & np.int64(0x7FFFFFFFFFFFFFFF)
    return np.where(i < 0, -mag, mag)


def max_ulp(a, b):
    """Largest ulp distance between the real and imaginary components of two
    complex arrays; NaNs must coincide."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    worst = 0
    for x, y in ((a.real, b.real), (a.imag, b.imag)):
        nx, ny = np.isnan(x), np.isnan(y)
        assert np.array_equal(nx, ny), "NaN positions differ"
        m = ~nx
        if np.any(m):
            d = np.abs(ordered(x[m]).astype(object) - ordered(y[m]).astype(object))
            worst = max(worst, int(max(d)))
    return worst


def bitrev(v, bits):
    out = np.zeros_like(v)
    for b in range(bits):
        out |= ((v >> b) & 1) << (bits - 1 - b)
    return out


def ntt_domain_index(logN, log2N1):
    """perm such that gpu[pos] == natural[perm[pos]] for the library's
    NTT-domain order (position i1*N2 + i2 holds X[br(i1) + N1*br(i2)])."""
    N = 1 << logN
    m1 = log2N1
    m2 = logN - m1
    pos = np.arange(N, dtype=np.int64)
    i1 = pos >> m2
    i2 = pos & ((1 << m2) - 1)
    return bitrev(i1, m1) + (bitrev(i2, m2) << m1)
