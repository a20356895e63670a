"""Oracle: extended-precision reference DFTs and the error metrics.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper measures errors against a 106-bit MPFR FFT (Sec. 5.1).  MPFR is not
available here; mpmath (arbitrary precision, O(n^2) direct sum of the DFT
definition) serves for small n and numpy's long-double FFT (64-bit
significand) for large n.
"""

from __future__ import annotations

import mpmath
import numpy as np


def dft_mpmath(x, prec: int = 160):
    """Direct O(n^2) DFT y(k) = sum_j x(j) w_n^{jk}, w_n = exp(-2 pi i / n)
    (Sec. 3.2, Eq. dft), at `prec` bits.  Returns a list of mpc."""
    with mpmath.workprec(prec):
        xs = [mpmath.mpc(float(v.real), float(v.imag)) for v in np.asarray(x)]
        n = len(xs)
        out = []
        for k in range(n):
            s = mpmath.mpc(0)
            for j in range(n):
                # exact reduction of j*k mod n keeps the angle argument small
                s += xs[j] * mpmath.expjpi(mpmath.mpf(-2 * ((j * k) % n)) / n)
            out.append(s)
        return out


def dft_longdouble(x) -> np.ndarray:
    """DFT in long double (x86 80-bit) via numpy.fft on clongdouble."""
    return np.fft.fft(np.asarray(x).astype(np.clongdouble), axis=-1)


def rel_l2_error(y, ref) -> float:
    """Relative l2 error ||y - ref||_2 / ||ref||_2 (Sec. 5.1)."""
    y = np.asarray(y).astype(np.clongdouble)
    ref = np.asarray(ref).astype(np.clongdouble)
    den = np.sqrt(np.sum(np.abs(ref) ** 2))
    num = np.sqrt(np.sum(np.abs(y - ref) ** 2))
    return float(num / den) if den > 0 else float(num)


def max_rel_error(y, ref) -> float:
    """Maximum componentwise relative error (Sec. 5.1), over the components
    whose reference value is non-zero."""
    y = np.asarray(y).astype(np.clongdouble)
    ref = np.asarray(ref).astype(np.clongdouble)
    out = 0.0
    for a, b in ((y.real, ref.real), (y.imag, ref.imag)):
        m = b != 0
        if np.any(m):
            out = max(out, float(np.max(np.abs((a[m] - b[m]) / b[m]))))
    return out


def mpc_to_clongdouble(vals) -> np.ndarray:
    re = np.array([np.longdouble(mpmath.nstr(v.real, 30)) for v in vals], dtype=np.longdouble)
    im = np.array([np.longdouble(mpmath.nstr(v.imag, 30)) for v in vals], dtype=np.longdouble)
    out = np.empty(len(vals), dtype=np.clongdouble)
    out.real = re
    out.imag = im
    return out
