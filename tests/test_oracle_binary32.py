"""Pins of the oracle's binary32 target precision (no GPU).

The binary32 transform is the binary64 method on the exactly widened input
with the cap K, rounded once to binary32.  Pinned against closed forms (unit
impulse, constant vector, single frequency), against the exact DFT within
binary32 accuracy for K = 2 (and shown to miss it with K = 1, so that a
dropped slice is caught), and the inverse against the forward by the
definition of the inverse DFT."""

import numpy as np
import pytest

import workloads as wl
from oracle import bluestein as bl


def _longdouble_dft(x):
    return np.fft.fft(np.asarray(x).astype(np.clongdouble))


def _rel_l2(y, ref):
    y = np.asarray(y).astype(np.clongdouble)
    return float(np.sqrt(np.sum(np.abs(y - ref) ** 2)) / np.sqrt(np.sum(np.abs(ref) ** 2)))


@pytest.mark.parametrize("n", [1, 5, 16, 100, 128])
def test_impulse_gives_ones(n):
    x = np.zeros(n, dtype=np.complex64)
    x[0] = 1.0
    y = bl.fft_binary32(x, 2, 3, bl.KernelPlan(n, 2, 3))
    assert y.dtype == np.complex64
    assert np.array_equal(y.real, np.ones(n, dtype=np.float32))
    assert np.all(np.abs(y.imag) <= 2.0 ** -24)


@pytest.mark.parametrize("n", [4, 9, 64])
def test_constant_gives_n_at_zero(n):
    x = np.full(n, 1.0 + 0.0j, dtype=np.complex64)
    y = bl.fft_binary32(x, 2, 3, bl.KernelPlan(n, 2, 3))
    assert y[0].real == np.float32(n) and abs(y[0].imag) <= n * 2.0 ** -24
    assert np.all(np.abs(y[1:]) <= n * 2.0 ** -22)


@pytest.mark.parametrize("n,k0", [(32, 3), (50, 7)])
def test_single_frequency(n, k0):
    j = np.arange(n)
    x = np.exp(2j * np.pi * k0 * j / n).astype(np.complex64)
    y = bl.fft_binary32(x, 2, 3, bl.KernelPlan(n, 2, 3))
    want = np.zeros(n, dtype=np.complex128)
    want[k0] = n
    assert np.max(np.abs(y - want)) <= n * 2.0 ** -20


@pytest.mark.parametrize("n", [256, 1000])
def test_binary32_accuracy_needs_two_slices(n):
    x = wl.paper_phi(n, 1.0, seed=3, batch=1)[0].astype(np.complex64)
    ref = _longdouble_dft(x.astype(np.complex128))
    y2 = bl.fft_binary32(x, 2, 3, bl.KernelPlan(n, 2, 3))
    y1 = bl.fft_binary32(x, 1, 3, bl.KernelPlan(n, 1, 3))
    rounding = _rel_l2(ref.astype(np.complex128).astype(np.complex64), ref)   # the exact DFT rounded
    assert _rel_l2(y2, ref) < 2.0 ** -24
    assert _rel_l2(y2, ref) <= 1.05 * rounding       # two slices: only the final rounding is seen
    assert _rel_l2(y1, ref) > 2.0 ** -24             # one slice of about 20 bits is not enough


def test_inverse_of_forward():
    n = 96
    x = wl.paper_phi(n, 0.0, seed=4, batch=1)[0].astype(np.complex64)
    kp = bl.KernelPlan(n, 2, 3)
    back = bl.ifft_binary32(bl.fft_binary32(x, 2, 3, kp), 2, 3, kp)
    assert _rel_l2(back, x.astype(np.clongdouble)) < 2.0 ** -22
    # adjoint = n * inverse up to the final roundings
    y = bl.fft_binary32(x, 2, 3, kp)
    a = bl.adjoint_binary32(y, 2, 3, kp)
    assert _rel_l2(a / n, x.astype(np.clongdouble)) < 2.0 ** -22
