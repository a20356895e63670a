"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.

This module only draws random numbers and builds arrays; it contains none
of the transform's arithmetic.  All generators use numpy's PCG64
``default_rng(seed)`` and draw in a fixed order, so every caller sees the
same bits.

Workloads (complex128 unless noted):

plain_1k       one transform, n = 2^10, Re/Im i.i.d. uniform[-1, 1]
batch_16k      64 transforms, n = 2^14, uniform[-1, 1] (round-trip checked)
batch_prime    64 transforms, prime n = 10007, uniform[-1, 1]
wide_256k      B transforms, n = 2^18, magnitudes log-uniform in
               [2^-30, 2^30] with uniform phase
mixed_256      256 transforms of lengths log-uniform in [2^10, 2^16], every
               third length moved to the next prime, uniform[-1, 1]
grad_64k       32 transforms, n = 2^16, uniform[-1, 1], plus weights
               uniform[0, 1] for the loss sum(w |X|^2)
paper_phi      the paper's accuracy generator (rand - 0.5) exp(phi randn),
               rand uniform on (0, 1], randn standard normal (Sec. 5.1),
               applied to Re and Im independently
"""

from __future__ import annotations

import numpy as np


def _complex_uniform(rng, shape):
    u = rng.uniform(-1.0, 1.0, tuple(shape) + (2,))
    return u[..., 0] + 1j * u[..., 1]


def plain_1k(seed: int = 0):
    rng = np.random.default_rng(seed)
    return _complex_uniform(rng, (1, 1024))


def batch_16k(seed: int = 0, batch: int = 64, n: int = 16384):
    rng = np.random.default_rng(seed)
    return _complex_uniform(rng, (batch, n))


def batch_prime(seed: int = 0, batch: int = 64, n: int = 10007):
    rng = np.random.default_rng(seed)
    return _complex_uniform(rng, (batch, n))


def wide_256k(seed: int = 0, batch: int = 8, n: int = 1 << 18, lo: float = -30.0, hi: float = 30.0):
    rng = np.random.default_rng(seed)
    m = np.exp2(rng.uniform(lo, hi, (batch, n)))
    th = rng.uniform(0.0, 2.0 * np.pi, (batch, n))
    return m * (np.cos(th) + 1j * np.sin(th))


def is_prime(v: int) -> bool:
    if v < 2:
        return False
    if v % 2 == 0:
        return v == 2
    d = 3
    while d * d <= v:
        if v % d == 0:
            return False
        d += 2
    return True


def next_prime(v: int) -> int:
    while not is_prime(v):
        v += 1
    return v


def mixed_lengths(seed: int = 0, count: int = 256, lo: float = 10.0, hi: float = 16.0):
    rng = np.random.default_rng(seed)
    e = rng.uniform(lo, hi, count)
    ns = []
    for i, ei in enumerate(e):
        v = int(round(2.0 ** ei))
        if i % 3 == 0:
            v = next_prime(v)
            if v > (1 << int(hi)):
                v = 65521
        ns.append(v)
    return ns, rng


def mixed_256(seed: int = 0, count: int = 256):
    """Returns (lengths, list of complex vectors)."""
    ns, rng = mixed_lengths(seed, count)
    xs = []
    for n in ns:
        u = rng.uniform(-1.0, 1.0, (n, 2))
        xs.append(u[:, 0] + 1j * u[:, 1])
    return ns, xs


def grad_64k(seed: int = 0, batch: int = 32, n: int = 1 << 16, wseed: int = 1):
    rng = np.random.default_rng(seed)
    x = _complex_uniform(rng, (batch, n))
    w = np.random.default_rng(wseed).uniform(0.0, 1.0, (batch, n))
    return x, w


def paper_phi(n: int, phi: float, seed: int = 0, batch: int = 1):
    rng = np.random.default_rng(seed)

    def draw():
        rand = 1.0 - rng.random((batch, n))          # uniform on (0, 1]
        return (rand - 0.5) * np.exp(phi * rng.standard_normal((batch, n)))

    re = draw()
    im = draw()
    return re + 1j * im


def uniform(n: int, batch: int = 1, seed: int = 0):
    rng = np.random.default_rng(seed)
    return _complex_uniform(rng, (batch, n))
