"""Pins for oracle.ntt: constants, NTT, convolution theorem, CRT (CPU only)."""

import json
import os
import random

import numpy as np
import pytest

from oracle import ntt as nt

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def _is_prime(v):
    if v < 2:
        return False
    d = 2
    while d * d <= v:
        if v % d == 0:
            return False
        d += 1
    return True


def _factor(v):
    f, d = {}, 2
    while d * d <= v:
        while v % d == 0:
            f[d] = f.get(d, 0) + 1
            v //= d
        d += 1
    if v > 1:
        f[v] = f.get(v, 0) + 1
    return f


def test_primes_match_paper():
    assert nt.P0 == GOLDEN["primes"]["p0"] and nt.P1 == GOLDEN["primes"]["p1"]
    for p in nt.PRIMES:
        assert _is_prime(p) and p < 2 ** 31 and 2 * p < 2 ** 32


def test_generators_are_primitive_roots():
    for p in nt.PRIMES:
        g = nt.GENERATORS[p]
        for q in _factor(p - 1):
            assert pow(g, (p - 1) // q, p) != 1
        # and it is the smallest one
        for h in range(2, g):
            assert any(pow(h, (p - 1) // q, p) == 1 for q in _factor(p - 1))


def test_derived_constants():
    assert (nt.P0 * nt.P0_INV_MOD_P1) % nt.P1 == 1
    assert nt.P0_INV_MOD_P1 == 2113929091
    assert pow(nt.P1, -1, nt.P0) == 127
    import math
    assert math.gcd(nt.P0 - 1, nt.P1 - 1) == 2 ** nt.MAX_LOG2_N
    assert nt.PP < 2 ** 62


@pytest.mark.parametrize("p", nt.PRIMES)
def test_roots_of_unity(p):
    for logn in range(0, nt.MAX_LOG2_N + 1):
        N = 1 << logn
        w = nt.root_of_unity(p, N)
        assert pow(w, N, p) == 1
        if N > 1:
            assert pow(w, N // 2, p) == p - 1   # primitive: w^(N/2) = -1


@pytest.mark.parametrize("p", nt.PRIMES)
@pytest.mark.parametrize("logn", range(0, 7))
def test_ntt_matches_definition(p, logn):
    N = 1 << logn
    rng = random.Random(1000 * logn + p % 97)
    x = [rng.randrange(p) for _ in range(N)]
    for inv in (False, True):
        got = nt.ntt(np.array(x, dtype=np.uint64), p, inverse=inv).tolist()
        assert got == nt.ntt_direct(x, p, inverse=inv)


@pytest.mark.parametrize("p", nt.PRIMES)
def test_ntt_roundtrip_and_impulses(p):
    rng = np.random.default_rng(p % 1000)
    for logn in (1, 5, 10, 13, 16):
        N = 1 << logn
        x = rng.integers(0, p, N, dtype=np.int64).astype(np.uint64)
        assert np.array_equal(nt.ntt(nt.ntt(x, p), p, inverse=True), x)
        d = np.zeros(N, dtype=np.uint64)
        d[0] = 1
        assert np.all(nt.ntt(d, p) == 1)
        ones = np.ones(N, dtype=np.uint64)
        e = nt.ntt(ones, p)
        assert e[0] == N % p and np.all(e[1:] == 0)


@pytest.mark.parametrize("p", nt.PRIMES)
@pytest.mark.parametrize("N", [1, 2, 8, 32, 128])
def test_convolution_theorem(p, N):
    rng = random.Random(N * 7 + p % 13)
    a = [rng.randint(-(2 ** 20), 2 ** 20) for _ in range(N)]
    b = [rng.randint(-(2 ** 20), 2 ** 20) for _ in range(N)]
    A = nt.ntt(np.array(a, dtype=np.int64), p)
    B = nt.ntt(np.array(b, dtype=np.int64), p)
    z = nt.ntt((A * B) % np.uint64(p), p, inverse=True).tolist()
    direct = nt.cyclic_convolution_direct(a, b)
    assert z == [v % p for v in direct]


def test_symmetric_remainder_definition():
    for m in (7, 8, nt.PP):
        for a in list(range(-3 * 8, 3 * 8)) + [nt.PP // 2, -(nt.PP // 2), nt.PP, -nt.PP - 5]:
            r = nt.smod(a, m)
            assert (a - r) % m == 0
            assert -m <= 2 * r < m


def test_garner_matches_explicit_crt():
    rng = random.Random(5)
    vals = [rng.randrange(-nt.PP_HALF, nt.PP_HALF + 1) for _ in range(2000)]
    vals += [nt.PP_HALF, -nt.PP_HALF, 0, 1, -1, nt.P0, -nt.P1, nt.P0 * 12345, -nt.P1 * 98765]
    z0 = np.array([v % nt.P0 for v in vals], dtype=np.uint64)
    z1 = np.array([v % nt.P1 for v in vals], dtype=np.uint64)
    got = nt.garner_crt(z0, z1).tolist()
    assert got == vals
    for v, a, b in zip(vals[:200], z0.tolist(), z1.tolist()):
        assert nt.crt_explicit([a, b], [nt.P0, nt.P1]) == v


def test_crt_wraps_outside_range():
    # one past the symmetric range wraps to the other end (why alpha matters)
    v = nt.PP_HALF + 1
    got = nt.garner_crt(np.array([v % nt.P0], dtype=np.uint64), np.array([v % nt.P1], dtype=np.uint64))
    assert int(got[0]) == v - nt.PP == -nt.PP_HALF
