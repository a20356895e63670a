"""Pins of the oracle's three-modulus variant (d = 3 CRT; no GPU).

The third modulus is checked to be a prime with the stated generator and
power-of-two part; Garner's mixed-radix CRT with d = 3 against the explicit
CRT formula (Sec. 3.3) and special values; the split width against
Sec. 4.2's inequality with the product of three moduli; the whole integer
pipeline against a direct rational evaluation of the convolutions of the
retained slices; a CRT range planted too small must break that pin; and the
accuracy of K = 2 with three moduli against the long-double DFT."""

from fractions import Fraction

import numpy as np
import pytest

import workloads as wl
from oracle import bluestein as bl
from oracle import ntt as nt
from oracle import ozaki as oz

U = 2.0 ** -53


def _is_prime(p):
    """Deterministic Miller-Rabin for p < 3.3e24 (bases 2 .. 41)."""
    if p < 2:
        return False
    d, r = p - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41):
        if a % p == 0:
            continue
        x = pow(a, d, p)
        if x in (1, p - 1):
            continue
        for _ in range(r - 1):
            x = x * x % p
            if x == p - 1:
                break
        else:
            return False
    return True


def test_third_prime():
    p = nt.P2
    assert _is_prime(p) and p < 2 ** 31 and p - 1 == 15 * 2 ** 27
    # 31 is a primitive root: p - 1 = 2^27 3 5, no proper power of 31 in those quotients is 1
    for q in (2, 3, 5):
        assert pow(31, (p - 1) // q, p) != 1
    # and the smallest one
    assert all(any(pow(g, (p - 1) // q, p) == 1 for q in (2, 3, 5)) for g in range(2, 31))
    assert nt.GENERATORS[p] == 31
    assert (p - 1) % (1 << nt.MAX_LOG2_N) == 0
    assert nt.PPP == nt.P0 * nt.P1 * nt.P2 and 2 ** 92 < nt.PPP < 2 ** 93


@pytest.mark.parametrize("N", [1, 2, 8, 32])
def test_ntt_mod_p2_matches_definition(N):
    rng = np.random.default_rng(N)
    x = rng.integers(0, nt.P2, N)
    assert [int(v) for v in nt.ntt(x, nt.P2)] == [int(v) for v in nt.ntt_direct(x, nt.P2)]
    back = nt.ntt(nt.ntt(x, nt.P2), nt.P2, inverse=True)
    assert [int(v) for v in back] == [int(v) for v in x]


def test_garner3_matches_explicit_crt():
    rng = np.random.default_rng(3)
    m = nt.PRIMES3
    vals = [0, 1, -1, nt.PPP_HALF, -nt.PPP_HALF, 2 ** 91 + 12345, -(2 ** 90) - 7, nt.PP, -nt.PP]
    vals += [int(v) for v in rng.integers(-2 ** 62, 2 ** 62, 50)]
    vals += [int(a) * 2 ** 30 + int(b) for a, b in zip(rng.integers(-2 ** 61, 2 ** 61, 50),
                                                         rng.integers(0, 2 ** 30, 50))]
    res = [[v % p for v in vals] for p in m]
    got = nt.garner_crt3(np.array(res[0], dtype=np.uint64), np.array(res[1], dtype=np.uint64),
                         np.array(res[2], dtype=np.uint64))
    assert [int(g) for g in got] == vals
    for v, r0, r1, r2 in zip(vals, *res):
        assert nt.crt_explicit((r0, r1, r2), m) == v
    # (M + 1) / 2 is the smallest residue class taken negative
    top = (nt.PPP + 1) // 2
    z = nt.garner_crt3(*(np.array([top % p], dtype=np.uint64) for p in m))
    assert int(z[0]) == top - nt.PPP


def test_alpha_three_moduli():
    # n = 2^18, L = 3: alpha = 36, so that two slices give 72 bits
    assert oz.alpha_crt(1 << 18, 3, nt.PPP) == 36
    for lg in (0, 5, 10, 17, 18, 20, 24):
        for L in (1, 3, 12):
            n = 1 << lg
            a = oz.alpha_crt(n, L, nt.PPP)
            assert 2 * L * n * 4 ** a <= nt.PPP < 2 * L * n * 4 ** (a + 1)
    assert bl.KernelPlan(1 << 10, 2, 3, cyclic=True, primes=3).alpha == oz.alpha_crt(1 << 10, 3, nt.PPP)


def _truncated_exact(slices, alpha):
    out = None
    for a, E in slices:
        v = [Fraction(int(q)) * Fraction(2) ** (E - alpha) for q in a]
        out = v if out is None else [u + w for u, w in zip(out, v)]
    return out


@pytest.mark.parametrize("n,K,L,cyclic", [(8, 2, 3, True), (17, 2, 3, False), (33, 1, 1, False),
                                          (64, 3, 3, True), (40, 2, 2, False)])
def test_integer_pipeline_is_exact_three_moduli(n, K, L, cyclic):
    """y' = RN(sum over the four convolutions of the exact products of the
    retained slices): NTT mod p0, p1, p2, grouping, Garner with d = 3 and
    recombination pinned by a direct rational evaluation."""
    x = wl.paper_phi(n, 1.0, seed=n)[0]
    plan = bl.KernelPlan(n, K, L, cyclic=cyclic, primes=3)
    tr = bl.forward_trace(x, K, L, plan)
    assert tr["alpha"] == oz.alpha_crt(n, L, nt.PPP) > oz.alpha_crt(n, L)
    X = [_truncated_exact(tr["slices"][v], tr["alpha"]) for v in range(2)]
    W = [_truncated_exact(plan.slices[v], tr["alpha"]) for v in range(2)]
    for tgt, out in ((0, tr["ypr"]), (1, tr["ypi"])):
        for k in range(n):
            acc = Fraction(0)
            for (pa, pb, t, sg) in bl.CONVS:
                if t != tgt or not X[pa] or not W[pb]:
                    continue
                acc += sg * sum(X[pa][j] * W[pb][abs(k - j)] for j in range(n))
            assert out[k] == bl._round_fraction(acc), (tgt, k)


def test_two_moduli_range_is_caught_by_pin(monkeypatch):
    """Planting the two-prime Garner into the three-prime pipeline (a CRT
    range of p0 p1 for products sized for p0 p1 p2) must break the pin."""
    n = 32
    x = wl.uniform(n, seed=9)[0]
    monkeypatch.setattr(nt, "garner_crt3", lambda a, b, c: nt.garner_crt(a, b))
    plan = bl.KernelPlan(n, 2, 1, cyclic=True, primes=3)
    tr = bl.forward_trace(x, 2, 1, plan)
    X = [_truncated_exact(tr["slices"][v], tr["alpha"]) for v in range(2)]
    W = [_truncated_exact(plan.slices[v], tr["alpha"]) for v in range(2)]
    acc = Fraction(0)
    for (pa, pb, t, sg) in bl.CONVS:
        if t == 0:
            acc += sg * sum(X[pa][j] * W[pb][abs(0 - j)] for j in range(n))
    assert tr["ypr"][0] != bl._round_fraction(acc)


@pytest.mark.parametrize("n", [256, 1000])
def test_two_slices_reach_binary64_with_three_moduli(n):
    x = wl.paper_phi(n, 1.0, seed=7, batch=1)[0]
    ref = np.fft.fft(x.astype(np.clongdouble))

    def rel(y):
        y = np.asarray(y).astype(np.clongdouble)
        return float(np.sqrt(np.sum(np.abs(y - ref) ** 2)) / np.sqrt(np.sum(np.abs(ref) ** 2)))

    e3 = rel(bl.fft(x, plan=bl.KernelPlan(n, 2, 3, primes=3)))
    e2 = rel(bl.fft(x, plan=bl.KernelPlan(n, 3, 3)))
    e1 = rel(bl.fft(x, plan=bl.KernelPlan(n, 1, 3, primes=3)))
    assert e3 < 4 * U and e3 <= 1.5 * e2       # K = 2 with ~40-bit slices: the K = 3 two-prime accuracy
    assert e1 > 2.0 ** -48 and e1 > 100 * e3   # one slice of about 40 bits is not enough
