"""Pins for oracle.bluestein: chirp, padding, Alg. 8 schedule, counts, the
exactness of the integer pipeline, and the whole DFT (CPU only)."""

from fractions import Fraction
import json
import os

import mpmath
import numpy as np
import pytest

import workloads as wl
from oracle import bluestein as bl
from oracle import ntt as nt
from oracle import ozaki as oz
from oracle import reference as ref

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
U = 2.0 ** -53


def test_conv_length():
    cases = {1: 1, 2: 4, 3: 8, 5: 16, 1024: 2048, 1025: 4096, 10007: 32768, 16384: 32768,
             65536: 131072, 65521: 131072, 1 << 18: 1 << 19}
    for n, N in cases.items():
        assert bl.conv_length(n) == N
        assert N >= 2 * n - 1 and (N == 1 or N // 2 < 2 * n - 1)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 12, 17, 64, 100, 127, 1000])
def test_chirp_correctly_rounded(n):
    c, s = bl.chirp(n)
    with mpmath.workprec(320):
        for j in range(n):
            th = mpmath.pi * ((j * j) % (2 * n)) / n
            cc, ss = mpmath.cos(th), mpmath.sin(th)
            for got, exact in ((c[j], cc), (s[j], ss)):
                if abs(exact) < mpmath.mpf(2) ** -200:
                    assert got == 0.0 and np.signbit(got) == False  # noqa: E712
                    continue
                # |got - exact| <= half an ulp of got, i.e. got = RN(exact)
                err = abs(mpmath.mpf(got) - exact)
                assert err <= mpmath.mpf(np.spacing(abs(got))) / 2


def test_chirp_symmetries():
    for n in (7, 101, 10007):
        c, s = bl.chirp(n)
        # odd n: (n-j)^2 = j^2 + n (mod 2n), so w(n-j) = -w(j)
        j = np.arange(1, n)
        assert np.array_equal(c[n - j], -c[j]) and np.array_equal(s[n - j], -s[j])
    for n in (8, 1024):
        c, s = bl.chirp(n)
        j = np.arange(1, n)
        assert np.array_equal(c[n - j], c[j]) and np.array_equal(s[n - j], s[j])


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13])
def test_padding_turns_cyclic_into_bluestein_convolution(n):
    rng = np.random.default_rng(n)
    a = rng.integers(-50, 50, n)
    b = rng.integers(-50, 50, n)
    N = bl.conv_length(n)
    cyc = nt.cyclic_convolution_direct(bl.pad_input(a, N), bl.pad_kernel(b, N))
    for k in range(n):
        assert cyc[k] == sum(int(a[j]) * int(b[abs(k - j)]) for j in range(n))


def test_alg8_gapless_groups():
    alpha = 21
    E = [0, -alpha, -2 * alpha]
    g3 = bl.alg8_groups(E, E, 3)
    assert [len(g) for g in g3] == [1, 2, 3, 2, 1]
    assert g3[0] == [(2, 2)] and g3[-1] == [(0, 0)]
    g1 = bl.alg8_groups(E, E, 1)
    assert len(g1) == 9 and all(len(g) == 1 for g in g1)
    g2 = bl.alg8_groups(E, E, 2)
    assert [len(g) for g in g2] == [1, 2, 2, 1, 2, 1]
    # every pair exactly once
    for gs in (g1, g2, g3):
        pairs = sorted(p for g in gs for p in g)
        assert pairs == [(s, t) for s in range(3) for t in range(3)]
    # a gap in the first operand splits the anti-diagonals
    Eg = [0, -alpha - 5, -2 * alpha - 5]
    gg = bl.alg8_groups(Eg, E, 3)
    keys = [[Eg[s] + E[t] for s, t in g] for g in gg]
    assert all(len(set(k)) == 1 for k in keys)
    assert bl.alg8_groups([], E, 3) == []


def test_count_closed_forms():
    # Sec. 4.5: L >= K and gapless -> 24K - 8 total, 20K - 8 runtime; L = 1 -> 8K + 8K^2
    alpha = 21
    for K in (1, 2, 3, 4):
        E = [-k * alpha for k in range(K)]
        inv3 = 2 * 4 * len(bl.alg8_groups(E, E, K))
        inv1 = 2 * 4 * len(bl.alg8_groups(E, E, 1))
        assert 4 * K + 4 * K + inv3 == 24 * K - 8
        assert 4 * K + inv3 == 20 * K - 8
        assert 4 * K + 4 * K + inv1 == 8 * K + 8 * K * K


def _counts(n, phi, K, L, seed=0):
    alpha = oz.alpha_crt(n, L)
    c, s = bl.chirp(n)
    x = wl.paper_phi(n, phi, seed)[0]
    xr, xi = bl.premultiply(x.real.copy(), x.imag.copy(), c, s)
    sx = [oz.split(v, alpha, K)[0] for v in (xr, xi)]
    sw = [oz.split(v, alpha, K)[0] for v in (c, s)]
    EX = [[E for _, E in q] for q in sx]
    EW = [[E for _, E in q] for q in sw]
    g = [len(bl.alg8_groups(EX[a], EW[b], L)) for (a, b, _, _) in bl.CONVS]
    return 2 * (len(sx[0]) + len(sx[1]) + len(sw[0]) + len(sw[1])) + 2 * sum(g), [len(q) for q in sw]


def test_printed_counts():
    gc = GOLDEN["ntt_counts"]
    for n in (1 << 10, 1 << 12, 1 << 14):
        for phi in (0.0, 1.0):
            assert _counts(n, phi, 3, 3)[0] == gc["K3_L3_total_phi01"]
        for phi in (0.0, 1.0, 4.0):
            assert _counts(n, phi, 3, 1)[0] == gc["K3_L1_total"]
    assert gc["K3_L3_total_phi01"] - 12 == gc["K3_L3_runtime"]


@pytest.mark.parametrize("n", [1 << 10, 1 << 12])
def test_oracle_ntt_counts_printed(n):
    """The oracle's own counter (ntt_counts) on full forward traces against
    the printed totals: 64 transforms at K = L = 3 for phi = 0, 1 (Sec. 5.4),
    52 of them at runtime (Sec. 5.5), 96 at K = 3, L = 1 (Sec. 5.3); and the
    split of the totals into runtime forward, offline forward and inverse
    transforms that the closed forms of Sec. 4.5 give for gapless splits:
    4K + 4K offline / runtime forward, 8(2K - 1) inverse (L >= K) or 8K^2
    (L = 1)."""
    gc = GOLDEN["ntt_counts"]
    K = 3
    for L, phis, total in ((3, (0.0, 1.0), gc["K3_L3_total_phi01"]), (1, (0.0, 1.0, 4.0), gc["K3_L1_total"])):
        kp = bl.KernelPlan(n, K, L)
        for phi in phis:
            x = wl.paper_phi(n, phi, 0)[0]
            c = bl.ntt_counts(bl.forward_trace(x, K, L, kp), kp)
            assert c["total"] == total
            assert c["forward_offline"] == 4 * K and c["forward_runtime"] == 4 * K
            assert c["inverse"] == (8 * (2 * K - 1) if L >= K else 8 * K * K)
            assert c["runtime"] == c["forward_runtime"] + c["inverse"]
            assert c["total"] == c["runtime"] + c["forward_offline"]
            if L == 3:
                assert c["runtime"] == gc["K3_L3_runtime"]
                assert c["total"] == 24 * K - 8 and c["runtime"] == 20 * K - 8
            else:
                assert c["total"] == 8 * K + 8 * K * K


def test_oracle_ntt_counts_planted_mistakes():
    """ntt_counts must see both primes and the offline kernel transforms: a
    trace with one slice fewer per input part drops exactly 2 x 2 runtime
    forward transforms, and a three-modulus plan counts 3 per vector."""
    n, K = 1 << 10, 3
    kp = bl.KernelPlan(n, K, 3)
    x = wl.paper_phi(n, 0.0, 0)[0]
    tr = bl.forward_trace(x, K, 3, kp)
    c = bl.ntt_counts(tr, kp)
    short = dict(tr, slices=[tr["slices"][0][:-1], tr["slices"][1][:-1]])
    cs = bl.ntt_counts(short, kp)
    assert c["forward_runtime"] - cs["forward_runtime"] == 4
    assert cs["inverse"] == c["inverse"] and cs["forward_offline"] == c["forward_offline"]
    kp3 = bl.KernelPlan(n, 2, 3, primes=3)
    c3 = bl.ntt_counts(bl.forward_trace(x, 2, 3, kp3), kp3)
    assert c3["forward_offline"] == 3 * 2 * 2 and c3["forward_runtime"] == 3 * 2 * 2
    assert c3["inverse"] % 3 == 0


@pytest.mark.slow
def test_kernel_split_count_large_n():
    g = GOLDEN["kernel_split_count_large_n"]
    for n in g["n"]:
        c, s = bl.chirp(n)
        for v in (c, s):
            sl, _, _ = oz.split(v, oz.alpha_crt(n, 1), None)
            assert len(sl) == g["kw"]


def _truncated_exact(v_slices, alpha):
    n = len(v_slices[0][0]) if v_slices else 0
    out = [Fraction(0)] * n
    for a, E in v_slices:
        sc = Fraction(2) ** (E - alpha)
        for j in range(n):
            out[j] += int(a[j]) * sc
    return out


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 16, 17, 31, 64])
def test_integer_pipeline_is_exact_uncapped(n):
    """K uncapped: every split is exact, so y' must equal RN of the exact
    convolution of the binary64 x' and chirp (closed form, no NTT/CRT)."""
    x = wl.uniform(n, seed=100 + n)[0]
    plan = bl.KernelPlan(n, None, 1)
    tr = bl.forward_trace(x, None, 1, plan)
    yr, yi = bl.exact_convolution_rounded(tr["xpr"], tr["xpi"], plan.c, plan.s)
    assert np.array_equal(yr, tr["ypr"]) and np.array_equal(yi, tr["ypi"])


@pytest.mark.parametrize("n,K,L", [(8, 3, 3), (17, 3, 3), (33, 2, 1), (64, 3, 3), (50, 1, 1), (40, 3, 2)])
def test_integer_pipeline_is_exact_capped(n, K, L):
    """K capped: y' = RN(sum over the four convolutions of the exact products
    of the retained slices) -- NTT, grouping, CRT and recombination pinned
    by a direct rational evaluation."""
    x = wl.paper_phi(n, 1.0, seed=n)[0]
    plan = bl.KernelPlan(n, K, L)
    tr = bl.forward_trace(x, K, L, plan)
    a = alpha = tr["alpha"]
    X = [_truncated_exact(tr["slices"][v], alpha) for v in range(2)]
    W = [_truncated_exact(plan.slices[v], a) for v in range(2)]
    for tgt, out in ((0, tr["ypr"]), (1, tr["ypi"])):
        for k in range(n):
            acc = Fraction(0)
            for (pa, pb, t, sg) in bl.CONVS:
                if t != tgt or not X[pa] or not W[pb]:
                    continue
                acc += sg * sum(X[pa][j] * W[pb][abs(k - j)] for j in range(n))
            assert out[k] == bl._round_fraction(acc), (tgt, k)


def test_crt_range_violation_is_caught_by_pin(monkeypatch):
    """Planting alpha+1 (too wide) must break the exactness pin (Sec. 4.2 /
    4.4: alpha bounds the CRT range)."""
    n = 64
    x = wl.uniform(n, seed=9)[0] * 1.0
    real_alpha = oz.alpha_crt

    def wide(nn, L=1, modulus_product=nt.PP):
        return real_alpha(nn, L, modulus_product) + 2

    monkeypatch.setattr(oz, "alpha_crt", wide)
    plan = bl.KernelPlan(n, None, 1)
    tr = bl.forward_trace(x, None, 1, plan)
    yr, yi = bl.exact_convolution_rounded(tr["xpr"], tr["xpi"], plan.c, plan.s)
    assert not (np.array_equal(yr, tr["ypr"]) and np.array_equal(yi, tr["ypi"]))


def test_wrong_kernel_padding_is_caught_by_pin(monkeypatch):
    n = 16
    x = wl.uniform(n, seed=11)[0]
    monkeypatch.setattr(bl, "pad_kernel", bl.pad_input)   # plant: no wrap-around
    plan = bl.KernelPlan(n, None, 1)
    tr = bl.forward_trace(x, None, 1, plan)
    yr, yi = bl.exact_convolution_rounded(tr["xpr"], tr["xpi"], plan.c, plan.s)
    assert not (np.array_equal(yr, tr["ypr"]) and np.array_equal(yi, tr["ypi"]))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 16, 17, 64, 100, 127])
@pytest.mark.parametrize("KL", [(None, 1), (3, 3)])
def test_dft_accuracy_vs_mpmath(n, KL):
    K, L = KL
    x = wl.paper_phi(n, 1.0, seed=n)[0]
    y = bl.fft(x, K, L)
    r = ref.mpc_to_clongdouble(ref.dft_mpmath(x))
    assert ref.rel_l2_error(y, r) < 8 * U


@pytest.mark.parametrize("n,phi", [(4096, 0.0), (4096, 4.0), (10007, 1.0)])
def test_dft_accuracy_vs_longdouble(n, phi):
    x = wl.paper_phi(n, phi, seed=3)[0]
    y = bl.fft(x, 3, 3)
    r = ref.dft_longdouble(x)
    # Sec. 5.3: K = 3 relative errors lie in [1e-16, 1e-15]
    assert ref.rel_l2_error(y, r) < 1e-15


def test_dft_identities():
    n = 48
    plan = bl.KernelPlan(n, 3, 3)
    d = np.zeros(n, complex)
    d[0] = 1
    assert np.max(np.abs(bl.fft(d, plan=plan) - 1)) < 4 * U
    one = np.ones(n, complex)
    y = bl.fft(one, plan=plan)
    assert abs(y[0] - n) < 8 * n * U and np.max(np.abs(y[1:])) < 8 * n * U
    m = 5
    e = np.zeros(n, complex)
    e[m] = 1
    k = np.arange(n)
    with mpmath.workprec(200):
        want = np.array([complex(mpmath.expjpi(mpmath.mpf(-2 * ((m * kk) % n)) / n)) for kk in range(n)])
    assert np.max(np.abs(bl.fft(e, plan=plan) - want)) < 8 * U
    x = wl.uniform(n, seed=2)[0]
    g = wl.uniform(n, seed=3)[0]
    y = bl.fft(x, plan=plan)
    # Parseval
    assert abs(np.sum(np.abs(y) ** 2) - n * np.sum(np.abs(x) ** 2)) < 1e-13 * n * np.sum(np.abs(x) ** 2)
    # shift <-> modulation: DFT(x(j - 1)) = w^k DFT(x)
    ys = bl.fft(np.roll(x, 1), plan=plan)
    assert np.max(np.abs(ys - np.exp(-2j * np.pi * k / n) * y)) < 1e-14 * np.max(np.abs(y))
    # linearity
    y2 = bl.fft(x + 2 * g, plan=plan)
    assert np.max(np.abs(y2 - y - 2 * bl.fft(g, plan=plan))) < 1e-14 * np.max(np.abs(y2))
    # adjoint: <F x, g> = <x, F^H g>
    lhs = np.vdot(g, y)
    rhs = np.vdot(bl.adjoint(g, plan=plan), x)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    # round trip
    assert np.max(np.abs(bl.ifft(y, plan=plan) - x)) < 1e-15


def test_nonfinite_and_range_status():
    x = wl.uniform(16, seed=1)[0]
    x[3] = np.nan
    tr = bl.forward_trace(x, 3, 3)
    assert tr["status"] == oz.STATUS_NONFINITE and np.all(np.isnan(tr["y"].real))
    x = wl.uniform(16, seed=1)[0] * 2.0 ** 1000
    tr = bl.forward_trace(x, 3, 3)
    assert tr["status"] == oz.STATUS_RANGE
    z = np.zeros(16, complex)
    y = bl.fft(z)
    assert np.all(y == 0)


def test_signed_zeros_follow_ieee_products():
    """A zero input gives y' = +0; y = y' (.) w is formed by IEEE products and
    sums, so the output's zeros carry the signs those operations give."""
    n = 100
    kp = bl.KernelPlan(n, 3, 3)
    y = bl.fft(np.zeros(n, complex), plan=kp)
    zr, zi = np.zeros(n), np.zeros(n)
    want_r = zr * kp.c + zi * kp.s
    want_i = zi * kp.c - zr * kp.s
    assert np.array_equal(np.signbit(y.real), np.signbit(want_r))
    assert np.array_equal(np.signbit(y.imag), np.signbit(want_i))
    assert np.any(np.signbit(y.imag))


# ---------------------------------------------------------------------------
# Power-of-two special case: cyclic embedding N = n (Sec. 3.2)

def test_chirp_index_has_period_n_for_even_n():
    """q(j) = j^2 mod 2n: (j + n)^2 = j^2 + 2jn + n^2 and n^2 = 2n (n/2), so for
    even n the index (and with it w*) has period n and is even in j; for odd n
    it does not, which is why the embedding is limited to even (here
    power-of-two) n."""
    for n in (2, 4, 6, 8, 10, 64, 1000):
        q = [(j * j) % (2 * n) for j in range(3 * n)]
        assert all(q[j + n] == q[j] for j in range(2 * n))
        assert all(q[(n - j) % n] == q[j] for j in range(n))
    for n in (3, 5, 7, 9):
        assert any(((j + n) ** 2) % (2 * n) != (j * j) % (2 * n) for j in range(n))


def test_cyclic_conv_length():
    for n in (1, 2, 4, 1024, 1 << 18):
        assert bl.conv_length(n, cyclic=True) == n
    for n in (3, 6, 10007):
        with pytest.raises(ValueError):
            bl.conv_length(n, cyclic=True)


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 64])
def test_cyclic_embedding_exact_uncapped(n):
    """N = n, K uncapped: y' must still be RN of the exact linear convolution
    of x' with the chirp (closed form, no NTT)."""
    x = wl.uniform(n, seed=200 + n)[0]
    plan = bl.KernelPlan(n, None, 1, cyclic=True)
    tr = bl.forward_trace(x, None, 1, plan)
    assert tr["N"] == n
    yr, yi = bl.exact_convolution_rounded(tr["xpr"], tr["xpi"], plan.c, plan.s)
    assert np.array_equal(yr, tr["ypr"]) and np.array_equal(yi, tr["ypi"])


@pytest.mark.parametrize("n,K,L", [(8, 3, 3), (32, 2, 1), (64, 3, 3)])
def test_cyclic_embedding_exact_capped(n, K, L):
    """N = n, K capped: direct rational evaluation of the retained slice
    products over |k - j| (the linear Bluestein convolution)."""
    x = wl.paper_phi(n, 1.0, seed=n + 1)[0]
    plan = bl.KernelPlan(n, K, L, cyclic=True)
    tr = bl.forward_trace(x, K, L, plan)
    alpha = tr["alpha"]
    X = [_truncated_exact(tr["slices"][v], alpha) for v in range(2)]
    W = [_truncated_exact(plan.slices[v], alpha) for v in range(2)]
    for tgt, out in ((0, tr["ypr"]), (1, tr["ypi"])):
        for k in range(n):
            acc = Fraction(0)
            for (pa, pb, t, sg) in bl.CONVS:
                if t != tgt or not X[pa] or not W[pb]:
                    continue
                acc += sg * sum(X[pa][j] * W[pb][abs(k - j)] for j in range(n))
            assert out[k] == bl._round_fraction(acc), (tgt, k)


@pytest.mark.parametrize("n", [2, 16, 256, 1024])
def test_cyclic_embedding_equals_padded(n):
    """Same slices, exponents, groups and CRT integers as the padded
    embedding, so the outputs are bit-identical."""
    x = wl.paper_phi(n, 4.0, seed=7)[0]
    tp = bl.forward_trace(x, 3, 3, bl.KernelPlan(n, 3, 3))
    tc = bl.forward_trace(x, 3, 3, bl.KernelPlan(n, 3, 3, cyclic=True))
    assert tc["N"] == n and tp["N"] == bl.conv_length(n)
    assert tc["groups"] == tp["groups"]
    for gc, gp in zip(tc["group_z"], tp["group_z"]):
        for (zc, ec), (zp, ep) in zip(gc, gp):
            assert ec == ep and np.array_equal(zc, zp)
    assert np.array_equal(tc["y"].view(np.uint64), tp["y"].view(np.uint64))


def test_cyclic_embedding_without_wrap_is_caught_by_pin(monkeypatch):
    """Planted mistake: a length-n kernel whose negative lags are dropped
    (b(j) only for the first half, zeros after) breaks the closed-form pin."""
    n = 16

    def half(b, N):
        out = np.zeros(N, dtype=np.int64)
        out[: n // 2] = np.asarray(b)[: n // 2]
        return out

    x = wl.uniform(n, seed=12)[0]
    monkeypatch.setattr(bl, "pad_kernel", half)
    plan = bl.KernelPlan(n, None, 1, cyclic=True)
    tr = bl.forward_trace(x, None, 1, plan)
    yr, yi = bl.exact_convolution_rounded(tr["xpr"], tr["xpi"], plan.c, plan.s)
    assert not (np.array_equal(yr, tr["ypr"]) and np.array_equal(yi, tr["ypi"]))
