"""The NTT-domain accumulation schedules (host logic, no GPU).

The per-convolution schedule must be Alg. 8 as the oracle implements it; the
complex schedule must visit every slice pair once, give the products of an
x' part shifted by xsh the weight 2^xsh, keep a group's weights within the
CRT range, and its signed group sums, the shifted part's products times
2^xsh, must reproduce the exact integer sums of the member convolutions
(brute force on tiny inputs)."""

import itertools

import numpy as np
import pytest

import workloads as wl
from oracle import bluestein as bl
from oracle import ntt as nt
from oracle import ozaki as oz
from tests.accum_schedule import P, acc_limit, component_schedule, group_residues, part_shift


def _random_exps(rng, k, gaps):
    E = [int(rng.integers(-5, 5))]
    for _ in range(k - 1):
        E.append(E[-1] - 20 - (int(rng.integers(0, 3)) * 20 if gaps else 0))
    return E


@pytest.mark.parametrize("seed", range(40))
def test_per_conv_is_alg8(seed):
    rng = np.random.default_rng(seed)
    K = int(rng.integers(1, 6))
    L = int(rng.integers(1, 5))
    gaps = bool(seed % 2)
    EX = [_random_exps(rng, int(rng.integers(0, K + 1)), gaps) for _ in range(2)]
    EW = [_random_exps(rng, int(rng.integers(1, K + 1)), gaps) for _ in range(2)]
    sched = component_schedule(EX, EW, L, "per_conv", L)
    want = [[(c, s, t) for s, t in g]
            for c in range(4) for g in bl.alg8_groups(EX[bl.CONVS[c][0]], EW[bl.CONVS[c][1]], L)]
    assert sched[0] + sched[1] == want


@pytest.mark.parametrize("seed", range(40))
def test_complex_schedule_properties(seed):
    rng = np.random.default_rng(100 + seed)
    K = int(rng.integers(1, 6))
    L = int(rng.integers(1, 5))
    limit = int(rng.integers(L, 9))
    alpha = int(rng.integers(26, 31))
    gaps = bool(seed % 2)
    EX = [_random_exps(rng, int(rng.integers(0, K + 1)), gaps) for _ in range(2)]
    EW = [_random_exps(rng, int(rng.integers(1, K + 1)), gaps) for _ in range(2)]
    sched = component_schedule(EX, EW, L, "complex", limit, weights=True, alpha=alpha)
    xsh = part_shift(EX, EW, limit, alpha)
    assert min(xsh) == 0 and max(xsh) <= 2 and alpha + max(xsh) <= 30
    if max(xsh):              # only the part with the larger top exponent, by the difference
        p = xsh.index(max(xsh))
        assert EX[p][0] - EX[1 - p][0] == xsh[p]
    for tg in range(2):
        members = [m[:3] for g in sched[tg] for m in g]
        # every pair of the component's two convolutions exactly once
        want = set()
        for c in (2 * tg, 2 * tg + 1):
            kA, kB = len(EX[bl.CONVS[c][0]]), len(EW[bl.CONVS[c][1]])
            want |= {(c, s, t) for s in range(kA) for t in range(kB)}
        assert len(members) == len(want) and set(members) == want
        # anti-diagonals descending
        ds = [s + t for _, s, t in members]
        assert ds == sorted(ds, reverse=True)
        for g in sched[tg]:
            assert all(sh == xsh[bl.CONVS[c][0]] for c, _, _, sh in g)
            keys = {EX[bl.CONVS[c][0]][s] - sh + EW[bl.CONVS[c][1]][t] for c, s, t, sh in g}
            assert len(g) >= 1 and len(keys) == 1 and sum(1 << sh for *_, sh in g) <= limit
        # never more groups than the per-convolution schedule when no exponent gaps
        if not gaps:
            per = component_schedule(EX, EW, L, "per_conv", L)
            assert len(sched[tg]) <= len(per[tg])


def test_acc_limit_values():
    # n = 2^18, L = 3: alpha = 20 and 7 n 4^20 <= (P-1)/2 < 8 n 4^20
    assert oz.alpha_crt(1 << 18, 3) == 20 and acc_limit(1 << 18, 20) == 7
    assert oz.alpha_crt(1 << 17, 3) == 21 and acc_limit(1 << 17, 21) == 3
    for lg in range(0, 24):
        for L in (1, 2, 3, 5, 8):
            n = 1 << lg
            a = oz.alpha_crt(n, L)
            if a < 1:
                continue
            lim = acc_limit(n, a)
            assert lim >= L                                       # alpha leaves room for L products
            assert lim * (n << (2 * a)) <= (P - 1) // 2 < (lim + 1) * (n << (2 * a)) or lim == 128


def test_bench_shape_groups():
    # gap-free, equal top exponents, K = L = 3: five anti-diagonals per component
    EX = [[0, -20, -40], [0, -20, -40]]
    EW = [[1, -19, -39], [1, -19, -39]]
    assert [len(g) for g in component_schedule(EX, EW, 3, "per_conv", 3)] == [10, 10]
    assert [len(g) for g in component_schedule(EX, EW, 3, "complex", 7, alpha=20)] == [5, 5]
    # a CRT bound of 3 products (odd log2 n) still saves groups
    assert [len(g) for g in component_schedule(EX, EW, 3, "complex", 3, alpha=20)] == [8, 8]
    # Re and Im parts one binade apart: Re x' is taken times 2, its products weigh 2
    EX2 = [[0, -20, -40], [-1, -21, -41]]
    assert part_shift(EX2, EW, 7, 20) == [1, 0]
    sched = component_schedule(EX2, EW, 3, "complex", 7, weights=True, alpha=20)
    assert [len(g) for g in sched] == [6, 6]
    assert sched[0][0] == [(0, 2, 2, 1), (1, 2, 2, 0)]
    # with a bound of 3 an anti-diagonal of weight-2 products does not fit: no shift, no merging
    assert part_shift(EX2, EW, 3, 20) == [0, 0]
    assert [len(g) for g in component_schedule(EX2, EW, 3, "complex", 3, alpha=20)] == [10, 10]
    # two binades apart with a bound of 12: Im x' times 4
    EX4 = [[-2, -22, -42], [0, -20, -40]]
    assert part_shift(EX4, EW, 12, 20) == [0, 2]
    assert [len(g) for g in component_schedule(EX4, EW, 3, "complex", 12, alpha=20)] == [6, 6]   # middle: 3 + 3 * 4 > 12
    # slice integers times 2^d must stay below 2^30: alpha + d <= 30
    assert part_shift(EX4, EW, 12, 28) == [0, 2] and part_shift(EX4, EW, 12, 29) == [0, 0]
    assert part_shift(EX2, EW, 7, 29) == [1, 0] and part_shift(EX2, EW, 7, 30) == [0, 0]
    # three binades apart: nothing merges
    EX3 = [[0, -20, -40], [-3, -23, -43]]
    assert part_shift(EX3, EW, 128, 20) == [0, 0]
    assert [len(g) for g in component_schedule(EX3, EW, 3, "complex", 7, alpha=20)] == [10, 10]


@pytest.mark.parametrize("n,cyclic,seed,im_scale,xsh", [
    (8, True, 0, 1.0, None), (16, True, 1, 1.0, None), (5, False, 2, 1.0, None), (12, False, 3, 1.0, None),
    (16, True, 4, 0.3, [1, 0]), (16, True, 4, 3.0, [0, 1]), (6, False, 6, 0.2, [0, 1]),
    (12, False, 8, 0.25, [2, 0]), (12, False, 8, 4.0, [0, 2])])
def test_complex_groups_exact(n, cyclic, seed, im_scale, xsh):
    """Signed NTT-domain sums of the complex schedule give, after the CRT,
    the exact integer sum of the member convolutions (computed by the
    definition of cyclic convolution), the shifted part's products counted
    2^xsh times.  im_scale != 1 moves the top exponents of Re x' and Im x'
    apart so that the part shift (xsh) is exercised."""
    K, L = 3, 3
    kp = bl.KernelPlan(n, K, L, cyclic=cyclic)
    x = wl.paper_phi(n, 1.0, seed=seed, batch=1)[0]
    x = x.real + 1j * im_scale * x.imag
    tr = bl.forward_trace(x, K, L, kp)
    N = tr["N"]
    EX = [[E for _, E in tr["slices"][v]] for v in range(2)]
    EW = [kp.exps(v) for v in range(2)]
    lim = acc_limit(n, tr["alpha"])
    sched = component_schedule(EX, EW, L, "complex", lim, weights=True, alpha=tr["alpha"])
    if xsh is not None:
        assert part_shift(EX, EW, lim, tr["alpha"]) == xsh
    for tg in range(2):
        for g in sched[tg]:
            z0, z1 = group_residues(tr, kp, g)
            got = nt.garner_crt(z0, z1)
            exact = np.zeros(N, dtype=object)
            for c, s, t, sh in g:
                pa, pb, _, sign = bl.CONVS[c]
                a = bl.pad_input(tr["slices"][pa][s][0], N)
                b = bl.pad_kernel(kp.slices[pb][t][0], N)
                exact = exact + (sign << sh) * np.array(nt.cyclic_convolution_direct(a, b), dtype=object)
            assert [int(v) for v in got] == [int(v) for v in exact[:n]]


def test_complex_worst_case_fits_crt():
    """acc_limit products of the largest magnitude n 4^alpha, all of one sign,
    stay inside the symmetric CRT range; one more would not."""
    for n in (1 << 10, 1 << 17, 1 << 18, 1000):
        a = oz.alpha_crt(n, 3)
        lim = acc_limit(n, a)
        worst = lim * n * (1 << a) * (1 << a)
        assert worst <= (P - 1) // 2
        assert (lim + 1) * n * 4 ** a > (P - 1) // 2
        # the CRT maps the residues of +-worst back to +-worst
        for v in (worst, -worst):
            assert int(nt.garner_crt(np.uint64(v % nt.P0), np.uint64(v % nt.P1))) == v


def test_members_fit_128_positions():
    # the library walks at most 2 K^2 <= 128 positions per component
    EX = [list(range(0, -160, -20))] * 2
    EW = [list(range(0, -160, -20))] * 2
    for mode in ("per_conv", "complex"):
        sched = component_schedule(EX, EW, 8, mode, 128, alpha=20)
        assert sum(len(g) for g in sched[0]) == 128
    assert list(itertools.chain(*component_schedule(EX, EW, 8, "complex", 128, alpha=20)[0]))[0] == (0, 7, 7)
