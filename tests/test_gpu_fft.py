"""GPU parity of the full transform against the oracle.

Every intermediate the library exposes is compared bit for bit with the
oracle's (chirp, x', slice counts and exponents, forward NTTs of the slices,
kernel NTTs, inverse-NTT residues of every accumulation group); the binary64
outputs must agree within 2 ulp per component (the method is deterministic
and the expected distance is 0)."""

import numpy as np
import pytest

import workloads as wl
from oracle import bluestein as bl
from oracle import ntt as nt
from oracle import ozaki as oz_or
from oracle import reference as ref
from tests.accum_schedule import acc_limit, component_schedule, group_residues, part_shift
from tests.gpu_helpers import max_ulp, ntt_domain_index

pytestmark = pytest.mark.gpu
ULP_TOL = 2


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


def _gpu(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).cuda()


_KPLANS = {}


def kplan(n, K, L, cyclic=None):
    """Oracle plan with the library's embedding: by default (cyclic=None) the
    cyclic N = n for power-of-two n, as the library's default plans."""
    if cyclic is None:
        cyclic = bl.is_pow2(n)
    cyclic = bool(cyclic) and bl.is_pow2(n)
    key = (n, K, L, cyclic)
    if key not in _KPLANS:
        _KPLANS[key] = bl.KernelPlan(n, K, L, cyclic=cyclic)
    return _KPLANS[key]


def check_stages(plan, idx, tr, kp, K):
    """Bit-exact comparison of the exposed intermediates of one transform."""
    n, N = tr["n"], tr["N"]
    info = plan.transform_info(idx)
    assert info["status"] == tr["status"]
    assert info["N"] == N and info["alpha"] == tr["alpha"]
    # chirp
    ch = plan.debug_dump(5, idx)
    assert np.array_equal(ch.real, kp.c) and np.array_equal(ch.imag, kp.s)
    if tr["status"]:
        return
    # x'
    xp = plan.debug_dump(1, idx)
    assert np.array_equal(xp.real, tr["xpr"]) and np.array_equal(xp.imag, tr["xpi"])
    # slice counts and exponents
    for part in range(2):
        assert info["kx"][part] == len(tr["slices"][part])
        assert info["Ex"][part] == [E for _, E in tr["slices"][part]]
        assert info["kw"][part] == len(kp.slices[part])
        assert info["Ew"][part] == [E for _, E in kp.slices[part]]
    # accumulation schedule: group counts per output component
    complex_acc = plan.info()["accumulation"] == 1
    limit = acc_limit(n, tr["alpha"]) if complex_acc else tr["L"]
    assert info["acc_limit"] == limit
    EX = [[E for _, E in tr["slices"][v]] for v in range(2)]
    EW = [kp.exps(v) for v in range(2)]
    sched = component_schedule(EX, EW, tr["L"], "complex" if complex_acc else "per_conv", limit, weights=True,
                                alpha=tr["alpha"])
    if not complex_acc:       # the paper's schedule: the oracle's Alg. 8 groups, convolution by convolution
        assert [[(s, t) for _, s, t, _ in g] for g in sched[0] + sched[1]] == [
            list(g) for c in range(4) for g in tr["groups"][c]]
    assert info["ngroups"] == [len(g) for g in sched]
    xsh = part_shift(EX, EW, limit, tr["alpha"]) if complex_acc else [0, 0]
    assert info["xsh"] == xsh
    logN = N.bit_length() - 1
    perm = ntt_domain_index(logN, info["ntt_log2N1"])
    # forward NTTs of the slices (part p's times 2^xsh[p])
    X = plan.debug_dump(2, idx).reshape(2, K, 2, N)
    for part in range(2):
        for k in range(len(tr["slices"][part])):
            for ip, p in enumerate(nt.PRIMES):
                want = (tr["X"][part][k][ip] * np.uint64(1 << xsh[part])) % np.uint64(p)
                assert np.array_equal(X[part, k, ip].astype(np.uint64), want[perm]), (part, k, ip)
    # kernel NTTs (times N^-1)
    W = plan.debug_dump(4, idx).reshape(2, K, 2, N)
    for part in range(2):
        for t in range(len(kp.slices[part])):
            for ip, p in enumerate(nt.PRIMES):
                want = (kp.ntts[part][t][ip] * np.uint64(pow(N, -1, p))) % np.uint64(p)
                assert np.array_equal(W[part, t, ip].astype(np.uint64), want[perm]), (part, t, ip)
    # inverse NTT residues of every group (signed sums: ImIm enters Re y' negated)
    Z = plan.debug_dump(3, idx).reshape(4 * K * K, 2, (n + 3) // 4 * 4)[:, :, :n]
    for tg in range(2):
        for g, grp in enumerate(sched[tg]):
            slot = tg * 2 * K * K + g
            if complex_acc:
                want = group_residues(tr, kp, grp)
            else:             # the oracle's group integers, convolution by convolution
                c = grp[0][0]
                j = sum(1 for h in sched[tg][:g] if h[0][0] == c)
                z = tr["group_z"][c][j][0] * bl.CONVS[c][3]
                want = [np.mod(z, p).astype(np.uint64) for p in nt.PRIMES]
            for ip in range(2):
                assert np.array_equal(Z[slot, ip].astype(np.uint64), want[ip]), (tg, g, ip)


@pytest.mark.parametrize("cyclic", [True, False])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 16, 17, 31, 64, 100, 127, 1000, 1024, 2047, 2048, 2049, 4097])
def test_forward_small(torch_mod, n, cyclic):
    import paper_2603_29129_amd as oz
    torch = torch_mod
    K, L = 3, 3
    x = wl.paper_phi(n, 1.0, seed=n, batch=2)
    plan = oz.Plan(n, 2, K=K, L=L, cyclic=cyclic)
    xd = _gpu(torch, x)              # held: stage 1 is rebuilt from the input
    y = plan.forward(xd).cpu().numpy()
    kp = kplan(n, K, L, cyclic)
    for b in range(2):
        tr = bl.forward_trace(x[b], K, L, kp)
        check_stages(plan, b, tr, kp, K)
        assert max_ulp(y[b], tr["y"]) <= ULP_TOL


def test_plain_1k_config(torch_mod):
    """One transform, n = 2^10 with the padded convolution length N = 2048,
    uniform[-1, 1], seed 0; the cyclic embedding (N = 1024) gives the same
    bits."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    x = wl.plain_1k(0)
    ys = []
    for cyclic, N in ((False, 2048), (True, 1024)):
        for mode in ("plain", "batched"):
            plan = oz.Plan(1024, 1, mode=mode, cyclic=cyclic)
            xd = _gpu(torch, x)              # held: stage 1 is rebuilt from the input
            y = plan.forward(xd).cpu().numpy()
            kp = kplan(1024, 3, 3, cyclic)
            tr = bl.forward_trace(x[0], 3, 3, kp)
            assert plan.transform_info(0)["N"] == N
            check_stages(plan, 0, tr, kp, 3)
            assert max_ulp(y[0], tr["y"]) == 0
            assert ref.rel_l2_error(y[0], ref.dft_longdouble(x[0])) < 1e-15
            ys.append(y)
    assert all(np.array_equal(v.view(np.uint64), ys[0].view(np.uint64)) for v in ys)


@pytest.mark.parametrize("n", [8192, 1 << 16])
def test_cyclic_embedding_two_pass(torch_mod, n):
    """Power-of-two n in the two-pass NTT range: the cyclic embedding's
    intermediates match the cyclic oracle and its outputs are bit-identical
    to the padded embedding's, batched and plain."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    x = wl.paper_phi(n, 1.0, seed=5, batch=3)
    xd = _gpu(torch, x)
    outs = []
    for cyclic in (True, False):
        for mode in ("batched", "plain"):
            plan = oz.Plan(n, 3, mode=mode, cyclic=cyclic)
            outs.append(plan.forward(xd).cpu().numpy())
            assert plan.transform_info(0)["N"] == (n if cyclic else 2 * n)
            if cyclic and mode == "batched" and n == 8192:
                kp = kplan(n, 3, 3, True)
                tr = bl.forward_trace(x[1], 3, 3, kp)
                check_stages(plan, 1, tr, kp, 3)
                assert max_ulp(outs[-1][1], tr["y"]) == 0
    assert all(np.array_equal(v.view(np.uint64), outs[0].view(np.uint64)) for v in outs)


def _spiked(n, spikes, seed=0):
    """Small noise with x_0 set per transform: x'_0 = x_0 (the chirp is 1
    there), so the spike fixes the top exponents of Re x' and Im x'."""
    x = wl.paper_phi(n, 0.0, seed=seed, batch=len(spikes)) * 2.0 ** -6
    x[:, 0] = spikes
    return x


@pytest.mark.parametrize("n,xsh", [(12, [[1, 0], [0, 1], [0, 0], [2, 0]]),
                                   (1 << 16, [[1, 0], [0, 1], [0, 0], [0, 0]])])
def test_part_shift(torch_mod, n, xsh):
    """Re x' and Im x' with top exponents 1 or 2 binades apart: the larger
    part is taken times 2^xsh (when an anti-diagonal of its products still
    fits the group bound) and its products share groups with the other
    part's.  Intermediates bit-exact, outputs 0 ulp from the oracle; at
    n = 2^16 (bound 7, three kernel slices) a shift of 2 would not fit."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    x = _spiked(n, [1 + 0.4j, 0.4 + 1j, 1 + 1j, 1 + 0.2j])
    plan = oz.Plan(n, 4)
    xd = _gpu(torch, x)              # held: stage 1 is rebuilt from the input
    y = plan.forward(xd).cpu().numpy()
    kp = kplan(n, 3, 3)
    for b in range(4):
        tr = bl.forward_trace(x[b], 3, 3, kp)
        check_stages(plan, b, tr, kp, 3)
        assert plan.transform_info(b)["xsh"] == xsh[b], b
        assert max_ulp(y[b], tr["y"]) == 0, b
    if n > 12:                # 10 groups per component unshifted, 6 shifted, 5 with equal exponents
        assert [plan.transform_info(b)["ngroups"] for b in range(4)] == [[6, 6], [6, 6], [5, 5], [10, 10]]


def test_part_shift_lowest_grid(torch_mod):
    """Regression: the shifted part's last slice on the lowest grid
    2^-1022 (alpha = 27 at n = 12; scaled by 2^-968 the Re x' slices have
    exponents -968, -995 and Im x' -970, so Re x' is taken times 2^2 and its
    second slice is scaled by 2^(alpha - E + 2) = 2^1024, beyond binary64;
    the slice itself must be scaled, not the factor formed).  Both the
    batched and the plain form, 0 ulp from the oracle, every stage exact."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    n = 12
    base = _spiked(n, [1 + 1j, 1 + 1j, 1 + 1j, 1 + 0.2j])[3]
    x = np.stack([base * 2.0 ** -968, base * 2.0 ** -966, base * 2.0 ** -967])
    kp = kplan(n, 3, 3)
    want_ex = ([-968, -995], [-966, -993], [-967, -994])
    for mode in ("batched", "plain"):
        plan = oz.Plan(n, 3, mode=mode)
        xd = _gpu(torch, x)              # held: stage 1 is rebuilt from the input
        y = plan.forward(xd).cpu().numpy()
        for b in range(3):
            tr = bl.forward_trace(x[b], 3, 3, kp)
            info = plan.transform_info(b)
            assert info["status"] == 0 and info["xsh"] == [2, 0], (mode, b)
            assert info["Ex"][0] == want_ex[b], (mode, b)
            check_stages(plan, b, tr, kp, 3)
            assert max_ulp(y[b], tr["y"]) == 0, (mode, b)


def test_part_shift_headline_length(torch_mod):
    """n = 2^18 (folded forward rows, fused column pass): a transform with
    the Re x' top exponent one above Im x' next to one with them equal, in
    one launch; full outputs 0 ulp from the oracle."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    n = 1 << 18
    x = _spiked(n, [1 + 0.4j, 1 + 1j], seed=3)
    plan = oz.Plan(n, 2)
    xd = _gpu(torch, x)              # held: stage 1 is rebuilt from the input
    y = plan.forward(xd).cpu().numpy()
    kp = kplan(n, 3, 3)
    for b, (xs, ng) in enumerate((([1, 0], [6, 6]), ([0, 0], [5, 5]))):
        info = plan.transform_info(b)
        assert info["xsh"] == xs and info["ngroups"] == ng, b
        assert max_ulp(y[b], bl.fft(x[b], plan=kp)) == 0, b


@pytest.mark.parametrize("K,L", [(1, 1), (2, 1), (3, 1), (2, 2), (4, 3), (6, 1), (8, 8)])
def test_K_L_variants(torch_mod, K, L):
    import paper_2603_29129_amd as oz
    torch = torch_mod
    n = 777
    x = wl.paper_phi(n, 4.0, seed=K * 10 + L, batch=1)
    plan = oz.Plan(n, 1, K=K, L=L)
    xd = _gpu(torch, x)              # held: stage 1 is rebuilt from the input
    y = plan.forward(xd).cpu().numpy()
    kp = kplan(n, K, L)
    tr = bl.forward_trace(x[0], K, L, kp)
    check_stages(plan, 0, tr, kp, K)
    assert max_ulp(y[0], tr["y"]) == 0


@pytest.mark.parametrize("direction", [1, 2])
def test_inverse_and_adjoint(torch_mod, direction):
    import paper_2603_29129_amd as oz
    torch = torch_mod
    for n in (64, 1000, 10007):
        x = wl.uniform(n, batch=1, seed=n)
        plan = oz.Plan(n, 1)
        y = plan.execute(_gpu(torch, x), direction).cpu().numpy()
        kp = kplan(n, 3, 3)
        want = bl.ifft(x[0], plan=kp) if direction == 1 else bl.adjoint(x[0], plan=kp)
        assert max_ulp(y[0], want) == 0


def test_modes_identical_and_uneven_lengths(torch_mod):
    import paper_2603_29129_amd as oz
    torch = torch_mod
    lengths = [1, 3, 1024, 1031, 5000, 4096, 4099, 257, 10007, 2]
    rng = np.random.default_rng(5)
    xs = [rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n) for n in lengths]
    flat = np.concatenate(xs)
    outs = {}
    for mode in ("plain", "batched"):
        plan = oz.Plan(lengths=lengths, mode=mode)
        outs[mode] = plan.forward(_gpu(torch, flat)).cpu().numpy()
        # run twice: the graph replay must give the same bits
        again = plan.forward(_gpu(torch, flat)).cpu().numpy()
        assert np.array_equal(again.view(np.uint64), outs[mode].view(np.uint64))
    assert np.array_equal(outs["plain"].view(np.uint64), outs["batched"].view(np.uint64))
    off = 0
    for n, x in zip(lengths, xs):
        want = bl.fft(x, 3, 3, kplan(n, 3, 3))
        assert max_ulp(outs["batched"][off:off + n], want) == 0, n
        off += n


def test_special_inputs(torch_mod):
    import paper_2603_29129_amd as oz
    torch = torch_mod
    n = 100
    x = wl.uniform(n, batch=4, seed=3)
    x[0] = 0
    x[1, 7] = np.nan
    x[2] *= 2.0 ** 1000
    x[3, 5] = 1e-300          # tiny element next to O(1) values: split stops early
    plan = oz.Plan(n, 4)
    xd = _gpu(torch, x)              # held: stage 1 is rebuilt from the input
    y = plan.forward(xd).cpu().numpy()
    # a zero input gives y' = +0; the postmultiply's IEEE products then carry
    # the chirp's signs into signed zeros, exactly as in the oracle
    assert np.all(y[0] == 0)
    assert np.array_equal(y[0].view(np.uint64), bl.fft(x[0], 3, 3, kplan(n, 3, 3)).view(np.uint64))
    assert plan.transform_info(1)["status"] == oz_or.STATUS_NONFINITE and np.all(np.isnan(y[1].real))
    assert plan.transform_info(2)["status"] == oz_or.STATUS_RANGE and np.all(np.isnan(y[2].imag))
    kp = kplan(n, 3, 3)
    for b in range(4):
        tr = bl.forward_trace(x[b], 3, 3, kp)
        assert plan.transform_info(b)["status"] == tr["status"]
        assert max_ulp(y[b], tr["y"]) == 0


def test_special_inputs_two_pass_runs(torch_mod):
    """Special transforms inside the multi-transform runs of the two-pass
    inverse (64 x n = 2^14, two transforms per inverse-row workgroup): an
    all-zero transform (no groups), a non-finite one and an out-of-range one
    (status set, skipped), one whose premultiplied input is real (no slices
    of Im x'), and their neighbours, all bit-identical to the oracle."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    n = 16384
    x = wl.batch_16k(1)
    x[1] = 0
    x[2, 100] = np.inf
    x[3] *= 2.0 ** 1000
    x[4] = 0
    x[4, 0] = 1.5             # x' = x (.) w is real: one slice of Re x', none of Im x'
    x[6, 9] = 1e-300
    plan = oz.Plan(n, 64, cyclic=False)         # N = 2^15: two transforms per inverse-row workgroup
    xd = _gpu(torch, x)              # held: stage 1 is rebuilt from the input
    y = plan.forward(xd).cpu().numpy()
    kp = kplan(n, 3, 3, False)
    for b in (0, 1, 2, 3, 4, 5, 6, 7, 63):
        tr = bl.forward_trace(x[b], 3, 3, kp)
        assert plan.transform_info(b)["status"] == tr["status"], b
        assert max_ulp(y[b], tr["y"]) == 0, b


@pytest.mark.parametrize("n", [1000, 8192])
def test_wide_exponent_span(torch_mod, n):
    """Half the entries 2^-300 times the others (K = 8): the split jumps from
    the O(1) entries to the tiny ones, the group exponents of one output
    component span about 400 bits and the recombination takes its wide
    accumulator; transforms with ordinary spans in the same launch take the
    fast one.  All bit-identical to the oracle."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    x = wl.uniform(n, batch=3, seed=21)
    x[1, ::2] *= 2.0 ** -300
    plan = oz.Plan(n, 3, K=8, L=3)
    xd = _gpu(torch, x)              # held: stage 1 is rebuilt from the input
    y = plan.forward(xd).cpu().numpy()
    kp = kplan(n, 8, 3)
    for b in range(3):
        tr = bl.forward_trace(x[b], 8, 3, kp)
        if b == 1:
            es = [e for conv in tr["group_z"] for (_z, e) in conv]
            assert max(es) - min(es) > 300
            check_stages(plan, b, tr, kp, 8)
        assert max_ulp(y[b], tr["y"]) == 0, b


def test_batch_16k_roundtrip(torch_mod):
    """64 transforms at n = 2^14 (N = 2^15): two sampled transforms compared
    with the oracle, all 64 round-tripped through the inverse."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    x = wl.batch_16k(0)
    plan = oz.Plan(16384, 64)
    xd = _gpu(torch, x)
    yd = plan.forward(xd)
    y = yd.cpu().numpy()
    kp = kplan(16384, 3, 3)
    for b in (0, 63):
        tr = bl.forward_trace(x[b], 3, 3, kp)
        check_stages(plan, b, tr, kp, 3)       # intermediates of the last execution
        assert max_ulp(y[b], tr["y"]) == 0
    z = plan.inverse(yd).cpu().numpy()
    assert np.max(np.abs(z - x)) < 1e-14
    assert ref.rel_l2_error(y[5], ref.dft_longdouble(x[5])) < 1e-15


def test_batch_prime_10007(torch_mod):
    import paper_2603_29129_amd as oz
    torch = torch_mod
    x = wl.batch_prime(0)
    plan = oz.Plan(10007, 64)
    xd = _gpu(torch, x)
    yd = plan.forward(xd)
    y = yd.cpu().numpy()
    kp = kplan(10007, 3, 3)
    for b in (0, 31):
        tr = bl.forward_trace(x[b], 3, 3, kp)
        check_stages(plan, b, tr, kp, 3)
        assert max_ulp(y[b], tr["y"]) == 0
    z = plan.inverse(yd).cpu().numpy()
    assert np.max(np.abs(z - x)) < 1e-14
