"""GPU parity at the benchmark workloads' full sizes.

n = 2^18 (wide dynamic range), the 256 mixed lengths in one batched launch,
and the differentiable transform on 32 x 2^16.  Where the oracle cannot
recompute everything in seconds, sampled transforms are compared exactly and
the rest is checked through properties that hold at any size (a transform
computed inside the batch equals the same transform planned alone; the plain
and batched forms agree bit for bit)."""

import numpy as np
import pytest

import workloads as wl
from oracle import bluestein as bl
from oracle import reference as ref
from tests.gpu_helpers import max_ulp, oracle_ffts, oracle_ffts_own_plans

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


def _gpu(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).cuda()


@pytest.fixture(scope="module")
def wide_plan():
    return bl.KernelPlan(1 << 18, 3, 3)


def test_wide_256k_batch8(torch_mod, wide_plan):
    """8 x n = 2^18, |x| log-uniform in [2^-30, 2^30]: transforms 0 and 7
    against the oracle, all 8 batched vs plain bit for bit."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    n, B = 1 << 18, 8
    x = wl.wide_256k(seed=0, batch=B, n=n)
    xd = _gpu(torch, x)
    yb = oz.Plan(n, B, mode="batched").forward(xd).cpu().numpy()
    yp = oz.Plan(n, B, mode="plain").forward(xd).cpu().numpy()
    assert np.array_equal(yb.view(np.uint64), yp.view(np.uint64))
    for b in (0, 7):
        want = bl.fft(x[b], 3, 3, wide_plan)
        assert max_ulp(yb[b], want) == 0
    assert ref.rel_l2_error(yb[0], ref.dft_longdouble(x[0])) < 1e-15


def test_wide_256k_every_transform_vs_oracle(torch_mod, wide_plan):
    """Every transform of the headline workload (8 x n = 2^18, |x|
    log-uniform in [2^-30, 2^30], seed 0) against the oracle, 0 ulp; the
    oracle runs one transform per process."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    n, B = 1 << 18, 8
    x = wl.wide_256k(seed=0, batch=B, n=n)
    y = oz.Plan(n, B).forward(_gpu(torch, x)).cpu().numpy()
    want = oracle_ffts(list(x), 3, 3, wide_plan)
    for b in range(B):
        assert max_ulp(y[b], want[b]) == 0, b


def test_wide_256k_single_K6_L1(torch_mod):
    """Single transform at n = 2^18 with K = 6, L = 1 (uncapped for this
    distribution's dynamic range)."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    n = 1 << 18
    x = wl.wide_256k(seed=0, batch=1, n=n)
    plan = oz.Plan(n, 1, K=6, L=1)
    y = plan.forward(_gpu(torch, x)).cpu().numpy()
    want = bl.fft(x[0], 6, 1, bl.KernelPlan(n, 6, 1))
    assert max_ulp(y[0], want) == 0
    info = plan.transform_info(0)
    assert info["alpha"] == 21


def test_mixed_256_one_launch(torch_mod):
    """256 transforms of lengths log-uniform in [2^10, 2^16] (a third prime)
    in one batched execution: every eighth transform and one per convolution
    length class against the oracle (over a pool of processes), a subset
    equal to the same transform computed by a plan of its own, and the graph
    replay stable."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    ns, xs = wl.mixed_256(0)
    flat = _gpu(torch, np.concatenate(xs))
    plan = oz.Plan(lengths=ns)
    y1 = plan.forward(flat).cpu().numpy()
    y2 = plan.forward(flat).cpu().numpy()
    assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64))
    offs = np.concatenate([[0], np.cumsum(ns)])
    # every eighth transform and one per convolution-length class
    by_N = {}
    for i, n in enumerate(ns):
        by_N.setdefault(bl.conv_length(n), i)
    sample = sorted(set(range(0, 256, 8)) | set(by_N.values()))
    wants = oracle_ffts_own_plans([xs[i] for i in sample], 3, 3)
    for i, want in zip(sample, wants):
        assert max_ulp(y1[offs[i]:offs[i + 1]], want) == 0, (i, ns[i])
    for i in range(0, 256, 37):
        single = oz.Plan(ns[i], 1).forward(_gpu(torch, xs[i][None, :])).cpu().numpy()[0]
        assert np.array_equal(single.view(np.uint64), y1[offs[i]:offs[i + 1]].view(np.uint64)), i


def test_autograd_backward_is_oracle_adjoint(torch_mod):
    """loss = sum(w |X|^2) on 32 x 2^16: the gradient equals the oracle's
    adjoint DFT of 2 w X (sampled rows, bit for bit) and central finite
    differences (h = 1e-6) along the gradient and random directions."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    x, w = wl.grad_64k(0)
    n = x.shape[1]
    xd = _gpu(torch, x).requires_grad_(True)
    wd = torch.from_numpy(w).cuda()
    X = oz.OzakiDFT.apply(xd)
    seen = []
    X.register_hook(lambda gX: seen.append(gX.detach().clone()))
    loss = (wd * X.abs() ** 2).sum()
    loss.backward()
    g = xd.grad.detach().cpu().numpy()
    gX = seen[0].cpu().numpy()
    Xh = X.detach().cpu().numpy()
    # the incoming gradient is 2 w X (torch's convention for real losses)
    assert np.allclose(gX, 2.0 * w * Xh, rtol=1e-14, atol=0)
    kp = bl.KernelPlan(n, 3, 3)
    for b in (0, 31):
        want = bl.adjoint(gX[b], plan=kp)          # backward = DFT^H of the incoming gradient
        assert max_ulp(g[b], want) == 0
    # finite differences of the loss along directions v: (L(x+hv)-L(x-hv))/(2h) = Re<grad, v>
    def L(xx):
        with torch.no_grad():
            Y = oz.fft(xx)
            return float((wd * Y.abs() ** 2).sum())
    h = 1e-6
    gn = np.linalg.norm(g)
    rng = np.random.default_rng(4)
    dirs = [g / gn]
    for _ in range(2):
        v = rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)
        dirs.append(v / np.linalg.norm(v))
    for k, v in enumerate(dirs):
        vd = _gpu(torch, v)
        fd = (L(xd.detach() + h * vd) - L(xd.detach() - h * vd)) / (2 * h)
        an = float(np.real(np.vdot(g, v)))   # torch grads are conjugate Wirtinger: dL = Re<g, dx>
        tol = 1e-6 if k == 0 else 1e-3
        assert abs(fd - an) <= tol * max(abs(an), gn), (k, fd, an)


def test_autograd_gradcheck_small(torch_mod):
    import paper_2603_29129_amd as oz
    torch = torch_mod
    x = _gpu(torch, wl.uniform(12, batch=2, seed=1)).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda t: oz.OzakiDFT.apply(t), (x,), eps=1e-6, atol=1e-7, rtol=1e-5)


@pytest.mark.parametrize("n", [1 << 24, (1 << 23) - 1])
def test_maximum_length(torch_mod, n):
    """The largest convolution length both primes support, N = 2^24 (cyclic
    n = 2^24; padded n = 2^23 - 1, the largest length that is not a power
    of two; 2^23 + 1 is rejected at plan time): the oracle cannot run this size in
    seconds, so the checks are properties that hold at any size: accuracy
    against numpy's complex128 FFT, the inverse round trip, and bit-identity
    of a transform computed in a batch of two with the same transform alone."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    x = wl.uniform(n, batch=1, seed=3)
    xd = _gpu(torch, x)
    plan = oz.Plan(n, 1)
    assert plan.transform_info(0)["N"] == 1 << 24
    y = plan.forward(xd)
    ref_y = np.fft.fft(x[0])
    yh = y.cpu().numpy()[0]
    assert np.linalg.norm(yh - ref_y) / np.linalg.norm(ref_y) < 1e-14
    z = plan.inverse(y).cpu().numpy()[0]
    assert np.max(np.abs(z - x[0])) < 1e-13
    del plan
    torch.cuda.empty_cache()
    if n == 1 << 24:
        x2 = np.concatenate([wl.uniform(n, batch=1, seed=4), x])
        p2 = oz.Plan(n, 2)
        y2 = p2.forward(_gpu(torch, x2)).cpu().numpy()
        assert np.array_equal(y2[1].view(np.uint64), yh.view(np.uint64))


def test_prime_near_2_18(torch_mod):
    """n = 262139 (prime, convolution length 2^19, N1 = 1024: the pipelined
    row pass, then the column pass and the recombination as separate
    kernels): both transforms of a batch 0 ulp from the oracle on wide-range
    inputs, and equal to the plain form (one launch per NTT)."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    n = 262139
    x = wl.wide_256k(seed=2, batch=2, n=n)
    xd = _gpu(torch, x)
    plan = oz.Plan(n, 2)
    assert plan.transform_info(0)["N"] == 1 << 19 and plan.transform_info(0)["ntt_log2N1"] == 10
    y = plan.forward(xd).cpu().numpy()
    yp = oz.Plan(n, 2, mode="plain").forward(xd).cpu().numpy()
    assert np.array_equal(y.view(np.uint64), yp.view(np.uint64))
    kp = bl.KernelPlan(n, 3, 3)
    for b in range(2):
        assert max_ulp(y[b], bl.fft(x[b], 3, 3, kp)) == 0, b


def test_padded_2_18_and_wide_span(torch_mod):
    """The padded embedding of n = 2^18 (N = 2^19) gives the cyclic
    embedding's bits; a transform whose group exponents span about 300 bits
    (wide accumulator in the recombination) is 0 ulp from the oracle in
    both."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    n = 1 << 18
    x = wl.uniform(n, batch=2, seed=31)
    x[1, ::2] *= 2.0 ** -300
    xd = _gpu(torch, x)
    yc = oz.Plan(n, 2, K=8).forward(xd).cpu().numpy()
    pad = oz.Plan(n, 2, K=8, cyclic=False)
    assert pad.transform_info(0)["N"] == 1 << 19
    yp = pad.forward(xd).cpu().numpy()
    assert np.array_equal(yc.view(np.uint64), yp.view(np.uint64))
    want = bl.fft(x[1], 8, 3, bl.KernelPlan(n, 8, 3))
    assert max_ulp(yp[1], want) == 0


def test_length_2_19_two_pass_n1_1024_n2_1024(torch_mod):
    """n = 2^19 - 1 (N = 2^20: N1 = N2 = 1024, the general row pass and the
    unfused column pass): batched equals plain, and the transform is 0 ulp
    from the oracle."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    n = (1 << 19) - 1
    x = wl.uniform(n, batch=1, seed=32)
    xd = _gpu(torch, x)
    plan = oz.Plan(n, 1)
    assert plan.transform_info(0)["N"] == 1 << 20
    y = plan.forward(xd).cpu().numpy()
    yp = oz.Plan(n, 1, mode="plain").forward(xd).cpu().numpy()
    assert np.array_equal(y.view(np.uint64), yp.view(np.uint64))
    assert max_ulp(y[0], bl.fft(x[0], 3, 3, bl.KernelPlan(n, 3, 3))) == 0
