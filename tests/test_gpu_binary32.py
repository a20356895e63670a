"""GPU parity of the binary32 target precision (complex64 in and out).

The oracle widens the complex64 input exactly, runs the binary64 method with
the cap K (2 by default for this target) and rounds each output component
once to binary32.  The library's binary64 results equal the oracle's (0 ulp
observed, 2 ulp allowed), so the rounded results are compared with a
tolerance of 1 ulp of binary32 per component (0 expected)."""

import numpy as np
import pytest

import workloads as wl
from oracle import bluestein as bl
from tests.accum_schedule import acc_limit, component_schedule

pytestmark = pytest.mark.gpu
ULP32_TOL = 1


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


def _ordered32(a):
    i = np.ascontiguousarray(a, dtype=np.float32).view(np.int32).astype(np.int64)
    mag = i & 0x7FFFFFFF
    return np.where(i < 0, -mag, mag)


def max_ulp32(a, b):
    a = np.asarray(a, dtype=np.complex64)
    b = np.asarray(b, dtype=np.complex64)
    worst = 0
    for x, y in ((a.real, b.real), (a.imag, b.imag)):
        nx, ny = np.isnan(x), np.isnan(y)
        assert np.array_equal(nx, ny), "NaN positions differ"
        m = ~nx
        if np.any(m):
            worst = max(worst, int(np.max(np.abs(_ordered32(x[m]) - _ordered32(y[m])))))
    return worst


def _kp(n, K=2, L=3):
    return bl.KernelPlan(n, K, L, cyclic=bl.is_pow2(n))


@pytest.mark.parametrize("mode", ["batched", "plain"])
@pytest.mark.parametrize("n", [1, 3, 64, 1000, 1024, 4097, 16384])
def test_binary32_forward(torch_mod, n, mode):
    import paper_2603_29129_amd as oz
    torch = torch_mod
    x = wl.paper_phi(n, 1.0, seed=n, batch=2).astype(np.complex64)
    plan = oz.Plan(n, 2, precision="fp32", mode=mode)
    assert plan.info()["precision"] == oz.PREC_FP32 and plan.K == 2
    y = plan.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    assert y.dtype == np.complex64
    kp = _kp(n)
    for b in range(2):
        assert max_ulp32(y[b], bl.fft_binary32(x[b], 2, 3, kp)) <= ULP32_TOL, b
        # the schedule of K = 2: 2 (kx0 + kx1) forward NTTs, 2 per group
        info = plan.transform_info(b)
        tr = bl.forward_trace(x[b].astype(np.complex128), 2, 3, kp)
        EX = [[E for _, E in tr["slices"][v]] for v in range(2)]
        sched = component_schedule(EX, [kp.exps(0), kp.exps(1)], 3, "complex", acc_limit(n, tr["alpha"]),
                                    alpha=tr["alpha"])
        assert info["ngroups"] == [len(g) for g in sched]
        assert info["forward_runtime"] == 2 * sum(info["kx"]) and max(info["kx"]) <= 2


@pytest.mark.parametrize("n", [1000, 4096])
def test_binary32_inverse_adjoint(torch_mod, n):
    import paper_2603_29129_amd as oz
    torch = torch_mod
    x = wl.paper_phi(n, 0.0, seed=5, batch=1).astype(np.complex64)
    plan = oz.Plan(n, 1, precision="fp32")
    xd = torch.from_numpy(x).cuda()
    kp = _kp(n)
    assert max_ulp32(plan.inverse(xd).cpu().numpy()[0], bl.ifft_binary32(x[0], 2, 3, kp)) <= ULP32_TOL
    assert max_ulp32(plan.adjoint(xd).cpu().numpy()[0], bl.adjoint_binary32(x[0], 2, 3, kp)) <= ULP32_TOL


def test_binary32_k3_and_in_place(torch_mod):
    import paper_2603_29129_amd as oz
    torch = torch_mod
    n = 2048
    x = wl.paper_phi(n, 4.0, seed=9, batch=2).astype(np.complex64)
    plan = oz.Plan(n, 2, K=3, precision="fp32")
    xd = torch.from_numpy(x).cuda()
    y = plan.forward(xd).cpu().numpy()
    kp = _kp(n, 3)
    for b in range(2):
        assert max_ulp32(y[b], bl.fft_binary32(x[b], 3, 3, kp)) <= ULP32_TOL
    plan.forward(xd, out=xd)                         # in place
    assert np.array_equal(xd.cpu().numpy().view(np.uint32), y.view(np.uint32))


def test_binary32_special_inputs_and_types(torch_mod):
    import paper_2603_29129_amd as oz
    torch = torch_mod
    n = 256
    x = np.zeros((3, n), dtype=np.complex64)
    x[1, 7] = np.nan
    x[2] = wl.paper_phi(n, 1.0, seed=2, batch=1)[0].astype(np.complex64)
    plan = oz.Plan(n, 3, precision="fp32")
    y = plan.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.all(y[0] == 0)
    assert np.all(np.isnan(y[1].real)) and np.all(np.isnan(y[1].imag))
    assert max_ulp32(y[2], bl.fft_binary32(x[2], 2, 3, _kp(n))) <= ULP32_TOL
    with pytest.raises(TypeError):
        plan.forward(torch.from_numpy(x.astype(np.complex128)).cuda())


def test_binary32_headline_length(torch_mod):
    """n = 2^18 (the headline length), one transform, full comparison; and
    the error against the long-double DFT is the binary32 rounding alone."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    n = 1 << 18
    x = wl.wide_256k(seed=0, batch=1, n=n).astype(np.complex64)
    plan = oz.Plan(n, 1, precision="fp32")
    y = plan.forward(torch.from_numpy(x).cuda()).cpu().numpy()[0]
    assert max_ulp32(y, bl.fft_binary32(x[0], 2, 3, _kp(n))) <= ULP32_TOL
    ref = np.fft.fft(x[0].astype(np.clongdouble))

    def rel(v):
        v = np.asarray(v).astype(np.clongdouble)
        return float(np.sqrt(np.sum(np.abs(v - ref) ** 2)) / np.sqrt(np.sum(np.abs(ref) ** 2)))

    rounding = rel(ref.astype(np.complex128).astype(np.complex64))
    assert rel(y) <= 1.05 * rounding
