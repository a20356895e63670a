"""Boundary behaviour on the GPU: in-place execution, user streams, the
graph cache across buffers and directions."""

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("mode", ["batched", "plain"])
@pytest.mark.parametrize("n", [1000, 1 << 14])
def test_in_place_equals_out_of_place(torch_mod, mode, n):
    """in == out is allowed: each input is consumed by the premultiply before
    any output is written."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    x = torch.from_numpy(wl.uniform(n, batch=3, seed=8)).cuda()
    plan = oz.Plan(n, 3, mode=mode)
    ref = plan.forward(x.clone())
    buf = x.clone()
    plan.forward(buf, out=buf)
    assert torch.equal(buf.view(torch.float64), ref.view(torch.float64))
    back = buf.clone()
    plan.inverse(back, out=back)
    assert torch.equal(back.view(torch.float64), plan.inverse(ref).view(torch.float64))


def test_user_stream_and_graph_cache(torch_mod):
    """Executions on a user stream and into several output buffers (more than
    the plan caches graphs for) give the same bits as the default stream."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    n = 1 << 14
    x = torch.from_numpy(wl.uniform(n, batch=2, seed=9)).cuda()
    plan = oz.Plan(n, 2)
    ref = plan.forward(x)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    outs = []
    with torch.cuda.stream(s):
        for _ in range(6):
            outs.append(plan.forward(x))
        inv = plan.inverse(outs[-1])
    s.synchronize()
    for o in outs:
        assert torch.equal(o.view(torch.float64), ref.view(torch.float64))
    assert float((inv - x).abs().max()) < 1e-14
    again = plan.forward(x)
    assert torch.equal(again.view(torch.float64), ref.view(torch.float64))


@pytest.mark.parametrize("primes", [2, 3])
def test_graph_replays_with_new_data(torch_mod, primes):
    """The batched plan captures one graph per (in, out, direction) and
    replays it: four replays into the same buffers with new input data each
    time, eager torch work and synchronisations in between, every replay
    equal bit for bit to the eager plain form (two moduli) or to a fresh
    plan's first execution (three moduli)."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    n, B = 4096 + 7, 3
    plan = oz.Plan(n, B, primes=primes)
    xin = torch.empty((B, n), dtype=torch.complex128, device="cuda")
    yout = torch.empty_like(xin)
    noise = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
    for r in range(4):
        x = torch.from_numpy(wl.paper_phi(n, float(r), seed=40 + r, batch=B)).cuda()
        xin.copy_(x)
        plan.forward(xin, out=yout)
        noise.mul_(1.0001).add_(0.5)                   # eager work between the replays
        torch.cuda.synchronize()
        if primes == 2:
            want = oz.Plan(n, B, mode="plain").forward(x)
        else:
            want = oz.Plan(n, B, primes=3).forward(x)
        assert torch.equal(yout.view(torch.float64), want.view(torch.float64)), r
