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
    """in == out is allowed: each input is consumed by the split (the
    premultiply and the extraction passes, which recompute x' from it)
    before any output is written.  The debug copy of x' rebuilds it from the
    input and so is refused after an in-place execution."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    x = torch.from_numpy(wl.uniform(n, batch=3, seed=8)).cuda()
    plan = oz.Plan(n, 3, mode=mode)
    ref = plan.forward(x.clone())
    buf = x.clone()
    plan.forward(buf, out=buf)
    assert torch.equal(buf.view(torch.float64), ref.view(torch.float64))
    with pytest.raises(oz.FftOzakiError, match="in-place"):
        plan.debug_dump(1, 0)
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


def test_autotuned_plans_bit_identical(torch_mod, tmp_path):
    """Plans with autotuned tile shapes give the default plan's bits (and the
    oracle's on a sampled transform); a second plan reads the tune cache and
    takes the same shapes."""
    import paper_2603_29129_amd as oz
    from oracle import bluestein as bl
    from tests.gpu_helpers import max_ulp
    torch = torch_mod
    cache = str(tmp_path / "tune.txt")
    ns, xs = wl.mixed_256(seed=0, count=24)          # lengths over the classes N = 2^12 .. 2^17
    cases = [[1 << 14] * 2, [1 << 18] * 2, ns]
    for lengths in cases:
        if lengths is ns:
            x = np.concatenate(xs)
        else:
            x = wl.uniform(lengths[0], batch=len(lengths), seed=3).reshape(-1)
        xd = torch.from_numpy(x).cuda()
        ref = oz.Plan(lengths=lengths).forward(xd).cpu().numpy()
        p1 = oz.Plan(lengths=lengths, autotune=True, tune_cache=cache)
        y1 = p1.forward(xd).cpu().numpy()
        assert np.array_equal(y1.view(np.uint64), ref.view(np.uint64)), lengths[:2]
        shapes1 = [(p1.transform_info(i)["tile_cols_log2"], p1.transform_info(i)["tile_rows_log2"])
                   for i in range(len(lengths))]
        p2 = oz.Plan(lengths=lengths, autotune=True, tune_cache=cache)
        y2 = p2.forward(xd).cpu().numpy()
        shapes2 = [(p2.transform_info(i)["tile_cols_log2"], p2.transform_info(i)["tile_rows_log2"])
                   for i in range(len(lengths))]
        assert shapes1 == shapes2
        assert np.array_equal(y2.view(np.uint64), ref.view(np.uint64))
        if lengths[0] == 1 << 14:
            want = bl.fft(x[: 1 << 14], 3, 3, bl.KernelPlan(1 << 14, 3, 3, cyclic=True))
            assert max_ulp(y1[: 1 << 14], want) == 0
    with open(cache) as f:
        keys = [line.split()[0] for line in f if line.strip()]
    # key: architecture, log2 N, scratch vectors (4 K per transform, rounded up to a power of two)
    assert any(k.split(":")[-2:] == ["18", "32"] for k in keys)
    assert any(k.split(":")[-2:] == ["14", "32"] for k in keys)


def test_injected_allocation_failure(torch_mod, monkeypatch):
    """A device allocation that fails during planning returns
    FFT_OZAKI_ERR_NOMEM with a message, releases what was allocated, and
    leaves the library usable."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    x = torch.from_numpy(wl.uniform(1 << 14, batch=2, seed=4)).cuda()
    want = oz.Plan(1 << 14, 2).forward(x).cpu().numpy()
    free0 = torch.cuda.mem_get_info()[0]
    for k in (1, 2, 5, 9, 13):
        monkeypatch.setenv("FFT_OZAKI_TEST_FAIL_ALLOC", str(k))
        with pytest.raises(oz.FftOzakiError, match=r"out of memory \(-2\).*injected"):
            oz.Plan(1 << 14, 2)
    monkeypatch.delenv("FFT_OZAKI_TEST_FAIL_ALLOC")
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] >= free0 - (64 << 20)      # the failed plans freed their workspace
    got = oz.Plan(1 << 14, 2).forward(x).cpu().numpy()
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


def test_log_lines(tmp_path):
    """FFT_OZAKI_LOG=1 reports the plan and the graph capture on stderr."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import torch, paper_2603_29129_amd as oz\n"
            "p = oz.Plan(1 << 14, 2)\n"
            "for i in range(8):\n"
            "    x = torch.full((2, 1 << 14), float(i), dtype=torch.complex128, device='cuda')\n"
            "    p.forward(x); p.inverse(x)\n"
            "torch.cuda.synchronize(); print('done', flush=True)\n")
    env = dict(os.environ, FFT_OZAKI_LOG="1", PYTHONPATH=root)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=100, cwd=root)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "[fft_ozaki] plan: 2 transforms" in r.stderr
    assert "class N=2^14" in r.stderr
    # eight (in, out) pairs per direction, one capture per direction
    assert r.stderr.count("captured the batched schedule for direction 0") == 1
    assert r.stderr.count("captured the batched schedule for direction 1") == 1


def test_rotating_buffers_reuse_the_graph(torch_mod):
    """Executions over eight (in, out) pairs in turn, both directions, through
    one batched plan (one captured graph per direction, its pointers
    rebound per call) give the plain form's bits every time."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    n, B = 1 << 14, 2
    plan = oz.Plan(n, B)
    ref = oz.Plan(n, B, mode="plain")
    xs = [torch.from_numpy(wl.uniform(n, batch=B, seed=40 + i)).cuda() for i in range(8)]
    outs = [torch.empty_like(xs[0]) for _ in range(8)]
    for rnd in range(2):
        for i in range(8):
            d = (i + rnd) % 2
            plan.execute(xs[i], d, out=outs[i])
            want = ref.execute(xs[i], d)
            assert torch.equal(outs[i].view(torch.float64), want.view(torch.float64)), (rnd, i)


@pytest.mark.parametrize("primes", [2, 3])
def test_stage_timing_in_the_graph(torch_mod, primes):
    """Stage timing (the batched launches on the stream with HIP events at
    the stage boundaries): the outputs keep the graph replay's bits, every
    stage of every length class gets a nonnegative device time, and the times
    add up to no more than the execution's own device time; switched off,
    the plan replays its graph again.  Three length classes: a fused
    two-pass length (N = 2^14), a single-block length (N = 2^11 for
    n = 1000) and an unfused two-pass length (N = 2^20: N1 = 1024); two and
    three moduli."""
    import paper_2603_29129_amd as oz
    torch = torch_mod
    lengths = [1 << 14, 1000, (1 << 19) - 1, 1 << 14]
    x = torch.from_numpy(np.concatenate([wl.uniform(n, batch=1, seed=60 + i).ravel()
                                         for i, n in enumerate(lengths)])).cuda()
    plan = oz.Plan(lengths=lengths, primes=primes)
    ref = plan.forward(x)
    with pytest.raises(oz.FftOzakiError, match="no stage times"):
        plan.stage_times()
    plan.stage_timing(True)
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for rep in range(3):
        a.record(s)
        y = plan.forward(x)
        b.record(s)
        torch.cuda.synchronize()
        assert torch.equal(y.view(torch.float64), ref.view(torch.float64)), rep
        t = plan.stage_times()
        assert len(t["classes"]) == 3
        vals = [t["split"]] + [v for c in t["classes"] for v in c.values()]
        assert all(v >= 0 for v in vals), t
        assert t["split"] > 0 and all(c["forward"] > 0 and c["rows"] > 0 for c in t["classes"]), t
        assert sum(vals) <= a.elapsed_time(b) * 1.05 + 0.01, (t, a.elapsed_time(b))
    # the single-block class has no separate column pass
    assert t["classes"][1]["cols"] < 0.01, t
    plan.stage_timing(False)
    y = plan.forward(x)
    assert torch.equal(y.view(torch.float64), ref.view(torch.float64))
    with pytest.raises(oz.FftOzakiError, match="no stage times"):
        plan.stage_times()
    with pytest.raises(oz.FftOzakiError):
        oz.Plan(1000, 1, mode="plain").stage_timing(True)
