"""The allocation-free entry point fft_ozaki_execute_static against the
planned entry point (fft_ozaki_plan + fft_ozaki_execute) on the same seeded
inputs: outputs must agree bit for bit (the tolerance of the parity tests is
2 ulp; both paths run the same kernels, so 0 is expected and required)."""

import ctypes

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _static(oz, torch, x, direction):
    """One call through the C ABI; the output buffer comes from torch."""
    out = torch.empty_like(x)
    n = x.shape[-1]
    batch = x.numel() // n
    stream = torch.cuda.current_stream(x.device).cuda_stream
    rc = oz.lib().fft_ozaki_execute_static(n, batch, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                           direction, ctypes.c_void_p(stream))
    oz._check(rc)
    return out


def test_static_matches_planned_calls_in_a_row():
    """Calls in a row share the device's static workspace: a two-pass length,
    the same size again (tables kept), then a smaller input (tables rebuilt),
    then the first size once more."""
    import torch

    import paper_2603_29129_amd as oz
    assert torch.cuda.is_available()
    calls = [(1 << 14, 4, oz.FORWARD, 11), (1 << 14, 4, oz.ADJOINT, 12), (1000, 3, oz.INVERSE, 13),
             (1 << 14, 2, oz.FORWARD, 14)]
    for n, batch, direction, seed in calls:
        print(f"static call n={n} batch={batch} direction={direction} seed={seed}", flush=True)
        x = torch.from_numpy(wl.uniform(n, batch=batch, seed=seed)).cuda()
        got = _static(oz, torch, x, direction)
        torch.cuda.synchronize()
        want = oz.Plan(n, batch).execute(x, direction)
        torch.cuda.synchronize()
        g = got.cpu().numpy().view(np.uint64)
        w = want.cpu().numpy().view(np.uint64)
        assert np.array_equal(g, w), f"n={n} batch={batch}: static output differs from the planned output"


def test_static_python_wrapper_and_rejections():
    """The package wrapper gives the same bits; a size beyond the static
    workspace is rejected with an error naming it."""
    import torch

    import paper_2603_29129_amd as oz
    x = torch.from_numpy(wl.uniform(1 << 10, batch=5, seed=21)).cuda()
    got = oz.execute_static(x)
    want = oz.Plan(1 << 10, 5).forward(x)
    assert torch.equal(got.view(torch.float64), want.view(torch.float64))
    big = torch.zeros(1, 1 << 18, dtype=torch.complex128, device="cuda")
    with pytest.raises(oz.FftOzakiError, match="static workspace"):
        oz.execute_static(big)
