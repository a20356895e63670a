"""GPU parity of the library's 32-bit NTT against the oracle (bit-exact)."""

import numpy as np
import pytest

from oracle import ntt as nt
from tests.gpu_helpers import ntt_domain_index

pytestmark = pytest.mark.gpu

LOGNS = [0, 1, 2, 3, 4, 5, 7, 8, 11, 12, 13, 14, 15, 16, 17, 19, 20]


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("logN", LOGNS)
@pytest.mark.parametrize("prime", [0, 1, 2])
def test_forward_matches_oracle(torch_mod, logN, prime):
    import paper_2603_29129_amd as oz
    torch = torch_mod
    p = nt.PRIMES3[prime]
    N = 1 << logN
    count = 3 if logN <= 17 else 2
    rng = np.random.default_rng(1000 + 17 * logN + prime)
    x = rng.integers(0, p, (count, N), dtype=np.int64).astype(np.uint32)
    x[0, :] = np.arange(N) % p if N > 1 else 5          # a structured row too
    d = torch.from_numpy(x.view(np.int32)).cuda()
    oz.ntt(d, prime, inverse=False)
    got = d.cpu().numpy().view(np.uint32)
    perm = ntt_domain_index(logN, oz.ntt_layout(logN))
    for r in range(count):
        want = nt.ntt(x[r].astype(np.uint64), p)
        assert np.array_equal(got[r].astype(np.uint64), want[perm]), f"row {r}"
    # inverse of the forward output recovers the input
    oz.ntt(d, prime, inverse=True)
    back = d.cpu().numpy().view(np.uint32)
    assert np.array_equal(back, x)


@pytest.mark.parametrize("logN", [3, 12, 13, 16])
@pytest.mark.parametrize("prime", [0, 1, 2])
def test_inverse_matches_oracle(torch_mod, logN, prime):
    import paper_2603_29129_amd as oz
    torch = torch_mod
    p = nt.PRIMES3[prime]
    N = 1 << logN
    rng = np.random.default_rng(77 + logN + prime)
    Xnat = rng.integers(0, p, N, dtype=np.int64).astype(np.uint64)
    perm = ntt_domain_index(logN, oz.ntt_layout(logN))
    d = torch.from_numpy(Xnat[perm].astype(np.uint32).view(np.int32)[None, :].copy()).cuda()
    oz.ntt(d, prime, inverse=True)
    got = d.cpu().numpy().view(np.uint32)[0].astype(np.uint64)
    assert np.array_equal(got, nt.ntt(Xnat, p, inverse=True))
