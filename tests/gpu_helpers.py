"""Helpers shared by the GPU parity tests (no method arithmetic here)."""

import numpy as np


def ordered(a):
    """Map binary64 values to integers whose differences count ulps
    (+0 and -0 both map to 0)."""
    i = np.ascontiguousarray(a, dtype=np.float64).view(np.int64)
    mag = i & np.int64(0x7FFFFFFFFFFFFFFF)
    return np.where(i < 0, -mag, mag)


def max_ulp(a, b):
    """Largest ulp distance between the real and imaginary components of two
    complex arrays; NaNs must coincide."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    worst = 0
    for x, y in ((a.real, b.real), (a.imag, b.imag)):
        nx, ny = np.isnan(x), np.isnan(y)
        assert np.array_equal(nx, ny), "NaN positions differ"
        m = ~nx
        if np.any(m):
            d = np.abs(ordered(x[m]).astype(object) - ordered(y[m]).astype(object))
            worst = max(worst, int(max(d)))
    return worst


def bitrev(v, bits):
    out = np.zeros_like(v)
    for b in range(bits):
        out |= ((v >> b) & 1) << (bits - 1 - b)
    return out


def ntt_domain_index(logN, log2N1):
    """perm such that gpu[pos] == natural[perm[pos]] for the library's
    NTT-domain order (position i1*N2 + i2 holds X[br(i1) + N1*br(i2)])."""
    N = 1 << logN
    m1 = log2N1
    m2 = logN - m1
    pos = np.arange(N, dtype=np.int64)
    i1 = pos >> m2
    i2 = pos & ((1 << m2) - 1)
    return bitrev(i1, m1) + (bitrev(i2, m2) << m1)


# The oracle over a pool of processes (one transform per task), for parity
# checks at sizes where one process would take minutes.  Spawned workers
# (the parent holds a GPU context); the kernel plan is sent once per worker.
_POOL_PLAN = None


def _pool_init(plan):
    global _POOL_PLAN
    _POOL_PLAN = plan


def _pool_fft(args):
    from oracle import bluestein as bl
    x, K, L = args
    return bl.fft(x, K, L, _POOL_PLAN)


def oracle_ffts(xs, K, L, plan, procs=8):
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(min(procs, len(xs)), initializer=_pool_init, initargs=(plan,)) as pool:
        return pool.map_async(_pool_fft, [(x, K, L) for x in xs], chunksize=1).get(timeout=600)


def _own_plan_fft(args):
    from oracle import bluestein as bl
    x, K, L = args
    n = len(x)
    return bl.fft(x, K, L, bl.KernelPlan(n, K, L, cyclic=bl.is_pow2(n)))


def oracle_ffts_own_plans(xs, K, L, procs=16):
    """The oracle for vectors of different lengths, each worker building the
    kernel plan of the length it is given."""
    import multiprocessing as mp
    import os
    procs = max(1, min(procs, len(xs), os.cpu_count() or 1))
    with mp.get_context("spawn").Pool(procs) as pool:
        return pool.map_async(_own_plan_fft, [(x, K, L) for x in xs], chunksize=1).get(timeout=900)
