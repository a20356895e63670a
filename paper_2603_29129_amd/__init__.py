"""Python binding of libfft_ozaki: FP64-accurate DFTs on MI355X computed by
Bluestein's algorithm with Ozaki integer slices and two-prime 32-bit NTT
convolution (Kawakami & Takahashi, "Computing FFTs at Target Precision Using
Lower-Precision FFTs").

Every step of the transform runs in the HIP library; this module only
marshals arguments (device pointers from torch tensors, the current HIP
stream) through ctypes.  There is no CPU fallback: if the library is not
built, using it raises an error.

    import torch, paper_2603_29129_amd as oz
    x = torch.randn(8, 1 << 18, dtype=torch.complex128, device="cuda")
    y = oz.fft(x)                 # forward DFT along the last axis
    z = oz.ifft(y)                # inverse
    y = oz.OzakiDFT.apply(x)      # differentiable (backward = adjoint DFT)
"""

from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfft_ozaki.so")

FORWARD, INVERSE, ADJOINT = 0, 1, 2
MODE_PLAIN, MODE_BATCHED = 0, 1
EMBED_PADDED, EMBED_AUTO = 0, 1
ACCUM_PER_CONV, ACCUM_COMPLEX = 0, 1
_ACCUMS = {"per_conv": ACCUM_PER_CONV, "complex": ACCUM_COMPLEX}
PREC_FP64, PREC_FP32 = 0, 1
_PRECS = {"fp64": PREC_FP64, "fp32": PREC_FP32}
_MODES = {"plain": MODE_PLAIN, "batched": MODE_BATCHED}


class FftOzakiError(RuntimeError):
    pass


class _Options(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int), ("L", ctypes.c_int), ("mode", ctypes.c_int),
                ("autotune", ctypes.c_int), ("tune_cache", ctypes.c_char_p), ("embedding", ctypes.c_int),
                ("accumulation", ctypes.c_int), ("precision", ctypes.c_int), ("primes", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64), ("total_length", ctypes.c_int64), ("K", ctypes.c_int),
                ("L", ctypes.c_int), ("mode", ctypes.c_int), ("num_length_classes", ctypes.c_int),
                ("workspace_bytes", ctypes.c_int64), ("embedding", ctypes.c_int), ("accumulation", ctypes.c_int),
                ("precision", ctypes.c_int), ("primes", ctypes.c_int)]


class _TInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("N", ctypes.c_int64), ("alpha", ctypes.c_int), ("status", ctypes.c_int),
                ("kx", ctypes.c_int * 2), ("Ex", (ctypes.c_int * 8) * 2), ("kw", ctypes.c_int * 2),
                ("Ew", (ctypes.c_int * 8) * 2), ("ngroups", ctypes.c_int * 2), ("acc_limit", ctypes.c_int),
                ("xsh", ctypes.c_int * 2),
                ("forward_runtime", ctypes.c_int),
                ("forward_offline", ctypes.c_int), ("inverse", ctypes.c_int), ("ntt_log2N1", ctypes.c_int),
                ("tile_cols_log2", ctypes.c_int), ("tile_rows_log2", ctypes.c_int)]


_lib = None
_lib_lock = threading.Lock()


def lib():
    """The loaded HIP library (raises FftOzakiError if it is not built)."""
    global _lib
    if _lib is None:
        with _lib_lock:
            if _lib is None:
                if not os.path.exists(LIB_PATH):
                    raise FftOzakiError(f"{LIB_PATH} not found: build it with "
                                        "`python -m paper_2603_29129_amd.build_lib`")
                L = ctypes.CDLL(LIB_PATH)
                vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
                sig = {
                    "fft_ozaki_default_options": ([ctypes.POINTER(_Options)], ci),
                    "fft_ozaki_plan": ([ctypes.POINTER(vp), i64, i64], ci),
                    "fft_ozaki_plan_ex": ([ctypes.POINTER(vp), ctypes.POINTER(i64), i64, ctypes.POINTER(_Options)], ci),
                    "fft_ozaki_execute": ([vp, vp, vp, ci, vp], ci),
                    "fft_ozaki_forward": ([vp, vp, vp, vp], ci),
                    "fft_ozaki_inverse": ([vp, vp, vp, vp], ci),
                    "fft_ozaki_query": ([vp, ctypes.POINTER(_Info)], ci),
                    "fft_ozaki_query_transform": ([vp, i64, ctypes.POINTER(_TInfo)], ci),
                    "fft_ozaki_debug_dump": ([vp, ci, i64, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)], ci),
                    "fft_ozaki_destroy": ([vp], ci),
                    "fft_ozaki_profile_stage": ([vp, ci, ci, vp], ci),
                    "fft_ozaki_stage_timing": ([vp, ci], ci),
                    "fft_ozaki_stage_times": ([vp, ctypes.POINTER(ctypes.c_float), ci, ctypes.POINTER(ci)], ci),
                    "fft_ozaki_error_string": ([ci], ctypes.c_char_p),
                    "fft_ozaki_last_error_message": ([], ctypes.c_char_p),
                    "fft_ozaki_ntt": ([ci, ci, i64, vp, ci, vp], ci),
                    "fft_ozaki_ntt_layout": ([ci, ctypes.POINTER(ci)], ci),
                    "fft_ozaki_execute_static": ([i64, i64, vp, vp, ci, vp], ci),
                }
                for name, (args, res) in sig.items():
                    f = getattr(L, name)
                    f.argtypes = args
                    f.restype = res
                _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        L = lib()
        raise FftOzakiError(f"{L.fft_ozaki_error_string(rc).decode()} ({rc}): "
                            f"{L.fft_ozaki_last_error_message().decode()}")


def _stream_handle(torch, device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Plan:
    """A plan for `lengths` transforms (or `batch` transforms of length `n`).

    cyclic: for power-of-two lengths use the cyclic embedding N = n instead of
    padding to N = 2^ceil(log2(2n-1)) (Sec. 3.2); the outputs are the same
    bit for bit, the NTTs half as long.

    accumulation: "complex" (default) walks the two real convolutions of each
    output component together so that products of equal scale share an
    inverse NTT (ReRe - ImIm, ImRe + ReIm); "per_conv" is Alg. 8 applied to
    each real convolution on its own.  Outputs are bit-identical.

    precision: "fp64" (complex128 in and out) or "fp32" (complex64 in and
    out: inputs widened exactly, the transform computed as for fp64 with this
    plan's K, each output component rounded once to binary32).  K defaults to
    3 for fp64 and 2 (about 40 bits per part) for fp32.

    primes: 2 (p0, p1) or 3 (p0, p1, p2: the CRT with d = 3 moduli, slices
    of about 36 bits at n = 2^18; K then defaults to 2; batched mode only)."""

    def __init__(self, n: int | None = None, batch: int = 1, *, lengths=None, K: int | None = None, L: int = 3,
                 mode: str = "batched", autotune: bool = False, tune_cache: str | None = None,
                 cyclic: bool = True, accumulation: str = "complex", precision: str = "fp64", primes: int = 2):
        if lengths is None:
            if n is None:
                raise ValueError("give n (and batch) or lengths")
            lengths = [int(n)] * int(batch)
        self.lengths = [int(v) for v in lengths]
        if K is None:
            K = 2 if precision == "fp32" or primes == 3 else 3
        self.K, self.L, self.mode, self.precision, self.primes = K, L, mode, precision, primes
        opts = _Options(K, L, _MODES[mode], int(bool(autotune)), tune_cache.encode() if tune_cache else None,
                        EMBED_AUTO if cyclic else EMBED_PADDED, _ACCUMS[accumulation], _PRECS[precision],
                        int(primes))
        arr = (ctypes.c_int64 * len(self.lengths))(*self.lengths)
        h = ctypes.c_void_p()
        _check(lib().fft_ozaki_plan_ex(ctypes.byref(h), arr, len(self.lengths), ctypes.byref(opts)))
        self._h = h
        self.total = sum(self.lengths)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().fft_ozaki_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def execute(self, x, direction: int = FORWARD, out=None, stream=None):
        """Run on a contiguous CUDA tensor (complex128, or complex64 for an
        fp32 plan) holding the transforms back to back (e.g. shape
        (batch, n)); returns `out`."""
        import torch
        want = torch.complex64 if self.precision == "fp32" else torch.complex128
        if x.dtype != want or not x.is_cuda:
            raise TypeError(f"x must be a {want} CUDA tensor")
        if out is not None and (out.dtype != want or not out.is_cuda or out.numel() != self.total
                                or not out.is_contiguous()):
            raise TypeError(f"out must be a contiguous {want} CUDA tensor of {self.total} elements")
        if x.numel() != self.total:
            raise ValueError(f"x has {x.numel()} elements, the plan needs {self.total}")
        x = x.contiguous()
        if out is None:
            out = torch.empty_like(x)
        s = stream if stream is not None else _stream_handle(torch, x.device)
        _check(lib().fft_ozaki_execute(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                       int(direction), ctypes.c_void_p(s)))
        return out

    def forward(self, x, out=None):
        return self.execute(x, FORWARD, out)

    def inverse(self, x, out=None):
        return self.execute(x, INVERSE, out)

    def adjoint(self, x, out=None):
        return self.execute(x, ADJOINT, out)

    def profile_stage(self, stage: int, reps: int = 1, stream=None):
        """Enqueue `reps` repetitions of one stage of the batched schedule
        (see fft_ozaki_profile_stage) on the current stream."""
        import torch
        s = stream if stream is not None else _stream_handle(torch, torch.cuda.current_device())
        _check(lib().fft_ozaki_profile_stage(self._h, int(stage), int(reps), ctypes.c_void_p(s)))

    def stage_timing(self, enable: bool = True):
        """Launch later batched executions on the stream in the graph's order
        with a HIP event at each stage boundary (see fft_ozaki_stage_timing);
        False returns to graph replays."""
        _check(lib().fft_ozaki_stage_timing(self._h, int(bool(enable))))

    def stage_times(self) -> dict:
        """Device ms of the stages of the last execution (see
        fft_ozaki_stage_times): {"split": t, "classes": [{"forward", "rows",
        "cols", "recombine"} per length class]}."""
        n = ctypes.c_int(0)
        lib().fft_ozaki_stage_times(self._h, None, 0, ctypes.byref(n))
        buf = (ctypes.c_float * n.value)()
        _check(lib().fft_ozaki_stage_times(self._h, buf, n.value, ctypes.byref(n)))
        v = list(buf)
        keys = ("forward", "rows", "cols", "recombine")
        return {"split": v[0],
                "classes": [dict(zip(keys, v[1 + 4 * c: 5 + 4 * c])) for c in range((n.value - 1) // 4)]}

    def info(self) -> dict:
        i = _Info()
        _check(lib().fft_ozaki_query(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in _Info._fields_}

    def transform_info(self, index: int) -> dict:
        i = _TInfo()
        _check(lib().fft_ozaki_query_transform(self._h, index, ctypes.byref(i)))
        d = {f: getattr(i, f) for f, _ in _TInfo._fields_}
        d["kx"] = list(i.kx)
        d["kw"] = list(i.kw)
        d["Ex"] = [list(i.Ex[p])[: i.kx[p]] for p in range(2)]
        d["Ew"] = [list(i.Ew[p])[: i.kw[p]] for p in range(2)]
        d["ngroups"] = list(i.ngroups)
        d["xsh"] = list(i.xsh)
        return d

    def debug_dump(self, stage: int, index: int) -> np.ndarray:
        need = ctypes.c_size_t()
        _check(lib().fft_ozaki_debug_dump(self._h, stage, index, None, 0, ctypes.byref(need)))
        buf = np.empty(need.value, dtype=np.uint8)
        _check(lib().fft_ozaki_debug_dump(self._h, stage, index, buf.ctypes.data, need.value, None))
        if stage in (1, 5):
            return buf.view(np.complex128)
        return buf.view(np.uint32)


_plans: dict = {}
_plans_lock = threading.Lock()


def _plan_for(shape, device, K, L, primes=2, stream=0) -> Plan:
    # one plan per stream as well: a plan's workspace serves one execution
    # at a time, and executions on different streams may overlap
    key = (tuple(shape), str(device), K, L, primes, int(stream))
    with _plans_lock:
        p = _plans.get(key)
        if p is None:
            n = shape[-1]
            batch = int(np.prod(shape[:-1])) if len(shape) > 1 else 1
            import torch
            with torch.cuda.device(device):
                p = Plan(n, batch, K=K, L=L, primes=primes)
            _plans[key] = p
    return p


def _run(x, direction, K, L, primes=2):
    import torch
    if x.dtype != torch.complex128:
        raise TypeError("expected complex128")
    xc = x.contiguous()
    stream = _stream_handle(torch, xc.device)
    p = _plan_for(xc.shape, xc.device, K, L, primes, stream)
    with torch.cuda.device(xc.device):
        return p.execute(xc, direction, stream=stream)


def fft(x, K: int | None = None, L: int = 3, primes: int = 2):
    """Forward DFT along the last axis (Sec. 3.2, Eq. dft).  K defaults to 3
    with two CRT moduli and to 2 with three."""
    return _run(x, FORWARD, K, L, primes)


def ifft(x, K: int | None = None, L: int = 3, primes: int = 2):
    """Inverse DFT along the last axis, conj(DFT(conj x)) / n (Eq. idft)."""
    return _run(x, INVERSE, K, L, primes)


def adjoint(x, K: int | None = None, L: int = 3, primes: int = 2):
    """Adjoint DFT along the last axis, conj(DFT(conj x))."""
    return _run(x, ADJOINT, K, L, primes)


def _autograd_class():
    import torch

    class OzakiDFT(torch.autograd.Function):
        """y = DFT(x) along the last axis.  For a C-linear map y = F x the
        vector-Jacobian product in PyTorch's convention is F^H g, so the
        backward pass is the adjoint transform through the same pipeline."""

        @staticmethod
        def forward(ctx, x, K=None, L=3, primes=2):
            ctx.K, ctx.L, ctx.primes = K, L, primes
            return _run(x, FORWARD, K, L, primes)

        @staticmethod
        def backward(ctx, g):
            return _run(g, ADJOINT, ctx.K, ctx.L, ctx.primes), None, None, None

    return OzakiDFT


class _LazyAutograd:
    _cls = None

    def __getattr__(self, name):
        if _LazyAutograd._cls is None:
            _LazyAutograd._cls = _autograd_class()
        return getattr(_LazyAutograd._cls, name)


OzakiDFT = _LazyAutograd()


def execute_static(x, direction: int = FORWARD, out=None):
    """DFT along the last axis of a contiguous complex128 CUDA tensor through
    the allocation-free entry point (fft_ozaki_execute_static: default
    options, the library's static device workspace, no device allocation by
    the library); `out` (same shape) is allocated by torch when not given."""
    import torch
    if x.dtype != torch.complex128 or not x.is_cuda or not x.is_contiguous():
        raise TypeError("x must be a contiguous complex128 CUDA tensor")
    if out is None:
        out = torch.empty_like(x)
    elif out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous() or out.device != x.device:
        raise TypeError("out must be a contiguous complex128 tensor shaped like x on its device")
    n = x.shape[-1]
    batch = x.numel() // n if n else 0
    with torch.cuda.device(x.device):
        _check(lib().fft_ozaki_execute_static(n, batch, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                              int(direction), ctypes.c_void_p(_stream_handle(torch, x.device))))
    return out


def ntt(data, prime: int, inverse: bool = False):
    """The library's NTT in place on a contiguous CUDA int32 tensor viewed as
    uint32 residues, shape (count, N) (see fft_ozaki_ntt in the header)."""
    import torch
    if data.dtype != torch.int32 or not data.is_cuda or not data.is_contiguous():
        raise TypeError("data must be a contiguous int32 CUDA tensor")
    count, N = data.shape
    logN = N.bit_length() - 1
    if 1 << logN != N:
        raise ValueError("N must be a power of two")
    _check(lib().fft_ozaki_ntt(prime, logN, count, ctypes.c_void_p(data.data_ptr()), int(inverse),
                               ctypes.c_void_p(_stream_handle(torch, data.device))))
    return data


def ntt_layout(log2N: int) -> int:
    m = ctypes.c_int()
    _check(lib().fft_ozaki_ntt_layout(log2N, ctypes.byref(m)))
    return m.value
