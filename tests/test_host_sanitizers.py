"""The host and C-ABI code built with AddressSanitizer and
UndefinedBehaviorSanitizer (host side only; no GPU here): argument
validation, error strings, layouts and the size checks of the
allocation-free entry point run without a sanitizer report."""

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHECKS = r"""
import ctypes, sys
L = ctypes.CDLL(sys.argv[1])
vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
L.fft_ozaki_error_string.restype = ctypes.c_char_p
L.fft_ozaki_last_error_message.restype = ctypes.c_char_p
L.fft_ozaki_plan.argtypes = [ctypes.POINTER(vp), i64, i64]
L.fft_ozaki_execute_static.argtypes = [i64, i64, vp, vp, ci, vp]
L.fft_ozaki_plan_ex.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(i64), i64, vp]
h = vp()
for code in (0, -1, -2, -3, -4, -99):
    assert L.fft_ozaki_error_string(code)
assert L.fft_ozaki_plan(ctypes.byref(h), 0, 1) == -1
assert L.fft_ozaki_plan(ctypes.byref(h), 16, 0) == -1
assert L.fft_ozaki_plan(ctypes.byref(h), (1 << 23) + 1, 1) == -1
assert b"exceeds" in L.fft_ozaki_last_error_message()
assert L.fft_ozaki_plan_ex(ctypes.byref(h), None, 1, None) == -1
arr = (i64 * 3)(16, 0, 5)
assert L.fft_ozaki_plan_ex(ctypes.byref(h), arr, 3, None) == -1
assert L.fft_ozaki_execute(None, None, None, 0, None) == -1
assert L.fft_ozaki_destroy(None) == -1
m = ci()
for lg in range(0, 25):
    assert L.fft_ozaki_ntt_layout(lg, ctypes.byref(m)) == 0
assert L.fft_ozaki_ntt_layout(25, ctypes.byref(m)) == -1
fake = vp(256)
assert L.fft_ozaki_execute_static(1 << 18, 1, fake, fake, 0, None) == -1
assert L.fft_ozaki_execute_static(1 << 14, 7, fake, fake, 0, None) == -1
assert L.fft_ozaki_execute_static(1 << 24, 1 << 24, fake, fake, 0, None) == -1
assert L.fft_ozaki_execute_static(-5, 1, fake, fake, 0, None) == -1
print("host checks ok", flush=True)
"""


@pytest.mark.slow
def test_host_code_under_sanitizers(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_2603_29129_amd import build_lib
    rts = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rts:
        pytest.skip("no AddressSanitizer runtime in this ROCm installation")
    lib = build_lib.build(sanitize=True, out=str(tmp_path / "libfft_ozaki_sanitized.so"))
    env = dict(os.environ, LD_PRELOAD=rts[0], ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", CHECKS, lib], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "host checks ok" in r.stdout, (r.stdout + r.stderr)[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
