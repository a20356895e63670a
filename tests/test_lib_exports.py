"""CPU checks of the built library: it loads and exports every entry point
declared in include/*.h (no compute calls: no GPU here)."""

import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2603_29129_amd", "libfft_ozaki.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(fft_ozaki_[a-z_0-9]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("fft_ozaki_plan", "fft_ozaki_plan_ex", "fft_ozaki_execute", "fft_ozaki_forward",
                 "fft_ozaki_inverse", "fft_ozaki_query", "fft_ozaki_debug_dump", "fft_ozaki_destroy",
                 "fft_ozaki_error_string"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_all_declared_symbols():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_only_calls():
    import paper_2603_29129_amd as oz
    L = oz.lib()
    assert L.fft_ozaki_error_string(0) == b"success"
    assert L.fft_ozaki_error_string(-1) == b"invalid argument"
    # argument validation happens before any device call
    h = ctypes.c_void_p()
    assert L.fft_ozaki_plan(ctypes.byref(h), 0, 1) == -1
    assert L.fft_ozaki_plan(ctypes.byref(h), 16, 0) == -1
    assert L.fft_ozaki_plan(ctypes.byref(h), (1 << 23) + 1, 1) == -1     # N would exceed 2^24
    assert b"exceeds" in L.fft_ozaki_last_error_message()
    opts = oz._Options(9, 3, 1, 0, None)
    arr = (ctypes.c_int64 * 1)(16)
    assert L.fft_ozaki_plan_ex(ctypes.byref(h), arr, 1, ctypes.byref(opts)) == -1
    opts = oz._Options(3, 0, 1, 0, None)
    assert L.fft_ozaki_plan_ex(ctypes.byref(h), arr, 1, ctypes.byref(opts)) == -1
    opts = oz._Options(3, 3, 1, 0, None, 2)                               # no such embedding
    assert L.fft_ozaki_plan_ex(ctypes.byref(h), arr, 1, ctypes.byref(opts)) == -1
    opts = oz._Options(3, 3, 1, 0, None, 1, 2)                            # no such accumulation
    assert L.fft_ozaki_plan_ex(ctypes.byref(h), arr, 1, ctypes.byref(opts)) == -1
    assert b"accumulation" in L.fft_ozaki_last_error_message()
    opts = oz._Options(3, 3, 1, 0, None, 1, 1, 0, 4)                      # no such number of moduli
    assert L.fft_ozaki_plan_ex(ctypes.byref(h), arr, 1, ctypes.byref(opts)) == -1
    assert b"primes" in L.fft_ozaki_last_error_message()
    opts = oz._Options(2, 3, 0, 0, None, 1, 1, 0, 3)                      # three moduli, plain mode
    assert L.fft_ozaki_plan_ex(ctypes.byref(h), arr, 1, ctypes.byref(opts)) == -4
    d = oz._Options()
    assert L.fft_ozaki_default_options(ctypes.byref(d)) == 0
    assert (d.K, d.L, d.mode, d.autotune, d.embedding) == (3, 3, 1, 0, oz.EMBED_AUTO)
    assert d.accumulation == oz.ACCUM_COMPLEX and d.primes == 2
    assert L.fft_ozaki_execute(None, None, None, 0, None) == -1
    assert L.fft_ozaki_destroy(None) == -1
    assert L.fft_ozaki_stage_timing(None, 1) == -1
    n = ctypes.c_int(-7)
    assert L.fft_ozaki_stage_times(None, None, 0, ctypes.byref(n)) == -1 and n.value == -7
    m = ctypes.c_int()
    assert L.fft_ozaki_ntt_layout(19, ctypes.byref(m)) == 0 and m.value == 10
    assert L.fft_ozaki_ntt_layout(12, ctypes.byref(m)) == 0 and m.value == 12
    assert L.fft_ozaki_ntt_layout(25, ctypes.byref(m)) == -1
    assert L.fft_ozaki_ntt(2, 10, 1, None, 0, None) == -1                 # data NULL
    assert L.fft_ozaki_ntt(3, 10, 0, None, 0, None) == -1                 # no prime 3
    # the allocation-free entry point checks its arguments before any device call
    fake = ctypes.c_void_p(256)
    assert L.fft_ozaki_execute_static(1 << 18, 1, fake, fake, 0, None) == -1
    assert b"static workspace" in L.fft_ozaki_last_error_message()
    assert L.fft_ozaki_execute_static(1 << 14, 7, fake, fake, 0, None) == -1   # 6 fit, 7 do not
    assert L.fft_ozaki_execute_static(0, 1, fake, fake, 0, None) == -1
    assert L.fft_ozaki_execute_static(16, 1, None, fake, 0, None) == -1
    assert L.fft_ozaki_execute_static(16, 1, fake, fake, 3, None) == -1
    assert L.fft_ozaki_execute_static(16, 1, ctypes.c_void_p(264), fake, 0, None) == -1   # misaligned
