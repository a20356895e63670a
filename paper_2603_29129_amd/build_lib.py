"""Builds the HIP library libfft_ozaki.so for gfx950 in the package folder.

    python -m paper_2603_29129_amd.build_lib

Each source is compiled to an object of its own (in parallel), then the
objects are linked; every object carries its own gfx950 code object.
"""

from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libfft_ozaki.so")
SOURCES = ["ntt_kernels.hip", "split_kernels.hip", "recombine_kernels.hip", "plan.hip"]

FLAGS = [
    "-O3",
    "--offload-arch=gfx950",
    "-fPIC",
    "-std=c++17",
    # every binary64 operation rounds on its own; fused forms are written explicitly
    "-ffp-contract=off",
    # never emit packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


# per-source additions: the NTT pass kernels let the backend raise each
# wave's priority while it issues its first loads and lower it before the
# arithmetic (s_setprio; 0.8% per step at the headline, same bits)
SOURCE_FLAGS = {"ntt_kernels.hip": ["-mllvm", "-amdgpu-set-wave-priority"]}


# host-side AddressSanitizer and UndefinedBehaviorSanitizer (the device code
# is built as usual): a checking build of the host and C-ABI code
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def build(verbose: bool = False, sanitize: bool = False, out: str | None = None) -> str:
    """Compiles the library to `out` (default: libfft_ozaki.so in the
    package); sanitize adds the host-side sanitizers."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = "-I" + os.path.join(ROOT, "include")
    lib = out or LIB
    extra = HOST_SANITIZE if sanitize else []
    with tempfile.TemporaryDirectory(prefix="fft_ozaki_build_") as tmpd:
        def compile_one(src):
            obj = os.path.join(tmpd, os.path.splitext(src)[0] + ".o")
            cmd = [hipcc, *FLAGS, *SOURCE_FLAGS.get(src, []), *extra, inc, "-c", "-o", obj, os.path.join(PKG, "csrc", src)]
            if verbose:
                print(" ".join(cmd), flush=True)
            res = subprocess.run(cmd, capture_output=True, text=True)
            return obj, res

        with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
            results = list(ex.map(compile_one, SOURCES))
        for obj, res in results:
            if res.returncode != 0:
                sys.stderr.write(res.stdout + res.stderr)
                raise RuntimeError(f"hipcc failed compiling {obj}")
        tmp = lib + ".tmp"
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *extra, "-o", tmp, *[o for o, _ in results],
               "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libfft_ozaki.so")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
