"""Oracle for the FP64-accurate Bluestein/Ozaki/NTT DFT -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, CPU implementation of what the GPU path
computes, written from the paper "Computing FFTs at Target Precision Using
Lower-Precision FFTs" (Kawakami & Takahashi).  It exists to check the GPU
library; it is never part of the product path.  Only the test-suite, the
smoke check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py``
may import it.  It shares no code with the HIP library or its Python binding.

Modules
-------
ntt        modular arithmetic over p0, p1 (and p2 for the d = 3 variant):
           roots, NTT / inverse NTT (Sec. 3.3), symmetric remainder
           (Sec. 3.1), Garner's CRT with two and three moduli (Sec. 3.3,
           Alg. 5 / Alg. 8 reconstruction step).
ozaki      split width alpha (Sec. 4.2 for the product of the moduli;
           Sec. 4.4 with the accumulation bound L) and the splitting
           procedure (Alg. 3 with the scaling of Alg. 6, carried out in
           binary64).
bluestein  chirp, premultiply, padding (Sec. 3.2, Alg. 1), the NTT-domain
           accumulation schedule (Alg. 8), the four real convolutions
           (Sec. 4.5), CRT, exact recombination and postmultiply; forward,
           inverse and adjoint DFT, the binary32 target and the
           three-modulus variant; NTT counts.
reference  extended-precision DFTs (mpmath and long-double) and the error
           metrics of Sec. 5.1.

Pins: every function here is checked in ``tests/test_oracle_*.py`` against
something other than itself (definitions evaluated by brute force, closed
forms, values printed in the paper, identities).  Functions without such a
pin are marked "parity unpinned" in their docstring.
"""

from . import ntt, ozaki, bluestein, reference  # noqa: F401
