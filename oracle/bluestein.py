"""Oracle: the FP64 DFT by Bluestein + Ozaki slices + two-prime NTT
convolution with NTT-domain accumulation + Garner CRT + exact recombination.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Pipeline for y = DFT(x), x in (F64 + i F64)^n, parameters (K, L):

1. chirp w(j) = w_2n^{j^2} = exp(-i pi q_j / n), q_j = j^2 mod 2n, each
   component correctly rounded to binary64 (Sec. 3.2; the paper converts a
   double-precision chirp to TS in Alg. 4).
2. x' = x (.) w, complex product with each real product and the final
   sum rounded separately (no fused multiply-add) (Sec. 3.2 Step 1, Alg. 1).
3. split Re x', Im x' (runtime) and Re w*, Im w* (input independent, done
   once per length as the paper precomputes them, Sec. 4.5) with
   :func:`oracle.ozaki.split`, one split per vector shared by the two
   convolutions that use it (the split caching of Sec. 4.5).
4. residues mod p0, p1, zero padding of the x' slices and wrap-around
   padding of the w* slices to N = 2^ceil(log2(2n-1)) (Sec. 3.2, ZeroPad and
   ZeroPad+-), forward NTTs.  For a power-of-two n the paper notes that the
   convolution is already cyclic of length n (Sec. 3.2): w*(j) depends on
   j^2 mod 2n, which for even n has period n in j and is even in j, so the
   length-n cyclic convolution with w* itself gives the same sums; this
   embedding (N = n, no padding) is selected with ``cyclic=True``.
5. four real convolutions Re*Re, Im*Im, Im*Re, Re*Im (Sec. 4.5), each by
   Alg. 8: walk the anti-diagonals s+t = k from k_x+k_y-2 down to 0 and
   accumulate X^(s) (.) Y^(t) in the NTT domain, starting a new group when L
   products have been accumulated or the scale c_x^(s) c_y^(t) changes.
6. each group: inverse NTTs, Garner CRT to the symmetric range, first n
   entries; the group's value is z * 2^(E_x^s + E_y^t - 2 alpha).
7. recombination: Re y' = sum(ReRe groups) - sum(ImIm groups),
   Im y' = sum(ImRe groups) + sum(ReIm groups), each sum computed exactly and
   rounded once to binary64 (replaces TSAdd and the final TS->double rounding
   of Alg. 4 / Alg. 8).
8. y = y' (.) w (Sec. 3.2 Step 3), same product rule as step 2.

Inverse: DFT^{-1}(y) = conj(DFT(conj y)) / n, componentwise division
(Sec. 3.2, Eq. idft).  Adjoint: DFT^H(g) = conj(DFT(conj g)).

Three moduli (d = 3, Sec. 3.3's CRT with d moduli; ``primes=3``): residues
mod p0, p1, p2, the split width from Sec. 4.2's formula with the product of
the three moduli (alpha = 36 at n = 2^18, L = 3), Garner's algorithm with
d = 3 in step 6; everything else as above.  With slices that wide K = 2
reaches the binary64 accuracy of K = 3 with two moduli.

Binary32 target precision (the paper reaches a target precision through the
number of splits, Sec. 6): a complex64 input is widened exactly to binary64,
the transform above runs with the cap K (2 slices of about 20 bits per part
cover binary32's 24), and each output component is rounded once to binary32.
"""

from __future__ import annotations

from fractions import Fraction
import math

import mpmath
import numpy as np

from . import ntt as nt
from . import ozaki as oz

DEFAULT_K = 3
DEFAULT_L = 3

# the four real convolutions of Sec. 4.5: (input part, kernel part, target, sign)
# parts: 0 = Re, 1 = Im; target 0 = Re y', 1 = Im y'
CONVS = ((0, 0, 0, +1), (1, 1, 0, -1), (1, 0, 1, +1), (0, 1, 1, +1))


def _cplx(re, im):
    """Complex array with exactly these real and imaginary parts (building it
    as re + 1j*im would add a zero product and drop the sign of zeros)."""
    out = np.empty(np.shape(re), dtype=np.complex128)
    out.real = re
    out.imag = im
    return out


def is_pow2(n: int) -> bool:
    return n >= 1 and (n & (n - 1)) == 0


def conv_length(n: int, cyclic: bool = False) -> int:
    """Bluestein cyclic-convolution length: smallest power of two >= 2n-1
    (Sec. 3.2, N >= 2n - 1); with ``cyclic`` and a power-of-two n, n itself
    (the paper's special case, Sec. 3.2)."""
    if n < 1:
        raise ValueError("n must be positive")
    if cyclic:
        if not is_pow2(n):
            raise ValueError("the cyclic embedding N = n needs a power-of-two n")
        return n
    return 1 << (2 * n - 2).bit_length() if n > 1 else 1


_CHIRP_CACHE: dict = {}


def _cospi_sinpi(num: int, den: int):
    key = (num, den)
    v = _CHIRP_CACHE.get(key)
    if v is None:
        with mpmath.workprec(192):
            t = mpmath.mpf(num) / den
            v = (float(mpmath.cospi(t)), float(mpmath.sinpi(t)))
        _CHIRP_CACHE[key] = v
    return v


def chirp(n: int):
    """(c, s) with c_j = RN(cos(pi q_j / n)), s_j = RN(sin(pi q_j / n)),
    q_j = j^2 mod 2n computed exactly (Sec. 3.2: w(j) = w_2n^{j^2}).
    Then w(j) = c_j - i s_j and w*(j) = c_j + i s_j."""
    c = np.empty(n, dtype=np.float64)
    s = np.empty(n, dtype=np.float64)
    for j in range(n):
        q = (j * j) % (2 * n)
        g = math.gcd(q, n)
        c[j], s[j] = _cospi_sinpi(q // g, n // g)
    return c, s


def premultiply(xr, xi, c, s):
    """x' = x (.) w with w = c - i s: Re = RN(RN(xr c) + RN(xi s)),
    Im = RN(RN(xi c) - RN(xr s)) (Sec. 3.2 Step 1).  numpy never fuses."""
    return xr * c + xi * s, xi * c - xr * s


postmultiply = premultiply  # y = y' (.) w, Sec. 3.2 Step 3


def pad_input(a, N: int) -> np.ndarray:
    """ZeroPad(a, N) (Sec. 3.2)."""
    out = np.zeros(N, dtype=np.int64)
    out[: len(a)] = a
    return out


def pad_kernel(b, N: int) -> np.ndarray:
    """ZeroPad+-(b, N): b(j) for j < n, 0 for n <= j < N-n+1, b(N-j) for
    N-n+1 <= j < N (Sec. 3.2).  With N = n (cyclic embedding of a
    power-of-two n) the kernel is b itself."""
    n = len(b)
    if N == n:
        return np.asarray(b, dtype=np.int64).copy()
    out = np.zeros(N, dtype=np.int64)
    out[:n] = b
    for j in range(N - n + 1, N):
        out[j] = b[N - j]
    return out


def alg8_groups(EA, EB, L: int):
    """NTT-domain accumulation schedule of Alg. 8.

    EA, EB: exponents E of the slices of the two operands (the paper's scale
    c^(s) = 2^(alpha - E^(s))).  Returns a list of groups, each a list of
    (s, t) pairs; a group is closed when L products are in it or the product
    scale changes.  Equal products of scales <=> equal E_A^s + E_B^t.
    """
    kA, kB = len(EA), len(EB)
    if kA == 0 or kB == 0:
        return []
    groups = []
    cur = []
    key = EA[kA - 1] + EB[kB - 1]
    count = 0
    for d in range(kA + kB - 2, -1, -1):
        for s in range(max(0, d - kB + 1), min(kA - 1, d) + 1):
            t = d - s
            if count >= L or key != EA[s] + EB[t]:
                groups.append(cur)
                cur = []
                key = EA[s] + EB[t]
                count = 0
            cur.append((s, t))
            count += 1
    groups.append(cur)
    return groups


def round_dyadic(S: int, e: int) -> float:
    """RN(S * 2^e) to binary64, ties to even, overflow to +-inf.  Uses
    CPython's correctly rounded int->float conversion and int/int true
    division."""
    if S == 0:
        return 0.0
    try:
        if e >= 0:
            return float(S << e)
        return S / (1 << (-e))
    except OverflowError:
        return math.copysign(math.inf, S)


class KernelPlan:
    """Input-independent part for one length n: chirp, splits of Re w* and
    Im w* and their forward NTTs (Sec. 4.5, precomputed offline)."""

    def __init__(self, n: int, K: int | None = DEFAULT_K, L: int = DEFAULT_L, cyclic: bool = False,
                 primes: int = 2):
        if primes not in (2, 3):
            raise ValueError("primes must be 2 or 3")
        self.n, self.K, self.L, self.cyclic = n, K, L, cyclic
        self.N = conv_length(n, cyclic)
        self.primes = nt.PRIMES if primes == 2 else nt.PRIMES3
        self.alpha = oz.alpha_crt(n, L, nt.PP if primes == 2 else nt.PPP)
        self.c, self.s = chirp(n)
        self.slices = []   # per part: list of (a, E)
        self.ntts = []     # per part: list of (W0, W1)
        for v in (self.c, self.s):
            sl, _, st = oz.split(v, self.alpha, K)
            assert st == oz.STATUS_OK
            self.slices.append(sl)
            self.ntts.append([tuple(nt.ntt(pad_kernel(a, self.N), p) for p in self.primes)
                              for a, _ in sl])

    def exps(self, part):
        return [E for _, E in self.slices[part]]


def forward_trace(x, K: int | None = DEFAULT_K, L: int = DEFAULT_L, plan: KernelPlan | None = None):
    """Forward DFT of one complex vector with every intermediate returned."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.size
    if plan is None:
        plan = KernelPlan(n, K, L)
    N, alpha = plan.N, plan.alpha
    xr, xi = premultiply(x.real.copy(), x.imag.copy(), plan.c, plan.s)
    tr = dict(n=n, N=N, alpha=alpha, K=K, L=L, xpr=xr, xpi=xi, status=oz.STATUS_OK)
    xs = []
    status = oz.STATUS_OK
    if not (np.all(np.isfinite(xr)) and np.all(np.isfinite(xi))):
        status = oz.STATUS_NONFINITE
    else:
        for v in (xr, xi):
            sl, _, st = oz.split(v, alpha, K)
            status |= st
            xs.append(sl)
    tr["status"] = status
    if status != oz.STATUS_OK:
        nan = np.full(n, np.nan)
        tr["y"] = _cplx(nan, nan)
        tr["slices"] = [[], []]
        tr["groups"] = [[] for _ in CONVS]
        return tr
    tr["slices"] = xs
    # forward NTTs of the input slices (zero padded), every prime
    X = [[tuple(nt.ntt(pad_input(a, N), p) for p in plan.primes) for a, _ in xs[v]] for v in range(2)]
    tr["X"] = X
    EX = [[E for _, E in xs[v]] for v in range(2)]
    tr["groups"] = []
    tr["group_z"] = []        # per conv: list of (z int64[n], e)
    terms = ([], [])          # per target: list of (sign, z, e)
    for (pa, pb, tgt, sign) in CONVS:
        groups = alg8_groups(EX[pa], plan.exps(pb), L)
        tr["groups"].append(groups)
        zs = []
        for grp in groups:
            zi = []
            for ip, p in enumerate(plan.primes):
                acc = np.zeros(N, dtype=np.uint64)
                for (s, t) in grp:
                    acc = (acc + X[pa][s][ip] * plan.ntts[pb][t][ip]) % np.uint64(p)
                zi.append(nt.ntt(acc, p, inverse=True)[:n])
            z = nt.garner_crt(zi[0], zi[1]) if len(zi) == 2 else nt.garner_crt3(zi[0], zi[1], zi[2])
            s0, t0 = grp[0]
            e = EX[pa][s0] + plan.exps(pb)[t0] - 2 * alpha
            zs.append((z, e))
            terms[tgt].append((sign, z, e))
        tr["group_z"].append(zs)
    yp = []
    for tgt in range(2):
        tl = terms[tgt]
        out = np.zeros(n, dtype=np.float64)
        if tl:
            emin = min(e for _, _, e in tl)
            cols = [(sg, z.tolist(), e - emin) for sg, z, e in tl]
            for k in range(n):
                S = 0
                for sg, zl, sh in cols:
                    S += sg * (zl[k] << sh)
                out[k] = round_dyadic(S, emin)
        yp.append(out)
    tr["ypr"], tr["ypi"] = yp
    yr, yi = postmultiply(yp[0], yp[1], plan.c, plan.s)
    tr["y"] = _cplx(yr, yi)
    return tr


def fft(x, K: int | None = DEFAULT_K, L: int = DEFAULT_L, plan: KernelPlan | None = None):
    """Forward DFT (Sec. 3.2, Eq. dft) of one vector by the method."""
    return forward_trace(x, K, L, plan)["y"]


def _conj(v):
    v = np.asarray(v, dtype=np.complex128)
    return _cplx(v.real, -v.imag)


def adjoint(g, K: int | None = DEFAULT_K, L: int = DEFAULT_L, plan: KernelPlan | None = None):
    """DFT^H g = conj(DFT(conj g))."""
    y = fft(_conj(g), K, L, plan)
    out = np.empty_like(y)
    out.real = y.real
    out.imag = -y.imag
    return out


def ifft(y, K: int | None = DEFAULT_K, L: int = DEFAULT_L, plan: KernelPlan | None = None):
    """DFT^{-1} y = conj(DFT(conj y)) / n (Sec. 3.2, Eq. idft), each component
    divided by n with one IEEE rounding."""
    a = adjoint(y, K, L, plan)
    n = float(len(a))
    out = np.empty_like(a)
    out.real = a.real / n
    out.imag = a.imag / n
    return out


def _to32(v):
    """Each component rounded once to binary32 (round to nearest even)."""
    return np.asarray(v, dtype=np.complex128).astype(np.complex64)


def _from32(x32):
    """complex64 widened exactly to complex128."""
    return np.asarray(x32, dtype=np.complex64).astype(np.complex128)


def fft_binary32(x32, K: int | None = 2, L: int = DEFAULT_L, plan: KernelPlan | None = None):
    """Forward DFT at the binary32 target (module docstring): complex64 in and out."""
    return _to32(fft(_from32(x32), K, L, plan))


def adjoint_binary32(g32, K: int | None = 2, L: int = DEFAULT_L, plan: KernelPlan | None = None):
    return _to32(adjoint(_from32(g32), K, L, plan))


def ifft_binary32(y32, K: int | None = 2, L: int = DEFAULT_L, plan: KernelPlan | None = None):
    return _to32(ifft(_from32(y32), K, L, plan))


def ntt_counts(tr, plan: KernelPlan):
    """32-bit transform counts (Sec. 4.5): forward NTTs of the input splits
    (runtime), of the kernel splits (offline), inverse NTTs (runtime)."""
    d = len(plan.primes)
    fwd_rt = d * sum(len(tr["slices"][v]) for v in range(2))
    fwd_off = d * sum(len(plan.slices[v]) for v in range(2))
    inv = d * sum(len(g) for g in tr["groups"])
    return dict(forward_runtime=fwd_rt, forward_offline=fwd_off, inverse=inv,
                runtime=fwd_rt + inv, total=fwd_rt + fwd_off + inv)


def exact_convolution_rounded(xr, xi, c, s):
    """RN of the exact Bluestein convolution y'(k) = sum_j x'(j) w*(|k-j|)
    (Sec. 3.2, Eq. bluestein_convolution, with the binary64 x' and chirp),
    each component summed in rationals and rounded once.  Brute force, small
    n only; used to pin the whole integer pipeline when no slice is dropped.
    """
    n = len(xr)
    fr = [Fraction(float(v)) for v in xr]
    fi = [Fraction(float(v)) for v in xi]
    fc = [Fraction(float(v)) for v in c]
    fs = [Fraction(float(v)) for v in s]
    yr = np.empty(n)
    yi = np.empty(n)
    for k in range(n):
        re = Fraction(0)
        im = Fraction(0)
        for j in range(n):
            m = abs(k - j)
            re += fr[j] * fc[m] - fi[j] * fs[m]
            im += fi[j] * fc[m] + fr[j] * fs[m]
        yr[k] = _round_fraction(re)
        yi[k] = _round_fraction(im)
    return yr, yi


def _round_fraction(f: Fraction) -> float:
    if f == 0:
        return 0.0
    try:
        return f.numerator / f.denominator
    except OverflowError:
        return math.copysign(math.inf, f)
