"""Expected NTT-domain accumulation schedule of the library (test code).

The complex convolution x' (*) w* is four real convolutions, numbered as
oracle.bluestein.CONVS: 0 ReRe (+ into Re y'), 1 ImIm (- into Re y'),
2 ImRe and 3 ReIm (+ into Im y').  Output component tg takes convolutions
2 tg and 2 tg + 1.  Its walk lists the slice pairs (c, s, t):

  per_conv  Alg. 8 for each convolution on its own (convolution 2 tg, then
            2 tg + 1; anti-diagonals s + t descending, s ascending); a group
            closes at L products, at a change of scale and at the change of
            convolution, so the groups are exactly the oracle's alg8_groups.
  complex   anti-diagonals descending; on each the pairs of convolution 2 tg,
            then of 2 tg + 1.  A group holds products of one scale; a
            product of x' part p weighs 2^xsh[p] and the weights of a group
            sum to at most acc_limit, the most products whose signed sum the
            symmetric CRT still recovers: acc_limit n 4^alpha <= (p0 p1 - 1) / 2.
            xsh (part_shift): when the top slice exponents of Re x' and Im x'
            differ by d = 1 or 2, max(kw) 2^d <= acc_limit and
            alpha + d <= 30 (slice integers stay below 2^30), the part with
            the larger one is taken times 2^d and its exponents count d lower,
            so that products of the two parts can share a scale.

The residues of a group are the inverse NTT of the signed NTT-domain sum of
its members' products, a member of part p multiplied by 2^xsh[p], computed
here with the oracle's NTT.
"""

import numpy as np

from oracle import bluestein as bl
from oracle import ntt as nt

P = nt.P0 * nt.P1
MAX_MEMBERS = 128


def acc_limit(n: int, alpha: int, primes: int = 2) -> int:
    M = P if primes == 2 else nt.PPP
    return min(MAX_MEMBERS, ((M - 1) // 2) // (n << (2 * alpha)))


def _pairs(kA: int, kB: int, d: int):
    return [(s, d - s) for s in range(max(0, d - kB + 1), min(kA - 1, d) + 1)]


def part_shift(EX, EW, limit: int, alpha: int):
    """xsh of the complex schedule: [shift of Re x', shift of Im x']."""
    xsh = [0, 0]
    if EX[0] and EX[1]:
        dl = EX[0][0] - EX[1][0]
        part, sh = (0, dl) if dl > 0 else (1, -dl)
        if 1 <= sh <= 2 and (max(len(EW[0]), len(EW[1])) << sh) <= limit and alpha + sh <= 30:
            xsh[part] = sh
    return xsh


def component_schedule(EX, EW, L: int, mode: str, limit: int, weights: bool = False, alpha: int | None = None):
    """Groups per output component: [groups of Re y', groups of Im y'], each
    group a list of (c, s, t), or of (c, s, t, shift) with weights=True.  EX,
    EW: slice exponents of (Re, Im) x' and w*; alpha (the slice width) is
    needed by the complex schedule."""
    if mode == "complex" and alpha is None:
        raise ValueError("the complex schedule needs alpha")
    xsh = part_shift(EX, EW, limit, alpha) if mode == "complex" else [0, 0]
    out = []
    for tg in range(2):
        convs = (2 * tg, 2 * tg + 1)
        k = {c: (len(EX[bl.CONVS[c][0]]), len(EW[bl.CONVS[c][1]])) for c in convs}
        k = {c: (a, b) if a and b else (0, 0) for c, (a, b) in k.items()}
        members = []
        if mode == "per_conv":
            for c in convs:
                kA, kB = k[c]
                for d in range(kA + kB - 2, -1, -1):
                    members += [(c, s, t) for s, t in _pairs(kA, kB, d)]
        else:
            dmax = max(a + b for a, b in k.values()) - 2
            for d in range(dmax, -1, -1):
                for c in convs:
                    members += [(c, s, t) for s, t in _pairs(*k[c], d)]
        lim = L if mode == "per_conv" else limit
        groups, cur, key, load = [], [], None, 0
        for c, s, t in members:
            pa = bl.CONVS[c][0]
            k2 = EX[pa][s] - xsh[pa] + EW[bl.CONVS[c][1]][t]
            wgt = 1 << xsh[pa]
            if cur:
                if mode == "per_conv":
                    fits = len(cur) < lim and k2 == key and c == cur[-1][0]
                else:
                    fits = k2 == key and load + wgt <= lim
                if not fits:
                    groups.append(cur)
                    cur, load = [], 0
            key = k2
            load += wgt
            cur.append((c, s, t, xsh[pa]))
        if cur:
            groups.append(cur)
        out.append([[m if weights else m[:3] for m in g] for g in groups])
    return out


def group_residues(tr, kp, group):
    """Inverse-NTT residues (first n, every prime of the kernel plan) of one
    group's signed, weighted sum (members (c, s, t) or (c, s, t, shift))."""
    n, N = tr["n"], tr["N"]
    res = []
    for ip, p in enumerate(kp.primes):
        pu = np.uint64(p)
        acc = np.zeros(N, dtype=np.uint64)
        for m in group:
            c, s, t = m[:3]
            pa, pb, _tg, sign = bl.CONVS[c]
            prod = (tr["X"][pa][s][ip] * kp.ntts[pb][t][ip]) % pu
            prod = (prod * np.uint64(1 << (m[3] if len(m) > 3 else 0))) % pu
            acc = (acc + prod) % pu if sign > 0 else (acc + (pu - prod)) % pu
        res.append(nt.ntt(acc, p, inverse=True)[:n])
    return res
