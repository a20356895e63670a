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
            then of 2 tg + 1; a group closes at a change of scale or at
            acc_limit products, the most whose signed sum the symmetric CRT
            still recovers: acc_limit n 4^alpha <= (p0 p1 - 1) / 2.

The residues of a group are the inverse NTT of the signed NTT-domain sum of
its members' products, computed here with the oracle's NTT.
"""

import numpy as np

from oracle import bluestein as bl
from oracle import ntt as nt

P = nt.P0 * nt.P1
MAX_MEMBERS = 128


def acc_limit(n: int, alpha: int) -> int:
    return min(MAX_MEMBERS, ((P - 1) // 2) // (n << (2 * alpha)))


def _pairs(kA: int, kB: int, d: int):
    return [(s, d - s) for s in range(max(0, d - kB + 1), min(kA - 1, d) + 1)]


def component_schedule(EX, EW, L: int, mode: str, limit: int):
    """Groups per output component: [groups of Re y', groups of Im y'], each
    group a list of (c, s, t).  EX, EW: slice exponents of (Re, Im) x' and w*."""
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
        groups, cur, key = [], [], None
        for c, s, t in members:
            k2 = EX[bl.CONVS[c][0]][s] + EW[bl.CONVS[c][1]][t]
            if cur and (len(cur) >= lim or k2 != key or (mode == "per_conv" and c != cur[-1][0])):
                groups.append(cur)
                cur = []
            cur.append((c, s, t))
            key = k2
        if cur:
            groups.append(cur)
        out.append(groups)
    return out


def group_residues(tr, kp, group):
    """Inverse-NTT residues (first n, both primes) of one group's signed sum."""
    n, N = tr["n"], tr["N"]
    res = []
    for ip, p in enumerate(nt.PRIMES):
        pu = np.uint64(p)
        acc = np.zeros(N, dtype=np.uint64)
        for c, s, t in group:
            pa, pb, _tg, sign = bl.CONVS[c]
            prod = (tr["X"][pa][s][ip] * kp.ntts[pb][t][ip]) % pu
            acc = (acc + prod) % pu if sign > 0 else (acc + (pu - prod)) % pu
        res.append(nt.ntt(acc, p, inverse=True)[:n])
    return res
