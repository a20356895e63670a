"""Accuracy and NTT-count study of the method on the GPU.

The paper's evaluation (Sec. 5.1 setup, Sec. 5.2 results) varies the split
cap K, the accumulation bound L and the input spread phi over n = 2^10 ..
2^18 with inputs (rand - 0.5) exp(phi randn) for the real and imaginary
parts.  This module runs the same grid through the library:

    python -m paper_2603_29129_amd.study [--nmin 10] [--nmax 18] [--batch 4]
                                          [--seed 0] [--json FILE]

For every (K, L, phi, n) it reports the maximum componentwise relative
error and the relative l2 error of the GPU result against numpy's FFT in
long double, the largest slice counts of Re x', Im x' over the batch, the
kernel slice counts, and the 32-bit NTTs per transform (runtime forward +
inverse, offline forward, total).  K = inf is the library's cap, K = 8.
The counts are those of the paper's schedule (Alg. 8 per real convolution,
accumulation="per_conv"); every case also runs the library's default
complex accumulation, whose runtime NTT count is reported beside them and
whose outputs must be bit-identical.
"""

from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np

KL_GRID = (("inf", 1), (1, 1), (2, 1), (3, 1), (3, 3))
PHIS = (0.0, 1.0, 4.0)
K_INF = 8


def longdouble_errors(y, x):
    """(max componentwise relative error, relative l2 error) of y against the
    long-double DFT of x (components with a zero reference are skipped in
    the first)."""
    ref = np.fft.fft(np.asarray(x).astype(np.clongdouble), axis=-1)
    yl = np.asarray(y).astype(np.clongdouble)
    rel = float(np.sqrt(np.sum(np.abs(yl - ref) ** 2)) / np.sqrt(np.sum(np.abs(ref) ** 2)))
    mx = 0.0
    for a, b in ((yl.real, ref.real), (yl.imag, ref.imag)):
        m = b != 0
        if np.any(m):
            mx = max(mx, float(np.max(np.abs((a[m] - b[m]) / b[m]))))
    return mx, rel


def inputs(n: int, phi: float, seed: int = 0, batch: int = 1):
    """The paper's test inputs (Sec. 5.1): real and imaginary parts each
    (rand - 0.5) exp(phi randn), rand uniform on (0, 1], drawn from numpy's
    PCG64 generator with the given seed: all real parts of the batch, then
    all imaginary parts, each as a (batch, n) block of rand then randn."""
    rng = np.random.default_rng(seed)

    def part():
        rand = 1.0 - rng.random((batch, n))
        return (rand - 0.5) * np.exp(phi * rng.standard_normal((batch, n)))

    re = part()
    return re + 1j * part()


def run_case(n: int, K, L: int, phi: float, batch: int = 4, seed: int = 0, x=None) -> dict:
    """One configuration on cuda:0 (inputs from `inputs` unless x, a
    (batch, n) complex128 array, is given)."""
    import torch
    import paper_2603_29129_amd as oz
    k = K_INF if K == "inf" else int(K)
    if x is None:
        x = inputs(n, phi, seed=seed, batch=batch)
    xt = torch.from_numpy(x).cuda()
    runs = {}
    for acc in ("per_conv", "complex"):
        plan = oz.Plan(n, batch, K=k, L=L, accumulation=acc)
        y = plan.forward(xt).cpu().numpy()
        runs[acc] = (y, [plan.transform_info(b) for b in range(batch)])
        plan.close()
    y, infos = runs["per_conv"]
    yc, infos_c = runs["complex"]
    errs = [longdouble_errors(y[b], x[b]) for b in range(batch)]
    i0 = infos[0]
    per = [d["forward_runtime"] + d["inverse"] for d in infos]
    per_c = [d["forward_runtime"] + d["inverse"] for d in infos_c]
    return {
        "n": n, "K": K, "L": L, "phi": phi, "batch": batch, "N": i0["N"], "alpha": i0["alpha"],
        "max_rel_error": max(e[0] for e in errs), "rel_l2_error": max(e[1] for e in errs),
        "kx": [max(d["kx"][0] for d in infos), max(d["kx"][1] for d in infos)], "kw": list(i0["kw"]),
        "groups": max(sum(d["ngroups"]) for d in infos),
        "ntt_runtime": max(per), "ntt_offline": i0["forward_offline"],
        "ntt_total": max(per) + i0["forward_offline"],
        "ntt_runtime_complex": max(per_c),
        "complex_identical": bool(np.array_equal(y.view(np.int64), yc.view(np.int64))),
        "status": max(d["status"] for d in infos),
    }


def run_study(nmin: int = 10, nmax: int = 18, batch: int = 4, seed: int = 0, progress=None) -> list:
    rows = []
    for K, L in KL_GRID:
        for phi in PHIS:
            for lg in range(nmin, nmax + 1):
                r = run_case(1 << lg, K, L, phi, batch, seed)
                rows.append(r)
                if progress:
                    progress(r)
    return rows


def table(rows) -> str:
    head = ("| (K, L) | phi | n | alpha | slices Re/Im x' | kernel slices | groups | NTTs runtime | NTTs total "
            "| NTTs runtime, complex acc. | max rel. error | rel. l2 error |\n"
            "|---|---|---|---|---|---|---|---|---|---|---|---|")
    out = [head]
    for r in rows:
        out.append(f"| ({r['K']}, {r['L']}) | {r['phi']:g} | 2^{int(math.log2(r['n']))} | {r['alpha']} "
                   f"| {r['kx'][0]}/{r['kx'][1]} | {r['kw'][0]}/{r['kw'][1]} | {r['groups']} | {r['ntt_runtime']} "
                   f"| {r['ntt_total']} | {r['ntt_runtime_complex']}{'' if r['complex_identical'] else ' (DIFFERS)'} "
                   f"| {r['max_rel_error']:.2e} | {r['rel_l2_error']:.2e} |")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--nmin", type=int, default=10)
    ap.add_argument("--nmax", type=int, default=18)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    rows = run_study(a.nmin, a.nmax, a.batch, a.seed,
                     progress=lambda r: print(f"# (K,L)=({r['K']},{r['L']}) phi={r['phi']:g} n={r['n']}: "
                                              f"rel_l2={r['rel_l2_error']:.2e} ntt_total={r['ntt_total']}",
                                              file=sys.stderr, flush=True))
    print(table(rows))
    if a.json:
        with open(a.json, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    main()
