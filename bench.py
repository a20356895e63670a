#!/usr/bin/env python3
"""Throughput of the FP64-accurate DFT (Bluestein + Ozaki slices + two-prime
32-bit NTT convolution) on one MI355X.

One step = one forward execution of the whole path (premultiply, split,
forward NTTs, NTT-domain multiply-accumulate, inverse NTTs, CRT,
recombination, postmultiply) over a batch of 8 transforms of length n = 2^18
whose magnitudes are log-uniform in [2^-30, 2^30] with uniform phase
(workload `wide_256k`, seed 0), inputs resident in HBM.  The metric is
GFLOP/s in the 5 n log2 n convention.  The headline plan uses the library's
default embedding: for a power-of-two n the convolution is cyclic of length
N = n (Sec. 3.2); the padded embedding (N = 2n) is timed beside it and must
give the same bits.

Prints one JSON line.  Besides the headline (batched form, HIP graph replay)
it reports the plain form on the same input, the relative l2 error against
a long-double DFT, per-stage device times, the roofline of the dominant
kernel, the binary32 target precision (complex64 in and out, K = 2) on the
same input rounded to binary32, the three-modulus CRT plan (K = 2 slices of
36 bits) on the same input, one transform of the workload on its own, and
the CPU oracle timed on a bounded sample.
"""

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FP64-accurate FFT GFLOP/s (5n·log2n) at n=2^18, batched vs plain; rel. error"
HBM_PEAK_GBS = 8000.0
# 32-bit integer VALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one
# operation per lane per cycle (no fused pair for integer work)
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# int32 operations of the algorithm (Shoup products, fully reduced results):
# forward DIF butterfly: add_mod 3 + (x - y + p) 2 + product 6; inverse DIT
# butterfly: product 6 + add_mod 3 + sub_mod 3; twiddle product 6; NTT-domain
# multiply-accumulate: product 6 + add_mod 3.  Butterflies whose root is 1
# are counted at full cost (the textbook (N/2) log2 N products).
OPS_FWD_BFLY, OPS_INV_BFLY, OPS_TWIDDLE, OPS_MAC = 11, 12, 6, 9
# CRT and exact accumulation per output and group: Garner (z0 mod p1 2,
# sub_mod 3, product 6, 64-bit z0 + h p0 4, symmetric fold 3) = 18; adding
# z 2^sh to the 256-bit accumulator: one add-with-carry per 32-bit limb = 8
OPS_CRT, OPS_ACC = 18, 8
PASS_STAGES = (4, 5, 6, 7, 8)
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2603_29129_amd", "csrc")


def fused_columns(info):
    """The batched form fuses the inverse column pass with the CRT and the
    recombination for 2^7 <= N1 <= 2^9."""
    logN, m1 = info["N"].bit_length() - 1, info["ntt_log2N1"]
    return logN > 12 and 7 <= m1 <= 9 and 12 - m1 <= logN - m1


def folded_rows(info, K):
    """The batched form folds the forward row pass into the inverse row pass
    (register form, K <= 3, 512-position row tiles: the pipelined row pass)."""
    logN, m1 = info["N"].bit_length() - 1, info["ntt_log2N1"]
    m2 = logN - m1
    li = min(max(9 - m2, 0), m1)
    return logN > 12 and K <= 3 and m2 + li == 9


def stage_kernels(info, K, primes=2):
    """Kernel launched by each pass stage (one launch per stage for a uniform
    batch) of a batched plan, by the name rocprofv3 reports (None: the stage
    launches nothing)."""
    logN, m1 = info["N"].bit_length() - 1, info["ntt_log2N1"]
    m2 = logN - m1
    # the folded row pass runs as the persistent pipelined kernel
    rows = f"k_inv_rows_pipe<{m2}, {primes}>" if folded_rows(info, K) else f"k_inv_rows<{m2}>"
    out = {4: f"k_fwd_cols<{m1}>", 5: None if folded_rows(info, K) else f"k_fwd_rows<{m2}>", 6: rows}
    if fused_columns(info):
        out.update({7: f"k_inv_cols_rec<{m1}, {primes}>", 8: f"k_recombine<true, {primes}>"})
    else:
        out.update({7: f"k_inv_cols<{m1}>", 8: f"k_recombine<false, {primes}>"})
    return out


def algorithmic_ops(infos):
    """Algorithmic int32 operations per launch of the NTT pass kernels."""
    out = {4: 0, 5: 0, 6: 0, 7: 0}
    for d in infos:
        N = d["N"]
        logN, m1 = N.bit_length() - 1, d["ntt_log2N1"]
        m2 = logN - m1
        N1, N2 = 1 << m1, 1 << m2
        vf = 2 * (d["kx"][0] + d["kx"][1])          # forward vectors (part, slice, prime)
        vi = 2 * sum(d["ngroups"])                   # inverse vectors (group, prime)
        pairs = sum(d["kx"][pa] * d["kw"][pb] for pa, pb in ((0, 0), (1, 1), (1, 0), (0, 1)))
        out[4] += vf * N2 * (N1 // 2) * m1 * OPS_FWD_BFLY
        # the forward row pass runs inside the inverse row pass where folded
        out[6 if folded_rows(d, 3) else 5] += vf * (N * OPS_TWIDDLE + N1 * (N2 // 2) * m2 * OPS_FWD_BFLY)
        out[6] += vi * (N1 * (N2 // 2) * m2 * OPS_INV_BFLY + N * OPS_TWIDDLE) + 2 * N * pairs * OPS_MAC
        out[7] += vi * N2 * (N1 // 2) * m1 * OPS_INV_BFLY
        if fused_columns(d):
            out[7] += d["n"] * (vi // 2) * (OPS_CRT + OPS_ACC)
    return out


def source_digest():
    """SHA-256 of the kernel sources and their compile flags: every .h and
    every .hip file under csrc except the host-only plan layer (plan.hip
    holds no device code), and the flags build_lib compiles them with."""
    import hashlib
    from paper_2603_29129_amd import build_lib
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".h")) and f != "plan.hip":
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
            h.update(" ".join(build_lib.FLAGS + build_lib.SOURCE_FLAGS.get(f, [])).encode() + b"\0")
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE and
    WRITE_SIZE counter summary, scaled by the copy-kernel calibration; None
    when no summary exists or the kernel sources changed since it was taken."""
    import glob
    for path in sorted(glob.glob(os.path.join(PROFILES, "*hbm_traffic*.md"))):
        with open(path) as fh:
            text = fh.read()
        if "```json" not in text:
            continue
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        if blob.get("source_sha256") != source_digest() or kernel not in blob.get("kernels", {}):
            continue
        k, cal = blob["kernels"][kernel], blob["calibration"]
        return round(k["fetch_kib"] * 1024 * cal["fetch_factor"] + k["write_kib"] * 1024 * cal["write_factor"])
    return None


def algorithmic_bytes(infos, K):
    """Algorithmic HBM bytes per launch of each pass kernel, from the actual
    slice and group counts (each value read once and written once)."""
    out = {4: 0, 5: 0, 6: 0, 7: 0, 8: 0}
    kernels_seen = set()
    for d in infos:
        n, N = d["n"], d["N"]
        vecs = 2 * (d["kx"][0] + d["kx"][1])          # forward NTT vectors (part, slice, prime)
        grp = 2 * sum(d["ngroups"])                    # inverse NTT vectors (group, prime)
        out[4] += vecs * (4 * n + 4 * N)               # read the n non-zero inputs, write N
        if not folded_rows(d, K):
            out[5] += vecs * 8 * N                     # read + write N
        out[6] += vecs * 4 * N + grp * 4 * N           # read the slice spectra, write the group rows
        key = (n, N)
        if key not in kernels_seen:                    # kernel spectra + Shoup companions, once per length
            kernels_seen.add(key)
            out[6] += 2 * (d["kw"][0] + d["kw"][1]) * 8 * N
        if fused_columns(d):
            out[7] += grp * 4 * N + 16 * n + 16 * n    # read the group rows; chirp in, y out
        else:
            out[7] += grp * (4 * N + 4 * n)            # read N, write the first n
            out[8] += grp * 4 * n + 16 * n + 16 * n    # residues + chirp in, y out
    return out


def time_events(torch, fn, reps):
    s = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(s)
    fn(reps)
    b.record(s)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def longdouble_errors(np, y, x):
    """Relative l2 and maximum componentwise relative error of y against the
    DFT of x computed in long double (numpy's FFT on clongdouble)."""
    ref = np.fft.fft(np.asarray(x).astype(np.clongdouble))
    yl = np.asarray(y).astype(np.clongdouble)
    rel = float(np.sqrt(np.sum(np.abs(yl - ref) ** 2)) / np.sqrt(np.sum(np.abs(ref) ** 2)))
    mx = 0.0
    for a, b in ((yl.real, ref.real), (yl.imag, ref.imag)):
        m = b != 0
        if np.any(m):
            mx = max(mx, float(np.max(np.abs((a[m] - b[m]) / b[m]))))
    return rel, mx


_ORACLE_PLAN = None


def _oracle_init(plan):
    global _ORACLE_PLAN
    _ORACLE_PLAN = plan


def _oracle_one(x):
    from oracle import bluestein as bl
    bl.forward_trace(x, 3, 3, _ORACLE_PLAN)
    return 1


def host_cpu():
    """The host's logical CPU count, the CPUs this process may run on and
    the processor model line."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_count": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)), "model": model}


def cpu_baseline(xs, n, budget_s, max_procs=16):
    """The oracle, as it is, on transforms of the same workload: one process
    transform after transform until about budget_s seconds have passed (at
    least one), then all transforms of the batch spread over a pool of
    processes (at most max_procs, the GPU host's CPU share).  The kernel plan
    is input independent and not timed (as on the GPU)."""
    import multiprocessing as mp
    from oracle import bluestein as bl
    # same embedding as the GPU plan (cyclic N = n for a power-of-two n)
    plan = bl.KernelPlan(n, 3, 3, cyclic=bl.is_pow2(n))
    t0 = time.perf_counter()
    done = 0
    while done < len(xs) and (done == 0 or time.perf_counter() - t0 < budget_s):
        bl.forward_trace(xs[done], 3, 3, plan)
        done += 1
    dt = time.perf_counter() - t0
    flop = 5.0 * n * math.log2(n)
    host = host_cpu()
    procs = max(1, min(max_procs, host["usable_cpus"], len(xs)))
    with mp.get_context("spawn").Pool(procs, initializer=_oracle_init, initargs=(plan,)) as pool:
        # every worker started and holding the plan (bounded waits: a worker
        # that dies would otherwise leave the pool waiting)
        pool.map_async(_oracle_init, [plan] * procs).get(timeout=600)
        t1 = time.perf_counter()
        pool.map_async(_oracle_one, list(xs), chunksize=1).get(timeout=600)
        dt_pool = time.perf_counter() - t1
    return {"value": round(len(xs) * flop / dt_pool / 1e9, 6), "unit": "GFLOP/s", "cores": procs,
            "kind": "oracle",
            "sample": f"all {len(xs)} transforms of the same workload (n={n}), K=3, L=3, kernel plan precomputed, "
                      f"one transform per task over {procs} worker processes (numpy/Python-int oracle, "
                      f"single-threaded per process); {dt_pool:.1f} s wall",
            "seconds": round(dt_pool, 2),
            "single_process": {"value": round(done * flop / dt / 1e9, 6), "cores": 1, "transforms": done,
                               "seconds": round(dt, 2)},
            "host": host}


def events_ms(torch, fn, reps, warmup=20):
    """Device time per call of fn() between HIP events on torch's current
    stream (the stream the library launches on), after warmup calls."""
    for _ in range(warmup):
        fn()
    return time_events(torch, lambda k: [fn() for _ in range(k)], reps)


def gflops(lengths, ms):
    return round(sum(5.0 * n * math.log2(n) for n in lengths if n > 1) / (ms * 1e-3) / 1e9, 2)


def config_plain_1k(np, torch, oz, wl, reps):
    """n = 2^10, one transform, uniform[-1, 1] (seed 0): latency of the
    batched form (graph replay) and of the plain form (one launch per NTT,
    host synchronisations included), same bits."""
    x = wl.plain_1k(seed=0)
    xd = torch.from_numpy(x).cuda()
    out = {}
    ys = {}
    for mode in ("batched", "plain"):
        plan = oz.Plan(1024, 1, mode=mode)
        y = torch.empty_like(xd)
        ms = events_ms(torch, lambda: plan.forward(xd, y), reps)
        ys[mode] = y.cpu().numpy()
        out[mode] = {"ms": round(ms, 4), "GFLOPs": gflops([1024], ms)}
        plan.close()
    rel, mx = longdouble_errors(np, ys["batched"][0], x[0])
    out.update({"N": 1024, "rel_l2_error": rel, "max_rel_error": mx,
                "plain_bit_identical": bool(np.array_equal(ys["plain"].view(np.uint64), ys["batched"].view(np.uint64)))})
    return out


def config_batch64(np, torch, oz, wl, reps, n, gen):
    """64 transforms of length n, uniform[-1, 1] (seed 0): forward and
    inverse (batched form), the round trip's largest error relative to the
    largest input magnitude."""
    x = gen(seed=0)
    xd = torch.from_numpy(x).cuda()
    plan = oz.Plan(n, x.shape[0])
    y = torch.empty_like(xd)
    z = torch.empty_like(xd)
    ms_f = events_ms(torch, lambda: plan.forward(xd, y), reps)
    ms_i = events_ms(torch, lambda: plan.inverse(y, z), reps)
    rel, mx = longdouble_errors(np, y[0].cpu().numpy(), x[0])
    rt = float((z - xd).abs().max() / xd.abs().max())
    info = plan.transform_info(0)
    plan.close()
    return {"n": n, "batch": int(x.shape[0]), "N": info["N"], "forward_ms": round(ms_f, 4),
            "forward_GFLOPs": gflops([n] * x.shape[0], ms_f), "inverse_ms": round(ms_i, 4),
            "inverse_GFLOPs": gflops([n] * x.shape[0], ms_i), "rel_l2_error": rel, "max_rel_error": mx,
            "round_trip_max_error": rt}


def config_mixed_256(np, torch, oz, wl, reps):
    """256 transforms, lengths log-uniform in [2^10, 2^16] (every third moved
    to a prime), uniform[-1, 1] entries, one graph replay per step; the plan
    is autotuned (tile shapes of its length classes)."""
    ns, xs = wl.mixed_256(seed=0)
    x = np.concatenate(xs)
    xd = torch.from_numpy(x).cuda()
    out = {"transforms": len(ns), "total_length": int(sum(ns)), "length_classes": None}
    for tag, kw in (("default", {}), ("autotuned", {"autotune": True})):
        plan = oz.Plan(lengths=ns, **kw)
        y = torch.empty_like(xd)
        ms = events_ms(torch, lambda: plan.forward(xd, y), reps)
        out[tag] = {"ms": round(ms, 4), "GFLOPs": gflops(ns, ms)}
        out["length_classes"] = plan.info()["num_length_classes"]
        if tag == "default":
            y0 = y.cpu().numpy()
        else:
            out["autotuned"]["bit_identical_to_default"] = bool(np.array_equal(y.cpu().numpy().view(np.uint64),
                                                                              y0.view(np.uint64)))
        plan.close()
    rel, mx = longdouble_errors(np, y0[:ns[0]], xs[0])
    out.update({"rel_l2_error_transform_0": rel, "max_rel_error_transform_0": mx})
    return out


def config_grad_64k(np, torch, oz, wl, reps):
    """32 x 2^16 uniform[-1, 1] (seed 0), weights uniform[0, 1] (seed 1):
    forward + backward of loss = sum(w |DFT(x)|^2) through OzakiDFT (the
    backward is the adjoint DFT through the same pipeline)."""
    x, w = wl.grad_64k(seed=0)
    xd = torch.from_numpy(x).cuda()
    wd = torch.from_numpy(w).cuda()

    def step():
        xx = xd.detach().requires_grad_(True)
        y = oz.OzakiDFT.apply(xx)
        loss = (wd * (y.real ** 2 + y.imag ** 2)).sum()
        loss.backward()
        return xx.grad

    ms = events_ms(torch, step, reps)
    n, B = x.shape[1], x.shape[0]
    return {"n": n, "batch": B, "ms_forward_backward": round(ms, 4),
            "GFLOPs": gflops([n] * (2 * B), ms), "transforms_per_step": 2 * B}


def rotating_buffers(np, torch, oz, plan, xd, out_ref, reps, pairs=8):
    """The headline plan executed over `pairs` (in, out) pairs in turn (one
    captured graph, its array pointers rebound per call) against the same
    plan on one fixed pair; the outputs of every pair equal the headline's."""
    xs = [xd.clone() for _ in range(pairs)]
    outs = [torch.empty_like(xd) for _ in range(pairs)]
    state = {"i": 0}

    def one():
        i = state["i"] % pairs
        plan.forward(xs[i], outs[i])
        state["i"] += 1

    ms_rot = events_ms(torch, one, reps * pairs, warmup=pairs)
    ms_fix = events_ms(torch, lambda: plan.forward(xd, out_ref), reps)
    same = all(torch.equal(o.view(torch.float64), out_ref.view(torch.float64)) for o in outs)
    return {"pairs": pairs, "ms_per_call_rotating": round(ms_rot, 4), "ms_per_call_fixed_pair": round(ms_fix, 4),
            "bit_identical": bool(same)}


def config_per_conv(np, torch, oz, xd, out_ref, reps):
    """The headline input through the paper's schedule (Alg. 8 for each real
    convolution, 12 + 40 NTTs per transform) instead of the library's
    complex accumulation (12 + 20); same bits."""
    n, B = xd.shape[1], xd.shape[0]
    plan = oz.Plan(n, B, accumulation="per_conv")
    y = torch.empty_like(xd)
    ms = events_ms(torch, lambda: plan.forward(xd, y), reps)
    i0 = plan.transform_info(0)
    res = {"ms_per_step": round(ms, 4), "value": gflops([n] * B, ms),
           "ntt_counts": {"forward_runtime": i0["forward_runtime"], "inverse": i0["inverse"]},
           "bit_identical_to_headline": bool(torch.equal(y.view(torch.float64), out_ref.view(torch.float64)))}
    plan.close()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    # about 0.1 s of timed steps after 50 ms of warmup: with 20 steps the
    # timed window (10 ms) still held the GPU's clock ramp (5-7% slower)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n", type=int, default=1 << 18)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--stage-reps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (for HBM counter calibration)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other configurations (n = 2^10, 64 x 2^14, 64 x 10007, 256 mixed lengths, "
                         "32 x 2^16 forward + backward)")
    ap.add_argument("--config-reps", type=int, default=100)
    ap.add_argument("--only-config", default=None,
                    choices=["plain_1k", "batch_16k", "batch_prime", "mixed_256", "grad_64k"],
                    help="run only this configuration and print its figures (for profiling)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(transforms shard by batch with no communication; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2603_29129_amd as oz
    import workloads as wl

    if args.only_config:
        r = args.config_reps
        c = args.only_config
        res = {"plain_1k": lambda: config_plain_1k(np, torch, oz, wl, r),
               "batch_16k": lambda: config_batch64(np, torch, oz, wl, r, 16384, wl.batch_16k),
               "batch_prime": lambda: config_batch64(np, torch, oz, wl, r, 10007, wl.batch_prime),
               "mixed_256": lambda: config_mixed_256(np, torch, oz, wl, r),
               "grad_64k": lambda: config_grad_64k(np, torch, oz, wl, r)}[c]()
        torch.cuda.synchronize()
        print(json.dumps({"config": c, **res}), flush=True)
        return

    n, B = args.n, args.batch
    print(f"# bench: n={n} batch={B} steps={args.steps} warmup={args.warmup}", file=sys.stderr, flush=True)
    x = wl.wide_256k(seed=0, batch=B, n=n)
    xd = torch.from_numpy(x).cuda()
    out = torch.empty_like(xd)
    flops = B * 5.0 * n * math.log2(n)

    plan = oz.Plan(n, B, mode="batched")
    for _ in range(args.warmup):
        plan.forward(xd, out)
    torch.cuda.synchronize()

    def run(k):
        for _ in range(k):
            plan.forward(xd, out)

    ms = time_events(torch, run, args.steps)
    value = flops / (ms * 1e-3) / 1e9
    # the pass kernels' device times where they run: right after the timed
    # region, steps of the same sequence launched on the stream with HIP
    # events at the stage boundaries (HIP takes no timestamps inside a graph
    # replay); the mean over the steps
    plan.stage_timing(True)
    seq = []
    for i in range(10 + args.stage_reps * 2):
        plan.forward(xd, out)
        if i >= 10:
            seq.append(plan.stage_times())
    plan.stage_timing(False)
    graph_times = {"split": statistics.mean(t["split"] for t in seq),
                   "classes": [{k: statistics.mean(t["classes"][c][k] for t in seq) for k in seq[0]["classes"][c]}
                               for c in range(len(seq[0]["classes"]))]}
    print(f"# batched: {ms:.3f} ms/step, {value:.1f} GFLOP/s", file=sys.stderr, flush=True)

    # the padded embedding (N = 2^ceil(log2(2n-1))) on the same input
    pplan_pad = oz.Plan(n, B, mode="batched", cyclic=False)
    out_pad = torch.empty_like(xd)
    for _ in range(args.warmup):
        pplan_pad.forward(xd, out_pad)
    torch.cuda.synchronize()
    ms_pad = time_events(torch, lambda k: [pplan_pad.forward(xd, out_pad) for _ in range(k)], args.steps)
    padded = {"N": pplan_pad.transform_info(0)["N"], "ms_per_step": round(ms_pad, 4),
              "value": round(flops / (ms_pad * 1e-3) / 1e9, 2),
              "bit_identical_to_headline": bool(torch.equal(out_pad.view(torch.float64), out.view(torch.float64)))}
    pplan_pad.close()
    del out_pad
    print(f"# padded embedding: {ms_pad:.3f} ms/step", file=sys.stderr, flush=True)

    # binary32 target precision (complex64 in and out, K = 2) on the same
    # input rounded to binary32; its error against the long-double DFT of
    # that input and the error of the exact DFT rounded to binary32
    x32 = x.astype(np.complex64)
    x32d = torch.from_numpy(x32).cuda()
    out32 = torch.empty_like(x32d)
    plan32 = oz.Plan(n, B, mode="batched", precision="fp32")
    for _ in range(args.warmup):
        plan32.forward(x32d, out32)
    torch.cuda.synchronize()
    ms32 = time_events(torch, lambda k: [plan32.forward(x32d, out32) for _ in range(k)], args.steps)
    i32 = plan32.transform_info(0)
    ref32 = np.fft.fft(x32[0].astype(np.clongdouble))
    rel32 = lambda v: float(np.sqrt(np.sum(np.abs(np.asarray(v).astype(np.clongdouble) - ref32) ** 2))
                            / np.sqrt(np.sum(np.abs(ref32) ** 2)))
    binary32 = {"K": plan32.K, "ms_per_step": round(ms32, 4), "value": round(flops / (ms32 * 1e-3) / 1e9, 2),
                "rel_l2_error": rel32(out32[0].cpu().numpy()),
                "rel_l2_error_of_rounded_exact_dft": rel32(ref32.astype(np.complex128).astype(np.complex64)),
                "ntt_counts": {"forward_runtime": i32["forward_runtime"], "inverse": i32["inverse"],
                               "forward_offline": i32["forward_offline"]}}
    plan32.close()
    del x32d, out32
    print(f"# binary32 target (K=2): {ms32:.3f} ms/step", file=sys.stderr, flush=True)

    # one transform of the same workload (the configuration's single case),
    # batched form: latency of one n = 2^18 transform
    plan1 = oz.Plan(n, 1, mode="batched")
    x1 = xd[:1].contiguous()
    out1 = torch.empty_like(x1)
    for _ in range(args.warmup):
        plan1.forward(x1, out1)
    torch.cuda.synchronize()
    ms1 = time_events(torch, lambda k: [plan1.forward(x1, out1) for _ in range(k)], args.steps)
    single = {"batch": 1, "ms_per_step": round(ms1, 4), "value": round(5.0 * n * math.log2(n) / (ms1 * 1e-3) / 1e9, 2),
              "bit_identical_to_headline_transform_0": bool(torch.equal(out1.view(torch.float64),
                                                                        out[:1].view(torch.float64)))}
    plan1.close()
    del out1, x1
    print(f"# single transform: {ms1:.3f} ms", file=sys.stderr, flush=True)

    # three CRT moduli (d = 3): K = 2 slices of alpha = 36 bits, same input
    # and output type, the same kernels with three primes per group
    plan3 = oz.Plan(n, B, mode="batched", primes=3)
    out3 = torch.empty_like(xd)
    for _ in range(args.warmup):
        plan3.forward(xd, out3)
    torch.cuda.synchronize()
    ms3 = time_events(torch, lambda k: [plan3.forward(xd, out3) for _ in range(k)], args.steps)
    i3 = plan3.transform_info(0)
    rel3, maxrel3 = longdouble_errors(np, out3[0].cpu().numpy(), x[0])
    three_moduli = {"K": plan3.K, "alpha": i3["alpha"], "acc_limit": i3["acc_limit"], "ms_per_step": round(ms3, 4),
                    "value": round(flops / (ms3 * 1e-3) / 1e9, 2), "rel_l2_error": rel3, "max_rel_error": maxrel3,
                    "ntt_counts": {"forward_runtime": i3["forward_runtime"], "inverse": i3["inverse"],
                                   "forward_offline": i3["forward_offline"]}}
    three_moduli["stages_ms"] = {st: round(time_events(torch, lambda k, st=st: plan3.profile_stage(st, k),
                                                       args.stage_reps), 4) for st in (1, 2, 4, 5, 6, 7, 8)}
    plan3.close()
    # the same with L = 12: alpha = 35, a CRT bound of 14 products, 3 groups per component
    plan3b = oz.Plan(n, B, mode="batched", primes=3, L=12)
    for _ in range(args.warmup):
        plan3b.forward(xd, out3)
    torch.cuda.synchronize()
    ms3b = time_events(torch, lambda k: [plan3b.forward(xd, out3) for _ in range(k)], args.steps)
    i3b = plan3b.transform_info(0)
    three_moduli["L12"] = {"alpha": i3b["alpha"], "acc_limit": i3b["acc_limit"], "ms_per_step": round(ms3b, 4),
                           "value": round(flops / (ms3b * 1e-3) / 1e9, 2),
                           "rel_l2_error": longdouble_errors(np, out3[0].cpu().numpy(), x[0])[0],
                           "ntt_counts": {"forward_runtime": i3b["forward_runtime"], "inverse": i3b["inverse"]}}
    plan3b.close()
    del out3
    print(f"# three moduli (K=2, alpha={i3['alpha']}): {ms3:.3f} ms/step; L=12 (alpha={i3b['alpha']}): "
          f"{ms3b:.3f} ms/step", file=sys.stderr, flush=True)

    y = out.cpu().numpy()
    infos = [plan.transform_info(b) for b in range(B)]
    rel, maxrel = longdouble_errors(np, y[0], x[0])

    # per-stage device times (same buffers, one launch of each stage per rep)
    stage_ms = {}
    for st in (1, 2, 4, 5, 6, 7, 8):
        stage_ms[st] = time_events(torch, lambda k, st=st: plan.profile_stage(st, k), args.stage_reps)
    plan.forward(xd, out)             # restore a consistent state
    torch.cuda.synchronize()
    print("# stages (ms): " + ", ".join(f"{k}:{v:.3f}" for k, v in stage_ms.items()), file=sys.stderr, flush=True)

    alg = algorithmic_bytes(infos, 3)
    ops = algorithmic_ops(infos)
    names = stage_kernels(infos[0], 3)
    # pass times in sequence (one length class): forward column pass (the
    # forward row pass is folded into the inverse row pass), inverse row
    # pass, fused column pass, wide-span recombination
    gc = graph_times["classes"][0]
    graph_ms = {4: gc["forward"], 6: gc["rows"], 7: gc["cols"], 8: gc["recombine"]}
    if names[5]:                      # forward row pass not folded: the forward time spans two kernels
        del graph_ms[4]
    # the dominant kernel (longest pass) is bound by its integer VALU work
    dom = max((s for s in (4, 6, 7) if names[s] and s in graph_ms), key=lambda s: graph_ms[s])
    t_dom = graph_ms[dom]
    achieved = ops[dom] / (t_dom * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 2), "unit": "TOP/s",
                "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": measured_traffic(names[dom]),
                "kernel": names[dom], "kernel_ms": round(t_dom, 4),
                "kernel_ms_timing": f"HIP events at the stage boundaries of the step's launch sequence on the stream, "
                                    f"mean of {len(seq)} steps after the timed region",
                "algorithmic_int32_ops_per_launch": ops[dom], "algorithmic_bytes_per_launch": alg[dom],
                "hbm_achieved_GBps": round(alg[dom] / (t_dom * 1e-3) / 1e9, 1),
                "hbm_frac": round(alg[dom] / (t_dom * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    per_kernel = {}
    for s in PASS_STAGES:
        if names[s] is None or s not in graph_ms:
            continue
        t = graph_ms[s]
        e = {"ms": round(t, 4), "ms_stage_repetitions": round(stage_ms[s], 4),
             "alg_GBps": round(alg[s] / (t * 1e-3) / 1e9, 1), "traffic": measured_traffic(names[s])}
        if s in ops:
            e["alu_TOPs"] = round(ops[s] / (t * 1e-3) / 1e12, 3)
            e["alu_frac"] = round(ops[s] / (t * 1e-3) / 1e12 / ALU_PEAK_TOPS, 4)
        per_kernel[names[s]] = e

    plain = None
    if not args.no_plain:
        pplan = oz.Plan(n, B, mode="plain")
        pout = torch.empty_like(xd)
        pplan.forward(xd, pout)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            pplan.forward(xd, pout)
        torch.cuda.synchronize()
        pms = (time.perf_counter() - t0) * 1e3 / args.plain_steps
        same = bool(torch.equal(pout.view(torch.float64), out.view(torch.float64)))
        pms_dev = events_ms(torch, lambda: pplan.forward(xd, pout), args.plain_steps, warmup=0)
        plain = {"ms_per_step": round(pms, 3), "value": round(flops / (pms * 1e-3) / 1e9, 2),
                 "batched_over_plain": round(pms / ms, 2), "bit_identical_to_batched": same,
                 "timing": "host wall clock (the plain form synchronises the host)",
                 "device_event_ms": round(pms_dev, 3),
                 "batched_over_plain_device_events": round(pms_dev / ms, 2)}
        pplan.close()
        print(f"# plain: {pms:.3f} ms/step", file=sys.stderr, flush=True)

    configs = None
    rotating = rotating_buffers(np, torch, oz, plan, xd, out, args.steps)
    print(f"# {rotating['pairs']} rotating buffer pairs: {rotating['ms_per_call_rotating']:.3f} ms per call "
          f"(fixed pair {rotating['ms_per_call_fixed_pair']:.3f})", file=sys.stderr, flush=True)
    per_conv = config_per_conv(np, torch, oz, xd, out, args.steps)
    print(f"# per-convolution schedule: {per_conv['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    if not args.no_configs:
        r = args.config_reps
        configs = {"plain_1k": config_plain_1k(np, torch, oz, wl, r)}
        print(f"# n=2^10: {configs['plain_1k']['batched']['ms']:.4f} ms batched, "
              f"{configs['plain_1k']['plain']['ms']:.4f} ms plain", file=sys.stderr, flush=True)
        configs["batch_16k"] = config_batch64(np, torch, oz, wl, r, 16384, wl.batch_16k)
        configs["batch_prime"] = config_batch64(np, torch, oz, wl, r, 10007, wl.batch_prime)
        print(f"# 64 x 2^14: {configs['batch_16k']['forward_ms']:.3f} ms, 64 x 10007: "
              f"{configs['batch_prime']['forward_ms']:.3f} ms", file=sys.stderr, flush=True)
        configs["mixed_256"] = config_mixed_256(np, torch, oz, wl, r)
        print(f"# 256 mixed lengths: {configs['mixed_256']['default']['ms']:.3f} ms "
              f"(autotuned {configs['mixed_256']['autotuned']['ms']:.3f} ms)", file=sys.stderr, flush=True)
        configs["grad_64k"] = config_grad_64k(np, torch, oz, wl, r)
        print(f"# 32 x 2^16 forward+backward: {configs['grad_64k']['ms_forward_backward']:.3f} ms",
              file=sys.stderr, flush=True)

    if args.calibrate_copy:
        a = torch.empty(1 << 25, dtype=torch.float64, device="cuda").fill_(1.0)
        for _ in range(5):
            a.clone()
        torch.cuda.synchronize()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(x, n, 12.0)
        print(f"# cpu oracle: {cpu['single_process']['seconds']} s (1 process), {cpu['seconds']} s "
              f"({cpu['cores']} processes)", file=sys.stderr, flush=True)

    counts = infos[0]
    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "dtype_note": "32-bit modular integer NTT/CRT; binary64 chirp, split and recombination",
        "data": "synthetic",
        "config": {"workload": "wide_256k: 8 transforms, n=2^18, |x| log-uniform in [2^-30,2^30], "
                               "uniform phase, seed 0; batched form (HIP graph replay)",
                   "n": n, "batch": B, "K": 3, "L": 3, "N": infos[0]["N"],
                   "embedding": "cyclic N=n for power-of-two n (Sec. 3.2)" if infos[0]["N"] == n else "padded",
                   "parallelism": "single GPU"},
        "padded_embedding": padded,
        "binary32_target": binary32,
        "three_moduli": three_moduli,
        "single_transform": single,
        "rel_l2_error": rel,
        "max_rel_error": maxrel,
        "ntt_counts": {"forward_runtime": counts["forward_runtime"], "inverse": counts["inverse"],
                       "forward_offline": counts["forward_offline"]},
        "plain": plain,
        "rotating_buffers": rotating,
        "per_conv_schedule": per_conv,
        "configs": configs,
        "stages_ms": {str(k): round(v, 4) for k, v in stage_ms.items()},
        "sequence_stage_ms": {"split": round(graph_times["split"], 4),
                           **{k: round(v, 4) for k, v in graph_times["classes"][0].items()}},
        "per_kernel": per_kernel,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
