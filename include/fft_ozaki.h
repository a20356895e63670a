/*
 * fft_ozaki.h -- C ABI of an FP64-accurate discrete Fourier transform for
 * AMD Instinct MI355X (gfx950), computed as in Kawakami & Takahashi,
 * "Computing FFTs at Target Precision Using Lower-Precision FFTs":
 *
 *   y = DFT(x),  y(k) = sum_j x(j) w_n^{jk},  w_n = exp(-2 pi i / n)
 *   (Sec. 3.2, Eq. dft; the inverse carries 1/n, Eq. idft),
 *
 * by Bluestein's algorithm (Sec. 3.2, Alg. 1) whose cyclic convolution is
 * split into integer slices by the Ozaki scheme (Alg. 3, with the split cap K
 * of Sec. 4.4), convolved exactly by 32-bit NTTs modulo p0 = 2130706433 and
 * p1 = 2113929217 with NTT-domain accumulation of at most L products
 * (Alg. 8), rebuilt by Garner's CRT (Sec. 3.3) and recombined to binary64.
 * Optionally a third modulus p2 = 2013265921 widens the CRT range (Sec. 3.3
 * with d = 3 moduli, see fft_ozaki_options.primes).
 * The four real convolutions of the complex convolution share their splits
 * (Sec. 4.5) and the kernel's splits and NTTs are computed once per plan
 * (Sec. 4.5, precomputed offline).  Outputs are deterministic: the integer
 * stages are exact and every binary64 operation has a fixed order; the
 * recombination is an exact sum rounded once.
 *
 * Conventions
 * -----------
 *  * Every function returns an int status: FFT_OZAKI_OK (0) or a negative
 *    FFT_OZAKI_ERR_* code.  fft_ozaki_error_string() describes a code;
 *    fft_ozaki_last_error_message() gives the detail of the last failure on
 *    the calling thread.
 *  * Complex data are arrays of interleaved binary64 pairs (re, im), i.e.
 *    double2 / complex128, 16-byte aligned (for an FFT_OZAKI_PREC_FP32
 *    plan: binary32 pairs, complex64, 8-byte aligned), in DEVICE memory of
 *    the device that was current when the plan was created.  Transform i occupies
 *    elements [off_i, off_i + n_i) where off_i is the sum of the preceding
 *    lengths; a uniform batch is therefore a row-major [batch][n] array.
 *    in == out is allowed.
 *  * A plan owns all device workspace (chirps, twiddles, kernel NTTs, slice
 *    and accumulator buffers).  The caller owns in, out and the stream.
 *  * `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Executions are asynchronous in the batched mode and synchronous (the
 *    host waits on `stream`) in the plain mode.  One execution may be in
 *    flight per plan.
 *  * Data-dependent faults are not returned by the call: a transform whose
 *    premultiplied input contains NaN/Inf (status bit 1) or whose largest
 *    value lies outside the supported exponent range, roughly 2^-1000 ..
 *    2^990 (status bit 2), has its output set to NaN; read the per-transform
 *    status with fft_ozaki_query_transform() after synchronising.
 */
#ifndef FFT_OZAKI_H
#define FFT_OZAKI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fft_ozaki_plan_s* fft_ozaki_plan_t;

enum {
  FFT_OZAKI_OK = 0,
  FFT_OZAKI_ERR_INVALID = -1,      /* bad argument (sizes, K, L, pointers, direction) */
  FFT_OZAKI_ERR_NOMEM = -2,        /* device or host allocation failed */
  FFT_OZAKI_ERR_HIP = -3,          /* a HIP runtime call or kernel launch failed */
  FFT_OZAKI_ERR_UNSUPPORTED = -4   /* valid request the library cannot serve */
};

enum {
  FFT_OZAKI_FORWARD = 0,           /* y = DFT(x) */
  FFT_OZAKI_INVERSE = 1,           /* y = conj(DFT(conj x)) / n  (= DFT^{-1}, Eq. idft) */
  FFT_OZAKI_ADJOINT = 2            /* y = conj(DFT(conj x))      (= DFT^H) */
};

enum {
  FFT_OZAKI_MODE_PLAIN = 0,        /* host-driven: one transform at a time, one kernel launch per NTT */
  FFT_OZAKI_MODE_BATCHED = 1       /* all transforms per launch, device-side schedule, HIP graph replay */
};

/* Convolution embedding (Sec. 3.2).  PADDED: cyclic convolution of length
 * N = 2^ceil(log2(2n-1)) with the input zero-padded and the chirp kernel
 * wrapped (ZeroPad, ZeroPad+-).  AUTO: for a power-of-two n the convolution
 * is already cyclic of length n (the chirp index j^2 mod 2n has period n
 * and is even in j for even n), so N = n and nothing is padded; other n
 * are padded.  Both give bit-identical outputs: the slices, groups and CRT
 * integers are the same, only the NTT length differs. */
enum {
  FFT_OZAKI_EMBED_PADDED = 0,
  FFT_OZAKI_EMBED_AUTO = 1
};

/* NTT-domain accumulation (Alg. 8, Sec. 4.4).  The complex convolution
 * x' (*) w* is four real convolutions: ReRe and ImIm give Re y' = ReRe - ImIm,
 * ImRe and ReIm give Im y' = ImRe + ReIm.  PER_CONV: Alg. 8 for each real
 * convolution on its own (a group holds at most L products of one
 * convolution), 2 inverse NTTs per group.  COMPLEX: the products of the two
 * convolutions of one output component are walked together, anti-diagonal by
 * anti-diagonal, and products of equal scale share a group (the ImIm ones
 * subtracted) up to acc_limit products, the most for which the signed sum
 * stays within the CRT range: acc_limit n 4^alpha <= (p0 p1 - 1) / 2.  Both
 * give bit-identical outputs (every output is the exact sum of all products,
 * rounded once); COMPLEX needs fewer inverse NTTs wherever the scales of the
 * real and imaginary parts agree. */
enum {
  FFT_OZAKI_ACCUM_PER_CONV = 0,
  FFT_OZAKI_ACCUM_COMPLEX = 1
};

/* Target precision (the method reaches a precision through the number of
 * splits, Sec. 6).  FP64: in / out are complex128 (interleaved binary64).
 * FP32: in / out are complex64; the input is widened exactly to binary64,
 * the transform runs as for FP64 with the plan's K, and each output
 * component is the binary64 result rounded once to binary32 (nearest even).
 * K = 2 (about 40 bits per part) suffices for binary32 targets. */
enum {
  FFT_OZAKI_PREC_FP64 = 0,
  FFT_OZAKI_PREC_FP32 = 1
};

/* Plan options.  K: cap on slices per vector (Sec. 4.4), 1..8, default 3.
 * L: NTT-domain accumulation bound (Sec. 4.4, Alg. 8), >= 1, default 3.
 * mode: FFT_OZAKI_MODE_*, default batched.  autotune: 1 = time the NTT tile
 * shapes at plan time and keep the fastest (results are identical for every
 * shape); tune_cache: optional file path where tuned shapes are stored and
 * looked up (NULL = none).  embedding: FFT_OZAKI_EMBED_*, default AUTO.
 * accumulation: FFT_OZAKI_ACCUM_*, default COMPLEX.  precision:
 * FFT_OZAKI_PREC_*, default FP64.  primes: number of CRT moduli, 2 (p0, p1;
 * default) or 3 (p0, p1 and p2 = 15 * 2^27 + 1, Sec. 3.3 with d = 3): the
 * split width then follows Sec. 4.2 with the product p0 p1 p2 (alpha = 36 at
 * n = 2^18, L = 3), so K = 2 slices of about 36 bits reach the binary64
 * accuracy that K = 3 needs with two moduli.  Three moduli: batched mode
 * only (FFT_OZAKI_ERR_UNSUPPORTED otherwise); group values reach 93 bits and
 * are rebuilt by Garner's mixed-radix form over the three moduli; the
 * buffers hold the three primes' residues where two-modulus plans hold two. */
typedef struct {
  int K;
  int L;
  int mode;
  int autotune;
  const char* tune_cache;
  int embedding;
  int accumulation;
  int precision;
  int primes;
} fft_ozaki_options;

/* Fills *opt with the defaults (K = 3, L = 3, batched, no autotune, AUTO
 * embedding, COMPLEX accumulation, FP64, two moduli). */
int fft_ozaki_default_options(fft_ozaki_options* opt);

/* Plan `batch` transforms of length n (uniform batch) with default options.
 * n >= 1 with convolution length N <= 2^24 (N = n for a power-of-two n,
 * else 2^ceil(log2(2n-1))); batch >= 1. */
int fft_ozaki_plan(fft_ozaki_plan_t* plan, int64_t n, int64_t batch);

/* Plan `count` transforms of the given (possibly different) lengths.
 * lengths: host array of `count` values, each as for fft_ozaki_plan.
 * opt may be NULL for the defaults.  Fails with FFT_OZAKI_ERR_INVALID when
 * the split width alpha = floor((log2(p0 p1 / 2) - log2(L n)) / 2) (Sec. 4.4)
 * would be < 1 or when L n 4^alpha > (p0 p1 - 1) / 2. */
int fft_ozaki_plan_ex(fft_ozaki_plan_t* plan, const int64_t* lengths, int64_t count,
                      const fft_ozaki_options* opt);

/* Execute the planned transforms in `direction` on device arrays in -> out. */
int fft_ozaki_execute(fft_ozaki_plan_t plan, const void* in, void* out, int direction, void* stream);
/* = fft_ozaki_execute(plan, in, out, FFT_OZAKI_FORWARD, stream) */
int fft_ozaki_forward(fft_ozaki_plan_t plan, const void* in, void* out, void* stream);
/* = fft_ozaki_execute(plan, in, out, FFT_OZAKI_INVERSE, stream) */
int fft_ozaki_inverse(fft_ozaki_plan_t plan, const void* in, void* out, void* stream);

/* Plan-level facts. */
typedef struct {
  int64_t count;                   /* number of transforms */
  int64_t total_length;            /* sum of the lengths */
  int K, L, mode, num_length_classes;
  int64_t workspace_bytes;         /* device memory held by the plan */
  int embedding;                   /* FFT_OZAKI_EMBED_* */
  int accumulation;                /* FFT_OZAKI_ACCUM_* */
  int precision;                   /* FFT_OZAKI_PREC_* */
  int primes;                      /* CRT moduli: 2 or 3 */
} fft_ozaki_info;
int fft_ozaki_query(fft_ozaki_plan_t plan, fft_ozaki_info* info);

/* Per-transform facts.  The data-dependent fields describe the last
 * execution and are valid once it has completed (the call synchronises the
 * device).  forward_runtime / inverse count the 32-bit NTTs performed per
 * execution, forward_offline those done once at plan time (Sec. 4.5). */
typedef struct {
  int64_t n, N;
  int alpha;
  int status;                      /* bit 1: non-finite input, bit 2: exponent range */
  int kx[2];                       /* slices of Re x', Im x' */
  int Ex[2][8];                    /* their exponents E = ceil(log2 max|r|) */
  int kw[2];                       /* slices of Re w*, Im w* */
  int Ew[2][8];
  int ngroups[2];                  /* accumulation groups of Re y', Im y' */
  int acc_limit;                   /* products per group: L (PER_CONV) or the CRT-range bound (COMPLEX) */
  int xsh[2];                      /* COMPLEX: slices of Re x', Im x' are taken times 2^xsh[part] (0, 1 or 2)
                                      and their products weigh 2^xsh[part] in a group; see debug stage 2 */
  int forward_runtime, forward_offline, inverse;
  int ntt_log2N1;                  /* NTT-domain layout: see fft_ozaki_ntt */
  int tile_cols_log2;              /* two-pass lengths: log2 of the columns per workgroup of the forward
                                      column pass (the autotuned shape when the plan was autotuned) */
  int tile_rows_log2;              /* log2 of the rows per workgroup of the standalone row passes */
} fft_ozaki_transform_info;
int fft_ozaki_query_transform(fft_ozaki_plan_t plan, int64_t index, fft_ozaki_transform_info* info);

/* Test hook: copy an intermediate buffer of transform `index` of the last
 * execution to host memory (synchronises the device).  P = the plan's CRT
 * moduli (2 or 3).  Stages:
 *   1  x' = x (.) w                          double2[n]  (not kept by the execution: rebuilt from its
 *                                            input, which must still hold the same values;
 *                                            FFT_OZAKI_ERR_UNSUPPORTED after an in-place execution)
 *   2  forward NTTs of the x' slices         uint32[2][K][P][N]  (part, slice, prime; NTT-domain order;
 *                                            part p's slices times 2^xsh[p], see fft_ozaki_transform_info)
 *   3  inverse NTT outputs per group         uint32[4*K*K][P][n4] (slot = component*2*K*K + group,
 *                                            component 0 = Re y', 1 = Im y'; prime;
 *                                            n4 = n rounded up to a multiple of 4, first n valid; where
 *                                            the batched form fuses the column pass with the CRT these
 *                                            are rebuilt from the stored row-pass output by the call)
 *   4  kernel NTTs times N^{-1}              uint32[2][K][P][N]
 *   5  chirp (cos, sin)                      double2[n]
 * `bytes` must be at least the stage size (FFT_OZAKI_ERR_INVALID otherwise);
 * the size is returned through *needed when not NULL. */
int fft_ozaki_debug_dump(fft_ozaki_plan_t plan, int stage, int64_t index, void* host_dst, size_t bytes,
                         size_t* needed);

/* Measurement hook: enqueue `reps` repetitions of one stage of the batched
 * schedule for all transforms of the plan, on `stream`, reusing the buffers
 * and the in/out pointers of the plan's last execution (they must still be
 * valid).  Stages: 1 split (premultiply, maxima, extraction passes),
 * 2 the accumulation schedule, 3 forward NTTs (both passes), 4 forward
 * column pass, 5 forward row pass, 6 inverse row pass with the fused
 * NTT-domain multiply-accumulate (for N <= 4096: the whole inverse),
 * 7 inverse column pass (for 2^13 <= N <= 2^18 fused with the CRT,
 * recombination and postmultiply; transforms whose exponent span needs the
 * wide accumulator only get their columns, written to the compact buffer),
 * 8 CRT/recombination/postmultiply (for the fused lengths: only those wide
 * transforms).  Stages 3-5 transform the slice
 * buffers again in place, so intermediates read with fft_ozaki_debug_dump
 * afterwards are not those of the last execution.  Batched plans only. */
int fft_ozaki_profile_stage(fft_ozaki_plan_t plan, int stage, int reps, void* stream);

/* Measurement hook: with enable != 0 every later batched execution of the
 * plan launches its kernels on `stream` itself, in the order of the captured
 * graph, with a HIP event recorded at each stage boundary (HIP records no
 * timestamps from inside a graph replay), so the device time of each stage
 * is taken where it runs, between its neighbours in the schedule and with
 * their data in the caches; enable = 0 returns to graph replays.  Batched
 * plans only; FFT_OZAKI_ERR_INVALID otherwise. */
int fft_ozaki_stage_timing(fft_ozaki_plan_t plan, int enable);

/* Device times in ms of the stages of the plan's last execution, which must
 * have run with stage timing on (FFT_OZAKI_ERR_INVALID otherwise); waits for
 * it to finish.  ms[0]: premultiply and split (from the state reset through
 * the last check); then for each length class c (the transforms of one
 * convolution length N; classes in the order in which their N first occurs
 * among the plan's transforms): ms[1 + 4c] forward NTTs
 * (with the folded row pass: the forward column pass), ms[2 + 4c] inverse
 * row pass (with the NTT-domain multiply-accumulate and the folded forward
 * rows; for N <= 4096 the whole inverse NTT), ms[3 + 4c] inverse column pass
 * (fused with the CRT, recombination and postmultiply where N1 <= 512),
 * ms[4 + 4c] the recombination launch (the wide-accumulator fallback where
 * fused).  *count (if not NULL) receives 1 + 4 x (length classes); an array
 * shorter than that (capacity) is FFT_OZAKI_ERR_INVALID. */
int fft_ozaki_stage_times(fft_ozaki_plan_t plan, float* ms, int capacity, int* count);

/* Release the plan and its device memory. */
int fft_ozaki_destroy(fft_ozaki_plan_t plan);

/* Static description of a status code; never NULL. */
const char* fft_ozaki_error_string(int status);
/* Detail of the last failing call on this thread ("" if none). */
const char* fft_ozaki_last_error_message(void);

/* The library's 32-bit NTT (Sec. 3.3, Eq. ntt / intt) on `count` contiguous
 * device vectors of length N = 2^log2N (1 <= N <= 2^24) modulo p0 (prime 0),
 * p1 (prime 1) or p2 = 2013265921 (prime 2, the third modulus of the
 * three-modulus plans), in place.  The forward transform reads natural order and
 * writes the NTT-domain order: position i1 * N2 + i2 holds X(br(i1) + N1 br(i2))
 * with N1 = 2^ntt_log2N1 (from fft_ozaki_ntt_layout), N2 = N / N1 and br the
 * bit reversal on log2 N1 resp. log2 N2 bits.  The inverse reads that order
 * and writes natural order including the factor N^{-1}.  Inputs must be
 * residues in [0, p). */
int fft_ozaki_ntt(int prime, int log2N, int64_t count, void* data, int inverse, void* stream);
int fft_ozaki_ntt_layout(int log2N, int* log2N1);

/* Allocation-free execution, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the forward / inverse / adjoint DFT of `batch` transforms of
 * length n with the default options (as fft_ozaki_plan(n, batch) followed by
 * fft_ozaki_execute; outputs are the same bit for bit), in -> out on device
 * arrays laid out as for fft_ozaki_execute, asynchronous on `stream`.
 *
 * All tables and buffers live in one region of device memory that the
 * library reserves statically, FFT_OZAKI_STATIC_WORKSPACE_BYTES per device
 * it runs on, held until the process ends; the call allocates and frees no
 * device memory (host bookkeeping only).  The region keeps the tables of the
 * last (n, batch): a call with another (n, batch) rebuilds them first, which
 * waits for `stream` and for the device (so it cannot be captured into a
 * graph: make one call with the size before capturing); calls with the size
 * of the previous call only enqueue kernels.  Sizes whose workspace would
 * exceed the region are rejected with FFT_OZAKI_ERR_INVALID before any device
 * call (the region holds up to 183 transforms of n = 2^10, 6 of n = 2^14 or
 * one of n = 2^16).
 * Every call on a device shares that device's region: calls that overlap on
 * one device (other streams, other threads) race and must be serialised by
 * the caller.  Data-dependent faults give NaN outputs as in the planned form;
 * the per-transform status is not queryable here. */
#define FFT_OZAKI_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int fft_ozaki_execute_static(int64_t n, int64_t batch, const void* in, void* out, int direction, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FFT_OZAKI_H */
