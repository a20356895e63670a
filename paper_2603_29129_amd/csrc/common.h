// Shared constants, modular arithmetic and plan-side data structures of the
// gfx950 implementation of the FP64-accurate DFT by Bluestein's algorithm,
// Ozaki integer slices and two-prime 32-bit NTT convolution (Kawakami &
// Takahashi, "Computing FFTs at Target Precision Using Lower-Precision FFTs").
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fo {

typedef uint32_t u32;
typedef uint64_t u64;
typedef int64_t i64;

// ---------------------------------------------------------------------------
// Moduli (Sec. 5.1): p0 = 127*2^24 + 1, p1 = 63*2^25 + 1, both < 2^31 so that
// 2p < 2^32 and every residue fits a 32-bit lane.
constexpr u32 P0 = 2130706433u;
constexpr u32 P1 = 2113929217u;
constexpr u32 G0 = 3u;   // primitive root mod p0
constexpr u32 G1 = 5u;   // primitive root mod p1
// Garner constant p0^{-1} mod p1 (Sec. 3.3) and its Shoup companion.
constexpr u32 P0_INV_MOD_P1 = 2113929091u;
constexpr u64 PP = (u64)P0 * (u64)P1;           // 4504162581568552961 < 2^62
constexpr u64 PP_HALF = (PP - 1) / 2;
constexpr int MAX_LOG2_N = 24;                  // 2^24 = gcd(p0-1, p1-1)
// Third modulus of the d = 3 CRT variant (Sec. 3.3 with three moduli):
// p2 = 15*2^27 + 1 < 2^31, smallest primitive root 31.
constexpr u32 P2 = 2013265921u;
constexpr u32 G2 = 31u;
constexpr int NPRIME_MAX = 3;

// Splitting limits.
constexpr int KMAX = 8;                         // cap on slices per vector
constexpr int MANTISSA = 53;                    // log2(u^{-1}) for binary64
constexpr int EMIN_GRID = -1022;                // smallest slice grid exponent E - alpha
constexpr int MAX_PAIRS = KMAX * KMAX;

// Status bits per transform.
constexpr int ST_NONFINITE = 1;
constexpr int ST_RANGE = 2;

// Block (single workgroup) NTT limit and twiddle table base.
constexpr int LOG2_BLOCK_MAX = 12;
constexpr int BLOCK_MAX = 1 << LOG2_BLOCK_MAX;

// Recombination accumulator widths (64-bit words).  The fast path covers
// exponent spans up to 64*W_FAST - 67 bits; the wide path covers every span
// that the exponent range rules allow.
constexpr int W_FAST = 4;
constexpr int W_WIDE = 50;

// ---------------------------------------------------------------------------
// Modular arithmetic on 32-bit lanes (all results in [0, p)).
//
// Shoup multiplication by a constant w with companion wq = floor(w 2^32 / p):
// q = floor(x wq / 2^32) and t = x w - q p lies in [0, 2p) for any x < 2^32.
__host__ __device__ __forceinline__ u32 umin32(u32 a, u32 b) { return a < b ? a : b; }
__host__ __device__ __forceinline__ u32 shoup_mul(u32 x, u32 w, u32 wq, u32 p) {
#ifdef __HIP_DEVICE_COMPILE__
  u32 q = __umulhi(x, wq);
#else
  u32 q = (u32)(((u64)x * wq) >> 32);
#endif
  u32 t = x * w - q * p;
  return umin32(t, t - p);        // t in [0, 2p): t - p wraps when t < p
}
// Shoup result left in [0, 2p).
__device__ __forceinline__ u32 shoup_mul_lazy(u32 x, u32 w, u32 wq, u32 p) {
  u32 q = __umulhi(x, wq);
  return x * w - q * p;
}
__host__ __device__ __forceinline__ u32 add_mod(u32 a, u32 b, u32 p) {
  u32 s = a + b;                  // < 2p < 2^32
  return umin32(s, s - p);
}
__host__ __device__ __forceinline__ u32 sub_mod(u32 a, u32 b, u32 p) {
  u32 d = a - b;                  // wraps above 2^32 - p when a < b
  return umin32(d, d + p);
}
__host__ __device__ inline u32 shoup_companion(u32 w, u32 p) {
  return (u32)(((u64)w << 32) / p);
}

// ---------------------------------------------------------------------------
// Device tables and per-transform records.

// Twiddles for block NTTs: w^e for e < BLOCK_MAX/2 with w a primitive
// BLOCK_MAX-th root, value and Shoup companion interleaved.
struct TwBlock {
  const uint2* fwd[NPRIME_MAX];   // per prime: (w^e, companion)
  const uint2* inv[NPRIME_MAX];   // per prime: (w^-e, companion)
};

// Twiddles between the two passes of a length-N NTT, w_N^e = lo[e & 4095] * hi[e >> 12].
struct TwStep {
  const uint2* lo[2][NPRIME_MAX];   // [dir][prime], 4096 entries
  const uint2* hi[2][NPRIME_MAX];   // [dir][prime], max(1, N/4096) entries
};

// Input-independent data for one distinct length n: the chirp and the
// forward NTTs of the slices of Re w* and Im w* (with N^{-1} folded in).
struct KernelDesc {
  int n, N, logN, alpha;
  const double2* chirp;    // (cos(pi q/n), sin(pi q/n)), q = j^2 mod 2n
  const u32* W;            // [part][t][prime][N] NTT-domain values * N^{-1} (prime < the plan's moduli)
  const u32* Wq;           // Shoup companions of W
  int kw[2];               // slice counts of Re w*, Im w*
  int Ew[2][KMAX];         // slice exponents
};

// NTT-domain accumulation schedule.  The four real convolutions of the
// complex product x' (*) w* are c = 0: Re x' Re w*, 1: Im x' Im w*,
// 2: Im x' Re w*, 3: Re x' Im w*; output component tg (0: Re y', 1: Im y')
// takes convolutions 2 tg (sign +) and 2 tg + 1 (sign - for tg = 0, + for
// tg = 1), so each component is one walk over the slice pairs of its two
// convolutions.  A group is a run of consecutive walk positions
// [start, start + count) of one component with the same exponent e; its
// residues are the signed NTT-domain sum of the members' products.
//
// Walk order (acc_mode of the transform):
//   ACC_PER_CONV  Alg. 8 for each convolution on its own: convolution 2 tg
//                 then 2 tg + 1, anti-diagonals s + t descending, s
//                 ascending; a group closes at L products, at a change of
//                 scale and at the change of convolution.
//   ACC_COMPLEX   anti-diagonals descending, on each the pairs of
//                 convolution 2 tg and then of 2 tg + 1 (s ascending); a
//                 group closes at a change of scale or when its products'
//                 weights would exceed acc_limit, the most products whose
//                 signed sum stays within the CRT range:
//                 acc_limit n 4^alpha <= (p0 p1 - 1) / 2.  Re y' = ReRe - ImIm
//                 and Im y' = ImRe + ReIm are then formed in the NTT domain
//                 wherever the scales agree.  When the top exponents of
//                 Re x' and Im x' differ by d = 1 or 2, the larger part's
//                 slice spectra enter the products times 2^d (xsh) and its
//                 exponents count d lower, so the two parts' scales line up;
//                 its products then weigh 2^d.  This is done when a full
//                 anti-diagonal of that part's products still fits
//                 acc_limit.
constexpr int ACC_PER_CONV = 0;
constexpr int ACC_COMPLEX = 1;
constexpr int MAX_MEMBERS = 2 * MAX_PAIRS;      // walk positions per output component
struct Group {
  int start, count, e;
};
// Buffer slot of group gi, groups numbered across the components (the ng0
// groups of Re y' first); each component owns 2 K^2 slots, its most groups.
__host__ __device__ inline int group_slot(int gi, int ng0, int K) { return gi < ng0 ? gi : 2 * K * K + gi - ng0; }

// Per-transform state written by the kernels during one execution.
struct TState {
  u64 mu[2][KMAX + 1];     // bit patterns of max |r_k| (atomicMax targets)
  int Espec[2][KMAX];      // exponents used by the current extraction pass
  int E[2][KMAX];          // final exponents
  int kx[2];               // final slice counts
  int start[2];            // first slice still to (re)extract
  int active[2];           // 1 while the part still needs an extraction pass
  int status;
  int nmem[2];             // per output component: walk positions
  unsigned char mc[2][MAX_MEMBERS], ms[2][MAX_MEMBERS], mt[2][MAX_MEMBERS];   // convolution, s, t
  int ngroups[2];
  Group groups[2][MAX_MEMBERS];
  u64 gend[2][2];          // bit w of the 128: walk position w closes its group
  int xsh[2];              // x' part p's slice spectra enter the products times 2^xsh[p]
  int emin[2];             // per output component: smallest group exponent
  int span[2];             // per output component: largest shift above emin
};

// The caller's input and output arrays of one execution, read by the
// kernels from device memory: a captured graph of the batched schedule then
// serves any (in, out) pair, the pointers being written before each replay.
struct IoPtrs {
  const void* in;
  void* out;
};

// Static per-transform descriptor.
struct TDesc {
  int n, N, logN, alpha;
  int acc_mode;            // ACC_PER_CONV or ACC_COMPLEX
  int acc_limit;           // products per group: L (ACC_PER_CONV) or the CRT-range bound (ACC_COMPLEX)
  int kd;                  // index into the KernelDesc array
  int zs;                  // row stride of the compact outputs: n rounded up to a multiple of 4
  i64 io_off;              // element offset of this transform in in/out
  i64 xp_off;              // element offset in the debug copy of x' (double2)
  i64 X_off;               // u32 offset of the slice/NTT buffer [part][k][prime][N]
  i64 G_off;               // u32 offset of the group buffer [slot][prime][N]
  i64 Z_off;               // u32 offset of the compact outputs [slot][prime][zs]
};

}  // namespace fo
