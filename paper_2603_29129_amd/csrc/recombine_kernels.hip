// Garner CRT, exact recombination to binary64 and chirp postmultiply.
//
// For each output index k < n and each group g of the Alg. 8 schedule the two
// inverse-NTT residues are combined by Garner's formula (Sec. 3.3)
//     z = z0 + ((z1 - z0) p0^{-1} mod p1) p0,  mapped to [-(P-1)/2, (P-1)/2],
// which is the exact integer convolution value because |z| <= L n 4^alpha
// <= (P-1)/2 (Sec. 4.2 / 4.4).  Each component of y' is then the exact sum
//     Re y' = sum_{ReRe} z 2^e - sum_{ImIm} z 2^e,  Im y' = sum_{ImRe} + sum_{ReIm},
// accumulated in a two's-complement fixed-point integer (4 x 64 bits when the
// exponents of the transform span <= 185 bits, 50 x 64 bits otherwise) and
// rounded once to binary64, round to nearest even, subnormals and overflow
// included.  The chirp postmultiply y = y' (.) w (Sec. 3.2 Step 3) uses the
// same unfused product rule as the premultiply.
#include "internal.h"

namespace fo {

constexpr u32 P0INV_Q = (u32)(((u64)P0_INV_MOD_P1 << 32) / P1);

__device__ __forceinline__ i64 garner(u32 z0, u32 z1) {
  const u32 z0m = umin32(z0, z0 - P1);                 // z0 mod p1 (z0 < p0 < 2 p1)
  const u32 dl = sub_mod(z1, z0m, P1);
  const u32 h = shoup_mul(dl, P0_INV_MOD_P1, P0INV_Q, P1);
  const u64 z = (u64)z0 + (u64)h * P0;                  // in [0, p0 p1)
  return z > PP_HALF ? (i64)(z - PP) : (i64)z;
}

template <int W>
__device__ __forceinline__ void acc_add(u64 (&acc)[W], i64 z, int sh) {
  const int wi = sh >> 6, b = sh & 63;
  const u64 ext = z < 0 ? ~0ull : 0ull;
  const u64 lo = (u64)z << b;
  const u64 hi = b ? (u64)(z >> (64 - b)) : ext;
  u64 carry = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const u64 add = w < wi ? 0ull : (w == wi ? lo : (w == wi + 1 ? hi : ext));
    const u64 s1 = acc[w] + add;
    const u64 c1 = s1 < add;
    const u64 s2 = s1 + carry;
    const u64 c2 = s2 < carry;
    acc[w] = s2;
    carry = c1 | c2;
  }
}

// RN(acc * 2^emin) with acc a W-word two's complement integer.
template <int W>
__device__ double acc_round(u64 (&acc)[W], int emin) {
  const bool neg = (i64)acc[W - 1] < 0;
  if (neg) {
    u64 carry = 1;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const u64 v = ~acc[w] + carry;
      carry = (carry && v == 0) ? 1 : 0;
      acc[w] = v;
    }
  }
  int wt = -1;
#pragma unroll
  for (int w = 0; w < W; ++w)
    if (acc[w]) wt = w;
  if (wt < 0) return 0.0;
  u64 top = 0, below = 0;
  bool lower_nz = false;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    if (w == wt) top = acc[w];
    if (w == wt - 1) below = acc[w];
    if (w < wt - 1 && acc[w]) lower_nz = true;
  }
  const int lz = __clzll(top);
  const int Lb = 64 * wt + 63 - lz;                     // leading bit position
  const u64 T = lz ? ((top << lz) | (below >> (64 - lz))) : top;
  const bool sticky = lower_nz || (lz ? ((below << lz) != 0) : (below != 0));
  const int E2 = Lb + emin;                             // value in [2^E2, 2^(E2+1))
  const int kept = E2 >= -1022 ? 53 : E2 + 1075;
  double res;
  if (kept <= 0) {
    res = (kept == 0 && (T != (1ull << 63) || sticky)) ? 0x1p-1074 : 0.0;
  } else {
    const int sh = 64 - kept;
    u64 mant = T >> sh;
    const u64 rem = T & ((1ull << sh) - 1);
    const u64 half = 1ull << (sh - 1);
    if (rem > half || (rem == half && (sticky || (mant & 1)))) ++mant;
    res = ldexp((double)mant, E2 - kept + 1);
  }
  return neg ? -res : res;
}

// Fast path: the accumulator as 2 W_FAST 32-bit limbs; z 2^sh is added at
// limb sh / 32 with one add-with-carry chain (the limb index is the same for
// every lane, so the chain is chosen by a scalar branch).
constexpr int NL_FAST = 2 * W_FAST;
template <int L>
__device__ __forceinline__ void limb_add_at(u32 (&acc)[NL_FAST], u32 l0, u32 l1, u32 l2, u32 ext) {
  u32 c;
  acc[L] = __builtin_addc(acc[L], l0, 0u, &c);
  if constexpr (L + 1 < NL_FAST) acc[L + 1] = __builtin_addc(acc[L + 1], l1, c, &c);
  if constexpr (L + 2 < NL_FAST) acc[L + 2] = __builtin_addc(acc[L + 2], l2, c, &c);
#pragma unroll
  for (int k = L + 3; k < NL_FAST; ++k) acc[k] = __builtin_addc(acc[k], ext, c, &c);
}
// acc += z 2^sh, two's complement; the caller guarantees the sum fits (sh <= span).
__device__ __forceinline__ void limb_add(u32 (&acc)[NL_FAST], i64 z, int sh) {
  const int b = sh & 31;
  const u64 lo = (u64)z << b;                                  // bits 0..63 of z 2^b
  const u32 l2 = (u32)((z >> 32) >> (32 - b));                 // bits 64..95 (b = 0: the sign)
  const u32 ext = (u32)(z >> 63);
  const u32 l0 = (u32)lo, l1 = (u32)(lo >> 32);
  switch (sh >> 5) {
    case 0: limb_add_at<0>(acc, l0, l1, l2, ext); break;
    case 1: limb_add_at<1>(acc, l0, l1, l2, ext); break;
    case 2: limb_add_at<2>(acc, l0, l1, l2, ext); break;
    case 3: limb_add_at<3>(acc, l0, l1, l2, ext); break;
    case 4: limb_add_at<4>(acc, l0, l1, l2, ext); break;
    case 5: limb_add_at<5>(acc, l0, l1, l2, ext); break;
    case 6: limb_add_at<6>(acc, l0, l1, l2, ext); break;
    default: limb_add_at<7>(acc, l0, l1, l2, ext); break;
  }
}
static_assert(NL_FAST == 8, "limb_add dispatches over eight limbs");

__device__ __constant__ int c_tconv[2][2] = {{0, 1}, {2, 3}};
__device__ __constant__ int c_tsign[2][2] = {{1, -1}, {1, 1}};

// Both outputs j, j + 1 of one component (j even; the compact rows are
// padded to a multiple of four, so j + 1 is always a readable position).
__device__ void recombine_fast2(const u32* Zb, const TState& s, int tg, int SL, int zs, int j, double& r0,
                                double& r1) {
  u32 a[NL_FAST], b[NL_FAST];
#pragma unroll
  for (int k = 0; k < NL_FAST; ++k) a[k] = b[k] = 0;
  const int emin = s.emin[tg];
  for (int ci = 0; ci < 2; ++ci) {
    const int c = c_tconv[tg][ci];
    const int sg = c_tsign[tg][ci];
    for (int g = 0; g < s.ngroups[c]; ++g) {
      const int slot = c * SL + g;
      const uint2 v0 = *reinterpret_cast<const uint2*>(Zb + (size_t)(slot * 2) * zs + j);
      const uint2 v1 = *reinterpret_cast<const uint2*>(Zb + (size_t)(slot * 2 + 1) * zs + j);
      i64 za = garner(v0.x, v1.x), zb = garner(v0.y, v1.y);
      if (sg < 0) {
        za = -za;
        zb = -zb;
      }
      const int sh = s.groups[c][g].e - emin;
      limb_add(a, za, sh);
      limb_add(b, zb, sh);
    }
  }
  u64 a64[W_FAST], b64[W_FAST];
#pragma unroll
  for (int w = 0; w < W_FAST; ++w) {
    a64[w] = (u64)a[2 * w] | ((u64)a[2 * w + 1] << 32);
    b64[w] = (u64)b[2 * w] | ((u64)b[2 * w + 1] << 32);
  }
  r0 = acc_round<W_FAST>(a64, emin);
  r1 = acc_round<W_FAST>(b64, emin);
}

template <int W>
__device__ double recombine_one(const u32* Zb, const TState& s, int tg, int SL, int zs, int j) {
  u64 acc[W];
#pragma unroll
  for (int w = 0; w < W; ++w) acc[w] = 0;
  const int emin = s.emin[tg];
  for (int ci = 0; ci < 2; ++ci) {
    const int c = c_tconv[tg][ci];
    const int sg = c_tsign[tg][ci];
    for (int g = 0; g < s.ngroups[c]; ++g) {
      const int slot = c * SL + g;
      const u32 z0 = Zb[(size_t)(slot * 2) * zs + j];
      const u32 z1 = Zb[(size_t)(slot * 2 + 1) * zs + j];
      i64 z = garner(z0, z1);
      if (sg < 0) z = -z;
      acc_add<W>(acc, z, s.groups[c][g].e - emin);
    }
  }
  return acc_round<W>(acc, emin);
}

// Postmultiply and direction handling of one output.
__device__ __forceinline__ double2 finish(double pr, double pi, double2 w, int dir, int n) {
  double yr = pr * w.x + pi * w.y;     // RN(RN(y'r c) + RN(y'i s))
  double yi = pi * w.x - pr * w.y;     // RN(RN(y'i c) - RN(y'r s))
  if (dir) {                           // inverse / adjoint: conj(F(conj x)) [/ n]
    yi = -yi;
    if (dir == 1) {
      const double nn = (double)n;
      yr = yr / nn;
      yi = yi / nn;
    }
  }
  return make_double2(yr, yi);
}

// WIDE = false: transforms whose exponent spans fit the fast accumulator (and
// those with a status, which get NaN), two outputs per thread;
// WIDE = true: the others, one output per thread.
template <bool WIDE>
__global__ void k_recombine(const u32* Z, double2* out, const TDesc* td, const TState* ts, const KernelDesc* kd,
                            const int* tlist, int K, int dir) {
  const int t = tlist[blockIdx.z];
  const TDesc& d = td[t];
  const TState& s = ts[t];
  const bool wide0 = s.span[0] > 64 * W_FAST - 71, wide1 = s.span[1] > 64 * W_FAST - 71;
  if (WIDE != (!s.status && (wide0 || wide1))) return;
  const double2* ch = kd[d.kd].chirp;
  const int SL = K * K;
  const u32* Zb = Z + d.Z_off;
  if (!WIDE) {
    for (int j = 2 * (blockIdx.x * blockDim.x + threadIdx.x); j < d.n; j += 2 * gridDim.x * blockDim.x) {
      double2 o0, o1;
      if (s.status) {
        o0 = o1 = make_double2(__builtin_nan(""), __builtin_nan(""));
      } else {
        double pr0, pr1, pi0, pi1;
        recombine_fast2(Zb, s, 0, SL, d.zs, j, pr0, pr1);
        recombine_fast2(Zb, s, 1, SL, d.zs, j, pi0, pi1);
        o0 = finish(pr0, pi0, ch[j], dir, d.n);
        o1 = j + 1 < d.n ? finish(pr1, pi1, ch[j + 1], dir, d.n) : o0;
      }
      out[d.io_off + j] = o0;
      if (j + 1 < d.n) out[d.io_off + j + 1] = o1;
    }
    return;
  }
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += gridDim.x * blockDim.x) {
    const double pr = wide0 ? recombine_one<W_WIDE>(Zb, s, 0, SL, d.zs, j) : recombine_one<W_FAST>(Zb, s, 0, SL, d.zs, j);
    const double pi = wide1 ? recombine_one<W_WIDE>(Zb, s, 1, SL, d.zs, j) : recombine_one<W_FAST>(Zb, s, 1, SL, d.zs, j);
    out[d.io_off + j] = finish(pr, pi, ch[j], dir, d.n);
  }
}

hipError_t launch_recombine(const u32* Z, double2* out, const TDesc* td, const TState* ts, const KernelDesc* kd,
                            const int* tlist, int count, int nmax, int K, int dir, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int b = (nmax + 255) / 256;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  const int b2 = (b + 1) / 2;      // two outputs per thread
  hipLaunchKernelGGL(k_recombine<false>, dim3(b2, 1, count), dim3(256), 0, s, Z, out, td, ts, kd, tlist, K, dir);
  hipLaunchKernelGGL(k_recombine<true>, dim3(b, 1, count), dim3(256), 0, s, Z, out, td, ts, kd, tlist, K, dir);
  return hipGetLastError();
}

}  // namespace fo
