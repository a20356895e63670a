// Device helpers of the CRT (two or three moduli) and the exact recombination
// (Sec. 3.3, 4.4), shared by the recombination kernels and the fused inverse
// column pass.
#pragma once
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

// Output element idx: complex128, or for a binary32 target complex64, each
// component rounded once (to nearest even) from the binary64 result.
__device__ __forceinline__ void put_out(void* out, i64 idx, double2 v, int io32) {
  if (io32) reinterpret_cast<float2*>(out)[idx] = make_float2((float)v.x, (float)v.y);
  else reinterpret_cast<double2*>(out)[idx] = v;
}

// ---------------------------------------------------------------------------
// Three moduli (Sec. 3.3's CRT with d = 3): Garner's mixed-radix form
// z = z0 + p0 h1 + p0 p1 h2 over p0, p1, p2 (p0 p1 p2 < 2^93).
constexpr u64 powmod_c(u64 b, u64 e, u64 p) {
  u64 r = 1;
  b %= p;
  while (e) {
    if (e & 1) r = r * b % p;
    b = b * b % p;
    e >>= 1;
  }
  return r;
}
constexpr u32 P0_MOD_P2 = P0 - P2;                                        // p0 < 2 p2
constexpr u32 P0_MOD_P2_Q = (u32)(((u64)P0_MOD_P2 << 32) / P2);
constexpr u32 PP_INV_MOD_P2 = (u32)powmod_c(PP % P2, P2 - 2, P2);        // (p0 p1)^{-1} mod p2
constexpr u32 PP_INV_MOD_P2_Q = (u32)(((u64)PP_INV_MOD_P2 << 32) / P2);
static_assert((PP % P2) * PP_INV_MOD_P2 % P2 == 1, "(p0 p1)^{-1} mod p2");
// M = p0 p1 p2 as two 64-bit words, from p0 p1 = hi32 2^32 + lo32.
constexpr u64 M_A = (PP & 0xFFFFFFFFull) * P2;                            // < 2^63
constexpr u64 M_B = (PP >> 32) * P2;                                      // < 2^61
constexpr u64 M_LO = M_A + (M_B << 32);
constexpr u64 M_HI = (M_B >> 32) + (M_LO < M_A ? 1 : 0);
// (M - 1) / 2 = M >> 1 (M odd)
constexpr u64 MH_LO = (M_LO >> 1) | (M_HI << 63);
constexpr u64 MH_HI = M_HI >> 1;

// z in [0, M) from its residues: h1 = (z1 - z0) p0^{-1} mod p1,
// h2 = (z2 - (z0 + p0 h1)) (p0 p1)^{-1} mod p2; then the symmetric remainder
// in [-(M-1)/2, (M-1)/2] as the two's complement 128-bit value hi 2^64 + lo.
__device__ __forceinline__ void garner3(u32 z0, u32 z1, u32 z2, u64& lo, i64& hi) {
  const u32 z0m1 = umin32(z0, z0 - P1);                       // z0 mod p1 (z0 < p0 < 2 p1)
  const u32 h1 = shoup_mul(sub_mod(z1, z0m1, P1), P0_INV_MOD_P1, P0INV_Q, P1);
  const u64 t = (u64)z0 + (u64)h1 * P0;                        // z mod p0 p1, in [0, p0 p1)
  const u32 z0m2 = umin32(z0, z0 - P2);                       // z0 mod p2 (z0 < p0 < 2 p2)
  const u32 tm2 = add_mod(z0m2, shoup_mul(h1, P0_MOD_P2, P0_MOD_P2_Q, P2), P2);   // t mod p2
  const u32 h2 = shoup_mul(sub_mod(z2, tm2, P2), PP_INV_MOD_P2, PP_INV_MOD_P2_Q, P2);
  u64 l = PP * (u64)h2;
  u64 h = __umul64hi(PP, (u64)h2);
  l += t;
  h += l < t ? 1ull : 0ull;
  if (h > MH_HI || (h == MH_HI && l > MH_LO)) {
    const u64 borrow = l < M_LO ? 1ull : 0ull;
    l -= M_LO;
    h = h - M_HI - borrow;
  }
  lo = l;
  hi = (i64)h;
}

// The signed group value of residues z[0 .. NP-1] added, times 2^sh, to the
// fast limbs: one piece for NP = 2 (|z| < 2^62); for NP = 3 (|z| < 2^92)
// z mod 2^62 (non-negative) at sh and z >> 62 (|.| < 2^31) at sh + 62.
template <int NP>
__device__ __forceinline__ void limb_add_crt(u32 (&acc)[NL_FAST], const u32 (&z)[NP], int sh) {
  if constexpr (NP == 2) {
    limb_add(acc, garner(z[0], z[1]), sh);
  } else {
    u64 lo;
    i64 hi;
    garner3(z[0], z[1], z[2], lo, hi);
    limb_add(acc, (i64)(lo & 0x3FFFFFFFFFFFFFFFull), sh);
    limb_add(acc, (hi << 2) | (i64)(lo >> 62), sh + 62);
  }
}
// The same into a W-word accumulator (the NP = 3 value as three pieces of at
// most 64 bits).
template <int NP, int W>
__device__ __forceinline__ void acc_add_crt(u64 (&acc)[W], const u32 (&z)[NP], int sh) {
  if constexpr (NP == 2) {
    acc_add<W>(acc, garner(z[0], z[1]), sh);
  } else {
    u64 lo;
    i64 hi;
    garner3(z[0], z[1], z[2], lo, hi);
    acc_add<W>(acc, (i64)(lo & 0xFFFFFFFFull), sh);
    acc_add<W>(acc, (i64)(lo >> 32), sh + 32);
    acc_add<W>(acc, hi, sh + 64);
  }
}

// A transform's exponent span needs the wide accumulator (output component
// tg): the fast limbs hold every sum while the span plus the group value's
// bits (63 for two moduli, 93 for three) and 7 bits of carries stays below
// their 64 W_FAST bits.
template <int NP>
__device__ __forceinline__ bool span_wide(const TState& s, int tg) {
  return s.span[tg] > 64 * W_FAST - (NP == 2 ? 71 : 104);
}

}  // namespace fo
