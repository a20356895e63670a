// The d = 3 CRT variant: three 31-bit moduli p0, p1, p2 (Sec. 3.3's CRT with
// d moduli) allow the split width of Sec. 4.2 with the product p0 p1 p2
// (alpha = 36 at n = 2^18, L = 3), so two slices per part carry 72 bits.
// The slice spectra and group sums of a length class are laid out prime by
// prime ([prime][transform][vector][N]) so that the forward and inverse
// NTTs run as the standalone transforms, one launch per class and prime;
// this file holds the NTT-domain multiply-accumulate over the three primes
// and Garner's mixed-radix reconstruction with the exact recombination.
#include "crt_dev.h"

namespace fo {

__device__ __forceinline__ u32 prime3_of(int q) { return q == 0 ? P0 : (q == 1 ? P1 : P2); }

// Garner constants for d = 3 (host-computed at compile time).
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
constexpr u32 P0INV_Q3 = (u32)(((u64)P0_INV_MOD_P1 << 32) / P1);
static_assert((PP % P2) * PP_INV_MOD_P2 % P2 == 1, "(p0 p1)^{-1} mod p2");
// M = p0 p1 p2 < 2^93 as two 64-bit words, from p0 p1 = hi32 2^32 + lo32.
constexpr u64 M_A = (PP & 0xFFFFFFFFull) * P2;                            // < 2^63
constexpr u64 M_B = (PP >> 32) * P2;                                      // < 2^61
constexpr u64 M_LO = M_A + (M_B << 32);
constexpr u64 M_HI = (M_B >> 32) + (M_LO < M_A ? 1 : 0);
// (M - 1) / 2 = M >> 1 (M odd)
constexpr u64 MH_LO = (M_LO >> 1) | (M_HI << 63);
constexpr u64 MH_HI = M_HI >> 1;

// z in [0, M) from its residues, mixed radix: z = z0 + p0 h1 + p0 p1 h2 with
// h1 = (z1 - z0) p0^{-1} mod p1 and h2 = (z2 - (z0 + p0 h1)) (p0 p1)^{-1}
// mod p2; then the symmetric remainder in [-(M-1)/2, (M-1)/2], returned as
// the two's complement 128-bit value hi 2^64 + lo.
__device__ __forceinline__ void garner3(u32 z0, u32 z1, u32 z2, u64& lo, i64& hi) {
  const u32 z0m1 = umin32(z0, z0 - P1);                       // z0 mod p1 (z0 < p0 < 2 p1)
  const u32 h1 = shoup_mul(sub_mod(z1, z0m1, P1), P0_INV_MOD_P1, P0INV_Q3, P1);
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

// acc += (hi 2^64 + lo) 2^sh, as three pieces of at most 64 bits each.
template <int W>
__device__ __forceinline__ void acc_add128(u64 (&acc)[W], u64 lo, i64 hi, int sh) {
  acc_add<W>(acc, (i64)(lo & 0xFFFFFFFFull), sh);
  acc_add<W>(acc, (i64)(lo >> 32), sh + 32);
  acc_add<W>(acc, hi, sh + 64);
}

// The fast accumulator (W_FAST words) holds every sum when the exponent span
// plus the 93 bits of a group value and 7 bits of carries stays below its width.
constexpr int SPAN_FAST3 = 64 * W_FAST - 104;

// ---------------------------------------------------------------------------
// NTT-domain multiply-accumulate: for every group g of component tg of the
// transform, G[slot] = sum over its members (c, s, t) of +- X_pa(c)^s (.)
// W_pb(c)^t mod p, the ImIm products (c = 1) subtracted.  blockIdx.y is the
// prime, blockIdx.z the transform; the schedule reads are uniform per block.
// Convolution c uses x' part ((c + 1) >> 1) & 1 and w* part c & 1.
__global__ void k_mac3(const u32* X, u32* G, const TDesc* td, const TState* ts, const KernelDesc* kd,
                       const int* tlist, int K) {
  const int t = tlist[blockIdx.z];
  const TState& s = ts[t];
  if (s.status) return;
  const TDesc& d = td[t];
  const KernelDesc& kk = kd[d.kd];
  const int q = blockIdx.y, logN = d.logN, SL = 2 * K * K;
  const u32 p = prime3_of(q);
  const size_t N = (size_t)1 << logN, wps = (size_t)(2 * K) << logN;
  const u32* Xb = X + d.X_off + q * d.xps;
  const u32* Wb = kk.W + q * wps;
  const u32* Qb = kk.Wq + q * wps;
  u32* Gb = G + d.G_off + q * d.gps;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    for (int tg = 0; tg < 2; ++tg) {
      for (int g = 0; g < s.ngroups[tg]; ++g) {
        const int m0 = s.groups[tg][g].start, m1 = m0 + s.groups[tg][g].count;
        u32 acc = 0;
        for (int m = m0; m < m1; ++m) {
          const int c = s.mc[tg][m], pa = ((c + 1) >> 1) & 1, pb = c & 1;
          const u32 xv = Xb[((size_t)(pa * K + s.ms[tg][m]) << logN) + e];
          const size_t wi = ((size_t)(pb * K + s.mt[tg][m]) << logN) + e;
          const u32 pr = shoup_mul(xv, Wb[wi], Qb[wi], p);
          acc = c == 1 ? sub_mod(acc, pr, p) : add_mod(acc, pr, p);
        }
        Gb[((size_t)(tg * SL + g) << logN) + e] = acc;
      }
    }
  }
}

// Shoup companions of the kernel spectra, W laid out [prime][part][k][N].
__global__ void k_companions3(const u32* W, u32* Wq, size_t per_prime) {
  const size_t total = 3 * per_prime;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x)
    Wq[i] = shoup_companion(W[i], prime3_of((int)(i / per_prime)));
}

// One component of y' at output j: the exact sum of the group values
// z_g 2^(e_g), rounded once to binary64.
template <int W>
__device__ double recombine3_one(const u32* G, const TDesc& d, const TState& s, int tg, int SL, int j) {
  u64 acc[W];
#pragma unroll
  for (int w = 0; w < W; ++w) acc[w] = 0;
  const int emin = s.emin[tg];
  for (int g = 0; g < s.ngroups[tg]; ++g) {
    const u32* z = G + d.G_off + ((size_t)(tg * SL + g) << d.logN) + j;
    u64 lo;
    i64 hi;
    garner3(z[0], z[d.gps], z[2 * d.gps], lo, hi);
    acc_add128<W>(acc, lo, hi, s.groups[tg][g].e - emin);
  }
  return acc_round<W>(acc, emin);
}

// WIDE = false: transforms whose spans fit the fast accumulator and those
// with a status (NaN outputs); WIDE = true: the others.
template <bool WIDE>
__global__ void k_recombine3(const u32* G, void* out, const TDesc* td, const TState* ts, const KernelDesc* kd,
                             const int* tlist, int K, int dir, int io32) {
  const int t = tlist[blockIdx.z];
  const TDesc& d = td[t];
  const TState& s = ts[t];
  const bool w0 = s.span[0] > SPAN_FAST3, w1 = s.span[1] > SPAN_FAST3;
  if (WIDE != (!s.status && (w0 || w1))) return;
  const double2* ch = kd[d.kd].chirp;
  const int SL = 2 * K * K;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += gridDim.x * blockDim.x) {
    double2 o;
    if (s.status) {
      o = make_double2(__builtin_nan(""), __builtin_nan(""));
    } else if (WIDE) {
      const double pr = w0 ? recombine3_one<W_WIDE>(G, d, s, 0, SL, j) : recombine3_one<W_FAST>(G, d, s, 0, SL, j);
      const double pi = w1 ? recombine3_one<W_WIDE>(G, d, s, 1, SL, j) : recombine3_one<W_FAST>(G, d, s, 1, SL, j);
      o = finish(pr, pi, ch[j], dir, d.n);
    } else {
      o = finish(recombine3_one<W_FAST>(G, d, s, 0, SL, j), recombine3_one<W_FAST>(G, d, s, 1, SL, j), ch[j], dir,
                 d.n);
    }
    put_out(out, d.io_off + j, o, io32);
  }
}

static int grid_for(size_t work) {
  size_t b = (work + 255) / 256;
  if (b > 2048) b = 2048;
  return b < 1 ? 1 : (int)b;
}

hipError_t launch_companions3(const u32* W, u32* Wq, int K, int logN, hipStream_t s) {
  const size_t per = (size_t)(2 * K) << logN;
  hipLaunchKernelGGL(k_companions3, dim3(grid_for(3 * per)), dim3(256), 0, s, W, Wq, per);
  return hipGetLastError();
}

hipError_t launch_mac3(const u32* X, u32* G, const TDesc* td, const TState* ts, const KernelDesc* kd,
                       const int* tlist, int count, int K, int logN, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mac3, dim3(grid_for((size_t)1 << logN), 3, count), dim3(256), 0, s, X, G, td, ts, kd, tlist,
                     K);
  return hipGetLastError();
}

hipError_t launch_recombine3(const u32* G, void* out, const TDesc* td, const TState* ts, const KernelDesc* kd,
                             const int* tlist, int count, int nmax, int K, int dir, int io32, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int b = grid_for((size_t)nmax);
  hipLaunchKernelGGL(k_recombine3<false>, dim3(b, 1, count), dim3(256), 0, s, G, out, td, ts, kd, tlist, K, dir,
                     io32);
  hipLaunchKernelGGL(k_recombine3<true>, dim3(b, 1, count), dim3(256), 0, s, G, out, td, ts, kd, tlist, K, dir,
                     io32);
  return hipGetLastError();
}

}  // namespace fo
