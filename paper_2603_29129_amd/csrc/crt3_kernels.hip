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
// NTT-domain multiply-accumulate: for every group g of component tg of a
// transform, G[slot] = sum over its members (c, s, t) of +- X_pa(c)^s (.)
// W_pb(c)^t mod p, the ImIm products (c = 1) subtracted.  A block takes 256
// positions of one prime (blockIdx.y) for a run of up to `tpr` transforms of
// the class (blockIdx.z), so the kernel spectra are loaded once per run
// (again only where the kernel changes).  Each thread keeps the values of
// its position in its own LDS column ([vector][256], conflict-free); the
// transform's walk is staged in LDS as operand offsets and sign per member.
// Convolution c uses x' part ((c + 1) >> 1) & 1 and w* part c & 1.
constexpr int MAC3_THREADS = 256;
__global__ void __launch_bounds__(MAC3_THREADS) k_mac3(const u32* __restrict__ X, u32* __restrict__ G,
                                                       const TDesc* td, const TState* ts, const KernelDesc* kd,
                                                       const int* tlist, int count, int K, int tpr) {
  extern __shared__ u32 sm[];
  const int V = 2 * K, SL = 2 * K * K, q = blockIdx.y;
  const u32 p = prime3_of(q);
  u32* cx = sm + threadIdx.x;                          // column of this thread: vector v at v * 256
  u32* cw = cx + V * MAC3_THREADS;
  u32* cq = cw + V * MAC3_THREADS;
  u32* code = sm + 3 * V * MAC3_THREADS;               // [component][walk position]
  const int b0 = blockIdx.z * tpr, b1 = min(count, b0 + tpr);
  int wkd = -1;
  for (int b = b0; b < b1; ++b) {
    const int t = tlist[b];
    const TState& s = ts[t];
    if (s.status) continue;
    const TDesc& d = td[t];
    const KernelDesc& kk = kd[d.kd];
    const int logN = d.logN;
    const size_t N = (size_t)1 << logN, e = blockIdx.x * (size_t)MAC3_THREADS + threadIdx.x;
    const bool live = e < N;
    __syncthreads();                                   // the previous transform's walk is consumed
    const int nm0 = s.nmem[0], nm = nm0 + s.nmem[1];
    for (int i = threadIdx.x; i < nm; i += MAC3_THREADS) {
      const int tg = i >= nm0, m = i - tg * nm0, c = s.mc[tg][m];
      const int xo = ((((c + 1) >> 1) & 1) * K + s.ms[tg][m]) * MAC3_THREADS;
      const int wo = ((c & 1) * K + s.mt[tg][m]) * MAC3_THREADS;
      code[tg * MAX_MEMBERS + m] = (u32)xo | ((u32)wo << 13) | (c == 1 ? 1u << 31 : 0u);
    }
    __syncthreads();
    if (!live) continue;
    if (d.kd != wkd) {
      const size_t wps = (size_t)V << logN;
      const u32* Wb = kk.W + q * wps;
      const u32* Qb = kk.Wq + q * wps;
      for (int v = 0; v < V; ++v)
        if (v - (v >= K) * K < kk.kw[v >= K]) {
          cw[v * MAC3_THREADS] = Wb[((size_t)v << logN) + e];
          cq[v * MAC3_THREADS] = Qb[((size_t)v << logN) + e];
        }
      wkd = d.kd;
    }
    const u32* Xb = X + d.X_off + q * d.xps;
    for (int v = 0; v < V; ++v)
      if (v - (v >= K) * K < s.kx[v >= K]) cx[v * MAC3_THREADS] = Xb[((size_t)v << logN) + e];
    u32* Gb = G + d.G_off + q * d.gps + e;
    for (int tg = 0; tg < 2; ++tg) {
      for (int g = 0; g < s.ngroups[tg]; ++g) {
        const int m0 = s.groups[tg][g].start, m1 = m0 + s.groups[tg][g].count;
        u32 acc = 0;
        for (int m = m0; m < m1; ++m) {
          const u32 cd = code[tg * MAX_MEMBERS + m];
          const int wo = (cd >> 13) & 0x1FFF;
          const u32 pr = shoup_mul(cx[cd & 0x1FFF], cw[wo], cq[wo], p);
          acc = (cd >> 31) ? sub_mod(acc, pr, p) : add_mod(acc, pr, p);
        }
        Gb[(size_t)(tg * SL + g) << logN] = acc;
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

// Fast path: the sum in NL_FAST 32-bit limbs; a group value v (|v| < 2^92)
// enters as v mod 2^62 (non-negative) at shift sh and v >> 62 (|.| < 2^31)
// at sh + 62, each one add-with-carry chain (sh <= SPAN_FAST3 keeps both
// inside the limbs).
__device__ double recombine3_fast(const u32* G, const TDesc& d, const TState& s, int tg, int SL, int j) {
  u32 acc[NL_FAST];
#pragma unroll
  for (int k = 0; k < NL_FAST; ++k) acc[k] = 0;
  const int emin = s.emin[tg];
  for (int g = 0; g < s.ngroups[tg]; ++g) {
    const u32* z = G + d.G_off + ((size_t)(tg * SL + g) << d.logN) + j;
    u64 lo;
    i64 hi;
    garner3(z[0], z[d.gps], z[2 * d.gps], lo, hi);
    const int sh = s.groups[tg][g].e - emin;
    limb_add(acc, (i64)(lo & 0x3FFFFFFFFFFFFFFFull), sh);
    limb_add(acc, (hi << 2) | (i64)(lo >> 62), sh + 62);
  }
  u64 a64[W_FAST];
#pragma unroll
  for (int w = 0; w < W_FAST; ++w) a64[w] = (u64)acc[2 * w] | ((u64)acc[2 * w + 1] << 32);
  return acc_round<W_FAST>(a64, emin);
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
__global__ void k_recombine3(const u32* G, const IoPtrs* io, const TDesc* td, const TState* ts, const KernelDesc* kd,
                             const int* tlist, int K, int dir, int io32) {
  const int t = tlist[blockIdx.z];
  void* out = io->out;
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
      o = finish(recombine3_fast(G, d, s, 0, SL, j), recombine3_fast(G, d, s, 1, SL, j), ch[j], dir, d.n);
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
  constexpr int TPR = 8;                                            // transforms per block
  // operand columns (at most 48 KiB for K <= 8) and the two walks' codes
  const size_t lds = sizeof(u32) * (3 * (size_t)(2 * K) * MAC3_THREADS + 2 * MAX_MEMBERS);
  const unsigned bx = (unsigned)((((size_t)1 << logN) + MAC3_THREADS - 1) / MAC3_THREADS);
  hipLaunchKernelGGL(k_mac3, dim3(bx, 3, (count + TPR - 1) / TPR), dim3(MAC3_THREADS), lds, s, X, G, td, ts, kd,
                     tlist, count, K, TPR);
  return hipGetLastError();
}

hipError_t launch_recombine3(const u32* G, const IoPtrs* io, const TDesc* td, const TState* ts, const KernelDesc* kd,
                             const int* tlist, int count, int nmax, int K, int dir, int io32, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int b = grid_for((size_t)nmax);
  hipLaunchKernelGGL(k_recombine3<false>, dim3(b, 1, count), dim3(256), 0, s, G, io, td, ts, kd, tlist, K, dir,
                     io32);
  hipLaunchKernelGGL(k_recombine3<true>, dim3(b, 1, count), dim3(256), 0, s, G, io, td, ts, kd, tlist, K, dir,
                     io32);
  return hipGetLastError();
}

}  // namespace fo
