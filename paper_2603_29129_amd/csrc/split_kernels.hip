// Chirp generation, premultiply, Ozaki slice extraction and the Alg. 8 group
// schedule on gfx950.
//
// All floating-point work here is binary64 with every operation rounded on
// its own (the library is compiled with -ffp-contract=off; fused operations
// appear only where written explicitly, in the double-double chirp code).
#include "schedule_dev.h"

namespace fo {

// ---------------------------------------------------------------------------
// Chirp w(j) = w_2n^{j^2} = exp(-i pi q/n), q = j^2 mod 2n (Sec. 3.2), stored
// as (c, s) = (RN(cos(pi q/n)), RN(sin(pi q/n))), so w = c - i s, w* = c + i s.
//
// q is reduced exactly in integers to an octant o = floor(4q/n) and a
// remainder r = 4q - o n in [0, n); the reduced angle (pi/4) r/n (or
// (pi/4)(n-r)/n in odd octants) lies in [0, pi/4].  Its sine and cosine are
// evaluated in double-double arithmetic (Dekker/Knuth error-free products and
// sums, Taylor series to x^31/31!), then rounded to binary64.  If the
// double-double value lies within its error bound of a rounding boundary the
// entry is flagged (the plan then fails) instead of risking a misrounding.

struct dd {
  double h, l;
};
__device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__device__ __forceinline__ dd fast_two_sum(double a, double b) {
  double s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
  double p = a.h * b.h;
  double e = __builtin_fma(a.h, b.h, -p);
  e = __builtin_fma(a.h, b.l, e);
  e = __builtin_fma(a.l, b.h, e);
  return fast_two_sum(p, e);
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  dd s = two_sum(a.h, b.h);
  double e = s.l + a.l + b.l;
  return fast_two_sum(s.h, e);
}

// (-1)^k / (2k+1)!  and  (-1)^k / (2k)!  as double-double, k = 0..15.
__device__ __constant__ double c_sin_dd[16][2] = {
    {0x1.0000000000000p+0, 0x0.0p+0},
    {-0x1.5555555555555p-3, -0x1.5555555555555p-57},
    {0x1.1111111111111p-7, 0x1.1111111111111p-63},
    {-0x1.a01a01a01a01ap-13, -0x1.a01a01a01a01ap-73},
    {0x1.71de3a556c734p-19, -0x1.c154f8ddc6c00p-73},
    {-0x1.ae64567f544e4p-26, 0x1.c062e06d1f209p-80},
    {0x1.6124613a86d09p-33, 0x1.f28e0cc748ebep-87},
    {-0x1.ae7f3e733b81fp-41, -0x1.1d8656b0ee8cbp-97},
    {0x1.952c77030ad4ap-49, 0x1.ac981465ddc6cp-103},
    {-0x1.2f49b46814157p-57, -0x1.2650f61dbdcb4p-112},
    {0x1.71b8ef6dcf572p-66, -0x1.d043ae40c4647p-120},
    {-0x1.761b41316381ap-75, 0x1.3423c7d91404fp-130},
    {0x1.3f3ccdd165fa9p-84, -0x1.58ddadf344487p-139},
    {-0x1.d1ab1c2dccea3p-94, -0x1.054d0c78aea14p-149},
    {0x1.259f98b4358adp-103, 0x1.eaf8c39dd9bc5p-157},
    {-0x1.434d2e783f5bcp-113, -0x1.0b87b91be9affp-167}};
__device__ __constant__ double c_cos_dd[16][2] = {
    {0x1.0000000000000p+0, 0x0.0p+0},
    {-0x1.0000000000000p-1, 0x0.0p+0},
    {0x1.5555555555555p-5, 0x1.5555555555555p-59},
    {-0x1.6c16c16c16c17p-10, 0x1.f49f49f49f49fp-65},
    {0x1.a01a01a01a01ap-16, 0x1.a01a01a01a01ap-76},
    {-0x1.27e4fb7789f5cp-22, -0x1.cbbc05b4fa99ap-76},
    {0x1.1eed8eff8d898p-29, -0x1.2aec959e14c06p-83},
    {-0x1.93974a8c07c9dp-37, -0x1.05d6f8a2efd1fp-92},
    {0x1.ae7f3e733b81fp-45, 0x1.1d8656b0ee8cbp-101},
    {-0x1.6827863b97d97p-53, -0x1.eec01221a8b0bp-107},
    {0x1.e542ba4020225p-62, 0x1.ea72b4afe3c2fp-120},
    {-0x1.0ce396db7f853p-70, 0x1.aebcdbd20331cp-124},
    {0x1.f2cf01972f578p-80, -0x1.9ada5fcc1ab14p-135},
    {-0x1.88e85fc6a4e5ap-89, 0x1.71c37ebd16540p-143},
    {0x1.0a18a2635085dp-98, 0x1.b9e2e28e1aa54p-153},
    {-0x1.3932c5047d60ep-108, -0x1.832b7b530a627p-162}};

// Rounds a double-double to binary64; sets *amb if the value is within `tol`
// (relative) of a midpoint between two binary64 neighbours.
__device__ __forceinline__ double dd_round(dd v, int* amb) {
  const double h = v.h, l = v.l;
  if (h == 0.0) return 0.0;
  const long long hb = __double_as_longlong(fabs(h));
  const double ulp_half = 0.5 * (__longlong_as_double(hb + 1) - fabs(h));   // exact: a power of two
  const double tol = fabs(h) * 0x1p-98;
  if (fabs(fabs(l) - ulp_half) <= tol) *amb = 1;
  return h;     // fast_two_sum normalisation makes h = RN(h + l) away from midpoints
}

// sin and cos of x = (pi/4) * t, t = num/den in [0, 1].
__device__ void sincos_quarter(long long num, long long den, dd* sn, dd* cs) {
  const double th = (double)num / (double)den;
  const double rem = __builtin_fma(-th, (double)den, (double)num);   // exact residual
  dd t = fast_two_sum(th, rem / (double)den);
  const dd pi4 = {0x1.921fb54442d18p-1, 0x1.1a62633145c07p-55};
  const dd x = dd_mul(pi4, t);
  const dd x2 = dd_mul(x, x);
  dd ps = {c_sin_dd[15][0], c_sin_dd[15][1]};
  dd pc = {c_cos_dd[15][0], c_cos_dd[15][1]};
  for (int k = 14; k >= 0; --k) {
    ps = dd_add(dd_mul(ps, x2), dd{c_sin_dd[k][0], c_sin_dd[k][1]});
    pc = dd_add(dd_mul(pc, x2), dd{c_cos_dd[k][0], c_cos_dd[k][1]});
  }
  *sn = dd_mul(ps, x);
  *cs = pc;
}

__global__ void k_chirp(double2* chirp, int n, int* flag) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const long long nn = n;
    const long long q = ((long long)j * j) % (2 * nn);
    const long long q4 = 4 * q;
    const int o = (int)(q4 / nn);
    const long long r = q4 - (long long)o * nn;
    dd S, C;
    if (o & 1) sincos_quarter(nn - r, nn, &S, &C);
    else sincos_quarter(r, nn, &S, &C);
    int amb = 0;
    const double s = dd_round(S, &amb), c = dd_round(C, &amb);
    // cos/sin of (pi/4)(o + r/n), reflected into [0, pi/4]
    double cv, sv;
    switch (o) {
      case 0: cv = c; sv = s; break;
      case 1: cv = s; sv = c; break;
      case 2: cv = -s; sv = c; break;
      case 3: cv = -c; sv = s; break;
      case 4: cv = -c; sv = -s; break;
      case 5: cv = -s; sv = -c; break;
      case 6: cv = s; sv = -c; break;
      default: cv = c; sv = -s; break;
    }
    if (cv == 0.0) cv = 0.0;   // exact zeros are +0
    if (sv == 0.0) sv = 0.0;
    if (amb) atomicOr(flag, 1);
    chirp[j] = make_double2(cv, sv);
  }
}

hipError_t launch_chirp(double2* chirp, int n, int* flag, hipStream_t s) {
  int blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_chirp, dim3(blocks), dim3(256), 0, s, chirp, n, flag);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-execution state reset; with io set the first workgroup also writes the
// execution's array pointers (a kernel, so that the write is an ordinary
// stream operation, also inside captured graphs).

__global__ void k_reset_io(TState* ts, const int* tlist, IoPtrs* io, const void* in, void* out) {
  const int t = tlist[blockIdx.x];
  u32* w = reinterpret_cast<u32*>(ts + t);
  for (int i = threadIdx.x; i < (int)(sizeof(TState) / 4); i += blockDim.x) w[i] = 0u;
  if (io && blockIdx.x == 0 && threadIdx.x == 0) {
    io->in = in;
    io->out = out;
  }
}

hipError_t launch_reset_io(TState* ts, const int* tlist, int count, IoPtrs* io, const void* in, void* out,
                           hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reset_io, dim3(count), dim3(RESET_THREADS), 0, s, ts, tlist, io, in, out);
  return hipGetLastError();
}
const void* reset_io_kernel() { return reinterpret_cast<const void*>(&k_reset_io); }

// ---------------------------------------------------------------------------
// Premultiply x' = x (.) w (Sec. 3.2 Step 1) and mu_0 = max |x'| per part.
// dir: 0 forward; 1, 2 (inverse, adjoint) transform conj(x).
// kernel_mode: x' is the kernel w* = (c, s) itself (input ignored).

__device__ __forceinline__ u64 abs_bits(double v) { return (u64)__double_as_longlong(v) & 0x7FFFFFFFFFFFFFFFull; }

__device__ __forceinline__ u64 wave_max_u64(u64 v) {
  for (int o = 32; o > 0; o >>= 1) {
    const u64 w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}
// Maximum over the workgroup (blockDim a multiple of 64, at most 1024),
// valid in thread 0; every thread must call it.  One atomic per workgroup
// instead of one per wave keeps the per-transform maxima from serialising.
__device__ __forceinline__ u64 block_max_u64(u64 v) {
  __shared__ u64 part[16];
  v = wave_max_u64(v);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  u64 m = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = part[w] > m ? part[w] : m;
  __syncthreads();
  return m;
}

// x'(j) of transform d: the input element times the chirp, or the kernel
// w* = (c, s) itself (kernel_mode).  The premultiply and every extraction
// pass compute it here, with the same binary64 operations, instead of
// keeping x' in memory.
__device__ __forceinline__ double2 xprime(const void* in, const TDesc& d, const double2* ch, int j, int dir,
                                          bool kernel_mode, int io32) {
  const double2 w = ch[j];
  if (kernel_mode) return w;
  double2 x;
  if (io32) {                       // binary32 input: widened exactly
    const float2 f = reinterpret_cast<const float2*>(in)[d.io_off + j];
    x = make_double2((double)f.x, (double)f.y);
  } else {
    x = reinterpret_cast<const double2*>(in)[d.io_off + j];
  }
  const double xr = x.x, xi = dir ? -x.y : x.y;
  return make_double2(xr * w.x + xi * w.y,      // RN(RN(xr c) + RN(xi s))
                      xi * w.x - xr * w.y);     // RN(RN(xi c) - RN(xr s))
}

// xp == nullptr: the maxima only (the execution); otherwise x' written to
// xp and no maxima (the debug copy).
__global__ void k_premul(const IoPtrs* io, double2* xp, const TDesc* td, const KernelDesc* kd, TState* ts,
                         const int* tlist, int dir, bool kernel_mode, int io32) {
  const int t = tlist[blockIdx.z];
  const void* in = kernel_mode ? nullptr : io->in;
  const TDesc& d = td[t];
  const double2* ch = kd[d.kd].chirp;
  u64 m0 = 0, m1 = 0;
#pragma unroll 4
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += gridDim.x * blockDim.x) {
    const double2 v = xprime(in, d, ch, j, dir, kernel_mode, io32);
    if (xp) {
      xp[d.xp_off + j] = v;
      continue;
    }
    const u64 a = abs_bits(v.x), b = abs_bits(v.y);
    m0 = a > m0 ? a : m0;
    m1 = b > m1 ? b : m1;
  }
  if (xp) return;
  m0 = block_max_u64(m0);
  m1 = block_max_u64(m1);
  if (threadIdx.x == 0) {
    if (m0) atomicMax((unsigned long long*)&ts[t].mu[0][0], (unsigned long long)m0);
    if (m1) atomicMax((unsigned long long*)&ts[t].mu[1][0], (unsigned long long)m1);
  }
}

// Workgroups of 256 threads per vector: 8 elements per thread.
static int chunks_for(int nmax) {
  int b = (nmax + 2047) / 2048;
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return b;
}

hipError_t launch_premul(const IoPtrs* io, double2* xp, const TDesc* td, const KernelDesc* kd, TState* ts,
                         const int* tlist, int count, int nmax, int dir, bool kernel_mode, int io32, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_premul, dim3(chunks_for(nmax), 1, count), dim3(256), 0, s, io, xp, td, kd, ts, tlist, dir,
                     kernel_mode, io32);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Split (Alg. 3 in binary64 with the cap K, Sec. 3.4 / 4.4):
//   mu_k = max|r_k|, E_k = ceil(log2 mu_k), sigma_k = 2^(E_k + 53 - alpha),
//   x_k = fl(fl(r_k + sigma_k) - sigma_k), a_k = x_k 2^(alpha - E_k),
//   r_{k+1} = r_k - x_k.
// Every E_k needs a reduction over the whole vector.  One pass extracts all
// K slices with the exponents speculated gap-free (E_{k+1} = E_k - alpha,
// the common case) and records max|r_{k+1}| under those exponents; a check
// then confirms each exponent in order and, at the first mismatch, restarts
// the extraction from that slice with the corrected exponent.  At most K
// passes are needed and the result equals the sequential algorithm.

__device__ __forceinline__ int ceil_log2_bits(u64 bits) {
  // bits: a positive finite binary64 pattern
  const int ex = (int)(bits >> 52);
  const u64 man = bits & 0xFFFFFFFFFFFFFull;
  if (ex == 0) {                      // subnormal: value = man * 2^-1074
    const int lz = __clzll(man);
    const int top = 63 - lz;          // value in [2^(top-1074), 2^(top-1073))
    const bool pow2 = (man & (man - 1)) == 0;
    return top - 1074 + (pow2 ? 0 : 1);
  }
  return ex - 1023 + (man ? 1 : 0);
}

__global__ void k_split_plan(const TDesc* td, TState* ts, const KernelDesc* kd, const int* tlist, int count, int K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int t = tlist[i];
  const TDesc& d = td[t];
  TState& s = ts[t];
  s.xsh[0] = s.xsh[1] = 0;
  const int alpha = d.alpha;
  int status = 0;
  for (int part = 0; part < 2; ++part) {
    const u64 mu = s.mu[part][0];
    s.active[part] = 0;
    s.kx[part] = 0;
    s.start[part] = 0;
    if (mu >= 0x7FF0000000000000ull) {
      status |= ST_NONFINITE;
      continue;
    }
    if (mu == 0) continue;
    const int E0 = ceil_log2_bits(mu);
    if (E0 - alpha < EMIN_GRID || E0 + MANTISSA - alpha > 1023) {
      status |= ST_RANGE;
      continue;
    }
    for (int k = 0; k < K; ++k) s.Espec[part][k] = E0 - k * alpha;
    s.E[part][0] = E0;
    s.active[part] = 1;
  }
  s.status = status;
  if (status) {
    s.active[0] = s.active[1] = 0;
    s.kx[0] = s.kx[1] = 0;
  } else if (d.acc_mode == ACC_COMPLEX && s.active[0] && s.active[1]) {
    // scale alignment for the complex accumulation: the part whose top
    // exponent lies sh = 1 or 2 binades above the other's is extracted
    // times 2^sh with exponents sh lower, when an anti-diagonal of its
    // products (each then weighing 2^sh) fits the group limit and the
    // scaled slice integers (at most 2^(alpha + sh)) stay below 2^30
    const int dl = s.E[0][0] - s.E[1][0], part = dl > 0 ? 0 : 1, sh = dl > 0 ? dl : -dl;
    const KernelDesc& kk = kd[d.kd];
    const int diag = max(kk.kw[0], kk.kw[1]);              // kernel slices, at most K
    if (sh >= 1 && sh <= 2 && (diag << sh) <= d.acc_limit && alpha + sh <= 30) s.xsh[part] = sh;
  }
}

hipError_t launch_split_plan(const TDesc* td, TState* ts, const KernelDesc* kd, const int* tlist, int count, int K,
                             hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_split_plan, dim3((count + 63) / 64), dim3(64), 0, s, td, ts, kd, tlist, count, K);
  return hipGetLastError();
}

// Residue of u < 2^64 modulo p by Barrett's reduction with m = floor(2^64 / p):
// q = floor(u m / 2^64) undershoots floor(u / p) by at most one, so
// u - q p lies in [0, 2p).
__device__ __forceinline__ u32 mod_barrett(u64 u, u32 p, u64 m) {
  const u64 r = u - __umul64hi(u, m) * (u64)p;
  return (u32)(r >= p ? r - p : r);
}
constexpr u64 BARRETT_P0 = ~0ull / P0, BARRETT_P1 = ~0ull / P1, BARRETT_P2 = ~0ull / P2;

// blockIdx.y = part.  Slices k >= start are written, times 2^xsh[part], as
// residues mod p0 .. p(NP-1) into X[((part*K + k)*NP + prime) N + j]; input
// slices go to positions j < n (the NTT treats the rest as zero), kernel
// slices are placed by ZeroPad+- (positions j and N - j), or at j alone when
// N = n (cyclic embedding).
template <int NP>
__global__ void k_split_extract(const IoPtrs* io, const KernelDesc* kd, u32* X, const TDesc* td, TState* ts,
                                const int* tlist, int K, int dir, bool kernel_mode, int io32) {
  const int t = tlist[blockIdx.z];
  const int part = blockIdx.y;
  TState& s = ts[t];
  if (!s.active[part]) return;
  const TDesc& d = td[t];
  const void* in = kernel_mode ? nullptr : io->in;
  const double2* ch = kd[d.kd].chirp;
  const int alpha = d.alpha, start = s.start[part], sh = s.xsh[part];
  int Ek[KMAX];
  int kend = K;
  for (int k = 0; k < K; ++k) {
    Ek[k] = k < start ? s.E[part][k] : s.Espec[part][k];
    if (Ek[k] - alpha < EMIN_GRID && kend == K) kend = k;
  }
  u64 mloc[KMAX];
  for (int k = 0; k < KMAX; ++k) mloc[k] = 0;
  u32* Xb = X + d.X_off;
  const size_t N = (size_t)1 << d.logN;
#pragma unroll 4
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += gridDim.x * blockDim.x) {
    const double2 v = xprime(in, d, ch, j, dir, kernel_mode, io32);
    double r = part ? v.y : v.x;
    for (int k = 0; k < kend; ++k) {
      const int E = Ek[k];
      const double sigma = ldexp(1.0, E + MANTISSA - alpha);
      const double x = (r + sigma) - sigma;
      r = r - x;
      if (k >= start) {
        // x is a multiple of 2^(E - alpha) with |x| <= 2^E, so scaling x itself is
        // exact; the factor 2^(alpha - E + sh) alone can exceed the binary64 range
        // (E - alpha down to -1022, sh up to 2)
        u32 res[NP];
        if constexpr (NP == 2) {
          const int a = (int)ldexp(x, alpha - E + sh);   // |a| <= 2^(alpha + sh) <= 2^30 < p0, p1
          res[0] = a < 0 ? (u32)(a + (int)P0) : (u32)a;
          res[1] = a < 0 ? (u32)(a + (int)P1) : (u32)a;
        } else {
          // three moduli: |a| <= 2^alpha with alpha up to 46, reduced as |a|
          // and negated
          const long long a = (long long)ldexp(x, alpha - E + sh);
          const u64 u = (u64)(a < 0 ? -a : a);
          const u32 m0 = mod_barrett(u, P0, BARRETT_P0), m1 = mod_barrett(u, P1, BARRETT_P1),
                    m2 = mod_barrett(u, P2, BARRETT_P2);
          res[0] = a < 0 && m0 ? P0 - m0 : m0;
          res[1] = a < 0 && m1 ? P1 - m1 : m1;
          res[2] = a < 0 && m2 ? P2 - m2 : m2;
        }
        u32* v0 = Xb + (((size_t)((part * K + k) * NP)) << d.logN);
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          v0[q * N + j] = res[q];
          if (kernel_mode && j > 0 && N != (size_t)d.n) v0[q * N + N - j] = res[q];   // ZeroPad+- (cyclic: no wrap)
        }
        const u64 rb = abs_bits(r);
        if (rb > mloc[k]) mloc[k] = rb;
      }
    }
  }
  for (int k = start; k < kend && k + 1 < K; ++k) {
    const u64 m = block_max_u64(mloc[k]);
    if (threadIdx.x == 0 && m) atomicMax((unsigned long long*)&s.mu[part][k + 1], (unsigned long long)m);
  }
}

hipError_t launch_split_extract(const IoPtrs* io, const KernelDesc* kd, u32* X, const TDesc* td, TState* ts,
                                const int* tlist, int count, int nmax, int K, int dir, bool kernel_mode, int io32,
                                int np, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (np == 3)
    hipLaunchKernelGGL(k_split_extract<3>, dim3(chunks_for(nmax), 2, count), dim3(256), 0, s, io, kd, X, td, ts, tlist,
                       K, dir, kernel_mode, io32);
  else
    hipLaunchKernelGGL(k_split_extract<2>, dim3(chunks_for(nmax), 2, count), dim3(256), 0, s, io, kd, X, td, ts, tlist,
                       K, dir, kernel_mode, io32);
  return hipGetLastError();
}

__global__ void k_split_check(const TDesc* td, TState* ts, const int* tlist, int count, int K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * count) return;
  const int t = tlist[i >> 1], part = i & 1;
  TState& s = ts[t];
  if (!s.active[part]) return;
  const int alpha = td[t].alpha;
  int kx = K;
  for (int k = s.start[part] + 1; k < K; ++k) {
    const u64 mu = s.mu[part][k];
    if (mu == 0) { kx = k; break; }
    const int Et = ceil_log2_bits(mu);
    if (Et - alpha < EMIN_GRID) { kx = k; break; }
    if (Et != s.Espec[part][k]) {
      // restart the extraction at slice k with the confirmed exponent
      s.E[part][k] = Et;
      for (int k2 = k; k2 < K; ++k2) s.Espec[part][k2] = Et - (k2 - k) * alpha;
      for (int k2 = k + 1; k2 <= K; ++k2) s.mu[part][k2] = 0;
      s.start[part] = k;
      return;
    }
    s.E[part][k] = Et;
  }
  s.kx[part] = kx;
  s.active[part] = 0;
}

hipError_t launch_split_check(const TDesc* td, TState* ts, const int* tlist, int count, int K, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_split_check, dim3((2 * count + 63) / 64), dim3(64), 0, s, td, ts, tlist, count, K);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The accumulation schedule of every transform.  One thread per transform.
__global__ void k_groups(const TDesc* td, TState* ts, const KernelDesc* kd, const int* tlist, int count, int K, int L) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int t = tlist[i];
  const TDesc& d = td[t];
  TState& s = ts[t];
  const KernelDesc& kk = kd[d.kd];
  __shared__ int sE[64][2][KMAX], sW[64][2][KMAX];
  int (&E)[2][KMAX] = sE[threadIdx.x];
  int (&Ew)[2][KMAX] = sW[threadIdx.x];
  for (int part = 0; part < 2; ++part)
    for (int k = 0; k < KMAX; ++k) {
      E[part][k] = s.E[part][k];
      Ew[part][k] = kk.Ew[part][k];
    }
  schedule_walk(d, s, kk, E, Ew, L);
  (void)K;
}

hipError_t launch_groups(const TDesc* td, TState* ts, const KernelDesc* kd, const int* tlist, int count, int K, int L,
                         hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_groups, dim3((count + 63) / 64), dim3(64), 0, s, td, ts, kd, tlist, count, K, L);
  return hipGetLastError();
}

}  // namespace fo
