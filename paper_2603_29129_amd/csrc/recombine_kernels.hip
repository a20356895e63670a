// Garner CRT, exact recombination to binary64 and chirp postmultiply.
//
// For each output index k < n and each group g of the accumulation schedule
// the inverse-NTT residues are combined by Garner's formula (Sec. 3.3)
//     z = z0 + ((z1 - z0) p0^{-1} mod p1) p0,  mapped to [-(P-1)/2, (P-1)/2]
// (with a third modulus p2 the mixed-radix form adds p0 p1 h2, P = p0 p1 p2),
// which is the exact signed integer value of the group's sum because at most
// acc_limit products of magnitude <= n 4^alpha enter it and
// acc_limit n 4^alpha <= (P-1)/2 (Sec. 4.2 / 4.4; the ImIm products enter Re y'
// with a minus sign, already applied in the NTT domain).  Each component of
// y' is then the exact sum of z 2^e over its groups,
// accumulated in a two's-complement fixed-point integer (4 x 64 bits when the
// exponents of the transform span <= 185 bits, 152 with three moduli; 50 x 64
// bits otherwise) and
// rounded once to binary64, round to nearest even, subnormals and overflow
// included.  The chirp postmultiply y = y' (.) w (Sec. 3.2 Step 3) uses the
// same unfused product rule as the premultiply.
#include "crt_dev.h"

namespace fo {

// Both outputs j, j + 1 of one component (j even; the compact rows are
// padded to a multiple of four, so j + 1 is always a readable position).
// Compact buffer: row (slot NP + prime) of zs words.
template <int NP>
__device__ void recombine_fast2(const u32* Zb, const TState& s, int tg, int SL, int zs, int j, double& r0,
                                double& r1) {
  u32 a[NL_FAST], b[NL_FAST];
#pragma unroll
  for (int k = 0; k < NL_FAST; ++k) a[k] = b[k] = 0;
  const int emin = s.emin[tg];
  for (int g = 0; g < s.ngroups[tg]; ++g) {
    const int slot = tg * SL + g;
    u32 z0[NP], z1[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const uint2 v = *reinterpret_cast<const uint2*>(Zb + (size_t)(slot * NP + q) * zs + j);
      z0[q] = v.x;
      z1[q] = v.y;
    }
    const int sh = s.groups[tg][g].e - emin;
    limb_add_crt<NP>(a, z0, sh);
    limb_add_crt<NP>(b, z1, sh);
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

template <int NP, int W>
__device__ double recombine_one(const u32* Zb, const TState& s, int tg, int SL, int zs, int j) {
  u64 acc[W];
#pragma unroll
  for (int w = 0; w < W; ++w) acc[w] = 0;
  const int emin = s.emin[tg];
  for (int g = 0; g < s.ngroups[tg]; ++g) {
    const int slot = tg * SL + g;
    u32 z[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) z[q] = Zb[(size_t)(slot * NP + q) * zs + j];
    acc_add_crt<NP, W>(acc, z, s.groups[tg][g].e - emin);
  }
  return acc_round<W>(acc, emin);
}

// WIDE = false: transforms whose exponent spans fit the fast accumulator (and
// those with a status, which get NaN), two outputs per thread;
// WIDE = true: the others, one output per thread.
template <bool WIDE, int NP>
__global__ void k_recombine(const u32* Z, const IoPtrs* io, const TDesc* td, const TState* ts, const KernelDesc* kd,
                            const int* tlist, int K, int dir, int io32) {
  const int t = tlist[blockIdx.z];
  void* out = io->out;
  const TDesc& d = td[t];
  const TState& s = ts[t];
  const bool wide0 = span_wide<NP>(s, 0), wide1 = span_wide<NP>(s, 1);
  if (WIDE != (!s.status && (wide0 || wide1))) return;
  const double2* ch = kd[d.kd].chirp;
  const int SL = 2 * K * K;                                   // slots per output component
  const u32* Zb = Z + d.Z_off;
  if (!WIDE) {
    for (int j = 2 * (blockIdx.x * blockDim.x + threadIdx.x); j < d.n; j += 2 * gridDim.x * blockDim.x) {
      double2 o0, o1;
      if (s.status) {
        o0 = o1 = make_double2(__builtin_nan(""), __builtin_nan(""));
      } else {
        double pr0, pr1, pi0, pi1;
        recombine_fast2<NP>(Zb, s, 0, SL, d.zs, j, pr0, pr1);
        recombine_fast2<NP>(Zb, s, 1, SL, d.zs, j, pi0, pi1);
        o0 = finish(pr0, pi0, ch[j], dir, d.n);
        o1 = j + 1 < d.n ? finish(pr1, pi1, ch[j + 1], dir, d.n) : o0;
      }
      put_out(out, d.io_off + j, o0, io32);
      if (j + 1 < d.n) put_out(out, d.io_off + j + 1, o1, io32);
    }
    return;
  }
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += gridDim.x * blockDim.x) {
    const double pr = wide0 ? recombine_one<NP, W_WIDE>(Zb, s, 0, SL, d.zs, j)
                            : recombine_one<NP, W_FAST>(Zb, s, 0, SL, d.zs, j);
    const double pi = wide1 ? recombine_one<NP, W_WIDE>(Zb, s, 1, SL, d.zs, j)
                            : recombine_one<NP, W_FAST>(Zb, s, 1, SL, d.zs, j);
    put_out(out, d.io_off + j, finish(pr, pi, ch[j], dir, d.n), io32);
  }
}

static int recombine_blocks(int nmax) {
  int b = (nmax + 255) / 256;
  if (b > 2048) b = 2048;
  return b < 1 ? 1 : b;
}

template <bool WIDE, int NP>
static void launch_rec(int blocks, int count, hipStream_t s, const u32* Z, const IoPtrs* io, const TDesc* td,
                       const TState* ts, const KernelDesc* kd, const int* tlist, int K, int dir, int io32) {
  hipLaunchKernelGGL((k_recombine<WIDE, NP>), dim3(blocks, 1, count), dim3(256), 0, s, Z, io, td, ts, kd, tlist, K,
                     dir, io32);
}

hipError_t launch_recombine(const u32* Z, const IoPtrs* io, const TDesc* td, const TState* ts, const KernelDesc* kd,
                            const int* tlist, int count, int nmax, int K, int dir, int io32, hipStream_t s, int np) {
  if (count <= 0) return hipSuccess;
  if (np != 2 && np != 3) return hipErrorInvalidValue;
  const int b = recombine_blocks(nmax), b2 = (b + 1) / 2;      // two outputs per thread in the fast kernel
  if (np == 3) {
    launch_rec<false, 3>(b2, count, s, Z, io, td, ts, kd, tlist, K, dir, io32);
    launch_rec<true, 3>(b, count, s, Z, io, td, ts, kd, tlist, K, dir, io32);
  } else {
    launch_rec<false, 2>(b2, count, s, Z, io, td, ts, kd, tlist, K, dir, io32);
    launch_rec<true, 2>(b, count, s, Z, io, td, ts, kd, tlist, K, dir, io32);
  }
  return hipGetLastError();
}

hipError_t launch_recombine_wide(const u32* Z, const IoPtrs* io, const TDesc* td, const TState* ts, const KernelDesc* kd,
                                 const int* tlist, int count, int nmax, int K, int dir, int io32, hipStream_t s,
                                 int np) {
  if (count <= 0) return hipSuccess;
  if (np != 2 && np != 3) return hipErrorInvalidValue;
  const int b = recombine_blocks(nmax);
  if (np == 3) launch_rec<true, 3>(b, count, s, Z, io, td, ts, kd, tlist, K, dir, io32);
  else launch_rec<true, 2>(b, count, s, Z, io, td, ts, kd, tlist, K, dir, io32);
  return hipGetLastError();
}

// One thread writes the execution's array pointers (a kernel, so that the
// write is an ordinary stream operation, also inside captured graphs).
__global__ void k_set_io(IoPtrs* io, const void* in, void* out) {
  io->in = in;
  io->out = out;
}
hipError_t launch_set_io(IoPtrs* io, const void* in, void* out, hipStream_t s) {
  hipLaunchKernelGGL(k_set_io, dim3(1), dim3(1), 0, s, io, in, out);
  return hipGetLastError();
}
}  // namespace fo
