// Garner CRT, exact recombination to binary64 and chirp postmultiply.
//
// For each output index k < n and each group g of the accumulation schedule
// the two inverse-NTT residues are combined by Garner's formula (Sec. 3.3)
//     z = z0 + ((z1 - z0) p0^{-1} mod p1) p0,  mapped to [-(P-1)/2, (P-1)/2],
// which is the exact signed integer value of the group's sum because at most
// acc_limit products of magnitude <= n 4^alpha enter it and
// acc_limit n 4^alpha <= (P-1)/2 (Sec. 4.2 / 4.4; the ImIm products enter Re y'
// with a minus sign, already applied in the NTT domain).  Each component of
// y' is then the exact sum of z 2^e over its groups,
// accumulated in a two's-complement fixed-point integer (4 x 64 bits when the
// exponents of the transform span <= 185 bits, 50 x 64 bits otherwise) and
// rounded once to binary64, round to nearest even, subnormals and overflow
// included.  The chirp postmultiply y = y' (.) w (Sec. 3.2 Step 3) uses the
// same unfused product rule as the premultiply.
#include "crt_dev.h"

namespace fo {

// Both outputs j, j + 1 of one component (j even; the compact rows are
// padded to a multiple of four, so j + 1 is always a readable position).
__device__ void recombine_fast2(const u32* Zb, const TState& s, int tg, int SL, int zs, int j, double& r0,
                                double& r1) {
  u32 a[NL_FAST], b[NL_FAST];
#pragma unroll
  for (int k = 0; k < NL_FAST; ++k) a[k] = b[k] = 0;
  const int emin = s.emin[tg];
  for (int g = 0; g < s.ngroups[tg]; ++g) {
    const int slot = tg * SL + g;
    const uint2 v0 = *reinterpret_cast<const uint2*>(Zb + (size_t)(slot * 2) * zs + j);
    const uint2 v1 = *reinterpret_cast<const uint2*>(Zb + (size_t)(slot * 2 + 1) * zs + j);
    const int sh = s.groups[tg][g].e - emin;
    limb_add(a, garner(v0.x, v1.x), sh);
    limb_add(b, garner(v0.y, v1.y), sh);
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
  for (int g = 0; g < s.ngroups[tg]; ++g) {
    const int slot = tg * SL + g;
    const u32 z0 = Zb[(size_t)(slot * 2) * zs + j];
    const u32 z1 = Zb[(size_t)(slot * 2 + 1) * zs + j];
    acc_add<W>(acc, garner(z0, z1), s.groups[tg][g].e - emin);
  }
  return acc_round<W>(acc, emin);
}

// WIDE = false: transforms whose exponent spans fit the fast accumulator (and
// those with a status, which get NaN), two outputs per thread;
// WIDE = true: the others, one output per thread.
template <bool WIDE>
__global__ void k_recombine(const u32* Z, const IoPtrs* io, const TDesc* td, const TState* ts, const KernelDesc* kd,
                            const int* tlist, int K, int dir, int io32) {
  const int t = tlist[blockIdx.z];
  void* out = io->out;
  const TDesc& d = td[t];
  const TState& s = ts[t];
  const bool wide0 = span_wide(s, 0), wide1 = span_wide(s, 1);
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
        recombine_fast2(Zb, s, 0, SL, d.zs, j, pr0, pr1);
        recombine_fast2(Zb, s, 1, SL, d.zs, j, pi0, pi1);
        o0 = finish(pr0, pi0, ch[j], dir, d.n);
        o1 = j + 1 < d.n ? finish(pr1, pi1, ch[j + 1], dir, d.n) : o0;
      }
      put_out(out, d.io_off + j, o0, io32);
      if (j + 1 < d.n) put_out(out, d.io_off + j + 1, o1, io32);
    }
    return;
  }
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += gridDim.x * blockDim.x) {
    const double pr = wide0 ? recombine_one<W_WIDE>(Zb, s, 0, SL, d.zs, j) : recombine_one<W_FAST>(Zb, s, 0, SL, d.zs, j);
    const double pi = wide1 ? recombine_one<W_WIDE>(Zb, s, 1, SL, d.zs, j) : recombine_one<W_FAST>(Zb, s, 1, SL, d.zs, j);
    put_out(out, d.io_off + j, finish(pr, pi, ch[j], dir, d.n), io32);
  }
}

hipError_t launch_recombine(const u32* Z, const IoPtrs* io, const TDesc* td, const TState* ts, const KernelDesc* kd,
                            const int* tlist, int count, int nmax, int K, int dir, int io32, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int b = (nmax + 255) / 256;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  const int b2 = (b + 1) / 2;      // two outputs per thread
  hipLaunchKernelGGL(k_recombine<false>, dim3(b2, 1, count), dim3(256), 0, s, Z, io, td, ts, kd, tlist, K, dir, io32);
  hipLaunchKernelGGL(k_recombine<true>, dim3(b, 1, count), dim3(256), 0, s, Z, io, td, ts, kd, tlist, K, dir, io32);
  return hipGetLastError();
}

}  // namespace fo

namespace fo {
hipError_t launch_recombine_wide(const u32* Z, const IoPtrs* io, const TDesc* td, const TState* ts, const KernelDesc* kd,
                                 const int* tlist, int count, int nmax, int K, int dir, int io32, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int b = (nmax + 255) / 256;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_recombine<true>, dim3(b, 1, count), dim3(256), 0, s, Z, io, td, ts, kd, tlist, K, dir, io32);
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
const void* set_io_kernel() { return reinterpret_cast<const void*>(&k_set_io); }
}  // namespace fo
