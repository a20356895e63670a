// Number-theoretic transforms modulo p0 = 2130706433 and p1 = 2113929217 on
// gfx950 (Sec. 3.3: y(k) = sum_j x(j) w_N^{jk} mod p, inverse with N^{-1}).
//
// Design:
//  * A block NTT of length M <= 4096 runs inside one workgroup on an LDS tile.
//    The forward transform is decimation in frequency (natural order in,
//    bit-reversed order out); the inverse is its exact mirror, decimation in
//    time (bit-reversed in, natural out), so no permutation pass is needed:
//    the pointwise products of the convolution work on bit-reversed data.
//  * Each thread holds 2^r elements (r <= 4) in registers and performs r
//    radix-2 stages between LDS exchanges, so a 4096-point transform takes
//    three LDS round trips.
//  * Lengths N > 4096 use two passes N = N1 * N2: column transforms of length
//    N1 (stride N2, a tile of C adjacent columns per workgroup so that global
//    accesses are C*4 bytes contiguous), the twiddle w_N^{j2 k1}, then
//    contiguous row transforms of length N2.
//  * Modular products are Shoup multiplications by precomputed constants
//    (value and floor(w 2^32 / p)); gfx950 issues v_mul_lo_u32 / v_mul_hi_u32
//    at full rate, so a butterfly is ~11 VALU instructions.
//  * The convolution's pointwise products and their NTT-domain accumulation
//    (Alg. 8) are fused into the first inverse pass; N^{-1} is folded into the
//    precomputed kernel transforms.
#include "internal.h"

namespace fo {

__device__ __forceinline__ u32 prime_of(int i) { return i ? P1 : P0; }
__device__ __forceinline__ u32 bitrev(u32 v, int bits) { return bits ? (__brev(v) >> (32 - bits)) : 0u; }

// LDS addressing of element i of vector v inside a tile.  COLS: vectors are
// interleaved (element i of all vectors adjacent), used by the column pass.
// Rows: one vector after another with one pad word every 32 elements.
__host__ __device__ inline int row_ld(int M) { return M + (M >> 5) + 1; }
template <bool COLS>
__device__ __forceinline__ int laddr(int v, int i, int lnvec, int ldr) {
  return COLS ? ((i << lnvec) + v) : (v * ldr + i + (i >> 5));
}

// r = RL radix-2 stages on the 2^RL registers of one group.  The group holds
// tile elements base + j*st (j < 2^RL) of a length-2^m vector and the round
// covers stages s0 .. s0+RL-1 (stage s pairs elements h = 2^(m-s-1) apart).
// tw[e] = (w_M^e, companion) for e < M/2 (forward or inverse roots).
template <int RL, bool INV>
__device__ __forceinline__ void radix_group(u32 (&a)[1 << RL], int base, int st, int m, int s0,
                                            const uint2* __restrict__ tw, u32 p) {
  constexpr int R = 1 << RL;
  if (!INV) {
#pragma unroll
    for (int ss = 0; ss < RL; ++ss) {
      const int s = s0 + ss;
      const int hd = R >> (ss + 1);
      const int hmask = (1 << (m - s - 1)) - 1;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        if (j & hd) continue;
        const uint2 w = tw[((base + j * st) & hmask) << s];
        const u32 x = a[j], y = a[j + hd];
        a[j] = add_mod(x, y, p);
        a[j + hd] = shoup_mul(x + p - y, w.x, w.y, p);   // x - y + p < 2p < 2^32
      }
    }
  } else {
#pragma unroll
    for (int ss = RL - 1; ss >= 0; --ss) {
      const int s = s0 + ss;
      const int hd = R >> (ss + 1);
      const int hmask = (1 << (m - s - 1)) - 1;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        if (j & hd) continue;
        const uint2 w = tw[((base + j * st) & hmask) << s];
        const u32 x = a[j];
        const u32 t = shoup_mul(a[j + hd], w.x, w.y, p);
        a[j] = add_mod(x, t, p);
        a[j + hd] = sub_mod(x, t, p);
      }
    }
  }
}

template <int RL, bool INV, bool COLS>
__device__ void ntt_round(u32* lds, int m, int s0, int lnvec, int ldr, const uint2* tw, u32 p) {
  constexpr int R = 1 << RL;
  const int lbk = m - s0;              // log2 of the block size
  const int lst = lbk - RL;            // log2 of the register stride
  const int st = 1 << lst;
  const int lgpv = m - RL;             // log2 groups per vector
  const int total = 1 << (lnvec + lgpv);
  for (int g = threadIdx.x; g < total; g += blockDim.x) {
    int v, q;
    if (COLS) {
      v = g & ((1 << lnvec) - 1);
      q = g >> lnvec;
    } else {
      v = g >> lgpv;
      q = g & ((1 << lgpv) - 1);
    }
    const int base = ((q >> lst) << lbk) + (q & (st - 1));
    u32 a[R];
#pragma unroll
    for (int j = 0; j < R; ++j) a[j] = lds[laddr<COLS>(v, base + j * st, lnvec, ldr)];
    radix_group<RL, INV>(a, base, st, m, s0, tw, p);
#pragma unroll
    for (int j = 0; j < R; ++j) lds[laddr<COLS>(v, base + j * st, lnvec, ldr)] = a[j];
  }
}

// In-place block NTT of 2^lnvec vectors of length 2^m held in LDS.  The caller
// synchronises after filling the tile; this routine ends synchronised.
template <bool INV, bool COLS>
__device__ void block_ntt(u32* lds, int m, int lnvec, int ldr, const uint2* tw, u32 p) {
  const int nr = (m + 3) >> 2;
  for (int rr = 0; rr < nr; ++rr) {
    const int round = INV ? (nr - 1 - rr) : rr;
    const int s0 = round << 2;
    const int r = min(4, m - s0);
    switch (r) {
      case 4: ntt_round<4, INV, COLS>(lds, m, s0, lnvec, ldr, tw, p); break;
      case 3: ntt_round<3, INV, COLS>(lds, m, s0, lnvec, ldr, tw, p); break;
      case 2: ntt_round<2, INV, COLS>(lds, m, s0, lnvec, ldr, tw, p); break;
      default: ntt_round<1, INV, COLS>(lds, m, s0, lnvec, ldr, tw, p); break;
    }
    __syncthreads();
  }
}

// Copies the roots w_M^e (e < M/2) of a length-2^m block NTT into LDS from the
// 4096-point table.
__device__ __forceinline__ void load_block_tw(uint2* tw, const uint2* __restrict__ src, int m) {
  const int half = m ? (1 << (m - 1)) : 0;
  for (int e = threadIdx.x; e < half; e += blockDim.x) tw[e] = src[e << (LOG2_BLOCK_MAX - m)];
}

// w_N^e (forward or inverse) applied to x, e < N.
__device__ __forceinline__ u32 step_twiddle(u32 x, u32 e, const uint2* __restrict__ lo,
                                            const uint2* __restrict__ hi, u32 p) {
  const uint2 a = lo[e & 4095u];
  x = shoup_mul(x, a.x, a.y, p);
  const uint2 b = hi[e >> 12];
  return shoup_mul(x, b.x, b.y, p);
}

// ---------------------------------------------------------------------------
// Transform bodies shared by the pipeline and the standalone kernels.

// Forward column pass on vector `vec` (elements >= valid read as zero).
__device__ void fwd_cols_body(u32* vec, int valid, int prime, const NttGeom g, int j2_0,
                              const uint2* twb, const uint2* lo, const uint2* hi, u32* smem) {
  const u32 p = prime_of(prime);
  const int m1 = g.m1, N2 = 1 << g.m2, lc = g.lc, C = 1 << lc;
  const u32 Nmask = (1u << g.logN) - 1;
  uint2* tw = reinterpret_cast<uint2*>(smem);
  u32* tile = smem + (1 << m1);
  load_block_tw(tw, twb, m1);
  const int tot = C << m1;
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int c = idx & (C - 1), i1 = idx >> lc;
    const int gi = i1 * N2 + j2_0 + c;
    tile[idx] = gi < valid ? vec[gi] : 0u;
  }
  __syncthreads();
  block_ntt<false, true>(tile, m1, lc, 0, tw, p);
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int c = idx & (C - 1), i1 = idx >> lc;
    const u32 e = ((u32)(j2_0 + c) * bitrev(i1, m1)) & Nmask;
    vec[i1 * N2 + j2_0 + c] = step_twiddle(tile[idx], e, lo, hi, p);
  }
}

// Forward row pass: rows [i1_0, i1_0 + 2^lrows) of vector vec.
__device__ void fwd_rows_body(u32* vec, int prime, const NttGeom g, int i1_0, const uint2* twb, u32* smem) {
  const u32 p = prime_of(prime);
  const int m2 = g.m2, N2 = 1 << m2, lr = g.lrows, ldr = row_ld(N2);
  uint2* tw = reinterpret_cast<uint2*>(smem);
  u32* tile = smem + N2;
  load_block_tw(tw, twb, m2);
  const int tot = N2 << lr;
  u32* src = vec + (size_t)i1_0 * N2;
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int r = idx >> m2, i = idx & (N2 - 1);
    tile[r * ldr + i + (i >> 5)] = src[idx];
  }
  __syncthreads();
  block_ntt<false, false>(tile, m2, lr, ldr, tw, p);
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int r = idx >> m2, i = idx & (N2 - 1);
    src[idx] = tile[r * ldr + i + (i >> 5)];
  }
}

// Forward single-workgroup transform of a vector of length 2^logN <= 4096.
__device__ void fwd_single_body(u32* vec, int valid, int prime, int logN, const uint2* twb, u32* smem) {
  const u32 p = prime_of(prime);
  const int N = 1 << logN, ldr = row_ld(N);
  uint2* tw = reinterpret_cast<uint2*>(smem);
  u32* tile = smem + N;
  load_block_tw(tw, twb, logN);
  for (int i = threadIdx.x; i < N; i += blockDim.x) tile[i + (i >> 5)] = i < valid ? vec[i] : 0u;
  __syncthreads();
  block_ntt<false, false>(tile, logN, 0, ldr, tw, p);
  for (int i = threadIdx.x; i < N; i += blockDim.x) vec[i] = tile[i + (i >> 5)];
}

// ---------------------------------------------------------------------------
// Standalone kernels (count contiguous vectors; blockIdx.z = vector).

__global__ void __launch_bounds__(NTT_THREADS) k_std_single(u32* data, int logN, int prime, bool inverse,
                                                            TwBlock tb) {
  extern __shared__ u32 smem[];
  u32* vec = data + ((size_t)blockIdx.z << logN);
  const int N = 1 << logN;
  if (!inverse) {
    fwd_single_body(vec, N, prime, logN, tb.fwd[prime], smem);
    return;
  }
  const u32 p = prime_of(prime);
  const int ldr = row_ld(N);
  uint2* tw = reinterpret_cast<uint2*>(smem);
  u32* tile = smem + N;
  load_block_tw(tw, tb.inv[prime], logN);
  for (int i = threadIdx.x; i < N; i += blockDim.x) tile[i + (i >> 5)] = vec[i];
  __syncthreads();
  block_ntt<true, false>(tile, logN, 0, ldr, tw, p);
  // N^{-1} = p - (p-1)/N
  const u32 ninv = p - ((p - 1) >> logN), ninvq = shoup_companion(ninv, p);
  for (int i = threadIdx.x; i < N; i += blockDim.x) vec[i] = shoup_mul(tile[i + (i >> 5)], ninv, ninvq, p);
}

__global__ void __launch_bounds__(NTT_THREADS) k_std_fwd_cols(u32* data, int prime, NttGeom g, TwBlock tb, TwStep ts) {
  extern __shared__ u32 smem[];
  u32* vec = data + ((size_t)blockIdx.z << g.logN);
  fwd_cols_body(vec, 1 << g.logN, prime, g, blockIdx.x << g.lc, tb.fwd[prime], ts.lo[0][prime], ts.hi[0][prime], smem);
}

__global__ void __launch_bounds__(NTT_THREADS) k_std_fwd_rows(u32* data, int prime, NttGeom g, TwBlock tb) {
  extern __shared__ u32 smem[];
  u32* vec = data + ((size_t)blockIdx.z << g.logN);
  fwd_rows_body(vec, prime, g, blockIdx.x << g.lrows, tb.fwd[prime], smem);
}

// Inverse row pass (standalone): DIT rows then w_N^{-j2 k1}.
__global__ void __launch_bounds__(NTT_THREADS) k_std_inv_rows(u32* data, int prime, NttGeom g, TwBlock tb, TwStep ts) {
  extern __shared__ u32 smem[];
  u32* vec = data + ((size_t)blockIdx.z << g.logN);
  const u32 p = prime_of(prime);
  const int m2 = g.m2, N2 = 1 << m2, lr = g.lrows, ldr = row_ld(N2);
  const u32 Nmask = (1u << g.logN) - 1;
  uint2* tw = reinterpret_cast<uint2*>(smem);
  u32* tile = smem + N2;
  load_block_tw(tw, tb.inv[prime], m2);
  const int i1_0 = blockIdx.x << lr;
  const int tot = N2 << lr;
  u32* src = vec + (size_t)i1_0 * N2;
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int r = idx >> m2, i = idx & (N2 - 1);
    tile[r * ldr + i + (i >> 5)] = src[idx];
  }
  __syncthreads();
  block_ntt<true, false>(tile, m2, lr, ldr, tw, p);
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int r = idx >> m2, j2 = idx & (N2 - 1);
    const u32 e = ((u32)j2 * bitrev(i1_0 + r, g.m1)) & Nmask;
    src[idx] = step_twiddle(tile[r * ldr + j2 + (j2 >> 5)], e, ts.lo[1][prime], ts.hi[1][prime], p);
  }
}

// Inverse column pass (standalone): DIT columns, times N^{-1}, natural order.
__global__ void __launch_bounds__(NTT_THREADS) k_std_inv_cols(u32* data, int prime, NttGeom g, TwBlock tb) {
  extern __shared__ u32 smem[];
  u32* vec = data + ((size_t)blockIdx.z << g.logN);
  const u32 p = prime_of(prime);
  const int m1 = g.m1, N2 = 1 << g.m2, lc = g.lc, C = 1 << lc;
  uint2* tw = reinterpret_cast<uint2*>(smem);
  u32* tile = smem + (1 << m1);
  load_block_tw(tw, tb.inv[prime], m1);
  const int j2_0 = blockIdx.x << lc;
  const int tot = C << m1;
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int c = idx & (C - 1), i1 = idx >> lc;
    tile[idx] = vec[i1 * N2 + j2_0 + c];
  }
  __syncthreads();
  block_ntt<true, true>(tile, m1, lc, 0, tw, p);
  const u32 ninv = p - ((p - 1) >> g.logN), ninvq = shoup_companion(ninv, p);
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int c = idx & (C - 1), i1 = idx >> lc;
    vec[i1 * N2 + j2_0 + c] = shoup_mul(tile[idx], ninv, ninvq, p);
  }
}

// ---------------------------------------------------------------------------
// Pipeline kernels.  blockIdx.z indexes the transform list.

struct FwdSel {
  u32* vec;
  int valid, prime;
};

__device__ __forceinline__ bool fwd_select(u32* X, const TDesc* td, const TState* ts, const int* tlist, int K,
                                           bool valid_full, int vi, FwdSel& o) {
  const int t = tlist[blockIdx.z];
  const TDesc& d = td[t];
  const TState& s = ts[t];
  const int part = vi / (2 * K), k = (vi >> 1) % K;
  if (s.status || k >= s.kx[part]) return false;
  o.vec = X + d.X_off + ((size_t)vi << d.logN);
  o.valid = valid_full ? d.N : d.n;
  o.prime = vi & 1;
  return true;
}

__global__ void __launch_bounds__(NTT_THREADS) k_fwd_single(u32* X, const TDesc* td, const TState* ts,
                                                            const int* tlist, int K, bool valid_full, int vi_lo,
                                                            int logN, TwBlock tb) {
  extern __shared__ u32 smem[];
  FwdSel o;
  if (!fwd_select(X, td, ts, tlist, K, valid_full, vi_lo + blockIdx.y, o)) return;
  fwd_single_body(o.vec, o.valid, o.prime, logN, tb.fwd[o.prime], smem);
}

__global__ void __launch_bounds__(NTT_THREADS) k_fwd_cols(u32* X, const TDesc* td, const TState* ts,
                                                          const int* tlist, int K, bool valid_full, int vi_lo,
                                                          NttGeom g, TwBlock tb, TwStep st) {
  extern __shared__ u32 smem[];
  FwdSel o;
  if (!fwd_select(X, td, ts, tlist, K, valid_full, vi_lo + blockIdx.y, o)) return;
  fwd_cols_body(o.vec, o.valid, o.prime, g, blockIdx.x << g.lc, tb.fwd[o.prime], st.lo[0][o.prime],
                st.hi[0][o.prime], smem);
}

__global__ void __launch_bounds__(NTT_THREADS) k_fwd_rows(u32* X, const TDesc* td, const TState* ts,
                                                          const int* tlist, int K, bool valid_full, int vi_lo,
                                                          NttGeom g, TwBlock tb) {
  extern __shared__ u32 smem[];
  FwdSel o;
  if (!fwd_select(X, td, ts, tlist, K, valid_full, vi_lo + blockIdx.y, o)) return;
  fwd_rows_body(o.vec, o.prime, g, blockIdx.x << g.lrows, tb.fwd[o.prime], smem);
}

// The four real convolutions (Sec. 4.5): input part pa with kernel part pb.
__device__ __constant__ int c_conv_pa[4] = {0, 1, 1, 0};
__device__ __constant__ int c_conv_pb[4] = {0, 1, 0, 1};

// Accumulates sum over the pairs of group (c, g) of X_pa^s (.) W_pb^t at
// NTT-domain position idx (Alg. 8, NTT-domain accumulation).
__device__ __forceinline__ u32 group_mac(const u32* __restrict__ Xb, const u32* __restrict__ Wb,
                                         const u32* __restrict__ Wqb, const TState& s, int c, const Group& gr,
                                         int K, int prime, int logN, size_t idx, u32 p) {
  const int pa = c_conv_pa[c], pb = c_conv_pb[c];
  u32 acc = 0;
  for (int w = gr.start; w < gr.start + gr.count; ++w) {
    const int ss = s.ps[c][w], tt = s.pt[c][w];
    const size_t xo = ((size_t)((pa * K + ss) * 2 + prime) << logN) + idx;
    const size_t wo = ((size_t)((pb * K + tt) * 2 + prime) << logN) + idx;
    acc = add_mod(acc, shoup_mul(Xb[xo], Wb[wo], Wqb[wo], p), p);
  }
  return acc;
}

// Single-workgroup inverse (N <= 4096): blockIdx.y = conv*2 + prime.
__global__ void __launch_bounds__(NTT_THREADS) k_inv_single(const u32* X, u32* Z, const TDesc* td, const TState* ts,
                                                            const KernelDesc* kd, const int* tlist, int K,
                                                            int slot_lo, int slot_hi, int logN, TwBlock tb) {
  extern __shared__ u32 smem[];
  const int t = tlist[blockIdx.z];
  const TDesc& d = td[t];
  const TState& s = ts[t];
  if (s.status) return;
  const int c = blockIdx.y >> 1, prime = blockIdx.y & 1;
  const u32 p = prime_of(prime);
  const KernelDesc& kk = kd[d.kd];
  const int N = 1 << logN, ldr = row_ld(N), SL = K * K;
  uint2* tw = reinterpret_cast<uint2*>(smem);
  u32* tile = smem + N;
  load_block_tw(tw, tb.inv[prime], logN);
  const u32* Xb = X + d.X_off;
  for (int gidx = 0; gidx < s.ngroups[c]; ++gidx) {
    const int slot = c * SL + gidx;
    if (slot < slot_lo || slot >= slot_hi) continue;
    const Group gr = s.groups[c][gidx];
    for (int i = threadIdx.x; i < N; i += blockDim.x)
      tile[i + (i >> 5)] = group_mac(Xb, kk.W, kk.Wq, s, c, gr, K, prime, logN, i, p);
    __syncthreads();
    block_ntt<true, false>(tile, logN, 0, ldr, tw, p);
    u32* zo = Z + d.Z_off + (size_t)(slot * 2 + prime) * d.n;
    for (int i = threadIdx.x; i < d.n; i += blockDim.x) zo[i] = tile[i + (i >> 5)];
    __syncthreads();
  }
}

// Two-pass inverse, first pass (rows): blockIdx.x = row tile, blockIdx.y = prime.
__global__ void __launch_bounds__(NTT_THREADS) k_inv_rows(const u32* X, u32* G, const TDesc* td, const TState* ts,
                                                          const KernelDesc* kd, const int* tlist, int K,
                                                          int slot_lo, int slot_hi, NttGeom g, TwBlock tb,
                                                          TwStep st) {
  extern __shared__ u32 smem[];
  const int t = tlist[blockIdx.z];
  const TDesc& d = td[t];
  const TState& s = ts[t];
  if (s.status) return;
  const int prime = blockIdx.y;
  const u32 p = prime_of(prime);
  const KernelDesc& kk = kd[d.kd];
  const int m2 = g.m2, N2 = 1 << m2, lr = g.lrows, ldr = row_ld(N2), SL = K * K;
  const u32 Nmask = (1u << g.logN) - 1;
  uint2* tw = reinterpret_cast<uint2*>(smem);
  u32* tile = smem + N2;
  load_block_tw(tw, tb.inv[prime], m2);
  const int i1_0 = blockIdx.x << lr;
  const int tot = N2 << lr;
  const size_t base = (size_t)i1_0 * N2;
  const u32* Xb = X + d.X_off;
  for (int c = 0; c < 4; ++c) {
    for (int gidx = 0; gidx < s.ngroups[c]; ++gidx) {
      const int slot = c * SL + gidx;
      if (slot < slot_lo || slot >= slot_hi) continue;
      const Group gr = s.groups[c][gidx];
      for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const int r = idx >> m2, i = idx & (N2 - 1);
        tile[r * ldr + i + (i >> 5)] = group_mac(Xb, kk.W, kk.Wq, s, c, gr, K, prime, g.logN, base + idx, p);
      }
      __syncthreads();
      block_ntt<true, false>(tile, m2, lr, ldr, tw, p);
      u32* go = G + d.G_off + ((size_t)(slot * 2 + prime) << g.logN) + base;
      for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const int r = idx >> m2, j2 = idx & (N2 - 1);
        const u32 e = ((u32)j2 * bitrev(i1_0 + r, g.m1)) & Nmask;
        go[idx] = step_twiddle(tile[r * ldr + j2 + (j2 >> 5)], e, st.lo[1][prime], st.hi[1][prime], p);
      }
      __syncthreads();
    }
  }
}

// Two-pass inverse, second pass (columns): blockIdx.y = slot*2 + prime.
// Writes the first n natural-order outputs to the compact buffer.
__global__ void __launch_bounds__(NTT_THREADS) k_inv_cols(const u32* G, u32* Z, const TDesc* td, const TState* ts,
                                                          const int* tlist, int K, int slot_lo, NttGeom g,
                                                          TwBlock tb) {
  extern __shared__ u32 smem[];
  const int t = tlist[blockIdx.z];
  const TDesc& d = td[t];
  const TState& s = ts[t];
  const int slot = slot_lo + (blockIdx.y >> 1), prime = blockIdx.y & 1;
  const int SL = K * K, c = slot / SL, gidx = slot % SL;
  if (s.status || gidx >= s.ngroups[c]) return;
  const u32 p = prime_of(prime);
  const int m1 = g.m1, N2 = 1 << g.m2, lc = g.lc, C = 1 << lc;
  uint2* tw = reinterpret_cast<uint2*>(smem);
  u32* tile = smem + (1 << m1);
  load_block_tw(tw, tb.inv[prime], m1);
  const int j2_0 = blockIdx.x << lc;
  const int tot = C << m1;
  const u32* gv = G + d.G_off + ((size_t)(slot * 2 + prime) << g.logN);
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int c2 = idx & (C - 1), i1 = idx >> lc;
    tile[idx] = gv[i1 * N2 + j2_0 + c2];
  }
  __syncthreads();
  block_ntt<true, true>(tile, m1, lc, 0, tw, p);
  u32* zo = Z + d.Z_off + (size_t)(slot * 2 + prime) * d.n;
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int c2 = idx & (C - 1), j1 = idx >> lc;
    const int gi = j1 * N2 + j2_0 + c2;
    if (gi < d.n) zo[gi] = tile[idx];
  }
}

// Kernel slices: W <- W * N^{-1}, Wq <- Shoup companion.  Layout [part][t][prime][N].
__global__ void k_kernel_finish(u32* W, u32* Wq, size_t total, int logN) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int prime = (int)((i >> logN) & 1);
    const u32 p = prime_of(prime);
    const u32 ninv = p - ((p - 1) >> logN);
    const u32 v = shoup_mul(W[i], ninv, shoup_companion(ninv, p), p);
    W[i] = v;
    Wq[i] = shoup_companion(v, p);
  }
}

// ---------------------------------------------------------------------------
// Host side.

NttGeom ntt_geom(int logN, int lc_override, int lrows_override) {
  NttGeom g{};
  g.logN = logN;
  if (logN <= LOG2_BLOCK_MAX) {
    g.m1 = logN;
    g.m2 = 0;
    g.lc = 0;
    g.lrows = 0;
    return g;
  }
  g.m1 = logN / 2;
  g.m2 = logN - g.m1;
  // column tile: C * N1 words <= 32K words (128 KiB), at most 32 columns
  int lc = 5;
  while (lc > 0 && (g.m1 + lc) > 15) --lc;
  if (lc > g.m2) lc = g.m2;
  // row tile: 4096 words per workgroup
  int lr = LOG2_BLOCK_MAX - g.m2;
  if (lr < 0) lr = 0;
  if (lr > g.m1) lr = g.m1;
  g.lc = lc_override >= 0 ? lc_override : lc;
  g.lrows = lrows_override >= 0 ? lrows_override : lr;
  return g;
}

static size_t smem_cols(const NttGeom& g) { return ((size_t)(1 << g.m1) + ((size_t)1 << (g.m1 + g.lc))) * 4; }
static size_t smem_rows(const NttGeom& g) {
  return ((size_t)(1 << g.m2) + ((size_t)row_ld(1 << g.m2) << g.lrows)) * 4;
}
static size_t smem_single(int logN) { return ((size_t)(1 << logN) + row_ld(1 << logN)) * 4; }

static hipError_t allow_big_lds() {
  static bool done = false;
  if (done) return hipSuccess;
  const int lim = 160 * 1024;
  const void* fns[] = {(const void*)k_std_single, (const void*)k_std_fwd_cols, (const void*)k_std_fwd_rows,
                       (const void*)k_std_inv_rows, (const void*)k_std_inv_cols, (const void*)k_fwd_single,
                       (const void*)k_fwd_cols, (const void*)k_fwd_rows, (const void*)k_inv_single,
                       (const void*)k_inv_rows, (const void*)k_inv_cols};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if (e != hipSuccess) return e;
  }
  done = true;
  return hipSuccess;
}

hipError_t launch_ntt_standalone(u32* data, int logN, int prime, int count, bool inverse, const NttGeom& g,
                                 const TwBlock& tb, const TwStep& ts, hipStream_t s) {
  hipError_t e = allow_big_lds();
  if (e != hipSuccess) return e;
  if (count <= 0) return hipSuccess;
  if (!g.two_pass()) {
    hipLaunchKernelGGL(k_std_single, dim3(1, 1, count), dim3(NTT_THREADS), smem_single(logN), s, data, logN, prime,
                       inverse, tb);
    return hipGetLastError();
  }
  const dim3 gc(1u << (g.m2 - g.lc), 1, count), gr(1u << (g.m1 - g.lrows), 1, count);
  if (!inverse) {
    hipLaunchKernelGGL(k_std_fwd_cols, gc, dim3(NTT_THREADS), smem_cols(g), s, data, prime, g, tb, ts);
    hipLaunchKernelGGL(k_std_fwd_rows, gr, dim3(NTT_THREADS), smem_rows(g), s, data, prime, g, tb);
  } else {
    hipLaunchKernelGGL(k_std_inv_rows, gr, dim3(NTT_THREADS), smem_rows(g), s, data, prime, g, tb, ts);
    hipLaunchKernelGGL(k_std_inv_cols, gc, dim3(NTT_THREADS), smem_cols(g), s, data, prime, g, tb);
  }
  return hipGetLastError();
}

hipError_t launch_fwd_pipeline(u32* X, const TDesc* td, const TState* ts, const int* tlist, int count, int K,
                               bool valid_full, int vi_lo, int vi_hi, const NttGeom& g, const TwBlock& tb,
                               const TwStep& st, hipStream_t s) {
  hipError_t e = allow_big_lds();
  if (e != hipSuccess) return e;
  const int nv = vi_hi - vi_lo;
  if (count <= 0 || nv <= 0) return hipSuccess;
  if (!g.two_pass()) {
    hipLaunchKernelGGL(k_fwd_single, dim3(1, nv, count), dim3(NTT_THREADS), smem_single(g.logN), s, X, td, ts, tlist,
                       K, valid_full, vi_lo, g.logN, tb);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_fwd_cols, dim3(1u << (g.m2 - g.lc), nv, count), dim3(NTT_THREADS), smem_cols(g), s, X, td, ts,
                     tlist, K, valid_full, vi_lo, g, tb, st);
  hipLaunchKernelGGL(k_fwd_rows, dim3(1u << (g.m1 - g.lrows), nv, count), dim3(NTT_THREADS), smem_rows(g), s, X, td,
                     ts, tlist, K, valid_full, vi_lo, g, tb);
  return hipGetLastError();
}

hipError_t launch_inv_pipeline(const u32* X, u32* G, u32* Z, const TDesc* td, const TState* ts,
                               const KernelDesc* kd, const int* tlist, int count, int K, int slot_lo, int slot_hi,
                               const NttGeom& g, const TwBlock& tb, const TwStep& st, hipStream_t s) {
  hipError_t e = allow_big_lds();
  if (e != hipSuccess) return e;
  if (count <= 0 || slot_hi <= slot_lo) return hipSuccess;
  if (!g.two_pass()) {
    hipLaunchKernelGGL(k_inv_single, dim3(1, 8, count), dim3(NTT_THREADS), smem_single(g.logN), s, X, Z, td, ts, kd,
                       tlist, K, slot_lo, slot_hi, g.logN, tb);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_inv_rows, dim3(1u << (g.m1 - g.lrows), 2, count), dim3(NTT_THREADS), smem_rows(g), s, X, G,
                     td, ts, kd, tlist, K, slot_lo, slot_hi, g, tb, st);
  hipLaunchKernelGGL(k_inv_cols, dim3(1u << (g.m2 - g.lc), 2 * (slot_hi - slot_lo), count), dim3(NTT_THREADS),
                     smem_cols(g), s, G, Z, td, ts, tlist, K, slot_lo, g, tb);
  return hipGetLastError();
}

hipError_t launch_fwd_stage(u32* X, const TDesc* td, const TState* ts, const int* tlist, int count, int K, int vi_lo,
                            int vi_hi, const NttGeom& g, const TwBlock& tb, const TwStep& st, int which, hipStream_t s) {
  if (which == 0) return launch_fwd_pipeline(X, td, ts, tlist, count, K, false, vi_lo, vi_hi, g, tb, st, s);
  hipError_t e = allow_big_lds();
  if (e != hipSuccess) return e;
  const int nv = vi_hi - vi_lo;
  if (which == 1)
    hipLaunchKernelGGL(k_fwd_cols, dim3(1u << (g.m2 - g.lc), nv, count), dim3(NTT_THREADS), smem_cols(g), s, X, td,
                       ts, tlist, K, false, vi_lo, g, tb, st);
  else
    hipLaunchKernelGGL(k_fwd_rows, dim3(1u << (g.m1 - g.lrows), nv, count), dim3(NTT_THREADS), smem_rows(g), s, X, td,
                       ts, tlist, K, false, vi_lo, g, tb);
  return hipGetLastError();
}

hipError_t launch_inv_stage(const u32* X, u32* G, u32* Z, const TDesc* td, const TState* ts, const KernelDesc* kd,
                            const int* tlist, int count, int K, int slot_lo, int slot_hi, const NttGeom& g,
                            const TwBlock& tb, const TwStep& st, int which, hipStream_t s) {
  hipError_t e = allow_big_lds();
  if (e != hipSuccess) return e;
  if (!g.two_pass()) {
    if (which == 1) return launch_inv_pipeline(X, G, Z, td, ts, kd, tlist, count, K, slot_lo, slot_hi, g, tb, st, s);
    return hipSuccess;
  }
  if (which == 1)
    hipLaunchKernelGGL(k_inv_rows, dim3(1u << (g.m1 - g.lrows), 2, count), dim3(NTT_THREADS), smem_rows(g), s, X, G,
                       td, ts, kd, tlist, K, slot_lo, slot_hi, g, tb, st);
  else
    hipLaunchKernelGGL(k_inv_cols, dim3(1u << (g.m2 - g.lc), 2 * (slot_hi - slot_lo), count), dim3(NTT_THREADS),
                       smem_cols(g), s, G, Z, td, ts, tlist, K, slot_lo, g, tb);
  return hipGetLastError();
}

hipError_t launch_kernel_finish(u32* W, u32* Wq, int K, int logN, hipStream_t s) {
  const size_t total = (size_t)(2 * K * 2) << logN;
  const int blocks = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_kernel_finish, dim3(blocks), dim3(256), 0, s, W, Wq, total, logN);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Twiddle tables (plan time, exact host integer arithmetic).

static u32 powmod(u64 b, u64 e, u32 p) {
  u64 r = 1;
  b %= p;
  while (e) {
    if (e & 1) r = r * b % p;
    b = b * b % p;
    e >>= 1;
  }
  return (u32)r;
}

static u32 root_of_unity(int prime, u64 N) {
  const u32 p = prime ? P1 : P0, gen = prime ? G1 : G0;
  return powmod(gen, (u64)(p - 1) / N, p);
}

static hipError_t upload_powers(uint2** dst, u32 w, u32 count, u32 p) {
  uint2* h = (uint2*)malloc(sizeof(uint2) * count);
  if (!h) return hipErrorOutOfMemory;
  u64 v = 1;
  for (u32 e = 0; e < count; ++e) {
    h[e].x = (u32)v;
    h[e].y = shoup_companion((u32)v, p);
    v = v * w % p;
  }
  hipError_t err = hipMalloc(dst, sizeof(uint2) * count);
  if (err == hipSuccess) err = hipMemcpy(*dst, h, sizeof(uint2) * count, hipMemcpyHostToDevice);
  free(h);
  return err;
}

int build_block_twiddles(TwBlock* out, void** allocs) {
  for (int prime = 0; prime < 2; ++prime) {
    const u32 p = prime ? P1 : P0;
    const u32 w = root_of_unity(prime, BLOCK_MAX);
    const u32 wi = powmod(w, p - 2, p);
    uint2 *f = nullptr, *iv = nullptr;
    if (upload_powers(&f, w, BLOCK_MAX / 2, p) != hipSuccess) return -1;
    if (upload_powers(&iv, wi, BLOCK_MAX / 2, p) != hipSuccess) return -1;
    out->fwd[prime] = f;
    out->inv[prime] = iv;
    allocs[2 * prime] = f;
    allocs[2 * prime + 1] = iv;
  }
  return 0;
}

int build_step_twiddles(int logN, TwStep* out, void** allocs) {
  const u64 N = 1ull << logN;
  const u32 nhi = N > 4096 ? (u32)(N >> 12) : 1u;
  int a = 0;
  for (int prime = 0; prime < 2; ++prime) {
    const u32 p = prime ? P1 : P0;
    const u32 w = root_of_unity(prime, N);
    const u32 wi = powmod(w, p - 2, p);
    for (int dir = 0; dir < 2; ++dir) {
      const u32 base = dir ? wi : w;
      uint2 *lo = nullptr, *hi = nullptr;
      if (upload_powers(&lo, base, 4096, p) != hipSuccess) return -1;
      if (upload_powers(&hi, powmod(base, 4096, p), nhi, p) != hipSuccess) return -1;
      out->lo[dir][prime] = lo;
      out->hi[dir][prime] = hi;
      allocs[a++] = lo;
      allocs[a++] = hi;
    }
  }
  return 0;
}

}  // namespace fo
