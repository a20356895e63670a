// Number-theoretic transforms modulo p0 = 2130706433 and p1 = 2113929217 (and
// p2 = 2013265921 for plans with three moduli) on gfx950 (Sec. 3.3:
// y(k) = sum_j x(j) w_N^{jk} mod p, inverse with N^{-1}).  NP is the number
// of moduli of a plan; the slice spectra are laid out
// [part][k][prime][N] and the group values [slot][prime][N], prime < NP.
//
// Design:
//  * A block NTT of length M <= 4096 runs inside one workgroup on an LDS tile.
//    The forward transform is decimation in frequency (natural order in,
//    bit-reversed order out); the inverse is its exact mirror, decimation in
//    time (bit-reversed in, natural out), so no permutation pass is needed:
//    the pointwise products of the convolution work on bit-reversed data.
//  * Each thread holds 2^r elements (r <= 3) in registers and performs r
//    radix-2 stages between LDS exchanges (a 512-point transform takes three
//    LDS round trips); eight registers per group keep the register file
//    small enough for four to five waves per SIMD.  The round structure is
//    instantiated per transform length, so LDS and twiddle addresses are
//    compile-time offsets and the butterflies whose root is 1 skip the
//    product.
//  * Lengths N > 4096 use two passes N = N1 * N2: column transforms of length
//    N1 (stride N2, a tile of C adjacent columns per workgroup so that global
//    accesses are C*4 bytes contiguous), the twiddle w_N^{j2 k1}, then
//    contiguous row transforms of length N2.
//  * Global traffic uses 16-byte accesses, several in flight per thread
//    before their LDS writes, so each wave keeps the memory pipe busy.
//  * Modular products are Shoup multiplications by precomputed constants
//    (value and floor(w 2^32 / p)); gfx950 issues v_mul_lo_u32 / v_mul_hi_u32
//    at full rate, so a butterfly is ~11 VALU instructions.
//  * The convolution's pointwise products and their NTT-domain accumulation
//    (Alg. 8) are fused into the first inverse pass: for four adjacent
//    positions a thread loads the NTT-domain slices of one input part and of
//    one kernel part once and forms every group sum of that convolution from
//    registers.  N^{-1} is folded into the precomputed kernel transforms.
#include <algorithm>

#include "crt_dev.h"
#include "internal.h"
#include "schedule_dev.h"

#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <unordered_set>
#include <utility>

namespace fo {

__device__ __forceinline__ u32 prime_of(int i) { return i == 0 ? P0 : (i == 1 ? P1 : P2); }
__device__ __forceinline__ u32 bitrev(u32 v, int bits) { return bits ? (__brev(v) >> (32 - bits)) : 0u; }

// Row layout of a tile: vector v at v * ldr, element i at pad8(i) = i + 8 (i / 64)
// (eight pad words per 64 keep 16-byte chunks contiguous, make the addresses
// of a radix group an affine function of its index -- compile-time offsets --
// and spread the strided accesses of the radix rounds over the LDS banks).
// Column layout (COLS): element i of all 2^lnvec vectors adjacent.
__host__ __device__ constexpr int pad8(int i) { return i + ((i >> 6) << 3); }
// Row stride: rows shorter than 512 words are offset by four banks (a wave's
// radix groups then span several rows); longer rows need no offset.
__host__ __device__ constexpr int row_ld(int M) { return pad8(M) + (M >= 512 ? 0 : 4); }
// Second row layout, for kernels that touch rows only element by element: one
// pad word per eight, element i at pad9(i) = i + i / 8, rows M + M/8 apart.
// The eight elements of a unit-stride radix group then start at 9q, so the
// 64 lanes of a wave reach 64 different banks in every round (with pad8 the
// unit-stride round puts eight lanes on each bank); 16-byte chunks stay
// contiguous but not aligned.  PL selects the layout (8 or 9).
__host__ __device__ constexpr int pad9(int i) { return i + (i >> 3); }
template <int PL>
__host__ __device__ constexpr int padl(int i) { return PL == 9 ? pad9(i) : pad8(i); }
// Column stride of the column passes' wave-local tiles: each column of
// N1 = 2^m1 values is a pad9 row; the stride is 8 mod 64 words so that the
// columns written or read together at one tile position fall on different
// LDS banks.
__host__ __device__ constexpr int rec_ldc(int m1) { return pad9(1 << m1) + ((8 - pad9(1 << m1)) & 63); }
template <int PL>
__host__ __device__ constexpr int row_ldl(int M) { return PL == 9 ? pad9(M) : row_ld(M); }

constexpr int UNR = 4;           // 16-byte global loads in flight per thread
constexpr int INV_TILE_ROWS = 20;        // group rows per inverse chunk: the 20 groups of K = L = 3 fit, 3 workgroups per CU
constexpr int KT = 3;            // slices per operand handled from registers in the fused MAC
// Group tiles (INV_ROW_THREADS = 512 positions each: nr rows of N2) in the
// LDS of the pipelined row pass, whatever N2: forward slice tiles (2K) and
// inverse group tiles share them.
constexpr int PIPE_TILES = 20;

// RL radix-2 stages (s = S0 .. S0+RL-1) on the 2^RL registers of one group of
// a length-2^M transform.  The group holds elements base + j*ST, base =
// blk * 2^RL * ST + off with off < ST.  At stage s the partners are hd =
// 2^RL >> (s - S0 + 1) registers apart and pair (j, j + hd) uses w_M^e with
// e = (off + (j mod hd) * ST) << s: hd distinct roots per stage, at
// compile-time offsets from tw + (off << s).  When ST = 1 (off = 0) the roots
// of the round are the same for every group (`twr`, preloaded) and those with
// j mod hd = 0 are 1, so those butterflies skip the product.
template <int RL, int S0, int ST, bool INV, bool HOIST>
__device__ __forceinline__ void radix_group_t(u32 (&a)[1 << RL], int off, const uint2* __restrict__ tw,
                                              const uint2 (&twr)[1 << RL], u32 p) {
  constexpr int R = 1 << RL;
#pragma unroll
  for (int k = 0; k < RL; ++k) {
    const int ss = INV ? RL - 1 - k : k;
    const int hd = R >> (ss + 1);
    const int s = S0 + ss;
    const uint2* tws = tw + (off << s);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (j & hd) continue;
      const int jj = j & (hd - 1);
      const bool trivial = (ST == 1) && jj == 0;
      uint2 w = make_uint2(1u, 0u);
      if (!trivial) w = (ST == 1 || HOIST) ? twr[hd + jj] : tws[(jj * ST) << s];
      const u32 x = a[j], y = a[j + hd];
      if (!INV) {
        a[j] = add_mod(x, y, p);
        a[j + hd] = trivial ? sub_mod(x, y, p) : shoup_mul(x + p - y, w.x, w.y, p);   // x - y + p < 2p
      } else {
        const u32 t = trivial ? y : shoup_mul(y, w.x, w.y, p);
        a[j] = add_mod(x, t, p);
        a[j + hd] = sub_mod(x, t, p);
      }
    }
  }
}

// The groups of one round.  HOIST: every group a thread visits has the same
// offset (row layout with blockDim a multiple of the groups per vector), so
// its roots were loaded into twr once for the round.  In the column layout
// a thread transforms two groups per iteration (g and g + blockDim): their
// independent instruction streams interleave and hide the latency of the
// dependent product chains (at the tail the second group repeats the first
// and is not stored).  The row kernels keep one group per iteration: there
// the extra registers cost a wave per SIMD, which is worth more.
template <int M, int S0, int RL, bool INV, bool COLS, bool HOIST, int PL = 8>
__device__ __forceinline__ void round_groups(u32* lds, int nv, int ldr, const uint2* __restrict__ tw,
                                             const uint2 (&twr)[1 << RL], u32 p, int tid, int nthr) {
  constexpr int R = 1 << RL, LBK = M - S0, LST = LBK - RL, ST = 1 << LST, LGPV = M - RL;
  const int total = COLS ? (1 << (nv + LGPV)) : (nv << LGPV);
  const int sst = COLS ? (ST << nv) : 0;     // element stride of a group, column layout
  auto locate = [&](int g, int& off) -> u32* {
    int v, q;
    if (COLS) {
      v = g & ((1 << nv) - 1);
      q = g >> nv;
    } else {
      v = g >> LGPV;
      q = g & ((1 << LGPV) - 1);
    }
    off = q & (ST - 1);
    const int base = ((q >> LST) << LBK) + off;
    return COLS ? lds + (base << nv) + v : lds + v * ldr + padl<PL>(base);
  };
  auto load = [&](u32 (&a)[R], const u32* p0) {
    if (!COLS && ST == 1 && R >= 4 && PL == 8) {
      // 8-byte accesses: a wave's 16-byte accesses to groups 8 words apart
      // meet half the banks (measured slower)
#pragma unroll
      for (int j = 0; j < R; j += 2) {
        const uint2 t = *reinterpret_cast<const uint2*>(p0 + j);
        a[j] = t.x;
        a[j + 1] = t.y;
      }
    } else {
#pragma unroll
      for (int j = 0; j < R; ++j) a[j] = COLS ? p0[j * sst] : p0[padl<PL>(j * ST)];
    }
  };
  auto store = [&](const u32 (&a)[R], u32* p0) {
    if (!COLS && ST == 1 && R >= 4 && PL == 8) {
#pragma unroll
      for (int j = 0; j < R; j += 2) *reinterpret_cast<uint2*>(p0 + j) = make_uint2(a[j], a[j + 1]);
    } else {
#pragma unroll
      for (int j = 0; j < R; ++j) {
        if (COLS) p0[j * sst] = a[j];
        else p0[padl<PL>(j * ST)] = a[j];
      }
    }
  };
  if (!COLS) {
    for (int g = tid; g < total; g += nthr) {
      int off;
      u32* p0 = locate(g, off);
      u32 a[R];
      load(a, p0);
      radix_group_t<RL, S0, ST, INV, HOIST>(a, off, tw, twr, p);
      store(a, p0);
    }
    return;
  }
  for (int g = tid; g < total; g += 2 * nthr) {
    const int g2 = g + nthr;
    const bool two = g2 < total;
    int off1, off2;
    u32* p1 = locate(g, off1);
    u32* p2 = locate(two ? g2 : g, off2);
    u32 a[R], b[R];
    load(a, p1);
    load(b, p2);
    radix_group_t<RL, S0, ST, INV, HOIST>(a, off1, tw, twr, p);
    radix_group_t<RL, S0, ST, INV, HOIST>(b, off2, tw, twr, p);
    store(a, p1);
    if (two) store(b, p2);
  }
}

// One round of a length-2^M block NTT over the vectors of a tile.
// nv: number of vectors (row layout) or log2 of it (column layout).  The
// roots a thread needs are read from LDS once per round when they are the
// same for all its groups (twr[hd + jj] for stage S0 + ss, hd = R >> (ss+1)):
// always when ST = 1, and in the row layout when blockDim is a multiple of
// the groups per vector (then the lanes of a stage would otherwise read the
// strided table w^((off + jj ST) 2^s) once per group, on few LDS banks).
template <int M, int S0, int RL, bool INV, bool COLS, int PL = 8>
__device__ __forceinline__ void round_t(u32* lds, int nv, int ldr, const uint2* __restrict__ tw, u32 p, int tid,
                                        int nthr) {
  constexpr int R = 1 << RL, LBK = M - S0, LST = LBK - RL, ST = 1 << LST, LGPV = M - RL;
  uint2 twr[R];
  if (ST == 1) {
#pragma unroll
    for (int ss = 0; ss < RL; ++ss) {
      const int hd = R >> (ss + 1);
#pragma unroll
      for (int jj = 1; jj < hd; ++jj) twr[hd + jj] = tw[jj << (S0 + ss)];
    }
    round_groups<M, S0, RL, INV, COLS, false, PL>(lds, nv, ldr, tw, twr, p, tid, nthr);
    return;
  }
  if (!COLS && (nthr & ((1 << LGPV) - 1)) == 0) {
    const int off = (tid & ((1 << LGPV) - 1)) & (ST - 1);
#pragma unroll
    for (int ss = 0; ss < RL; ++ss) {
      const int hd = R >> (ss + 1);
#pragma unroll
      for (int jj = 0; jj < hd; ++jj) twr[hd + jj] = tw[(off + jj * ST) << (S0 + ss)];
    }
    round_groups<M, S0, RL, INV, COLS, true, PL>(lds, nv, ldr, tw, twr, p, tid, nthr);
    return;
  }
  round_groups<M, S0, RL, INV, COLS, false, PL>(lds, nv, ldr, tw, twr, p, tid, nthr);
}

// Orders the LDS accesses of one wave around this point (a wave's LDS
// instructions are performed in issue order, so no workgroup barrier is
// needed when only this wave reads what it wrote).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Rounds I.. of a length-2^M block NTT: ceil(M/3) rounds, the M stages spread
// evenly (the first M mod nr rounds take one stage more); the inverse runs
// the mirrored rounds in reverse order.  The groups of a round are spread
// over nthr threads (tid = this thread's index among them).  WAVE: the
// threads are the lanes of one wave, which alone works on these vectors,
// so the rounds are separated by wave_sync instead of a workgroup barrier.
template <int M, int I, bool INV, bool COLS, int PL = 8, bool WAVE = false>
__device__ __forceinline__ void rounds_t(u32* lds, int nv, int ldr, const uint2* tw, u32 p, int tid, int nthr) {
  constexpr int NR = (M + 2) / 3, RB = NR ? M / NR : 0, RX = NR ? M % NR : 0;
  if constexpr (I < NR) {
    constexpr int IDX = INV ? NR - 1 - I : I;
    constexpr int S0 = IDX * RB + (IDX < RX ? IDX : RX);
    constexpr int RL = RB + (IDX < RX ? 1 : 0);
    round_t<M, S0, RL, INV, COLS, PL>(lds, nv, ldr, tw, p, tid, nthr);
    if constexpr (WAVE) wave_sync();
    else __syncthreads();
    rounds_t<M, I + 1, INV, COLS, PL, WAVE>(lds, nv, ldr, tw, p, tid, nthr);
  }
}

// In-place block NTT of the vectors of a tile (length 2^M each, M <= 12).  The
// caller synchronises after filling the tile; this routine ends
// synchronised.  Every kernel is instantiated per block length, so the
// rounds inline with compile-time geometry.
template <int M, bool INV, bool COLS, int PL = 8>
__device__ __forceinline__ void block_ntt(u32* lds, int nv, int ldr, const uint2* tw, u32 p) {
  rounds_t<M, 0, INV, COLS, PL>(lds, nv, ldr, tw, p, (int)threadIdx.x, (int)blockDim.x);
}

// Copies the roots w_M^e (e < M/2) of a length-2^m block NTT into LDS from the
// 4096-point table.
__device__ __forceinline__ void load_block_tw(uint2* tw, const uint2* __restrict__ src, int m) {
  const int half = m ? (1 << (m - 1)) : 0;
  for (int e = threadIdx.x; e < half; e += blockDim.x) tw[e] = src[e << (LOG2_BLOCK_MAX - m)];
}

// floor(v 2^32 / p) for v < p, exactly, in integer arithmetic: p is one of
// the NTT primes, so each branch divides by a compile-time constant (which
// the compiler turns into multiplications).
__device__ __forceinline__ u32 companion_dev(u32 v, u32 p) {
  const u64 w = (u64)v << 32;
  return (u32)(p == P0 ? w / P0 : (p == P1 ? w / P1 : w / P2));
}

// (w_N^e, companion) from the two-level step tables.
__device__ __forceinline__ uint2 step_root(u32 e, const uint2* __restrict__ lo, const uint2* __restrict__ hi, u32 p) {
  const uint2 a = lo[e & 4095u], b = hi[e >> 12];
  const u32 v = shoup_mul(a.x, b.x, b.y, p);
  return make_uint2(v, companion_dev(v, p));
}

// Twiddles of a row pass: rows r < nr of the tile are rows i1_0 + r of the
// N1 x N2 matrix, with k1 = br(i1_0 + r); element j2 of row r is multiplied
// by w_N^{j2 k1} (forward) or its inverse.  With j2 = jh 2^lb + jl the root
// factors as A_r[jl] * B_r[jh]; both small tables live in LDS with their
// Shoup companions (A: nr << lb entries, B: nr << (m2 - lb) entries).
struct RowTw {
  uint2* A;
  uint2* B;
  int lb;
};
__host__ __device__ inline int rowtw_lb(int m2) { return m2 < 6 ? m2 : 6; }
__host__ __device__ inline int rowtw_words(int m2, int nr) {
  const int lb = rowtw_lb(m2);
  return 2 * ((nr << lb) + (nr << (m2 - lb)));
}
__device__ void build_rowtw(RowTw& t, u32* mem, int nr, int i1_0, int m1, int m2, u32 Nmask,
                            const uint2* __restrict__ lo, const uint2* __restrict__ hi, u32 p) {
  t.lb = rowtw_lb(m2);
  t.A = reinterpret_cast<uint2*>(mem);
  t.B = t.A + (nr << t.lb);
  const int na = nr << t.lb, nb = nr << (m2 - t.lb);
  for (int i = threadIdx.x; i < na + nb; i += blockDim.x) {
    if (i < na) {
      const int r = i >> t.lb, jl = i & ((1 << t.lb) - 1);
      t.A[i] = step_root(((u32)jl * bitrev(i1_0 + r, m1)) & Nmask, lo, hi, p);
    } else {
      const int k = i - na, r = k >> (m2 - t.lb), jh = k & ((1 << (m2 - t.lb)) - 1);
      t.B[k] = step_root(((u32)(jh << t.lb) * bitrev(i1_0 + r, m1)) & Nmask, lo, hi, p);
    }
  }
}
__device__ __forceinline__ u32 apply_rowtw(const RowTw& t, u32 x, int r, int j2, int m2, u32 p) {
  const uint2 a = t.A[(r << t.lb) + (j2 & ((1 << t.lb) - 1))];
  const uint2 b = t.B[(r << (m2 - t.lb)) + (j2 >> t.lb)];
  return shoup_mul(shoup_mul(x, a.x, a.y, p), b.x, b.y, p);
}

__device__ __forceinline__ uint4 zero_from(uint4 w, int e, int valid) {
  if (e + 3 >= valid) {
    if (e >= valid) w.x = 0;
    if (e + 1 >= valid) w.y = 0;
    if (e + 2 >= valid) w.z = 0;
    w.w = 0;
  }
  return w;
}

// ---------------------------------------------------------------------------
// Tile movers.

// `nrows` rows of M = 2^m words (row r at src + r*M) into tile rows 0..nrows-1;
// flattened positions >= valid read as zero.
__device__ void load_rows(u32* tile, const u32* __restrict__ src, int nrows, int m, int ldr, int valid) {
  const int M = 1 << m;
  if (m < 2) {
    for (int e = threadIdx.x; e < (nrows << m); e += blockDim.x)
      tile[(e >> m) * ldr + pad8(e & (M - 1))] = e < valid ? src[e] : 0u;
    return;
  }
  const int tot4 = (nrows << m) >> 2;
  const uint4* s4 = reinterpret_cast<const uint4*>(src);
  for (int q0 = threadIdx.x; q0 < tot4; q0 += blockDim.x * UNR) {
    uint4 v[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int q = q0 + u * blockDim.x;
      if (q < tot4) v[u] = (q << 2) < valid ? s4[q] : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int q = q0 + u * blockDim.x;
      if (q < tot4) {
        const int e = q << 2;
        *reinterpret_cast<uint4*>(tile + (e >> m) * ldr + pad8(e & (M - 1))) = zero_from(v[u], e, valid);
      }
    }
  }
}

__device__ void store_rows(u32* __restrict__ dst, const u32* tile, int nrows, int m, int ldr) {
  const int M = 1 << m;
  if (m < 2) {
    for (int e = threadIdx.x; e < (nrows << m); e += blockDim.x) dst[e] = tile[(e >> m) * ldr + pad8(e & (M - 1))];
    return;
  }
  const int tot4 = (nrows << m) >> 2;
  uint4* d4 = reinterpret_cast<uint4*>(dst);
  for (int q = threadIdx.x; q < tot4; q += blockDim.x) {
    const int e = q << 2;
    d4[q] = *reinterpret_cast<const uint4*>(tile + (e >> m) * ldr + pad8(e & (M - 1)));
  }
}

// Column tile taken by workgroup x of a column pass over the 2^lt tiles of a
// vector (grid x dimension = 2^lt).  Workgroups go to the eight XCDs
// round-robin, so x and x + 8 run on one XCD at about the same time; giving
// them adjacent tiles lets their partial cache lines (a tile row is 16 to
// 128 bytes) meet in that XCD's L2 instead of being fetched by two XCDs.
__device__ __forceinline__ int col_tile(int x, int lt) { return lt < 3 ? x : (((x & 7) << (lt - 3)) | (x >> 3)); }

// Columns [j2_0, j2_0 + 2^lc) of a 2^m1 x 2^m2 row-major vector into the
// column-layout tile; positions >= valid read as zero.  Needs lc >= 2.
__device__ void load_cols(u32* tile, const u32* __restrict__ vec, int m1, int m2, int lc, int j2_0, int valid) {
  const int lq = lc - 2;
  const int tot4 = 1 << (m1 + lq);
  for (int q0 = threadIdx.x; q0 < tot4; q0 += blockDim.x * UNR) {
    uint4 v[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int q = q0 + u * blockDim.x;
      if (q < tot4) {
        const int i = q >> lq, c4 = (q & ((1 << lq) - 1)) << 2;
        const int gi = (i << m2) + j2_0 + c4;
        v[u] = gi < valid ? *reinterpret_cast<const uint4*>(vec + gi) : make_uint4(0, 0, 0, 0);
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int q = q0 + u * blockDim.x;
      if (q < tot4) {
        const int i = q >> lq, c4 = (q & ((1 << lq) - 1)) << 2;
        const int gi = (i << m2) + j2_0 + c4;
        *reinterpret_cast<uint4*>(tile + (i << lc) + c4) = zero_from(v[u], gi, valid);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Transform bodies shared by the pipeline and the standalone kernels.

// Forward column pass on vector `vec` (elements >= valid read as zero),
// written back in place; the twiddle w_N^{j2 k1} is applied by the row pass.
// With at least 8 columns per tile (one per wave of the COL_THREADS
// workgroup) the columns are stored as pad9 rows, each wave transforms
// whole columns with wave-local rounds (no workgroup barrier between the
// rounds), and the tile is transposed on the way in and out; narrower
// tiles keep the column layout and workgroup-wide rounds.
template <int M1>
__device__ __forceinline__ void fwd_cols_body(u32* vec, int valid, int prime, const NttGeom g, int j2_0, const uint2* twb,
                                              u32* smem) {
  const u32 p = prime_of(prime);
  constexpr int m1 = M1;
  const int m2 = g.m2, lc = g.lc, lq = lc - 2;
  uint2* tw = reinterpret_cast<uint2*>(smem);
  u32* tile = smem + (1 << m1);
  load_block_tw(tw, twb, m1);
  if (lc >= 3 && (1 << lc) >= (int)(blockDim.x >> 6)) {
    constexpr int LDC = rec_ldc(M1);
    const int tot4 = 1 << (m1 + lq);
    for (int q0 = threadIdx.x; q0 < tot4; q0 += blockDim.x * UNR) {
      uint4 v[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = q0 + u * blockDim.x;
        if (q < tot4) {
          const int gi = ((q >> lq) << m2) + j2_0 + ((q & ((1 << lq) - 1)) << 2);
          v[u] = gi < valid ? *reinterpret_cast<const uint4*>(vec + gi) : make_uint4(0, 0, 0, 0);
        }
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = q0 + u * blockDim.x;
        if (q < tot4) {
          const int i = q >> lq, c4 = (q & ((1 << lq) - 1)) << 2;
          const uint4 w = zero_from(v[u], (i << m2) + j2_0 + c4, valid);
          u32* b = tile + c4 * LDC + pad9(i);                // row i of columns c4 .. c4 + 3
          b[0] = w.x;
          b[LDC] = w.y;
          b[2 * LDC] = w.z;
          b[3 * LDC] = w.w;
        }
      }
    }
    __syncthreads();
    {
      const int cpw = (1 << lc) / (int)(blockDim.x >> 6);   // columns per wave
      int ln = threadIdx.x & 63;
      asm volatile("" : "+v"(ln));
      rounds_t<M1, 0, false, false, 9, true>(tile + (int)(threadIdx.x >> 6) * cpw * LDC, cpw, LDC, tw, p, ln, 64);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < tot4; q += blockDim.x) {
      const int i = q >> lq, c4 = (q & ((1 << lq) - 1)) << 2;
      const u32* b = tile + c4 * LDC + pad9(i);
      *reinterpret_cast<uint4*>(vec + (i << m2) + j2_0 + c4) = make_uint4(b[0], b[LDC], b[2 * LDC], b[3 * LDC]);
    }
    return;
  }
  load_cols(tile, vec, m1, m2, lc, j2_0, valid);
  __syncthreads();
  block_ntt<M1, false, true>(tile, lc, 0, tw, p);
  const int tot4 = 1 << (m1 + lq);
  for (int q = threadIdx.x; q < tot4; q += blockDim.x) {
    const int i = q >> lq, c4 = (q & ((1 << lq) - 1)) << 2;
    *reinterpret_cast<uint4*>(vec + (i << m2) + j2_0 + c4) = *reinterpret_cast<const uint4*>(tile + (i << lc) + c4);
  }
}

// Forward row pass: rows [i1_0, i1_0 + 2^lrows) of vector vec, each element
// first multiplied by w_N^{j2 k1}.
template <int M2>
__device__ __forceinline__ void fwd_rows_body(u32* vec, int prime, const NttGeom g, int i1_0, const uint2* twb,
                                              const uint2* lo, const uint2* hi, u32* smem) {
  const u32 p = prime_of(prime);
  constexpr int m2 = M2, N2 = 1 << m2, ldr = row_ld(N2);
  const int nr = 1 << g.lrows;
  const u32 Nmask = (1u << g.logN) - 1;
  uint2* tw = reinterpret_cast<uint2*>(smem);
  u32* tile = smem + N2;
  u32* twmem = tile + nr * ldr;
  load_block_tw(tw, twb, m2);
  RowTw rt;
  build_rowtw(rt, twmem, nr, i1_0, g.m1, m2, Nmask, lo, hi, p);
  u32* src = vec + ((size_t)i1_0 << m2);
  load_rows(tile, src, nr, m2, ldr, 1 << 30);
  __syncthreads();
  for (int e = threadIdx.x; e < (nr << m2); e += blockDim.x) {
    const int r = e >> m2, j2 = e & (N2 - 1);
    u32* q = tile + r * ldr + pad8(j2);
    *q = apply_rowtw(rt, *q, r, j2, m2, p);
  }
  __syncthreads();
  block_ntt<M2, false, false>(tile, nr, ldr, tw, p);
  store_rows(src, tile, nr, m2, ldr);
}

// Forward single-workgroup transform of a vector of length 2^logN <= 4096.
template <int M>
__device__ __forceinline__ void fwd_single_body(u32* vec, int valid, int prime, const uint2* twb, u32* smem) {
  const u32 p = prime_of(prime);
  constexpr int logN = M, ldr = row_ld(1 << logN);
  uint2* tw = reinterpret_cast<uint2*>(smem);
  u32* tile = smem + (1 << logN);
  load_block_tw(tw, twb, logN);
  load_rows(tile, vec, 1, logN, ldr, valid);
  __syncthreads();
  block_ntt<M, false, false>(tile, 1, ldr, tw, p);
  store_rows(vec, tile, 1, logN, ldr);
}

// ---------------------------------------------------------------------------
// Standalone kernels (count contiguous vectors; blockIdx.z = vector).

template <int M>
__global__ void __launch_bounds__(NTT_THREADS) k_std_single(u32* data, int prime, bool inverse, TwBlock tb) {
  extern __shared__ u32 smem[];
  constexpr int logN = M, N = 1 << logN;
  u32* vec = data + ((size_t)blockIdx.z << logN);
  if (!inverse) {
    fwd_single_body<M>(vec, N, prime, tb.fwd[prime], smem);
    return;
  }
  const u32 p = prime_of(prime);
  const int ldr = row_ld(N);
  uint2* tw = reinterpret_cast<uint2*>(smem);
  u32* tile = smem + N;
  load_block_tw(tw, tb.inv[prime], logN);
  load_rows(tile, vec, 1, logN, ldr, N);
  __syncthreads();
  block_ntt<M, true, false>(tile, 1, ldr, tw, p);
  // N^{-1} = p - (p-1)/N
  const u32 ninv = p - ((p - 1) >> logN), ninvq = shoup_companion(ninv, p);
  for (int i = threadIdx.x; i < N; i += blockDim.x) vec[i] = shoup_mul(tile[pad8(i)], ninv, ninvq, p);
}

template <int M1>
__global__ void __launch_bounds__(COL_THREADS) k_std_fwd_cols(u32* data, int prime, NttGeom g, TwBlock tb, TwStep ts) {
  extern __shared__ u32 smem[];
  u32* vec = data + ((size_t)blockIdx.z << g.logN);
  fwd_cols_body<M1>(vec, 1 << g.logN, prime, g, col_tile(blockIdx.x, g.m2 - g.lc) << g.lc, tb.fwd[prime], smem);
}

template <int M2>
__global__ void __launch_bounds__(NTT_THREADS) k_std_fwd_rows(u32* data, int prime, NttGeom g, TwBlock tb, TwStep ts) {
  extern __shared__ u32 smem[];
  u32* vec = data + ((size_t)blockIdx.z << g.logN);
  fwd_rows_body<M2>(vec, prime, g, blockIdx.x << g.lrows, tb.fwd[prime], ts.lo[0][prime], ts.hi[0][prime], smem);
}

// Inverse row pass (standalone): DIT rows then w_N^{-j2 k1}.
template <int M2>
__global__ void __launch_bounds__(NTT_THREADS) k_std_inv_rows(u32* data, int prime, NttGeom g, TwBlock tb, TwStep ts) {
  extern __shared__ u32 smem[];
  u32* vec = data + ((size_t)blockIdx.z << g.logN);
  const u32 p = prime_of(prime);
  constexpr int m2 = M2, N2 = 1 << m2, ldr = row_ld(N2);
  const int nr = 1 << g.lrows;
  const u32 Nmask = (1u << g.logN) - 1;
  uint2* tw = reinterpret_cast<uint2*>(smem);
  u32* tile = smem + N2;
  u32* twmem = tile + nr * ldr;
  load_block_tw(tw, tb.inv[prime], m2);
  const int i1_0 = blockIdx.x << g.lrows;
  RowTw rt;
  build_rowtw(rt, twmem, nr, i1_0, g.m1, m2, Nmask, ts.lo[1][prime], ts.hi[1][prime], p);
  u32* src = vec + ((size_t)i1_0 << m2);
  load_rows(tile, src, nr, m2, ldr, 1 << 30);
  __syncthreads();
  block_ntt<M2, true, false>(tile, nr, ldr, tw, p);
  for (int idx = threadIdx.x; idx < (nr << m2); idx += blockDim.x) {
    const int r = idx >> m2, j2 = idx & (N2 - 1);
    src[idx] = apply_rowtw(rt, tile[r * ldr + pad8(j2)], r, j2, m2, p);
  }
}

// Inverse column pass (standalone): DIT columns, times N^{-1}, natural order.
template <int M1>
__global__ void __launch_bounds__(COL_THREADS) k_std_inv_cols(u32* data, int prime, NttGeom g, TwBlock tb) {
  extern __shared__ u32 smem[];
  u32* vec = data + ((size_t)blockIdx.z << g.logN);
  const u32 p = prime_of(prime);
  constexpr int m1 = M1;
  const int m2 = g.m2, lc = g.lc, lq = lc - 2;
  uint2* tw = reinterpret_cast<uint2*>(smem);
  u32* tile = smem + (1 << m1);
  load_block_tw(tw, tb.inv[prime], m1);
  const int j2_0 = col_tile(blockIdx.x, m2 - lc) << lc;
  load_cols(tile, vec, m1, m2, lc, j2_0, 1 << 30);
  __syncthreads();
  block_ntt<M1, true, true>(tile, lc, 0, tw, p);
  const u32 ninv = p - ((p - 1) >> g.logN), ninvq = shoup_companion(ninv, p);
  const int tot4 = 1 << (m1 + lq);
  for (int q = threadIdx.x; q < tot4; q += blockDim.x) {
    const int i = q >> lq, c4 = (q & ((1 << lq) - 1)) << 2;
    uint4 w = *reinterpret_cast<const uint4*>(tile + (i << lc) + c4);
    w.x = shoup_mul(w.x, ninv, ninvq, p);
    w.y = shoup_mul(w.y, ninv, ninvq, p);
    w.z = shoup_mul(w.z, ninv, ninvq, p);
    w.w = shoup_mul(w.w, ninv, ninvq, p);
    *reinterpret_cast<uint4*>(vec + (i << m2) + j2_0 + c4) = w;
  }
}

// ---------------------------------------------------------------------------
// Pipeline kernels.  blockIdx.z indexes the transform list.

struct FwdSel {
  u32* vec;
  int valid, prime;
};

// vector vi = (part K + k) np + prime
__device__ __forceinline__ bool fwd_select(u32* X, const TDesc* td, const TState* ts, const int* tlist, int K, int np,
                                           bool valid_full, int vi, FwdSel& o) {
  const int t = tlist[blockIdx.z];
  const TDesc& d = td[t];
  const TState& s = ts[t];
  const int pk = vi / np, part = pk / K, k = pk - part * K;
  if (s.status || k >= s.kx[part]) return false;
  o.vec = X + d.X_off + ((size_t)vi << d.logN);
  o.valid = valid_full ? d.N : d.n;
  o.prime = vi - pk * np;
  return true;
}

// With a schedule walk attached (walk.ts set) the launch has one more
// vector slice: its first workgroup per transform computes the transform's
// accumulation schedule in one thread while the others transform, since the
// schedule and the forward NTTs depend only on the split.
struct WalkArgs {
  TState* ts = nullptr;
  const KernelDesc* kd = nullptr;
  int L = 0;
};
__device__ __forceinline__ bool walk_slice(const WalkArgs& w, const TDesc* td, const int* tlist, u32* smem) {
  if (!w.ts || blockIdx.y != gridDim.y - 1) return false;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int t = tlist[blockIdx.z];
    const TDesc& d = td[t];
    TState& s = w.ts[t];
    const KernelDesc& kk = w.kd[d.kd];
    int (&E)[2][KMAX] = *reinterpret_cast<int(*)[2][KMAX]>(smem);
    int (&Ew)[2][KMAX] = *reinterpret_cast<int(*)[2][KMAX]>(smem + 2 * KMAX);
    for (int part = 0; part < 2; ++part)
      for (int k = 0; k < KMAX; ++k) {
        E[part][k] = s.E[part][k];
        Ew[part][k] = kk.Ew[part][k];
      }
    schedule_walk(d, s, kk, E, Ew, w.L);
  }
  return true;
}

template <int M>
__global__ void __launch_bounds__(NTT_THREADS) k_fwd_single(u32* X, const TDesc* td, const TState* ts,
                                                            const int* tlist, int K, int np, bool valid_full,
                                                            int vi_lo, TwBlock tb, WalkArgs walk) {
  extern __shared__ u32 smem[];
  if (walk_slice(walk, td, tlist, smem)) return;
  FwdSel o;
  if (!fwd_select(X, td, ts, tlist, K, np, valid_full, vi_lo + blockIdx.y, o)) return;
  fwd_single_body<M>(o.vec, o.valid, o.prime, tb.fwd[o.prime], smem);
}

template <int M1>
__global__ void __launch_bounds__(COL_THREADS) k_fwd_cols(u32* X, const TDesc* td, const TState* ts,
                                                          const int* tlist, int K, int np, bool valid_full,
                                                          int vi_lo, NttGeom g, TwBlock tb, TwStep st, WalkArgs walk) {
  extern __shared__ u32 smem[];
  if (walk_slice(walk, td, tlist, smem)) return;
  FwdSel o;
  if (!fwd_select(X, td, ts, tlist, K, np, valid_full, vi_lo + blockIdx.y, o)) return;
  fwd_cols_body<M1>(o.vec, o.valid, o.prime, g, col_tile(blockIdx.x, g.m2 - g.lc) << g.lc, tb.fwd[o.prime], smem);
}

template <int M2>
__global__ void __launch_bounds__(NTT_THREADS) k_fwd_rows(u32* X, const TDesc* td, const TState* ts,
                                                          const int* tlist, int K, int np, bool valid_full,
                                                          int vi_lo, NttGeom g, TwBlock tb, TwStep st) {
  extern __shared__ u32 smem[];
  FwdSel o;
  if (!fwd_select(X, td, ts, tlist, K, np, valid_full, vi_lo + blockIdx.y, o)) return;
  fwd_rows_body<M2>(o.vec, o.prime, g, blockIdx.x << g.lrows, tb.fwd[o.prime], st.lo[0][o.prime], st.hi[0][o.prime], smem);
}

// The four real convolutions (Sec. 4.5): input part pa with kernel part pb.
__device__ __constant__ int c_conv_pa[4] = {0, 1, 1, 0};
__device__ __constant__ int c_conv_pb[4] = {0, 1, 0, 1};

// NTT-domain multiply-accumulate (Alg. 8) at the two positions e, e+1 of
// the NTT domain: every group sum
//     Z_g = sum over the members (c, s, t) of g of +- X_pa(c)^s (.) W_pb(c)^t   (mod p),
// with the minus sign for convolution 1 (Im x' Im w*, subtracted in Re y').
// Groups are numbered across the output components (group g of component tg
// has number gofs[tg] + g); those in [g0, g1) are written to LDS at
// lds0 + (number - g0) * rstride.  Members are visited in the component's
// walk order and `gend` marks the position closing each group.  With at
// most KT slices per operand the slices of the two positions are loaded
// once into registers and every product is formed from them.
struct MacArgs {
  const u32* X;      // this transform's slice spectra, [part][k][prime][N]
  const u32* W;      // kernel spectra of its length, same layout
  const u32* Wq;
  int K, logN, prime;
  u32 p;
  int kw0, kw1;      // kernel slice counts of Re w*, Im w*
  int np;            // moduli
};

__device__ __forceinline__ uint2 ld2(const u32* ptr) { return *reinterpret_cast<const uint2*>(ptr); }

__device__ __forceinline__ void mac_acc(uint2& acc, const uint2& x, const uint2& w, const uint2& q, u32 p) {
  acc.x = add_mod(acc.x, shoup_mul(x.x, w.x, q.x, p), p);
  acc.y = add_mod(acc.y, shoup_mul(x.y, w.y, q.y, p), p);
}

__device__ __forceinline__ void mac_acc(u32& acc, u32 x, u32 w, u32 q, u32 p) {
  acc = add_mod(acc, shoup_mul(x, w, q, p), p);
}
__device__ __forceinline__ void mac_sub(uint2& acc, const uint2& x, const uint2& w, const uint2& q, u32 p) {
  acc.x = sub_mod(acc.x, shoup_mul(x.x, w.x, q.x, p), p);
  acc.y = sub_mod(acc.y, shoup_mul(x.y, w.y, q.y, p), p);
}
__device__ __forceinline__ void mac_sub(u32& acc, u32 x, u32 w, u32 q, u32 p) {
  acc = sub_mod(acc, shoup_mul(x, w, q, p), p);
}
__device__ __forceinline__ void zero_acc(uint2& a) { a = make_uint2(0, 0); }
__device__ __forceinline__ void zero_acc(u32& a) { a = 0; }
__device__ __forceinline__ void put_acc(u32* ptr, const uint2& a) { *reinterpret_cast<uint2*>(ptr) = a; }
__device__ __forceinline__ void put_acc(u32* ptr, u32 a) { *ptr = a; }

// Both convolutions of one output component from register-held slices
// (all slice counts <= KT), in the component's walk order: convolution a
// (sign +) and b (sign - when NEGB).  V is u32 (one position) or uint2 (two
// adjacent positions).  Position w of the walk closes a group when bit w of
// gend is set; group g (numbered from gbase) goes to LDS row g - g0 when it
// lies in [g0, g1).
template <bool NEGB, typename V>
__device__ __forceinline__ void walk_step(V& acc, int h, const V& x, const V& w, const V& q, u32 p) {
  if (NEGB && h == 1) mac_sub(acc, x, w, q, p);
  else mac_acc(acc, x, w, q, p);
}
template <bool MERGED, bool NEGB, typename V>
__device__ __forceinline__ void walk_target(const V (&xa)[KT], const V (&wa)[KT], const V (&qa)[KT], int kAa, int kBa,
                                            const V (&xb)[KT], const V (&wb)[KT], const V (&qb)[KT], int kAb, int kBb,
                                            u64 gend, int gbase, int g0, int g1, u32* lds0, int rstride, u32 p) {
  int w = 0, g = gbase;
  V acc;
  zero_acc(acc);
  auto close = [&]() {
    if ((gend >> w) & 1) {
      if (g >= g0 && g < g1) put_acc(lds0 + (g - g0) * rstride, acc);
      zero_acc(acc);
      ++g;
    }
    ++w;
  };
  if constexpr (MERGED) {
#pragma unroll
    for (int d = 2 * KT - 2; d >= 0; --d) {
#pragma unroll
      for (int ss = (d - KT + 1 > 0 ? d - KT + 1 : 0); ss <= (KT - 1 < d ? KT - 1 : d); ++ss)
        if (ss < kAa && d - ss < kBa) {
          walk_step<NEGB>(acc, 0, xa[ss], wa[d - ss], qa[d - ss], p);
          close();
        }
#pragma unroll
      for (int ss = (d - KT + 1 > 0 ? d - KT + 1 : 0); ss <= (KT - 1 < d ? KT - 1 : d); ++ss)
        if (ss < kAb && d - ss < kBb) {
          walk_step<NEGB>(acc, 1, xb[ss], wb[d - ss], qb[d - ss], p);
          close();
        }
    }
  } else {
#pragma unroll
    for (int d = 2 * KT - 2; d >= 0; --d) {
#pragma unroll
      for (int ss = (d - KT + 1 > 0 ? d - KT + 1 : 0); ss <= (KT - 1 < d ? KT - 1 : d); ++ss)
        if (ss < kAa && d - ss < kBa) {
          walk_step<NEGB>(acc, 0, xa[ss], wa[d - ss], qa[d - ss], p);
          close();
        }
    }
#pragma unroll
    for (int d = 2 * KT - 2; d >= 0; --d) {
#pragma unroll
      for (int ss = (d - KT + 1 > 0 ? d - KT + 1 : 0); ss <= (KT - 1 < d ? KT - 1 : d); ++ss)
        if (ss < kAb && d - ss < kBb) {
          walk_step<NEGB>(acc, 1, xb[ss], wb[d - ss], qb[d - ss], p);
          close();
        }
    }
  }
}

// The same walk when all four slice counts equal C and every group of the
// component goes to LDS: fully unrolled, the only branches are the group
// ends (bit w of gend, w a compile-time position); group g is written to
// lds0 + g rstride.
template <bool MERGED, bool NEGB, int C, typename V>
__device__ __forceinline__ void walk_full(const V (&xa)[KT], const V (&wa)[KT], const V (&qa)[KT], const V (&xb)[KT],
                                          const V (&wb)[KT], const V (&qb)[KT], u64 gend, u32* lds0, int rstride,
                                          u32 p) {
  V acc;
  zero_acc(acc);
  u32* dst = lds0;
  int w = 0;
  auto close = [&]() {
    if ((gend >> w) & 1) {
      put_acc(dst, acc);
      zero_acc(acc);
      dst += rstride;
    }
    ++w;
  };
  if constexpr (MERGED) {
#pragma unroll
    for (int d = 2 * C - 2; d >= 0; --d) {
#pragma unroll
      for (int ss = (d - C + 1 > 0 ? d - C + 1 : 0); ss <= (C - 1 < d ? C - 1 : d); ++ss) {
        walk_step<NEGB>(acc, 0, xa[ss], wa[d - ss], qa[d - ss], p);
        close();
      }
#pragma unroll
      for (int ss = (d - C + 1 > 0 ? d - C + 1 : 0); ss <= (C - 1 < d ? C - 1 : d); ++ss) {
        walk_step<NEGB>(acc, 1, xb[ss], wb[d - ss], qb[d - ss], p);
        close();
      }
    }
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int d = 2 * C - 2; d >= 0; --d) {
#pragma unroll
        for (int ss = (d - C + 1 > 0 ? d - C + 1 : 0); ss <= (C - 1 < d ? C - 1 : d); ++ss) {
          if (h == 0) walk_step<NEGB>(acc, 0, xa[ss], wa[d - ss], qa[d - ss], p);
          else walk_step<NEGB>(acc, 1, xb[ss], wb[d - ss], qb[d - ss], p);
          close();
        }
      }
    }
  }
}
// One output component with operands read per walk position (any slice
// counts): the members (convolution, s, t) recorded by the schedule.
__device__ void walk_mem(const MacArgs& a, const TState& s, int tg, int gbase, int g0, int g1, size_t e, u32* lds0,
                         int rstride) {
  const size_t N = (size_t)1 << a.logN, sstride = a.np * N;
  int g = gbase;
  uint2 acc = make_uint2(0, 0);
  for (int w = 0; w < s.nmem[tg]; ++w) {
    const int c = s.mc[tg][w], ss = s.ms[tg][w], tt = s.mt[tg][w];
    const int pa = c_conv_pa[c], pb = c_conv_pb[c];
    const u32* xb = a.X + (size_t)((pa * a.K) * a.np + a.prime) * N + e;
    const u32* wb = a.W + (size_t)((pb * a.K) * a.np + a.prime) * N + e;
    const u32* qb = a.Wq + (size_t)((pb * a.K) * a.np + a.prime) * N + e;
    if (c == 1) mac_sub(acc, ld2(xb + ss * sstride), ld2(wb + tt * sstride), ld2(qb + tt * sstride), a.p);
    else mac_acc(acc, ld2(xb + ss * sstride), ld2(wb + tt * sstride), ld2(qb + tt * sstride), a.p);
    if ((s.gend[tg][w >> 6] >> (w & 63)) & 1) {
      if (g >= g0 && g < g1) *reinterpret_cast<uint2*>(lds0 + (g - g0) * rstride) = acc;
      acc = make_uint2(0, 0);
      ++g;
    }
  }
}

// Kernel-slice operands of positions e, e+1 held in registers (<= KT slices
// per part): Re w* slices with companions (w0, q0), Im w* (w1, q1).
template <typename V>
struct WRegs {
  V w0[KT], q0[KT], w1[KT], q1[KT];
};
__device__ __forceinline__ void ldv(uint2& v, const u32* ptr) { v = ld2(ptr); }
__device__ __forceinline__ const u32* at_byte(const u32* base, u32 byte_off) {
  return reinterpret_cast<const u32*>(reinterpret_cast<const char*>(base) + byte_off);
}
__device__ __forceinline__ void ldv(u32& v, const u32* ptr) { v = *ptr; }
template <int NP, typename V>
__device__ __forceinline__ void load_wregs(WRegs<V>& r, const u32* W, const u32* Wq, int K, int logN, int prime,
                                           int kw0, int kw1, u32 e) {
  // uniform row pointers plus a 32-bit byte offset per lane (e < N <= 2^24)
  const size_t N = (size_t)1 << logN, sstride = NP * N, part = (size_t)K * sstride;
  const u32 eb = e * 4u;
  const u32* wb = W + (size_t)prime * N;
  const u32* qb = Wq + (size_t)prime * N;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    if (k < kw0) {
      ldv(r.w0[k], at_byte(wb + k * sstride, eb));
      ldv(r.q0[k], at_byte(qb + k * sstride, eb));
    }
    if (k < kw1) {
      ldv(r.w1[k], at_byte(wb + part + k * sstride, eb));
      ldv(r.q1[k], at_byte(qb + part + k * sstride, eb));
    }
  }
}
// Slice spectra of Re x' (xr) and Im x' (xi) at positions e, e+1.
template <int NP, typename V>
__device__ __forceinline__ void load_xregs(V (&xr)[KT], V (&xi)[KT], const u32* X, int K, int logN, int prime, int kx0,
                                           int kx1, u32 e) {
  const size_t N = (size_t)1 << logN, sstride = NP * N, part = (size_t)K * sstride;
  const u32 eb = e * 4u;
  const u32* xb = X + (size_t)prime * N;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    if (k < kx0) ldv(xr[k], at_byte(xb + k * sstride, eb));
    if (k < kx1) ldv(xi[k], at_byte(xb + part + k * sstride, eb));
  }
}
// Both output components from register operands (Re y': ReRe - ImIm, then
// Im y': ImRe + ReIm); groups [g0, g1) go to LDS.
template <bool MERGED, typename V>
__device__ __forceinline__ void mac_regs_t(const V (&xr)[KT], const V (&xi)[KT], const V (&w0)[KT], const V (&q0)[KT],
                                           const V (&w1)[KT], const V (&q1)[KT], const TState& s, int kw0, int kw1,
                                           int tg_lo, int tg_hi, const int (&gofs)[2], int g0, int g1, u32* lds0,
                                           int rstride, u32 p) {
  const int kx0 = s.kx[0], kx1 = s.kx[1];
  if (tg_lo <= 0)
    walk_target<MERGED, true>(xr, w0, q0, kx0, kw0, xi, w1, q1, kx1, kw1, s.gend[0][0], gofs[0], g0, g1, lds0,
                              rstride, p);
  if (tg_hi >= 1)
    walk_target<MERGED, false>(xi, w0, q0, kx1, kw0, xr, w1, q1, kx0, kw1, s.gend[1][0], gofs[1], g0, g1, lds0,
                               rstride, p);
}
template <typename V>
__device__ __forceinline__ void mac_regs(const V (&xr)[KT], const V (&xi)[KT], const WRegs<V>& r,
                                         const TState& s, bool merged, int kw0, int kw1, const int (&gofs)[2], int g0,
                                         int g1, u32* lds0, int rstride, u32 p) {
  if (merged)
    mac_regs_t<true>(xr, xi, r.w0, r.q0, r.w1, r.q1, s, kw0, kw1, 0, 1, gofs, g0, g1, lds0, rstride, p);
  else
    mac_regs_t<false>(xr, xi, r.w0, r.q0, r.w1, r.q1, s, kw0, kw1, 0, 1, gofs, g0, g1, lds0, rstride, p);
}

// Both output components, all counts C, all groups to LDS rows 0 .. gtot-1.
template <int C, typename V>
__device__ __forceinline__ void mac_full(const V (&xr)[KT], const V (&xi)[KT], const WRegs<V>& r, const TState& s,
                                         bool merged, u32* lds0, int rstride, u32 p) {
  u32* lds1 = lds0 + s.ngroups[0] * rstride;
  if (merged) {
    walk_full<true, true, C>(xr, r.w0, r.q0, xi, r.w1, r.q1, s.gend[0][0], lds0, rstride, p);
    walk_full<true, false, C>(xi, r.w0, r.q0, xr, r.w1, r.q1, s.gend[1][0], lds1, rstride, p);
  } else {
    walk_full<false, true, C>(xr, r.w0, r.q0, xi, r.w1, r.q1, s.gend[0][0], lds0, rstride, p);
    walk_full<false, false, C>(xi, r.w0, r.q0, xr, r.w1, r.q1, s.gend[1][0], lds1, rstride, p);
  }
}

// Output components [tg_lo, tg_hi] at positions e, e+1 (e even).
__device__ void mac_pair(const MacArgs& a, const TState& s, bool merged, int tg_lo, int tg_hi, const int (&gofs)[2],
                         int g0, int g1, size_t e, u32* lds0, int rstride) {
  const size_t N = (size_t)1 << a.logN, sstride = a.np * N;
  const int kx0 = s.kx[0], kx1 = s.kx[1];
  if (kx0 <= KT && kx1 <= KT && a.kw0 <= KT && a.kw1 <= KT) {
    uint2 w0[KT], q0[KT], w1[KT], q1[KT], xr[KT], xi[KT];
    const u32* wb = a.W + (size_t)a.prime * N + e;
    const u32* qb = a.Wq + (size_t)a.prime * N + e;
    const u32* xb = a.X + (size_t)a.prime * N + e;
    const size_t part = (size_t)a.K * sstride;
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      if (k < a.kw0) {
        w0[k] = ld2(wb + k * sstride);
        q0[k] = ld2(qb + k * sstride);
      }
      if (k < a.kw1) {
        w1[k] = ld2(wb + part + k * sstride);
        q1[k] = ld2(qb + part + k * sstride);
      }
      if (k < kx0) xr[k] = ld2(xb + k * sstride);
      if (k < kx1) xi[k] = ld2(xb + part + k * sstride);
    }
    if (merged)
      mac_regs_t<true>(xr, xi, w0, q0, w1, q1, s, a.kw0, a.kw1, tg_lo, tg_hi, gofs, g0, g1, lds0, rstride, a.p);
    else
      mac_regs_t<false>(xr, xi, w0, q0, w1, q1, s, a.kw0, a.kw1, tg_lo, tg_hi, gofs, g0, g1, lds0, rstride, a.p);
    return;
  }
  for (int tg = tg_lo; tg <= tg_hi; ++tg) walk_mem(a, s, tg, gofs[tg], g0, g1, e, lds0, rstride);
}

// Scalar variant for vectors of length 1.
__device__ void mac_single(const MacArgs& a, const TState& s, int tg_lo, int tg_hi, const int (&gofs)[2], int g0,
                           int g1, size_t e, u32* lds0, int rstride) {
  const size_t N = (size_t)1 << a.logN;
  for (int tg = tg_lo; tg <= tg_hi; ++tg) {
    u32 acc = 0;
    int g = gofs[tg];
    for (int w = 0; w < s.nmem[tg]; ++w) {
      const int c = s.mc[tg][w], ss = s.ms[tg][w], tt = s.mt[tg][w];
      const int pa = c_conv_pa[c], pb = c_conv_pb[c];
      const u32* xb = a.X + (size_t)((pa * a.K) * a.np + a.prime) * N + e;
      const u32* wb = a.W + (size_t)((pb * a.K) * a.np + a.prime) * N + e;
      const u32* qb = a.Wq + (size_t)((pb * a.K) * a.np + a.prime) * N + e;
      const size_t xo = (size_t)ss * a.np * N, wo = (size_t)tt * a.np * N;
      if (c == 1) mac_sub(acc, xb[xo], wb[wo], qb[wo], a.p);
      else mac_acc(acc, xb[xo], wb[wo], qb[wo], a.p);
      if ((s.gend[tg][w >> 6] >> (w & 63)) & 1) {
        if (g >= g0 && g < g1) lds0[(g - g0) * rstride] = acc;
        acc = 0;
        ++g;
      }
    }
  }
}

// Rows of the group tile that fit the inverse's LDS budget.
// (about 512 words each; longer rows get proportionally fewer)
__host__ __device__ inline int inv_vmax(int m) {
  const int v = m <= 9 ? INV_TILE_ROWS : (INV_TILE_ROWS >> (m - 9));
  return v < 1 ? 1 : v;
}

// Workgroup index -> (tile, prime, transform).  When the tile-prime pairs
// divide evenly over the eight XCDs (workgroups are dispatched to XCDs
// round-robin), consecutive workgroups of one XCD take the same tile of
// consecutive transforms, so the kernel spectra they share stay in that
// XCD's L2.
__device__ __forceinline__ void decode_tile(int L, int pairs, int count, int& pair, int& b) {
  if ((pairs & 7) == 0) {
    const int xcd = L & 7, r = L >> 3;
    b = r % count;
    pair = (r / count) * 8 + xcd;
  } else {
    b = L / pairs;
    pair = L % pairs;
  }
}

// Single-workgroup inverse (N <= 4096): one workgroup per (transform, prime,
// output component).  For each chunk of groups: multiply-accumulate into LDS
// rows, inverse block NTTs, first n outputs to the compact buffer.
template <int M>
__global__ void __launch_bounds__(NTT_THREADS) k_inv_single(const u32* X, u32* Z, const TDesc* td, const TState* ts,
                                                            const KernelDesc* kd, const int* tlist, int count, int K,
                                                            int np, int slot_lo, int slot_hi, TwBlock tb) {
  constexpr int logN = M;
  extern __shared__ u32 smem[];
  int pair, b;
  decode_tile(blockIdx.x, 2 * np, count, pair, b);
  const int t = tlist[b];
  const TDesc& d = td[t];
  const TState& s = ts[t];
  if (s.status) return;
  const int tg = pair / np, prime = pair - tg * np;
  const int ng = s.ngroups[tg];
  if (ng == 0) return;
  const u32 p = prime_of(prime);
  const KernelDesc& kk = kd[d.kd];
  const int N = 1 << logN, ldr = row_ld(N), SL = 2 * K * K, vmax = inv_vmax(logN);
  const bool merged = d.acc_mode == ACC_COMPLEX;
  uint2* tw = reinterpret_cast<uint2*>(smem);
  u32* tile = smem + N;
  load_block_tw(tw, tb.inv[prime], logN);
  const MacArgs ma{X + d.X_off, kk.W, kk.Wq, K, logN, prime, p, kk.kw[0], kk.kw[1], np};
  const int gofs[2] = {0, 0};
  for (int g0 = 0; g0 < ng; g0 += vmax) {
    const int g1 = min(ng, g0 + vmax);
    if (tg * SL + g1 <= slot_lo || tg * SL + g0 >= slot_hi) continue;
    if (logN >= 1) {
      for (int q = threadIdx.x; q < (N >> 1); q += blockDim.x)
        mac_pair(ma, s, merged, tg, tg, gofs, g0, g1, (size_t)q << 1, tile + pad8(q << 1), ldr);
    } else {
      for (int i = threadIdx.x; i < N; i += blockDim.x) mac_single(ma, s, tg, tg, gofs, g0, g1, i, tile + pad8(i), ldr);
    }
    __syncthreads();
    block_ntt<M, true, false>(tile, g1 - g0, ldr, tw, p);
    for (int gi = g0; gi < g1; ++gi) {
      const int slot = tg * SL + gi;
      if (slot < slot_lo || slot >= slot_hi) continue;
      u32* zo = Z + d.Z_off + (size_t)(slot * np + prime) * d.zs;
      const u32* row = tile + (gi - g0) * ldr;
      for (int i = threadIdx.x; i < d.n; i += blockDim.x) zo[i] = row[pad8(i)];
    }
    __syncthreads();
  }
}

// Group rows [g0, g1) of the tile: times w_N^{-j2 k1}, stored to their slots.
// The (row, quad) items of all groups are spread over the whole workgroup;
// when blockDim is a multiple of the quads per group row, a thread always
// handles the same quad, so its four twiddles are loaded once.
template <int PL = 8>
__device__ __forceinline__ void store_group_rows(u32* G, const TDesc& d, const u32* tile, const u32* rtw,
                                                 const int (&gofs)[2], int g0, int g1, int SL, int slot_lo,
                                                 int slot_hi, int np, int prime, int logN, size_t base, int m2,
                                                 int nr, int ldr, u32 p) {
  const int quads = (nr << m2) >> 2, N2 = 1 << m2;
  const int items = (g1 - g0) * quads;
  const bool fixed = (blockDim.x % quads) == 0;
  uint4 w = make_uint4(0, 0, 0, 0), wq = w;
  if (fixed && (int)threadIdx.x < items) {
    const int e = ((int)threadIdx.x % quads) << 2;
    w = *reinterpret_cast<const uint4*>(rtw + e);          // roots and companions in separate arrays
    wq = *reinterpret_cast<const uint4*>(rtw + (nr << m2) + e);
  }
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int gi = g0 + it / quads, q = it % quads;
    const int slot = gi < gofs[1] ? gi : SL + gi - gofs[1];   // SL: slots per output component
    if (slot < slot_lo || slot >= slot_hi) continue;
    const int e = q << 2, r = e >> m2, j2 = e & (N2 - 1);
    uint4 v;
    if constexpr (PL == 8) {
      v = *reinterpret_cast<const uint4*>(tile + ((gi - g0) * nr + r) * ldr + pad8(j2));
    } else {                                  // j2..j2+3 share one eight-element block: contiguous
      const u32* q = tile + ((gi - g0) * nr + r) * ldr + padl<PL>(j2);
      v = make_uint4(q[0], q[1], q[2], q[3]);
    }
    if (!fixed) {
      w = *reinterpret_cast<const uint4*>(rtw + e);
      wq = *reinterpret_cast<const uint4*>(rtw + (nr << m2) + e);
    }
    v.x = shoup_mul(v.x, w.x, wq.x, p);
    v.y = shoup_mul(v.y, w.y, wq.y, p);
    v.z = shoup_mul(v.z, w.z, wq.z, p);
    v.w = shoup_mul(v.w, w.w, wq.w, p);
    reinterpret_cast<uint4*>(G + d.G_off + ((size_t)(slot * np + prime) << logN) + base)[q] = v;
  }
}

// Two-pass inverse, first pass (rows): one workgroup per (row tile, prime)
// and run of up to tpw consecutive transforms of the list.  Per transform:
// multiply-accumulate into LDS (normally all groups of the four
// convolutions at once), inverse row NTTs, twiddle w_N^{-j2 k1}, store the
// group rows.  The block roots and the row twiddles are set up once per run.
//
// Register form (K <= KT, row tile of INV_ROW_THREADS positions): one
// position per thread, the kernel-slice operands stay in registers for the
// run and the slice spectra of the next transform load while the current
// one is transformed; more groups than one chunk holds recompute the
// products from the registers per chunk.  (The batched schedule runs the
// pipelined form below, which also does the forward row pass; this one
// serves the per-group launches of the plain form, two moduli.)
constexpr int INV_ROW_THREADS = 512;
template <int M2>
__global__ void __launch_bounds__(INV_ROW_THREADS, 6) k_inv_rows_reg(const u32* X, u32* G, const TDesc* td,
                                                                  const TState* ts, const KernelDesc* kd,
                                                                  const int* tlist, int count, int K, int slot_lo,
                                                                  int slot_hi, NttGeom g, TwBlock tb, TwStep st,
                                                                  int tpw) {
  extern __shared__ u32 smem[];
  const int nruns = (count + tpw - 1) / tpw;
  int pair, run;
  decode_tile(blockIdx.x, 2 << (g.m1 - g.lrows_inv), nruns, pair, run);
  const int b_lo = run * tpw, b_hi = min(count, b_lo + tpw);
  const int prime = pair & 1;
  const u32 p = prime_of(prime);
  constexpr int PL = 9;                                       // row layout pad9: conflict-free rounds
  constexpr int m2 = M2, N2 = 1 << m2, ldr = row_ldl<PL>(N2);
  const int nr = 1 << g.lrows_inv, SL = 2 * K * K;           // slots per output component
  const int gch = max(1, inv_vmax(m2) >> g.lrows_inv);          // groups per chunk
  const u32 Nmask = (1u << g.logN) - 1;
  uint2* tw = reinterpret_cast<uint2*>(smem);                // inverse roots, entries 0 .. N2/2
  u32* rtw = smem + N2 + 4;                                   // w_N^{-j2 k1} per tile element, then companions
  u32* tile = rtw + 2 * (nr << m2) + 2 * nr;
  load_block_tw(tw, tb.inv[prime], m2);
  if (threadIdx.x == 0) tw[N2 >> 1] = make_uint2(p - 1, shoup_companion(p - 1, p));   // w^(-N2/2) = -1
  const int i1_0 = (pair >> 1) << g.lrows_inv;
  for (int e = threadIdx.x; e < (nr << m2); e += blockDim.x) {
    const uint2 r = step_root(((u32)(e & (N2 - 1)) * bitrev(i1_0 + (e >> m2), g.m1)) & Nmask, st.lo[1][prime],
                              st.hi[1][prime], p);
    rtw[e] = r.x;
    rtw[(nr << m2) + e] = r.y;
  }
  const size_t base = (size_t)i1_0 << m2;
  const int e_loc = threadIdx.x;                              // this thread's position in the tile
  const u32 pos = (u32)base + (u32)e_loc;                     // its position in the N2 x N1 matrix (< N)
  u32* lds_me = tile + (e_loc >> m2) * ldr + padl<PL>(e_loc & (N2 - 1));
  WRegs<u32> wr;
  int wkd = -1;
  u32 xr[KT], xi[KT];
  int bn = b_lo;                                              // transform whose slices are in xr, xi
  while (bn < b_hi && ts[tlist[bn]].status) ++bn;
  if (bn < b_hi) {
    const int t = tlist[bn];
    load_xregs<2>(xr, xi, X + td[t].X_off, K, g.logN, prime, ts[t].kx[0], ts[t].kx[1], pos);
  }
  while (bn < b_hi) {
    const int t = tlist[bn];
    const TDesc& d = td[t];
    const TState& s = ts[t];
    const KernelDesc& kk = kd[d.kd];
    if (d.kd != wkd) {
      load_wregs<2>(wr, kk.W, kk.Wq, K, g.logN, prime, kk.kw[0], kk.kw[1], pos);
      wkd = d.kd;
    }
    const int gofs[2] = {0, s.ngroups[0]};
    const int gtot = s.ngroups[0] + s.ngroups[1];
    int b2 = bn + 1;
    while (b2 < b_hi && ts[tlist[b2]].status) ++b2;
    for (int g0 = 0; g0 < gtot; g0 += gch) {
      const int g1 = min(gtot, g0 + gch);
      mac_regs(xr, xi, wr, s, d.acc_mode == ACC_COMPLEX, kk.kw[0], kk.kw[1], gofs, g0, g1, lds_me, nr * ldr, p);
      if (g1 == gtot && b2 < b_hi) {                          // slices consumed: fetch the next transform's
        const int t2 = tlist[b2];
        load_xregs<2>(xr, xi, X + td[t2].X_off, K, g.logN, prime, ts[t2].kx[0], ts[t2].kx[1], pos);
      }
      __syncthreads();
      block_ntt<M2, true, false, PL>(tile, (g1 - g0) * nr, ldr, tw, p);
      store_group_rows<PL>(G, d, tile, rtw, gofs, g0, g1, SL, slot_lo, slot_hi, 2, prime, g.logN, base, m2, nr, ldr,
                           p);
      __syncthreads();
    }
    if (gtot == 0 && b2 < b_hi) {                             // no groups (all-zero input): still advance
      const int t2 = tlist[b2];
      load_xregs<2>(xr, xi, X + td[t2].X_off, K, g.logN, prime, ts[t2].kx[0], ts[t2].kx[1], pos);
    }
    bn = b2;
  }
}

// Persistent, pipelined form of the folded inverse row pass (the batched
// schedule's row pass whenever fused_rows_ok holds; NP moduli).  The work
// units are (row tile, prime, transform); workgroup i of the grid (sized to
// the workgroups that fit the GPU at once) takes the contiguous units
// [i U / grid, (i + 1) U / grid), U = tiles x primes x transforms, in the
// order (tile, prime) major, transform minor, so a workgroup mostly stays on
// one tile and prime and keeps the kernel-slice operands of its position in
// registers.  One position of the tile per thread, as in k_inv_rows_reg.
//
// Per transform: the thread forms every group's NTT-domain sum at its
// position into the group tiles of LDS region A and, in the same step, the
// next transform's row-twiddled forward column output into region B; after
// one barrier every wave runs whole tiles (inverse row NTTs of the groups,
// forward row NTTs of the next transform's slices; 16 tiles over 8 waves at
// K = L = 3), each wave on its own tiles, so its rounds need no workgroup
// barrier; after a second barrier each thread twiddles and stores the group
// values of its own position and reads back the next transform's slice
// spectra.  Nothing else touches another thread's position, so two barriers
// per transform suffice.  The row twiddles w_N^{+-j2 k1} of the thread's
// position are formed in registers once per (tile, prime).
template <int M2, int NP>
__global__ void __launch_bounds__(INV_ROW_THREADS, 6) k_inv_rows_pipe(const u32* X, u32* G, const TDesc* td,
                                                                   const TState* ts, const KernelDesc* kd,
                                                                   const int* tlist, int count, int K, NttGeom g,
                                                                   TwBlock tb, TwStep st) {
  extern __shared__ u32 smem[];
  constexpr int PL = 9;
  constexpr int m2 = M2, N2 = 1 << m2, ldr = row_ldl<PL>(N2), NW = INV_ROW_THREADS / 64;
  const int lrows = g.lrows_inv, nr = 1 << lrows, SL = 2 * K * K;
  const int gch = PIPE_TILES;                                 // group tiles in LDS
  const int gA = gch - 2 * K;                                 // region A: inverse group tiles per chunk
  const int tstride = nr * ldr;                               // words per group tile
  const u32 Nmask = (1u << g.logN) - 1;
  uint2* tw = reinterpret_cast<uint2*>(smem);                // inverse roots, entries 0 .. N2/2
  uint2* twf = reinterpret_cast<uint2*>(smem + N2 + 4);      // forward roots, entries 0 .. N2/2 - 1
  u32* tileA = smem + 2 * N2 + 4;
  u32* tileB = tileA + gA * tstride;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int e_loc = threadIdx.x;
  const int r_loc = e_loc >> m2, j2 = e_loc & (N2 - 1);
  const int off_me = r_loc * ldr + padl<PL>(j2);
  const long units = (long)(NP << (g.m1 - lrows)) * count;
  const long u_lo = units * blockIdx.x / gridDim.x, u_hi = units * (blockIdx.x + 1) / gridDim.x;

  auto live = [&](int b) { return !ts[tlist[b]].status; };
  // wave w transforms tiles w, w + NW, ..: A tiles (inverse) first, then B (forward)
  // (the lane index passes through an empty asm statement per tile, so the
  // compiler recomputes the rounds' lane offsets instead of keeping them all
  // live across the kernel)
  auto run_tiles = [&](int nA, int nB, u32 p) {
    for (int r = wave; r < nA + nB; r += NW) {
      int ln = lane;
      asm volatile("" : "+v"(ln));
      if (r < nA) rounds_t<M2, 0, true, false, PL, true>(tileA + r * tstride, nr, ldr, tw, p, ln, 64);
      else rounds_t<M2, 0, false, false, PL, true>(tileB + (r - nA) * tstride, nr, ldr, twf, p, ln, 64);
    }
  };

  for (long u = u_lo; u < u_hi;) {
    const int pair = (int)(u / count), b_lo = (int)(u % count);
    const long seg_end = min(u_hi, (long)(pair + 1) * count);
    const int b_hi = (int)(seg_end - (long)pair * count);
    u = seg_end;
    const int rtile = pair / NP, prime = pair - rtile * NP;
    const u32 p = prime_of(prime);
    const int i1_0 = rtile << lrows;
    const size_t base = (size_t)i1_0 << m2;
    const u32 pos = (u32)base + (u32)e_loc;
    // tables of this (tile, prime): block roots in LDS, row twiddles of this position
    __syncthreads();                                          // the previous segment's rounds are done with tw
    load_block_tw(tw, tb.inv[prime], m2);
    load_block_tw(twf, tb.fwd[prime], m2);
    if (threadIdx.x == 0) tw[N2 >> 1] = make_uint2(p - 1, shoup_companion(p - 1, p));   // w^(-N2/2) = -1
    const u32 ek = ((u32)j2 * bitrev(i1_0 + r_loc, g.m1)) & Nmask;
    const uint2 fwt = step_root(ek, st.lo[0][prime], st.hi[0][prime], p);   // w_N^{j2 k1}
    const uint2 iwt = step_root(ek, st.lo[1][prime], st.hi[1][prime], p);   // w_N^{-j2 k1}
    WRegs<u32> wr;
    int wkd = -1;
    u32 xr[KT], xi[KT], yr[KT], yi[KT];
    int bn = b_lo;
    while (bn < b_hi && !live(bn)) ++bn;
    if (bn >= b_hi) continue;
    auto next_live = [&](int b) {
      ++b;
      while (b < b_hi && !live(b)) ++b;
      return b;
    };
    auto put_b = [&](int kx0, int kx1, int om) {              // row-twiddled column output into region B
#pragma unroll
      for (int k = 0; k < KT; ++k) {
        if (k < kx0) tileB[k * tstride + om] = shoup_mul(yr[k], fwt.x, fwt.y, p);
        if (k < kx1) tileB[(kx0 + k) * tstride + om] = shoup_mul(yi[k], fwt.x, fwt.y, p);
      }
    };
    auto get_b = [&](int kx0, int kx1, int om) {              // slice spectra back from region B
#pragma unroll
      for (int k = 0; k < KT; ++k) {
        if (k < kx0) xr[k] = tileB[k * tstride + om];
        if (k < kx1) xi[k] = tileB[(kx0 + k) * tstride + om];
      }
    };
    auto fetch = [&](int b) {                                 // column output of transform b into yr, yi
      const int t = tlist[b];
      load_xregs<NP>(yr, yi, X + td[t].X_off, K, g.logN, prime, ts[t].kx[0], ts[t].kx[1], pos);
    };
    // prologue: forward rows of the first live transform; the second one's
    // column output is fetched while they run
    {
      const int t = tlist[bn];
      const int kx0 = ts[t].kx[0], kx1 = ts[t].kx[1];
      fetch(bn);
      put_b(kx0, kx1, off_me);
      __syncthreads();                                        // tw and B complete
      const int b2 = next_live(bn);
      if (b2 < b_hi) fetch(b2);
      run_tiles(0, kx0 + kx1, p);
      __syncthreads();
      get_b(kx0, kx1, off_me);
    }
    while (bn < b_hi) {
      const int om = off_me;
      const int t = tlist[bn];
      const TDesc& d = td[t];
      const TState& s = ts[t];
      const KernelDesc& kk = kd[d.kd];
      if (d.kd != wkd) {
        load_wregs<NP>(wr, kk.W, kk.Wq, K, g.logN, prime, kk.kw[0], kk.kw[1], pos);
        wkd = d.kd;
      }
      const int b2 = next_live(bn);                           // its column output is in yr, yi
      const int b3 = b2 < b_hi ? next_live(b2) : b_hi;
      const int nkx0 = b2 < b_hi ? ts[tlist[b2]].kx[0] : 0, nkx1 = b2 < b_hi ? ts[tlist[b2]].kx[1] : 0;
      const int ng0 = s.ngroups[0], gtot = ng0 + s.ngroups[1];
      const int kx0 = s.kx[0], kx1 = s.kx[1];
      const bool merged = d.acc_mode == ACC_COMPLEX;
      const int cfull = (kx0 == kx1 && kx0 == kk.kw[0] && kx0 == kk.kw[1]) ? kx0 : 0;
      const int gofs[2] = {0, ng0};
      for (int g0 = 0;; g0 += gA) {
        const int g1 = min(gtot, g0 + gA);
        const bool last = g1 >= gtot;
        const int nB = last ? nkx0 + nkx1 : 0;
        if (nB) put_b(nkx0, nkx1, om);
        if (g1 > g0) {
          if (gtot <= gA && cfull == KT) mac_full<KT>(xr, xi, wr, s, merged, tileA + om, tstride, p);
          else if (gtot <= gA && cfull == 2) mac_full<2>(xr, xi, wr, s, merged, tileA + om, tstride, p);
          else mac_regs(xr, xi, wr, s, merged, kk.kw[0], kk.kw[1], gofs, g0, g1, tileA + om, tstride, p);
        }
        __syncthreads();                                      // A and B written
        if (last && b3 < b_hi) fetch(b3);                     // in flight during the rounds
        run_tiles(g1 - g0, nB, p);
        __syncthreads();                                      // rounds done
        for (int gi = g0; gi < g1; ++gi) {                    // this position of every group row
          const int slot = gi < ng0 ? gi : SL + gi - ng0;
          const u32 v = shoup_mul(tileA[(gi - g0) * tstride + om], iwt.x, iwt.y, p);
          G[d.G_off + ((size_t)(slot * NP + prime) << g.logN) + pos] = v;
        }
        if (nB) get_b(nkx0, nkx1, om);
        if (last) break;
      }
      bn = b2;
    }
  }
}

// General form (any slice counts and tile shape): operands read per
// position pair from memory, one transform after the other.
template <int M2>
__global__ void __launch_bounds__(NTT_THREADS) k_inv_rows(const u32* X, u32* G, const TDesc* td, const TState* ts,
                                                          const KernelDesc* kd, const int* tlist, int count, int K,
                                                          int np, int slot_lo, int slot_hi, NttGeom g, TwBlock tb,
                                                          TwStep st, int tpw) {
  extern __shared__ u32 smem[];
  const int nruns = (count + tpw - 1) / tpw;
  int pair, run;
  decode_tile(blockIdx.x, np << (g.m1 - g.lrows_inv), nruns, pair, run);
  const int b_lo = run * tpw, b_hi = min(count, b_lo + tpw);
  const int rtile = pair / np, prime = pair - rtile * np;
  const u32 p = prime_of(prime);
  constexpr int m2 = M2, N2 = 1 << m2, ldr = row_ld(N2);
  const int nr = 1 << g.lrows_inv, SL = 2 * K * K;           // slots per output component
  const int gch = max(1, inv_vmax(m2) >> g.lrows_inv);          // groups per chunk
  const u32 Nmask = (1u << g.logN) - 1;
  uint2* tw = reinterpret_cast<uint2*>(smem);
  u32* rtw = smem + N2;                                       // w_N^{-j2 k1} per tile element, then companions
  u32* tile = smem + N2 + 2 * (nr << m2);
  load_block_tw(tw, tb.inv[prime], m2);
  const int i1_0 = rtile << g.lrows_inv;
  for (int e = threadIdx.x; e < (nr << m2); e += blockDim.x) {
    const uint2 r = step_root(((u32)(e & (N2 - 1)) * bitrev(i1_0 + (e >> m2), g.m1)) & Nmask, st.lo[1][prime],
                              st.hi[1][prime], p);
    rtw[e] = r.x;
    rtw[(nr << m2) + e] = r.y;
  }
  const size_t base = (size_t)i1_0 << m2;
  const int quads = (nr << m2) >> 2;
  for (int b = b_lo; b < b_hi; ++b) {
    const int t = tlist[b];
    const TDesc& d = td[t];
    const TState& s = ts[t];
    if (s.status) continue;
    const KernelDesc& kk = kd[d.kd];
    const int gofs[2] = {0, s.ngroups[0]};
    const int gtot = s.ngroups[0] + s.ngroups[1];
    const MacArgs ma{X + d.X_off, kk.W, kk.Wq, K, g.logN, prime, p, kk.kw[0], kk.kw[1], np};
    for (int g0 = 0; g0 < gtot; g0 += gch) {
      const int g1 = min(gtot, g0 + gch);
      // tile vector (number - g0) * nr + r holds row r of that group
      for (int q = threadIdx.x; q < 2 * quads; q += blockDim.x) {
        const int e = q << 1, r = e >> m2, i = e & (N2 - 1);
        mac_pair(ma, s, d.acc_mode == ACC_COMPLEX, 0, 1, gofs, g0, g1, base + e, tile + r * ldr + pad8(i), nr * ldr);
      }
      __syncthreads();
      block_ntt<M2, true, false>(tile, (g1 - g0) * nr, ldr, tw, p);
      store_group_rows(G, d, tile, rtw, gofs, g0, g1, SL, slot_lo, slot_hi, np, prime, g.logN, base, m2, nr, ldr, p);
      __syncthreads();
    }
  }
}

// Two-pass inverse, second pass (columns).  The group vectors of a transform
// are numbered j = np gi + prime over the Alg. 8 groups gi of all four
// convolutions; workgroup (x, y, z) takes column tile x of vectors
// [y vpw, (y + 1) vpw) of transform z.  The tile of the next vector is
// loaded into registers while the current one is transformed, and the first
// n natural-order outputs go to the compact buffer.
constexpr int COL_PF = 8;        // 16-byte registers per thread staging the next tile (tile <= 16K words)

struct ColVecs {                 // group vectors of one transform (numbering j = np gi + prime)
  int ng0, SL, slot_lo, slot_hi, j_hi;   // ng0: groups of Re y'; SL: slots per output component
  int np;
  __device__ __forceinline__ int slot_of(int j) const {
    const int gi = j / np;
    return gi < ng0 ? gi : SL + gi - ng0;
  }
  // first vector >= j whose slot lies in [slot_lo, slot_hi), or j_hi
  __device__ __forceinline__ int next(int j) const {
    for (; j < j_hi; ++j) {
      const int sl = slot_of(j);
      if (sl >= slot_lo && sl < slot_hi) break;
    }
    return j;
  }
};

// The staged tile, in native 4-lane vectors (copies of the HIP uint4 struct
// go through memcpy, which kept the stage in scratch memory).
typedef u32 u32x4 __attribute__((ext_vector_type(4)));
struct ColStage {
  u32x4 v0, v1, v2, v3, v4, v5, v6, v7;
  template <int U>
  __device__ __forceinline__ u32x4& at() {
    static_assert(U >= 0 && U < COL_PF, "stage index");
    if constexpr (U == 0) return v0;
    else if constexpr (U == 1) return v1;
    else if constexpr (U == 2) return v2;
    else if constexpr (U == 3) return v3;
    else if constexpr (U == 4) return v4;
    else if constexpr (U == 5) return v5;
    else if constexpr (U == 6) return v6;
    else return v7;
  }
};
// part u of the tile: uint4 number q = threadIdx.x + u blockDim.x, row i, columns c4..c4+3
template <int U = 0>
__device__ __forceinline__ void fetch_col_tile(ColStage& b, const u32* __restrict__ gv, int tot4, int lq, int m2,
                                               int j2_0) {
  if constexpr (U < COL_PF) {
    const int q = threadIdx.x + U * blockDim.x;
    if (q < tot4) {
      const int i = q >> lq, c4 = (q & ((1 << lq) - 1)) << 2;
      b.at<U>() = *reinterpret_cast<const u32x4*>(gv + (i << m2) + j2_0 + c4);
    }
    fetch_col_tile<U + 1>(b, gv, tot4, lq, m2, j2_0);
  }
}
template <int U = 0>
__device__ __forceinline__ void put_col_tile(ColStage& b, u32* tile, int tot4, int lq, int lc) {
  if constexpr (U < COL_PF) {
    const int q = threadIdx.x + U * blockDim.x;
    if (q < tot4) {
      const int i = q >> lq, c4 = (q & ((1 << lq) - 1)) << 2;
      *reinterpret_cast<u32x4*>(tile + (i << lc) + c4) = b.at<U>();
    }
    put_col_tile<U + 1>(b, tile, tot4, lq, lc);
  }
}

template <int M1>
__global__ void __launch_bounds__(COL_THREADS) k_inv_cols(const u32* G, u32* Z, const TDesc* td, const TState* ts,
                                                          const int* tlist, int K, int np, int slot_lo, int slot_hi,
                                                          NttGeom g, TwBlock tb, int vpw) {
  extern __shared__ u32 smem[];
  const int t = tlist[blockIdx.z];
  const TDesc& d = td[t];
  const TState& s = ts[t];
  if (s.status) return;
  ColVecs cv;
  cv.ng0 = s.ngroups[0];
  cv.SL = 2 * K * K;
  cv.slot_lo = slot_lo;
  cv.slot_hi = slot_hi;
  cv.np = np;
  const int gtot = cv.ng0 + s.ngroups[1];
  const int j_lo = blockIdx.y * vpw;
  cv.j_hi = min(np * gtot, j_lo + vpw);
  if (j_lo >= cv.j_hi) return;
  constexpr int m1 = M1;
  const int m2 = g.m2, lc = g.lc_inv, lq = lc - 2, n = d.n;
  uint2* tw0 = reinterpret_cast<uint2*>(smem);             // roots of every prime, 2^(m1-1) entries each
  u32* tile = smem + (np << m1);
  for (int q = 0; q < np; ++q) load_block_tw(tw0 + (q << (m1 - 1)), tb.inv[q], m1);
  const int j2_0 = col_tile(blockIdx.x, m2 - lc) << lc;
  const int tot4 = 1 << (m1 + lq);
  const u32* gbase = G + d.G_off;
  ColStage buf;
  int j = cv.next(j_lo);
  auto vec_of = [&](int jj) { return gbase + ((size_t)(cv.slot_of(jj) * np + jj % np) << g.logN); };
  if (j < cv.j_hi) fetch_col_tile(buf, vec_of(j), tot4, lq, m2, j2_0);
  __syncthreads();                    // root tables
  while (j < cv.j_hi) {
    const int prime = j % np, slot = cv.slot_of(j);
    put_col_tile(buf, tile, tot4, lq, lc);
    __syncthreads();
    const int jn = cv.next(j + 1);
    if (jn < cv.j_hi) fetch_col_tile(buf, vec_of(jn), tot4, lq, m2, j2_0);
    block_ntt<M1, true, true>(tile, lc, 0, tw0 + (prime << (m1 - 1)), prime_of(prime));
    u32* zo = Z + d.Z_off + (size_t)(slot * np + prime) * d.zs;   // rows padded to a multiple of 4
    for (int q = threadIdx.x; q < tot4; q += blockDim.x) {
      const int j1 = q >> lq, c4 = (q & ((1 << lq) - 1)) << 2;
      const int gi = (j1 << m2) + j2_0 + c4;
      if (gi < n) *reinterpret_cast<uint4*>(zo + gi) = *reinterpret_cast<const uint4*>(tile + (j1 << lc) + c4);
    }
    __syncthreads();
    j = jn;
  }
}

// ---------------------------------------------------------------------------
// Fused inverse column pass, Garner CRT, exact recombination and chirp
// postmultiply (two-pass lengths with N1 <= 512, i.e. N <= 2^18; the tile
// rows of longer lengths would be 16 bytes).  One workgroup of
// REC_THREADS per (column tile of 2^(12 - M1) columns, transform): for every
// group the column vectors of all NP primes are transformed together,
// combined by Garner's formula and added, shifted by the group's exponent,
// to exact per-output accumulators held in registers (REC_OUT outputs per
// thread); the Re y' groups come first, then the Im y' groups, so one set of
// accumulators serves both components.  The group residues never go to
// memory.  Transforms whose exponent span needs the wide accumulator only
// get their column pass here, written to the compact buffer for the wide
// recombination.

constexpr int REC_THREADS = 1024, REC_OUT = 4;   // 4096-position tiles
// LDS of the fused column pass: the inverse roots of every prime and two
// buffers of one tile per prime.
__host__ __device__ constexpr size_t rec_smem_words(int m1, int np) {
  return ((size_t)np << m1) + 2 * (size_t)np * ((size_t)rec_ldc(m1) << (12 - m1));
}
template <int M1, int NP>
__global__ void __launch_bounds__(REC_THREADS) k_inv_cols_rec(const u32* G, u32* Z, const IoPtrs* io, const TDesc* td,
                                                              const TState* ts, const KernelDesc* kd,
                                                              const int* tlist, int K, int m2, TwBlock tb, int dir,
                                                              int io32) {
  constexpr int LC = 12 - M1, LQ = LC - 2, TILE = 1 << 12;
  static_assert(LC >= 2 && TILE == REC_THREADS * REC_OUT, "tile shape");
  extern __shared__ u32 smem[];
  const int t = tlist[blockIdx.z];
  const TDesc& d = td[t];
  const TState& s = ts[t];
  void* out = io->out;
  // a transform whose exponent span needs the wide accumulator only gets
  // its column pass here: the residues go to the compact buffer Z for the
  // wide recombination
  const bool wide = !s.status && (span_wide<NP>(s, 0) || span_wide<NP>(s, 1));
  const int n = d.n, N2 = 1 << m2;
  const int j2_0 = col_tile(blockIdx.x, m2 - LC) << LC;
  const double2* ch = kd[d.kd].chirp;
  if (s.status) {
#pragma unroll
    for (int k = 0; k < REC_OUT; ++k) {
      const int o = threadIdx.x + k * REC_THREADS;
      const int j = (o >> LC) * N2 + j2_0 + (o & ((1 << LC) - 1));
      if (j < n) put_out(out, d.io_off + j, make_double2(__builtin_nan(""), __builtin_nan("")), io32);
    }
    return;
  }
  uint2* tw = reinterpret_cast<uint2*>(smem);                // inverse roots, 2^(M1-1) per prime
  // the tile of each prime holds its 2^LC columns as pad9 rows (column c at
  // c LDC); two buffers of all primes' tiles: group v uses buffer v & 1, so
  // the next group's values are written while other waves still read this
  // one's.  Each wave owns CPW columns of one prime (CPW divides 2^LC) and
  // runs their inverse NTTs on its own (wave-local rounds); with three
  // primes the waves take a second turn for the columns beyond 32 CPW.
  // this thread's quad of the tile: row i, columns c4 .. c4 + 3
  const int qi = threadIdx.x >> LQ, qc = (threadIdx.x & ((1 << LQ) - 1)) << 2;
  constexpr int LDC = rec_ldc(M1), TT = LDC << LC;            // words per prime tile
  u32* tiles = smem + (NP << M1);
#pragma unroll
  for (int q = 0; q < NP; ++q) load_block_tw(tw + (q << (M1 - 1)), tb.inv[q], M1);
  constexpr int NWV = REC_THREADS / 64, CPW = (2 << LC) / NWV, NCOL = NP << LC;   // columns per wave, in all
  static_assert(CPW >= 1 && CPW * NWV == (2 << LC), "column split");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  auto put_tile = [&](u32* tile, const u32x4& q) {           // quad of row qi, columns qc .. qc + 3
    u32* b = tile + qc * LDC + pad9(qi);
    b[0] = q[0];
    b[LDC] = q[1];
    b[2 * LDC] = q[2];
    b[3 * LDC] = q[3];
  };
  auto at = [&](const u32* tile, int o) { return tile[(o & ((1 << LC) - 1)) * LDC + pad9(o >> LC)]; };
  auto columns_at = [&](u32* buf, int wcol) {
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const int wprime = wcol >> LC, wc0 = wcol & ((1 << LC) - 1);
    rounds_t<M1, 0, true, false, 9, true>(buf + wprime * TT + wc0 * LDC, CPW, LDC, tw + (wprime << (M1 - 1)),
                                          prime_of(wprime), ln, 64);
  };
  auto columns = [&](u32* buf) {
    if constexpr (NCOL == NWV * CPW) {
      columns_at(buf, wave * CPW);
    } else {
      for (int wcol = wave * CPW; wcol < NCOL; wcol += NWV * CPW) columns_at(buf, wcol);
    }
  };
  const int ng0 = s.ngroups[0], SL = 2 * K * K;
  const int V = ng0 + s.ngroups[1];                           // groups; Re y' groups are [0, ng0)
  auto slot_of = [&](int v) { return v < ng0 ? v : SL + v - ng0; };
  const u32* gb = G + d.G_off;
  const size_t goff = ((size_t)qi << m2) + j2_0 + qc;
  u32x4 st[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) st[q] = u32x4{0, 0, 0, 0};
  auto fetch = [&](int v) {
    const u32* vec = gb + ((size_t)(slot_of(v) * NP) << d.logN) + goff;
#pragma unroll
    for (int q = 0; q < NP; ++q) st[q] = *reinterpret_cast<const u32x4*>(vec + ((size_t)q << d.logN));
  };
  auto put_all = [&](u32* buf) {
#pragma unroll
    for (int q = 0; q < NP; ++q) put_tile(buf + q * TT, st[q]);
  };
  if (wide) {
    if (V > 0) fetch(0);
    for (int v = 0; v < V; ++v) {
      u32* buf = tiles + (v & 1) * NP * TT;
      put_all(buf);
      __syncthreads();                                        // tiles (and the root tables) complete
      if (v + 1 < V) fetch(v + 1);
      columns(buf);
      __syncthreads();                                        // columns done
      u32* z0 = Z + d.Z_off + (size_t)(slot_of(v) * NP) * d.zs;
#pragma unroll
      for (int k = 0; k < REC_OUT; ++k) {
        const int o = threadIdx.x + k * REC_THREADS;
        const int j = (o >> LC) * N2 + j2_0 + (o & ((1 << LC) - 1));
        if (j < n) {
#pragma unroll
          for (int q = 0; q < NP; ++q) z0[q * d.zs + j] = at(buf + q * TT, o);
        }
      }
    }
    return;
  }
  u32 acc[REC_OUT][NL_FAST];
  double pr[REC_OUT];
#pragma unroll
  for (int k = 0; k < REC_OUT; ++k) {
    pr[k] = 0.0;
#pragma unroll
    for (int l = 0; l < NL_FAST; ++l) acc[k][l] = 0;
  }
  if (V > 0) fetch(0);
  for (int v = 0; v < V; ++v) {
    u32* buf = tiles + (v & 1) * NP * TT;
    if (v == ng0 && v > 0) {                                  // Re y' complete
#pragma unroll
      for (int k = 0; k < REC_OUT; ++k) {
        u64 a64[W_FAST];
#pragma unroll
        for (int w = 0; w < W_FAST; ++w) a64[w] = (u64)acc[k][2 * w] | ((u64)acc[k][2 * w + 1] << 32);
        pr[k] = acc_round<W_FAST>(a64, s.emin[0]);
#pragma unroll
        for (int l = 0; l < NL_FAST; ++l) acc[k][l] = 0;
      }
    }
    put_all(buf);
    __syncthreads();                                          // tiles (and the root tables) complete
    if (v + 1 < V) fetch(v + 1);
    columns(buf);
    __syncthreads();                                          // columns done
    const int tg = v >= ng0 ? 1 : 0;                          // the signs are applied in the NTT domain
    const int sh = s.groups[tg][v - (tg ? ng0 : 0)].e - s.emin[tg];
#pragma unroll
    for (int k = 0; k < REC_OUT; ++k) {
      const int o = threadIdx.x + k * REC_THREADS;
      u32 z[NP];
#pragma unroll
      for (int q = 0; q < NP; ++q) z[q] = at(buf + q * TT, o);
      limb_add_crt<NP>(acc[k], z, sh);
    }
  }
  double pi[REC_OUT];
  const bool has_im = V > ng0;
#pragma unroll
  for (int k = 0; k < REC_OUT; ++k) {
    u64 a64[W_FAST];
#pragma unroll
    for (int w = 0; w < W_FAST; ++w) a64[w] = (u64)acc[k][2 * w] | ((u64)acc[k][2 * w + 1] << 32);
    const double r = acc_round<W_FAST>(a64, has_im ? s.emin[1] : s.emin[0]);
    pi[k] = has_im ? r : 0.0;
    if (!has_im) pr[k] = r;
  }
#pragma unroll
  for (int k = 0; k < REC_OUT; ++k) {
    const int o = threadIdx.x + k * REC_THREADS;
    const int j = (o >> LC) * N2 + j2_0 + (o & ((1 << LC) - 1));
    if (j < n) put_out(out, d.io_off + j, finish(pr[k], pi[k], ch[j], dir, n), io32);
  }
}

// Kernel slices: W <- W * N^{-1}, Wq <- Shoup companion.  Layout [part][t][prime][N].
__global__ void k_kernel_finish(u32* W, u32* Wq, size_t total, int logN, int np) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int prime = (int)((i >> logN) % np);
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
    g.lc_inv = 0;
    g.lrows = 0;
    return g;
  }
  g.m2 = logN / 2;
  g.m1 = logN - g.m2;
  // column tile: C * N1 words <= 16K words (64 KiB), 4 <= C <= 16 columns
  // (16 columns measured faster than 32 for N1 = 512: more workgroups); from
  // N1 = 1024 on the forward pass takes 8 columns (16 padded columns of 1024
  // allow two workgroups per CU; 8 columns measured faster there), the
  // unfused inverse pass keeps 16 (8 measured slower)
  int lc = 4;
  while (lc > 2 && (g.m1 + lc) > 14) --lc;
  if (lc > g.m2) lc = g.m2;
  g.lc_inv = lc;
  if (g.m1 >= 10 && lc > 3) lc = 3;
  // row tile: 4096 words per workgroup
  int lr = LOG2_BLOCK_MAX - g.m2;
  if (lr < 0) lr = 0;
  if (lr > g.m1) lr = g.m1;
  g.lc = lc_override >= 0 ? lc_override : lc;
  g.lrows = lrows_override >= 0 ? lrows_override : lr;
  // inverse rows: about 512 words per group row so that the groups of all
  // four convolutions fit the LDS tile together
  int li = 9 - g.m2;
  if (li < 0) li = 0;
  if (li > g.m1) li = g.m1;
  g.lrows_inv = li;
  return g;
}

static size_t smem_cols(const NttGeom& g) { return ((size_t)(1 << g.m1) + ((size_t)1 << (g.m1 + g.lc))) * 4; }
// The forward column pass: column layout, or the wave-local padded-row tile
// when there are at least as many columns as waves.
static size_t smem_fwd_cols(const NttGeom& g) {
  if (g.lc >= 3 && (1 << g.lc) >= COL_THREADS / 64)
    return ((size_t)(1 << g.m1) + ((size_t)rec_ldc(g.m1) << g.lc)) * 4;
  return smem_cols(g);
}
static size_t smem_inv_cols(const NttGeom& g, int np) {
  return ((size_t)(np << g.m1) + ((size_t)1 << (g.m1 + g.lc_inv))) * 4;
}
static size_t smem_rows(const NttGeom& g) {
  return ((size_t)(1 << g.m2) + ((size_t)row_ld(1 << g.m2) << g.lrows) + rowtw_words(g.m2, 1 << g.lrows)) * 4;
}
static size_t smem_single(int logN) { return ((size_t)(1 << logN) + row_ld(1 << logN)) * 4; }
static size_t smem_inv_rows(const NttGeom& g) {
  const int gch = std::max(1, inv_vmax(g.m2) >> g.lrows_inv);
  return ((size_t)(1 << g.m2) + 4 + ((size_t)2 << (g.m2 + g.lrows_inv)) + ((size_t)2 << g.lrows_inv) +
          (size_t)row_ld(1 << g.m2) * (size_t)(gch << g.lrows_inv)) * 4;
}
// LDS of k_inv_rows_pipe: inverse and forward block roots, then gch group
// tiles of nr pad9 rows.
static size_t smem_inv_pipe(const NttGeom& g) {
  const int gch = PIPE_TILES;
  return ((size_t)(2 << g.m2) + 4 + (size_t)gch * ((size_t)pad9(1 << g.m2) << g.lrows_inv)) * 4;
}
// Workgroups of `fn` that the device runs at once (occupancy x CUs), cached
// per device, kernel and LDS size.
static int resident_workgroups(const void* fn, int threads, size_t smem) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, size_t>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_tuple(dev, fn, smem);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int nb = 0, ncu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, smem) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const int slots = std::max(1, nb) * std::max(1, ncu);
  cache[key] = slots;
  return slots;
}
static size_t smem_inv_single(int logN) {
  return ((size_t)(1 << logN) + (size_t)row_ld(1 << logN) * (size_t)inv_vmax(logN)) * 4;
}

// Kernels are instantiated per block length: calls f(integral_constant<M>)
// for m in [LO, HI]; false when m is out of range.
template <int LO, int HI, typename F>
static bool with_m(int m, F&& f) {
  if constexpr (LO > HI) {
    return false;
  } else {
    if (m == LO) {
      f(std::integral_constant<int, LO>{});
      return true;
    }
    return with_m<LO + 1, HI>(m, std::forward<F>(f));
  }
}
// Column lengths 2^m1 and row lengths 2^m2 of the two-pass geometry
// (N = 2^13 .. 2^24) and single-workgroup lengths (N <= 2^12).
constexpr int M1_LO = 7, M1_HI = 12, M2_LO = 6, M2_HI = 12;

// Opts a kernel into the full 160 KiB of LDS once per process.
static hipError_t big_lds(const void* fn) {
  static std::mutex mu;
  static std::unordered_set<const void*> done;
  std::lock_guard<std::mutex> lk(mu);
  if (done.count(fn)) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e == hipSuccess) done.insert(fn);
  return e;
}

hipError_t launch_ntt_standalone(u32* data, int logN, int prime, int count, bool inverse, const NttGeom& g,
                                 const TwBlock& tb, const TwStep& ts, hipStream_t s, int which) {
  if (count <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
  if (!g.two_pass()) {
    if (!with_m<0, LOG2_BLOCK_MAX>(logN, [&](auto mc) {
          constexpr int M = decltype(mc)::value;
          if ((e = big_lds((const void*)k_std_single<M>)) != hipSuccess) return;
          hipLaunchKernelGGL(k_std_single<M>, dim3(1, 1, count), dim3(NTT_THREADS), smem_single(logN), s, data, prime,
                             inverse, tb);
        }))
      return hipErrorInvalidValue;
    return e != hipSuccess ? e : hipGetLastError();
  }
  const dim3 gc(1u << (g.m2 - g.lc), 1, count), gr(1u << (g.m1 - g.lrows), 1, count);
  auto cols = [&](auto mc) {
    constexpr int M1 = decltype(mc)::value;
    if (!inverse) {
      if ((e = big_lds((const void*)k_std_fwd_cols<M1>)) != hipSuccess) return;
      hipLaunchKernelGGL(k_std_fwd_cols<M1>, gc, dim3(COL_THREADS), smem_fwd_cols(g), s, data, prime, g, tb, ts);
    } else {
      if ((e = big_lds((const void*)k_std_inv_cols<M1>)) != hipSuccess) return;
      hipLaunchKernelGGL(k_std_inv_cols<M1>, gc, dim3(COL_THREADS), smem_cols(g), s, data, prime, g, tb);
    }
  };
  auto rows = [&](auto mc) {
    constexpr int M2 = decltype(mc)::value;
    if (!inverse) {
      if ((e = big_lds((const void*)k_std_fwd_rows<M2>)) != hipSuccess) return;
      hipLaunchKernelGGL(k_std_fwd_rows<M2>, gr, dim3(NTT_THREADS), smem_rows(g), s, data, prime, g, tb, ts);
    } else {
      if ((e = big_lds((const void*)k_std_inv_rows<M2>)) != hipSuccess) return;
      hipLaunchKernelGGL(k_std_inv_rows<M2>, gr, dim3(NTT_THREADS), smem_rows(g), s, data, prime, g, tb, ts);
    }
  };
  const bool do_cols = which != 2, do_rows = which != 1;
  if (!inverse) {
    if (do_cols && !with_m<M1_LO, M1_HI>(g.m1, cols)) return hipErrorInvalidValue;
    if (e != hipSuccess) return e;
    if (do_rows && !with_m<M2_LO, M2_HI>(g.m2, rows)) return hipErrorInvalidValue;
  } else {
    if (do_rows && !with_m<M2_LO, M2_HI>(g.m2, rows)) return hipErrorInvalidValue;
    if (e != hipSuccess) return e;
    if (do_cols && !with_m<M1_LO, M1_HI>(g.m1, cols)) return hipErrorInvalidValue;
  }
  return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_fwd_stage(u32* X, const TDesc* td, const TState* ts, const int* tlist, int count, int K, int np,
                            bool valid_full, int vi_lo, int vi_hi, const NttGeom& g, const TwBlock& tb,
                            const TwStep& st, int which, hipStream_t s, TState* walk_ts, const KernelDesc* kd, int L) {
  const int nv = vi_hi - vi_lo;
  if (count <= 0 || nv <= 0) return hipSuccess;
  if (np != 2 && np != 3) return hipErrorInvalidValue;
  WalkArgs walk;
  if (walk_ts && which != 2) {
    walk.ts = walk_ts;
    walk.kd = kd;
    walk.L = L;
  }
  const int ny = nv + (walk.ts ? 1 : 0);
  hipError_t e = hipSuccess;
  if (!g.two_pass()) {
    if (which == 2) return hipSuccess;
    if (!with_m<0, LOG2_BLOCK_MAX>(g.logN, [&](auto mc) {
          constexpr int M = decltype(mc)::value;
          if ((e = big_lds((const void*)k_fwd_single<M>)) != hipSuccess) return;
          // the walk slice stages 4 KMAX exponents in LDS
          const size_t lds = std::max(smem_single(g.logN), sizeof(int) * 4 * KMAX);
          hipLaunchKernelGGL(k_fwd_single<M>, dim3(1, ny, count), dim3(NTT_THREADS), lds, s, X, td, ts, tlist, K, np,
                             valid_full, vi_lo, tb, walk);
        }))
      return hipErrorInvalidValue;
    return e != hipSuccess ? e : hipGetLastError();
  }
  if (which != 2 && !with_m<M1_LO, M1_HI>(g.m1, [&](auto mc) {
        constexpr int M1 = decltype(mc)::value;
        if ((e = big_lds((const void*)k_fwd_cols<M1>)) != hipSuccess) return;
        const size_t lds = std::max(smem_fwd_cols(g), sizeof(int) * 4 * KMAX);
        hipLaunchKernelGGL(k_fwd_cols<M1>, dim3(1u << (g.m2 - g.lc), ny, count), dim3(COL_THREADS), lds, s, X, td, ts,
                           tlist, K, np, valid_full, vi_lo, g, tb, st, walk);
      }))
    return hipErrorInvalidValue;
  if (e != hipSuccess) return e;
  if (which != 1 && !with_m<M2_LO, M2_HI>(g.m2, [&](auto mc) {
        constexpr int M2 = decltype(mc)::value;
        if ((e = big_lds((const void*)k_fwd_rows<M2>)) != hipSuccess) return;
        hipLaunchKernelGGL(k_fwd_rows<M2>, dim3(1u << (g.m1 - g.lrows), nv, count), dim3(NTT_THREADS), smem_rows(g), s,
                           X, td, ts, tlist, K, np, valid_full, vi_lo, g, tb, st);
      }))
    return hipErrorInvalidValue;
  return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_fwd_pipeline(u32* X, const TDesc* td, const TState* ts, const int* tlist, int count, int K, int np,
                               bool valid_full, int vi_lo, int vi_hi, const NttGeom& g, const TwBlock& tb,
                               const TwStep& st, hipStream_t s) {
  return launch_fwd_stage(X, td, ts, tlist, count, K, np, valid_full, vi_lo, vi_hi, g, tb, st, 0, s);
}

bool fused_rows_ok(const NttGeom& g, int K) {
  // register form (K <= KT, 512-position row tiles), and the 2K forward
  // slice tiles leave room for inverse group tiles in the pipelined pass
  return g.two_pass() && K <= KT && (1 << (g.m2 + g.lrows_inv)) == INV_ROW_THREADS && 2 * K < PIPE_TILES;
}

hipError_t launch_inv_stage(const u32* X, u32* G, u32* Z, const TDesc* td, const TState* ts, const KernelDesc* kd,
                            const int* tlist, int count, int K, int np, int slot_lo, int slot_hi, const NttGeom& g,
                            const TwBlock& tb, const TwStep& st, int which, hipStream_t s,
                            bool fused_fwd) {
  if (fused_fwd && !fused_rows_ok(g, K)) return hipErrorInvalidValue;   // also keeps the forward rows inside the tile
  if (np != 2 && np != 3) return hipErrorInvalidValue;
  if (count <= 0 || slot_hi <= slot_lo) return hipSuccess;
  hipError_t e = hipSuccess;
  if (!g.two_pass()) {
    if (which == 2) return hipSuccess;
    if (!with_m<0, LOG2_BLOCK_MAX>(g.logN, [&](auto mc) {
          constexpr int M = decltype(mc)::value;
          if ((e = big_lds((const void*)k_inv_single<M>)) != hipSuccess) return;
          hipLaunchKernelGGL(k_inv_single<M>, dim3(2 * np * count), dim3(NTT_THREADS), smem_inv_single(g.logN), s, X,
                             Z, td, ts, kd, tlist, count, K, np, slot_lo, slot_hi, tb);
        }))
      return hipErrorInvalidValue;
    return e != hipSuccess ? e : hipGetLastError();
  }
  if (which != 2) {
    // runs of up to four transforms per workgroup while the grid keeps
    // at least about four workgroups per CU slot (3 per CU on 256 CUs)
    const long pairs = (long)np << (g.m1 - g.lrows_inv);
    int tpw = 1;
    while (tpw < 4 && 2 * tpw <= count && pairs * ((count + 2 * tpw - 1) / (2 * tpw)) >= 3072) tpw *= 2;
    const long runs = (count + tpw - 1) / tpw;
    // register form: slices fit the registers and the row tile has one
    // position per thread (without the folded forward rows: the plain
    // form's per-group launches, two moduli)
    const bool reg = K <= KT && (1 << (g.m2 + g.lrows_inv)) == INV_ROW_THREADS;
    if (!with_m<M2_LO, M2_HI>(g.m2, [&](auto mc) {
          constexpr int M2 = decltype(mc)::value;
          if constexpr ((1 << M2) <= INV_ROW_THREADS) {   // the register form exists only for these lengths
            if (reg && fused_fwd) {
              // persistent pipelined form (all groups): one workgroup per resident slot
              if (slot_lo != 0 || slot_hi < 4 * K * K) {
                e = hipErrorInvalidValue;
                return;
              }
              auto* kfn = np == 3 ? &k_inv_rows_pipe<M2, 3> : &k_inv_rows_pipe<M2, 2>;
              if ((e = big_lds((const void*)kfn)) != hipSuccess) return;
              const size_t sm = smem_inv_pipe(g);
              const long units = pairs * count;
              const int slots = resident_workgroups((const void*)kfn, INV_ROW_THREADS, sm);
              if (slots <= 0) {
                e = hipErrorInvalidValue;
                return;
              }
              hipLaunchKernelGGL(kfn, dim3((unsigned)std::min<long>(units, slots)), dim3(INV_ROW_THREADS), sm, s, X, G,
                                 td, ts, kd, tlist, count, K, g, tb, st);
              return;
            }
            if (reg && np == 2) {
              auto* kfn = &k_inv_rows_reg<M2>;
              if ((e = big_lds((const void*)kfn)) != hipSuccess) return;
              hipLaunchKernelGGL(kfn, dim3((unsigned)(pairs * runs)), dim3(INV_ROW_THREADS), smem_inv_rows(g), s, X,
                                 G, td, ts, kd, tlist, count, K, slot_lo, slot_hi, g, tb, st, tpw);
              return;
            }
          }
          {
            if ((e = big_lds((const void*)k_inv_rows<M2>)) != hipSuccess) return;
            hipLaunchKernelGGL(k_inv_rows<M2>, dim3((unsigned)(pairs * runs)), dim3(NTT_THREADS), smem_inv_rows(g), s,
                               X, G, td, ts, kd, tlist, count, K, np, slot_lo, slot_hi, g, tb, st, tpw);
          }
        }))
      return hipErrorInvalidValue;
    if (e != hipSuccess) return e;
  }
  if (which != 1) {
    // the staged next tile must fit COL_PF 16-byte registers per thread
    if (g.m1 + g.lc_inv > 14) return hipErrorInvalidValue;
    const int vecs = 4 * K * K * np, vpw = 4;    // group vectors (at most 4 K^2 groups, np primes)
    const dim3 grid(1u << (g.m2 - g.lc_inv), (vecs + vpw - 1) / vpw, count);
    if (!with_m<M1_LO, M1_HI>(g.m1, [&](auto mc) {
          constexpr int M1 = decltype(mc)::value;
          if ((e = big_lds((const void*)k_inv_cols<M1>)) != hipSuccess) return;
          hipLaunchKernelGGL(k_inv_cols<M1>, grid, dim3(COL_THREADS), smem_inv_cols(g, np), s, G, Z, td, ts, tlist, K,
                             np, slot_lo, slot_hi, g, tb, vpw);
        }))
      return hipErrorInvalidValue;
  }
  return e != hipSuccess ? e : hipGetLastError();
}

bool fused_cols_ok(const NttGeom& g) {
  return g.two_pass() && g.m1 >= 7 && g.m1 <= 9 && 12 - g.m1 <= g.m2;
}

hipError_t launch_inv_cols_rec(const u32* G, u32* Z, const IoPtrs* io, const TDesc* td, const TState* ts,
                               const KernelDesc* kd, const int* tlist, int count, int K, int np, const NttGeom& g,
                               const TwBlock& tb, int dir, int io32, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (!fused_cols_ok(g) || (np != 2 && np != 3)) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  with_m<7, 9>(g.m1, [&](auto mc) {
    constexpr int M1 = decltype(mc)::value;
    constexpr int LC = 12 - M1;
    auto* kfn = np == 3 ? &k_inv_cols_rec<M1, 3> : &k_inv_cols_rec<M1, 2>;
    const size_t smem = rec_smem_words(M1, np) * 4;
    if ((e = big_lds((const void*)kfn)) != hipSuccess) return;
    hipLaunchKernelGGL(kfn, dim3(1u << (g.m2 - LC), 1, count), dim3(REC_THREADS), smem, s, G, Z, io, td, ts, kd, tlist,
                       K, g.m2, tb, dir, io32);
  });
  return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_inv_pipeline(const u32* X, u32* G, u32* Z, const TDesc* td, const TState* ts,
                               const KernelDesc* kd, const int* tlist, int count, int K, int np, int slot_lo,
                               int slot_hi, const NttGeom& g, const TwBlock& tb, const TwStep& st, hipStream_t s) {
  return launch_inv_stage(X, G, Z, td, ts, kd, tlist, count, K, np, slot_lo, slot_hi, g, tb, st, 0, s);
}

hipError_t launch_kernel_finish(u32* W, u32* Wq, int K, int np, int logN, hipStream_t s) {
  const size_t total = (size_t)(2 * K * np) << logN;
  const int blocks = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_kernel_finish, dim3(blocks), dim3(256), 0, s, W, Wq, total, logN, np);
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
  const u32 p = prime == 0 ? P0 : (prime == 1 ? P1 : P2), gen = prime == 0 ? G0 : (prime == 1 ? G1 : G2);
  return powmod(gen, (u64)(p - 1) / N, p);
}

static hipError_t upload_powers(uint2** dst, u32 w, u32 count, u32 p, DevArena* arena) {
  uint2* h = (uint2*)malloc(sizeof(uint2) * count);
  if (!h) return hipErrorOutOfMemory;
  u64 v = 1;
  for (u32 e = 0; e < count; ++e) {
    h[e].x = (u32)v;
    h[e].y = shoup_companion((u32)v, p);
    v = v * w % p;
  }
  hipError_t err = hipSuccess;
  if (arena) {
    *dst = static_cast<uint2*>(arena->carve(sizeof(uint2) * count));
    if (!*dst) err = hipErrorOutOfMemory;
  } else {
    err = hipMalloc(dst, sizeof(uint2) * count);
  }
  if (err == hipSuccess) err = hipMemcpy(*dst, h, sizeof(uint2) * count, hipMemcpyHostToDevice);
  free(h);
  return err;
}

int build_block_twiddles(TwBlock* out, void** allocs, DevArena* arena) {
  for (int prime = 0; prime < NPRIME_MAX; ++prime) {
    const u32 p = prime == 0 ? P0 : (prime == 1 ? P1 : P2);
    const u32 w = root_of_unity(prime, BLOCK_MAX);
    const u32 wi = powmod(w, p - 2, p);
    uint2 *f = nullptr, *iv = nullptr;
    if (upload_powers(&f, w, BLOCK_MAX / 2, p, arena) != hipSuccess) return -1;
    if (upload_powers(&iv, wi, BLOCK_MAX / 2, p, arena) != hipSuccess) return -1;
    out->fwd[prime] = f;
    out->inv[prime] = iv;
    allocs[2 * prime] = arena ? nullptr : f;
    allocs[2 * prime + 1] = arena ? nullptr : iv;
  }
  return 0;
}

int build_step_twiddles(int logN, TwStep* out, void** allocs, DevArena* arena) {
  const u64 N = 1ull << logN;
  const u32 nhi = N > 4096 ? (u32)(N >> 12) : 1u;
  int a = 0;
  for (int prime = 0; prime < NPRIME_MAX; ++prime) {
    const u32 p = prime == 0 ? P0 : (prime == 1 ? P1 : P2);
    const u32 w = root_of_unity(prime, N);
    const u32 wi = powmod(w, p - 2, p);
    for (int dir = 0; dir < 2; ++dir) {
      const u32 base = dir ? wi : w;
      uint2 *lo = nullptr, *hi = nullptr;
      if (upload_powers(&lo, base, 4096, p, arena) != hipSuccess) return -1;
      if (upload_powers(&hi, powmod(base, 4096, p), nhi, p, arena) != hipSuccess) return -1;
      out->lo[dir][prime] = lo;
      out->hi[dir][prime] = hi;
      allocs[a++] = arena ? nullptr : lo;
      allocs[a++] = arena ? nullptr : hi;
    }
  }
  return 0;
}

}  // namespace fo
