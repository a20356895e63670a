// The NTT-domain accumulation schedule of one transform, shared by the
// schedule kernel and the forward NTT launch that runs it beside the
// transforms.
#pragma once
#include "internal.h"

namespace fo {

// Alg. 8 schedule for the four real convolutions of Sec. 4.5.  Per
// convolution the walk takes the anti-diagonals d = kA + kB - 2 .. 0,
// s = max(0, d - kB + 1) .. min(kA - 1, d), t = d - s; a new group starts
// when the group is full or the product scale (here the exponent sum
// E_A^s + E_B^t) changes.  The two convolutions of one output component are
// walked one after the other (the paper's schedule) or, anti-diagonal by
// anti-diagonal, together, so that equal scales of the two share a group.

// Convolution c uses x' part (c + 1) / 2 % 2 and w* part c % 2 (computed, not
// looked up: the walk is one serial chain per transform).
__device__ __forceinline__ int conv_pa(int c) { return ((c + 1) >> 1) & 1; }
__device__ __forceinline__ int conv_pb(int c) { return c & 1; }

// The schedule of one transform (the walk orders and group rules are
// described with TState), computed by one thread.  E, Ew: the slice
// exponents of x' and w*, staged by the caller in LDS (the walk reads them
// in data-dependent order).
__device__ inline void schedule_walk(const TDesc& d, TState& s, const KernelDesc& kk, const int (&E)[2][KMAX],
                                     const int (&Ew)[2][KMAX], int L) {
  const bool merged = d.acc_mode == ACC_COMPLEX;
  const int lim = merged ? d.acc_limit : L;
  const int xsh[2] = {merged ? s.xsh[0] : 0, merged ? s.xsh[1] : 0};
  for (int tg = 0; tg < 2; ++tg) {
    int np = 0, ng = 0, cnt = 0, gstart = 0, key = 0, cur = -1, load = 0;
    int emin = 0x7FFFFFFF, emax = -0x7FFFFFFF;
    u64 ge[2] = {0, 0};                                 // walk positions closing a group
    auto close = [&]() {
      s.groups[tg][ng].start = gstart;
      s.groups[tg][ng].count = cnt;
      s.groups[tg][ng].e = key - 2 * d.alpha;
      emin = min(emin, key - 2 * d.alpha);
      emax = max(emax, key - 2 * d.alpha);
      const int w = np - 1;
      ge[w >> 6] |= 1ull << (w & 63);
      ++ng;
      gstart = np;
      cnt = 0;
      load = 0;
    };
    auto visit = [&](int c, int ss, int tt) {
      const int pa = conv_pa(c), wgt = 1 << xsh[pa];
      const int k2 = E[pa][ss] - xsh[pa] + Ew[conv_pb(c)][tt];
      if (cnt > 0 && (load + wgt > lim || k2 != key || (!merged && c != cur))) close();
      key = k2;
      cur = c;
      load += wgt;
      s.mc[tg][np] = (unsigned char)c;
      s.ms[tg][np] = (unsigned char)ss;
      s.mt[tg][np] = (unsigned char)tt;
      ++np;
      ++cnt;
    };
    int kA[2], kB[2];
    for (int h = 0; h < 2; ++h) {
      const int c = 2 * tg + h;
      kA[h] = s.status ? 0 : s.kx[conv_pa(c)];
      kB[h] = kk.kw[conv_pb(c)];
      if (kA[h] == 0 || kB[h] == 0) kA[h] = kB[h] = 0;
    }
    if (merged) {
      const int dmax = max(kA[0] + kB[0], kA[1] + kB[1]) - 2;
      for (int dg = dmax; dg >= 0; --dg)
        for (int h = 0; h < 2; ++h)
          for (int ss = max(0, dg - kB[h] + 1); ss <= min(kA[h] - 1, dg); ++ss) visit(2 * tg + h, ss, dg - ss);
    } else {
      for (int h = 0; h < 2; ++h)
        for (int dg = kA[h] + kB[h] - 2; dg >= 0; --dg)
          for (int ss = max(0, dg - kB[h] + 1); ss <= min(kA[h] - 1, dg); ++ss) visit(2 * tg + h, ss, dg - ss);
    }
    if (cnt > 0) close();
    s.nmem[tg] = np;
    s.ngroups[tg] = ng;
    s.gend[tg][0] = ge[0];
    s.gend[tg][1] = ge[1];
    s.emin[tg] = ng ? emin : 0;
    s.span[tg] = ng ? emax - emin : 0;
  }
}

}  // namespace fo
