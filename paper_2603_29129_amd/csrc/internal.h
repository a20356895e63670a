// Internal interfaces between the plan/execution layer and the kernel files.
#pragma once

#include "common.h"

namespace fo {

constexpr int NTT_THREADS = 256;
constexpr int COL_THREADS = 512;     // column passes: 2 x 64 KiB tiles per CU, 16 waves

// Geometry of the NTT of length N = 2^logN: one workgroup block NTT when
// logN <= LOG2_BLOCK_MAX, else two passes N = N1 * N2 (columns of length N1
// strided by N2, then contiguous rows of length N2).  The NTT-domain order is
// position i1 * N2 + i2 holding X[br(i1) + N1 * br(i2)] (br = bit reversal
// over log2 N1 resp. log2 N2 bits); for the block case N1 = N, N2 = 1.
struct NttGeom {
  int logN, m1, m2;      // N1 = 2^m1, N2 = 2^m2
  int lc;                // log2 of the columns per workgroup (forward column pass, standalone passes)
  int lc_inv;            // log2 of the columns per workgroup (unfused inverse column pass)
  int lrows;             // log2 of the rows per workgroup (forward row pass)
  int lrows_inv;         // log2 of the rows per workgroup (inverse row pass, all groups in LDS)
  bool two_pass() const { return m2 > 0; }
};
NttGeom ntt_geom(int logN, int lc_override = -1, int lrows_override = -1);

struct TwTables {
  TwBlock blk;
  // step tables per logN (index logN), nullptr when unused
  TwStep step[MAX_LOG2_N + 1];
};

// Device memory of a plan: hipMalloc, or carved from one caller-given region
// (the allocation-free entry point), 256-byte aligned.  carve() returns
// nullptr when the region cannot hold the request.
struct DevArena {
  char* base = nullptr;
  size_t size = 0, used = 0;
  void* carve(size_t bytes) {
    const size_t off = (used + 255) & ~(size_t)255;
    if (off > size || bytes > size - off) return nullptr;
    used = off + bytes;
    return base + off;
  }
};

// Host-side table creation (plan time); with an arena the tables are carved
// from it (allocs then receives nullptr entries), otherwise hipMalloc'd.
int build_block_twiddles(TwBlock* out, void** allocs, DevArena* arena = nullptr);
int build_step_twiddles(int logN, TwStep* out, void** allocs, DevArena* arena = nullptr);

// --- NTT launches -----------------------------------------------------------
// Standalone transforms of `count` contiguous vectors (natural order in for the
// forward transform, NTT-domain order out; the inverse takes NTT-domain order
// and returns natural order multiplied by N^{-1}).
// which (two-pass lengths): 0 both passes, 1 the column pass only, 2 the
// row pass only (the autotuner times the passes separately).
hipError_t launch_ntt_standalone(u32* data, int logN, int prime, int count, bool inverse,
                                 const NttGeom& g, const TwBlock& tb, const TwStep& ts, hipStream_t s,
                                 int which = 0);

// Pipeline, np = 2 or 3 moduli: forward NTTs of the slice residues of the
// listed transforms (vector index vi = (part*K + k)*np + prime; only
// k < kx[part] are done).  valid_full: the vectors are fully populated
// (kernel slices) instead of holding zeros beyond n.  vi_lo/vi_hi restrict
// the vectors (plain form).
hipError_t launch_fwd_pipeline(u32* X, const TDesc* td, const TState* ts, const int* tlist, int count,
                               int K, int np, bool valid_full, int vi_lo, int vi_hi, const NttGeom& g,
                               const TwBlock& tb, const TwStep& st, hipStream_t s);

// Pipeline: NTT-domain multiply-accumulate of every Alg. 8 group followed by
// the inverse NTT; writes the first n outputs of each group and prime to the
// compact buffer.  slot_lo/slot_hi restrict the groups (plain form).
hipError_t launch_inv_pipeline(const u32* X, u32* G, u32* Z, const TDesc* td, const TState* ts,
                               const KernelDesc* kd, const int* tlist, int count, int K, int np,
                               int slot_lo, int slot_hi, const NttGeom& g, const TwBlock& tb,
                               const TwStep& st, hipStream_t s);

// Single passes of the above (measurement hook): which = 0 both passes,
// 1 column pass, 2 row pass (forward); 1 row pass with the fused
// multiply-accumulate, 2 column pass (inverse).  With walk_ts set (which 0
// or 1) the forward launch also computes every listed transform's
// accumulation schedule (as launch_groups) in one extra workgroup per
// transform.
hipError_t launch_fwd_stage(u32* X, const TDesc* td, const TState* ts, const int* tlist, int count, int K, int np,
                            bool valid_full, int vi_lo, int vi_hi, const NttGeom& g, const TwBlock& tb,
                            const TwStep& st, int which, hipStream_t s, TState* walk_ts = nullptr,
                            const KernelDesc* kd = nullptr, int L = 0);
// fused_fwd: the row pass also does the forward row NTTs of the slices (X
// holds the forward column pass's output); needs fused_rows_ok.
hipError_t launch_inv_stage(const u32* X, u32* G, u32* Z, const TDesc* td, const TState* ts, const KernelDesc* kd,
                            const int* tlist, int count, int K, int np, int slot_lo, int slot_hi, const NttGeom& g,
                            const TwBlock& tb, const TwStep& st, int which, hipStream_t s, bool fused_fwd = false);
// The register form of the inverse row pass applies (K <= 3, 512-position
// row tiles) and its group tile holds the 2K forward slice rows, so the
// forward row pass can be folded into it.
bool fused_rows_ok(const NttGeom& g, int K);

// Fused inverse column pass + CRT + recombination + postmultiply for the
// two-pass lengths with 2^7 <= N1 <= 2^9 (fused_cols_ok); transforms whose
// exponent span needs the wide accumulator only get their column pass,
// written to the compact buffer Z for launch_recombine_wide.
bool fused_cols_ok(const NttGeom& g);
hipError_t launch_inv_cols_rec(const u32* G, u32* Z, const IoPtrs* io, const TDesc* td, const TState* ts,
                               const KernelDesc* kd, const int* tlist, int count, int K, int np, const NttGeom& g,
                               const TwBlock& tb, int dir, int io32, hipStream_t s);

// Kernel slices: multiply by N^{-1} and build Shoup companions.
hipError_t launch_kernel_finish(u32* W, u32* Wq, int K, int np, int logN, hipStream_t s);

// --- split / chirp / groups / recombination --------------------------------
hipError_t launch_chirp(double2* chirp, int n, int* flag, hipStream_t s);
// Zeroes the per-execution state of the listed transforms; with io set it
// also writes the execution's array pointers there.  reset_io_kernel is that
// kernel: its node in a captured graph is the one whose pointer arguments
// change per execution (grid: count workgroups of RESET_THREADS).
constexpr int RESET_THREADS = 256;
hipError_t launch_reset_io(TState* ts, const int* tlist, int count, IoPtrs* io, const void* in, void* out,
                           hipStream_t s);
const void* reset_io_kernel();
// in / out of the transforms: complex128, or complex64 when io32 (binary32
// target precision: inputs widened exactly, outputs rounded once).
// x' = x (.) w is recomputed from the input by every pass that needs it:
// launch_premul with xp == nullptr takes the per-part maxima (the
// execution), otherwise it writes x' to xp (at each transform's xp_off)
// and takes no maxima (the debug copy).
hipError_t launch_premul(const IoPtrs* io, double2* xp, const TDesc* td, const KernelDesc* kd,
                         TState* ts, const int* tlist, int count, int nmax, int dir, bool kernel_mode,
                         int io32, hipStream_t s);
hipError_t launch_split_plan(const TDesc* td, TState* ts, const KernelDesc* kd, const int* tlist, int count, int K,
                             hipStream_t s);
hipError_t launch_split_extract(const IoPtrs* io, const KernelDesc* kd, u32* X, const TDesc* td, TState* ts,
                                const int* tlist, int count, int nmax, int K, int dir, bool kernel_mode, int io32,
                                int np, hipStream_t s);
hipError_t launch_split_check(const TDesc* td, TState* ts, const int* tlist, int count, int K,
                              hipStream_t s);
hipError_t launch_groups(const TDesc* td, TState* ts, const KernelDesc* kd, const int* tlist,
                         int count, int K, int L, hipStream_t s);
// Garner CRT over np = 2 or 3 moduli, exact recombination, postmultiply.
hipError_t launch_recombine(const u32* Z, const IoPtrs* io, const TDesc* td, const TState* ts,
                            const KernelDesc* kd, const int* tlist, int count, int nmax, int K,
                            int dir, int io32, hipStream_t s, int np);
// Only the transforms whose exponent span needs the wide accumulator.
hipError_t launch_recombine_wide(const u32* Z, const IoPtrs* io, const TDesc* td, const TState* ts,
                                 const KernelDesc* kd, const int* tlist, int count, int nmax, int K,
                                 int dir, int io32, hipStream_t s, int np);
// Writes the execution's array pointers to the plan's descriptor (one
// thread; the plain form's per-call write).
hipError_t launch_set_io(IoPtrs* io, const void* in, void* out, hipStream_t s);

}  // namespace fo
