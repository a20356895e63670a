// Plans, execution schedules and the C ABI of the library.
//
// A plan groups its transforms by convolution length N (one "length class"
// per distinct N); every stage is launched once per class for all of its
// transforms, and each kernel reads its transform's descriptor.  The
// input-independent part of the method -- chirp, splits of Re w* and Im w*
// and their forward NTTs (Sec. 4.5) -- is computed once per distinct n at
// plan time with the same kernels as the runtime path.
//
// Two execution modes:
//  * batched: a fixed launch sequence whose data-dependent parts (slice
//    counts, exponents, Alg. 8 groups) live in device tables; it is captured
//    once into a HIP graph per (in, out, direction) and replayed.
//  * plain: transform by transform, the host reads the slice counts and
//    groups back and issues one launch per NTT (per group and pass for the
//    inverse), like a library-call-per-NTT implementation.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "internal.h"
#include "fft_ozaki.h"

namespace fo {

static thread_local std::string g_err;

// FFT_OZAKI_LOG=1 (or higher) in the environment: plan decisions and
// failures are written to stderr, one line each.
static int log_level() {
  static const int lvl = [] {
    const char* v = getenv("FFT_OZAKI_LOG");
    return v ? atoi(v) : 0;
  }();
  return lvl;
}
#define FO_LOG(...)                          \
  do {                                       \
    if (log_level() > 0) {                   \
      fprintf(stderr, "[fft_ozaki] ");       \
      fprintf(stderr, __VA_ARGS__);          \
      fputc('\n', stderr);                   \
    }                                        \
  } while (0)

static int fail(int code, const std::string& msg) {
  g_err = msg;
  FO_LOG("error %d: %s", code, msg.c_str());
  return code;
}

// A range in the profiler's marker trace (rocprofv3 --marker-trace) around
// a host-side step: the execute calls, and each stage of the plain form and
// of the measurement hook, as in the paper's time breakdown (Sec. 5.5).
struct Range {
  explicit Range(const char* name) { roctxRangePush(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

#define HIPCHK(call)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return fail(FFT_OZAKI_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Split width of Sec. 4.4: the largest alpha with 2 L n 4^alpha <= P, i.e.
// alpha = floor((log2(P / 2) - log2(L n)) / 2) evaluated exactly, with P the
// product of the np moduli (p0 p1, or p0 p1 p2 for the d = 3 CRT).
static unsigned __int128 modulus_product(int np) {
  return np == 3 ? (unsigned __int128)PP * P2 : (unsigned __int128)PP;
}
static int alpha_for(i64 n, int L, int np = 2) {
  const unsigned __int128 P = modulus_product(np);
  int a = -1;
  for (int c = 0; c < 50; ++c) {
    const unsigned __int128 v = ((unsigned __int128)2 * (unsigned)L * (u64)n) << (2 * c);
    if (v > P) break;
    a = c;
  }
  return a;
}

// Products per group of the complex accumulation: the most c with
// c n 4^alpha <= (p0 p1 - 1) / 2, so that the signed sum of c products, each
// at most n 4^alpha in magnitude (n terms of two alpha-bit integers), is
// recovered exactly by the symmetric CRT (Sec. 3.3, Sec. 4.4).  At least L
// by the choice of alpha.
static int acc_limit_for(i64 n, int alpha, int np = 2) {
  const unsigned __int128 unit = (unsigned __int128)(u64)n << (2 * alpha);
  const unsigned __int128 lim = ((modulus_product(np) - 1) / 2) / unit;
  return lim > (unsigned __int128)MAX_MEMBERS ? MAX_MEMBERS : (int)lim;
}

// Bluestein convolution length: N = 2^ceil(log2(2n - 1)) (Sec. 3.2), or
// N = n for a power-of-two n with the cyclic embedding (Sec. 3.2).
static int conv_log2(i64 n, bool cyclic) {
  if (n <= 1) return 0;
  if (cyclic && (n & (n - 1)) == 0) {
    int l = 0;
    while (((i64)1 << l) < n) ++l;
    return l;
  }
  int l = 0;
  while (((i64)1 << l) < 2 * n - 1) ++l;
  return l;
}

struct KernelHost {
  i64 n;
  int logN, alpha;
  double2* chirp = nullptr;
  u32* W = nullptr;
  u32* Wq = nullptr;
  int kw[2] = {0, 0};
  int Ew[2][KMAX] = {};
};

struct LengthClass {
  int logN;
  NttGeom geom;
  std::vector<int> tids;
  int* d_tlist = nullptr;
  int nmax = 0;
};

// A captured batched schedule for one direction.  Its first node writes the
// execution's array pointers to the plan's descriptor; a new (in, out) pair
// only updates that node's arguments in the instantiated graph.
struct GraphEntry {
  int dir;
  hipGraph_t graph;          // kept alive: io_node belongs to it
  hipGraphExec_t exec;
  hipGraphNode_t io_node;
  const void* in;            // the pointers io_node currently writes
  void* out;
};

}  // namespace fo

struct fft_ozaki_plan_s {
  int device = 0;
  int K = 3, L = 3, mode = FFT_OZAKI_MODE_BATCHED;
  int autotune = 0;
  bool cyclic = true;               // FFT_OZAKI_EMBED_AUTO
  int accumulation = FFT_OZAKI_ACCUM_COMPLEX;
  int precision = FFT_OZAKI_PREC_FP64;  // FP32: complex64 in / out
  int primes = 2;                   // CRT moduli: 2 (p0, p1) or 3 (p0, p1, p2)
  std::string tune_cache;
  std::vector<fo::i64> lengths;
  fo::i64 total = 0;
  std::vector<fo::TDesc> td;
  std::vector<fo::KernelHost> kernels;
  std::vector<fo::LengthClass> classes;
  fo::TwBlock tb{};
  std::map<int, fo::TwStep> steps;
  fo::TDesc* d_td = nullptr;
  fo::KernelDesc* d_kd = nullptr;
  fo::TState* d_ts = nullptr;
  int* d_tall = nullptr;
  double2* xp = nullptr;            // x' of the transforms, filled only by the debug copy (stage 1)
  fo::u32* X = nullptr;
  fo::u32* G = nullptr;
  fo::u32* Z = nullptr;
  fo::IoPtrs* d_io = nullptr;       // the current execution's in / out (read by the kernels)
  std::vector<void*> allocs;
  fo::i64 bytes = 0;
  hipStream_t cap = nullptr;
  std::vector<fo::GraphEntry> graphs;
  // stage timing: HIP events at the stage boundaries of the batched
  // sequence, 2 + 4 (length classes); such executions launch the sequence
  // on the caller's stream instead of replaying the graph
  bool stage_timing = false;
  std::vector<hipEvent_t> tev;
  bool timed_last = false;          // the last execution recorded them
  const void* last_in = nullptr;
  void* last_out = nullptr;
  int last_dir = -1;
  // the batched form left X with the forward column pass only for the
  // lengths whose forward row pass is folded into the inverse row pass
  bool x_rows_pending = false;
  // non-null: all device memory is carved from this region (nothing is
  // allocated or freed, no capture stream is created)
  fo::DevArena* arena = nullptr;
  int fail_at = 0, alloc_count = 0;   // allocation-failure test hook
};

namespace fo {

// Test hook: FFT_OZAKI_TEST_FAIL_ALLOC=k makes the k-th device allocation of
// each plan build report failure (as hipMalloc running out of memory would),
// so the error path and the release of the earlier allocations can be tested.
static int fail_alloc_at() {
  const char* v = getenv("FFT_OZAKI_TEST_FAIL_ALLOC");
  return v ? atoi(v) : 0;
}

static int dmalloc(fft_ozaki_plan_s* p, void** ptr, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (p->fail_at > 0 && ++p->alloc_count == p->fail_at) {
    *ptr = nullptr;
    return fail(FFT_OZAKI_ERR_NOMEM, "device allocation " + std::to_string(p->alloc_count) + " of " +
                                         std::to_string(bytes) + " bytes failed (injected)");
  }
  if (p->arena) {
    *ptr = p->arena->carve(bytes);
    if (!*ptr) return fail(FFT_OZAKI_ERR_NOMEM, "static workspace exhausted");
    p->bytes += (i64)bytes;
    return FFT_OZAKI_OK;
  }
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) return fail(FFT_OZAKI_ERR_NOMEM, std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
  p->allocs.push_back(*ptr);
  p->bytes += (i64)bytes;
  return FFT_OZAKI_OK;
}

static void destroy_plan(fft_ozaki_plan_s* p) {
  if (!p) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  for (auto& g : p->graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
  }
  for (hipEvent_t e : p->tev) (void)hipEventDestroy(e);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  for (void* a : p->allocs) (void)hipFree(a);
  (void)hipSetDevice(cur);
  delete p;
}

static const TwStep& step_for(fft_ozaki_plan_s* p, int logN) {
  static const TwStep none{};
  auto it = p->steps.find(logN);
  return it == p->steps.end() ? none : it->second;
}

// --- autotuning of the NTT tile shapes -------------------------------------
// Two shapes per length class are tuned by timing them on scratch vectors as
// many as the class's slice vectors (4 K per transform, up to 256 MiB), with
// the plan's own twiddle tables:
//  * log2 columns per workgroup of the column passes: the forward column
//    pass alone (the same column body runs as the first pass of the batched
//    schedule's forward NTTs);
//  * log2 rows per workgroup of the standalone row passes: forward and
//    inverse row passes (they run in the three-modulus plans and in the
//    plain form).
// Every candidate computes the same transform, so results do not depend on
// the shapes.  The pipelined row pass sizes its grid from the device's
// occupancy and the fused column pass has a fixed 4096-position tile, so
// neither has a shape to tune.  The tune cache key holds the GPU
// architecture, log2 N and the scratch vector count rounded up to a power
// of two.

static std::string tune_key(int logN, int vecs) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t pr;
  (void)hipGetDeviceProperties(&pr, dev);
  int v = 1;
  while (v < vecs) v <<= 1;
  return std::string(pr.gcnArchName) + ":" + std::to_string(logN) + ":" + std::to_string(v);
}

static bool tune_lookup(const std::string& path, const std::string& key, int* lc, int* lr) {
  if (path.empty()) return false;
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (fgets(line, sizeof line, f)) {
    char k[400];
    int a, b;
    if (sscanf(line, "%399s %d %d", k, &a, &b) == 3 && key == k) {
      *lc = a;
      *lr = b;
      found = true;
    }
  }
  fclose(f);
  return found;
}

static void tune_store(const std::string& path, const std::string& key, int lc, int lr) {
  if (path.empty()) return;
  FILE* f = fopen(path.c_str(), "a");
  if (!f) return;
  fprintf(f, "%s %d %d\n", key.c_str(), lc, lr);
  fclose(f);
}

static int autotune_geom(fft_ozaki_plan_s* p, int logN, int transforms, NttGeom* out) {
  NttGeom def = ntt_geom(logN);
  *out = def;
  if (!def.two_pass()) return FFT_OZAKI_OK;
  const size_t vec_bytes = (size_t)4 << logN;
  const int vecs = (int)std::max<size_t>(1, std::min<size_t>((size_t)4 * p->K * transforms,
                                                             std::min<size_t>(65535, ((size_t)256 << 20) / vec_bytes)));
  const std::string key = tune_key(logN, vecs);
  auto lc_ok = [&](int c) { return c >= 2 && c <= 6 && def.m1 + c <= 14 && c <= def.m2; };
  auto lr_ok = [&](int r) { return r >= 0 && r <= 4 && def.m2 + r <= 14 && r <= def.m1; };
  int lc = -1, lr = -1;
  // a cached entry is used only if it is one of the shapes tried below
  if (tune_lookup(p->tune_cache, key, &lc, &lr) && lc_ok(lc) && lr_ok(lr)) {
    *out = ntt_geom(logN, lc, lr);
    FO_LOG("autotune N=2^%d (%d vectors): cached column tile 2^%d, row tile 2^%d", logN, vecs, lc, lr);
    return FFT_OZAKI_OK;
  }
  u32* buf = nullptr;
  HIPCHK(hipMalloc(&buf, vec_bytes * vecs));
  struct Free {
    u32* b;
    ~Free() { (void)hipFree(b); }
  } free_buf{buf};
  HIPCHK(hipMemset(buf, 0, vec_bytes * vecs));
  const TwStep& st = step_for(p, logN);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // time `reps` calls of run(g) after two untimed ones; a shape whose launch
  // fails is not a candidate (infinite time)
  auto time_shape = [&](const NttGeom& g, auto run) -> float {
    hipError_t le = hipSuccess;
    auto once = [&]() {
      const hipError_t e = run(g);
      if (le == hipSuccess) le = e;
    };
    once();
    once();
    if (hipEventRecord(e0, nullptr) != hipSuccess) return 1e30f;
    for (int w = 0; w < 5; ++w) once();
    if (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 1e30f;
    float ms = 0;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 1e30f;
    const hipError_t ke = hipGetLastError();
    return (le == hipSuccess && ke == hipSuccess) ? ms : 1e30f;
  };
  float best_c = 1e30f, best_r = 1e30f;
  int pick_c = def.lc, pick_r = def.lrows;
  for (int c = 2; c <= 6; ++c) {
    if (!lc_ok(c)) continue;
    const float ms = time_shape(ntt_geom(logN, c, def.lrows), [&](const NttGeom& g) {
      return launch_ntt_standalone(buf, logN, 0, vecs, false, g, p->tb, st, nullptr, 1);
    });
    FO_LOG("autotune N=2^%d (%d vectors): column tile 2^%d: %.4f ms", logN, vecs, c, ms);
    if (ms < best_c) {
      best_c = ms;
      pick_c = c;
    }
  }
  for (int r = 0; r <= 4; ++r) {
    if (!lr_ok(r)) continue;
    const float ms = time_shape(ntt_geom(logN, pick_c, r), [&](const NttGeom& g) {
      const hipError_t a = launch_ntt_standalone(buf, logN, 0, vecs, false, g, p->tb, st, nullptr, 2);
      const hipError_t b = launch_ntt_standalone(buf, logN, 0, vecs, true, g, p->tb, st, nullptr, 2);
      return a != hipSuccess ? a : b;
    });
    FO_LOG("autotune N=2^%d (%d vectors): row tile 2^%d: %.4f ms", logN, vecs, r, ms);
    if (ms < best_r) {
      best_r = ms;
      pick_r = r;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *out = ntt_geom(logN, pick_c, pick_r);
  tune_store(p->tune_cache, key, out->lc, out->lrows);
  return FFT_OZAKI_OK;
}

// --- kernel (chirp) preparation ---------------------------------------------

static int prepare_kernel(fft_ozaki_plan_s* p, KernelHost& kh, int idx) {
  const i64 n = kh.n;
  const size_t N = (size_t)1 << kh.logN;
  const int K = p->K, np = p->primes;
  int rc;
  if ((rc = dmalloc(p, (void**)&kh.chirp, sizeof(double2) * n))) return rc;
  if ((rc = dmalloc(p, (void**)&kh.W, 4 * (size_t)(2 * np * K) * N))) return rc;
  if ((rc = dmalloc(p, (void**)&kh.Wq, 4 * (size_t)(2 * np * K) * N))) return rc;
  HIPCHK(hipMemset(kh.W, 0, 4 * (size_t)(2 * np * K) * N));
  // temporaries of the kernel split (freed at the end; carved and left in
  // place with an arena)
  int* flag = nullptr;
  TState* ts = nullptr;
  TDesc* td = nullptr;
  KernelDesc* kd = nullptr;
  int* tl = nullptr;
  std::vector<void*> temps;
  auto tmalloc = [&](void** ptr, size_t bytes) -> int {
    if (p->arena) {
      *ptr = p->arena->carve(bytes);
      return *ptr ? FFT_OZAKI_OK : fail(FFT_OZAKI_ERR_NOMEM, "static workspace exhausted");
    }
    if (p->fail_at > 0 && ++p->alloc_count == p->fail_at)
      return fail(FFT_OZAKI_ERR_NOMEM, "device allocation " + std::to_string(p->alloc_count) + " failed (injected)");
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) return fail(FFT_OZAKI_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    temps.push_back(*ptr);
    return FFT_OZAKI_OK;
  };
  struct FreeTemps {
    std::vector<void*>& v;
    ~FreeTemps() {
      for (void* a : v) (void)hipFree(a);
    }
  } free_temps{temps};
  if ((rc = tmalloc((void**)&flag, sizeof(int))) ||
      (rc = tmalloc((void**)&ts, sizeof(TState))) || (rc = tmalloc((void**)&td, sizeof(TDesc))) ||
      (rc = tmalloc((void**)&kd, sizeof(KernelDesc))) || (rc = tmalloc((void**)&tl, sizeof(int))))
    return rc;
  HIPCHK(hipMemset(flag, 0, sizeof(int)));
  TDesc h{};
  h.n = (int)n;
  h.N = (int)N;
  h.logN = kh.logN;
  h.alpha = kh.alpha;
  h.kd = 0;
  KernelDesc hk{};
  hk.n = (int)n;
  hk.N = (int)N;
  hk.logN = kh.logN;
  hk.alpha = kh.alpha;
  hk.chirp = kh.chirp;
  const int zero = 0;
  HIPCHK(hipMemcpy(td, &h, sizeof h, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(kd, &hk, sizeof hk, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(tl, &zero, sizeof zero, hipMemcpyHostToDevice));
  HIPCHK(launch_chirp(kh.chirp, (int)n, flag, nullptr));
  HIPCHK(launch_reset_io(ts, tl, 1, nullptr, nullptr, nullptr, nullptr));
  HIPCHK(launch_premul(nullptr, nullptr, td, kd, ts, tl, 1, (int)n, 0, true, 0, nullptr));
  HIPCHK(launch_split_plan(td, ts, kd, tl, 1, K, nullptr));
  for (int r = 0; r < K; ++r) {
    HIPCHK(launch_split_extract(nullptr, kd, kh.W, td, ts, tl, 1, (int)n, K, 0, true, 0, np, nullptr));
    HIPCHK(launch_split_check(td, ts, tl, 1, K, nullptr));
  }
  TState hs;
  HIPCHK(hipMemcpy(&hs, ts, sizeof hs, hipMemcpyDeviceToHost));
  int hflag = 0;
  HIPCHK(hipMemcpy(&hflag, flag, sizeof hflag, hipMemcpyDeviceToHost));
  if (hs.status || hs.active[0] || hs.active[1]) return fail(FFT_OZAKI_ERR_UNSUPPORTED, "kernel split failed");
  if (hflag) return fail(FFT_OZAKI_ERR_UNSUPPORTED, "chirp value too close to a rounding boundary for n=" + std::to_string(n));
  for (int part = 0; part < 2; ++part) {
    kh.kw[part] = hs.kx[part];
    for (int k = 0; k < KMAX; ++k) kh.Ew[part][k] = k < hs.kx[part] ? hs.E[part][k] : 0;
  }
  // forward NTTs of the kernel slices (all N positions populated), then
  // N^{-1} folded in and the Shoup companions
  NttGeom g = ntt_geom(kh.logN);
  HIPCHK(launch_fwd_pipeline(kh.W, td, ts, tl, 1, K, np, true, 0, 2 * np * K, g, p->tb, step_for(p, kh.logN), nullptr));
  HIPCHK(launch_kernel_finish(kh.W, kh.Wq, K, np, kh.logN, nullptr));
  HIPCHK(hipDeviceSynchronize());
  (void)idx;
  return FFT_OZAKI_OK;
}

static int build_plan(fft_ozaki_plan_s* p) {
  const int K = p->K;
  const int count = (int)p->lengths.size();
  p->fail_at = fail_alloc_at();
  p->alloc_count = 0;
  HIPCHK(hipGetDevice(&p->device));
  void* tw_allocs[2 * NPRIME_MAX] = {};
  if (build_block_twiddles(&p->tb, tw_allocs, p->arena)) return fail(FFT_OZAKI_ERR_NOMEM, "twiddle tables");
  for (void* a : tw_allocs)
    if (a) p->allocs.push_back(a);
  // distinct lengths and N classes
  std::map<i64, int> kidx;
  std::map<int, int> cidx;
  for (i64 n : p->lengths) {
    if (!kidx.count(n)) {
      KernelHost kh;
      kh.n = n;
      kh.logN = conv_log2(n, p->cyclic);
      kh.alpha = alpha_for(n, p->L, p->primes);
      kidx[n] = (int)p->kernels.size();
      p->kernels.push_back(kh);
    }
    const int lg = conv_log2(n, p->cyclic);
    if (!cidx.count(lg)) {
      LengthClass lc;
      lc.logN = lg;
      cidx[lg] = (int)p->classes.size();
      p->classes.push_back(lc);
    }
  }
  std::map<int, int> class_count;
  for (i64 n : p->lengths) ++class_count[conv_log2(n, p->cyclic)];
  for (auto& lc : p->classes) {
    if (ntt_geom(lc.logN).two_pass() && !p->steps.count(lc.logN)) {
      void* sa[4 * NPRIME_MAX] = {};
      TwStep st{};
      if (build_step_twiddles(lc.logN, &st, sa, p->arena)) return fail(FFT_OZAKI_ERR_NOMEM, "step twiddles");
      for (void* a : sa)
        if (a) p->allocs.push_back(a);
      p->steps[lc.logN] = st;
    }
    lc.geom = ntt_geom(lc.logN);
    if (p->autotune) {
      int rc = autotune_geom(p, lc.logN, class_count[lc.logN], &lc.geom);
      if (rc) return rc;
    }
  }
  for (size_t i = 0; i < p->kernels.size(); ++i) {
    int rc = prepare_kernel(p, p->kernels[i], (int)i);
    if (rc) return rc;
  }
  // descriptors and workspace
  i64 io = 0, xo = 0, go = 0, zo = 0;
  const i64 SL = (i64)K * K;
  for (int t = 0; t < count; ++t) {
    const i64 n = p->lengths[t];
    TDesc d{};
    d.n = (int)n;
    d.logN = conv_log2(n, p->cyclic);
    d.N = 1 << d.logN;
    d.alpha = alpha_for(n, p->L, p->primes);
    d.acc_mode = p->accumulation == FFT_OZAKI_ACCUM_COMPLEX ? ACC_COMPLEX : ACC_PER_CONV;
    d.acc_limit = d.acc_mode == ACC_COMPLEX ? acc_limit_for(n, d.alpha, p->primes) : p->L;
    d.kd = kidx[n];
    d.zs = (int)((n + 3) & ~(i64)3);
    d.io_off = io;
    d.xp_off = io;
    d.X_off = xo;
    d.G_off = go;
    d.Z_off = zo;
    io += n;
    xo += (i64)(2 * p->primes * K) << d.logN;                    // [part][k][prime][N]
    if (ntt_geom(d.logN).two_pass()) go += (4 * SL * p->primes) << d.logN;   // [slot][prime][N], 4 K^2 slots
    zo += 4 * SL * p->primes * (i64)d.zs;                        // [slot][prime][zs]
    p->td.push_back(d);
    LengthClass& lc = p->classes[cidx[d.logN]];
    lc.tids.push_back(t);
    lc.nmax = std::max<int>(lc.nmax, (int)n);
  }
  p->total = io;
  for (auto& lc : p->classes)
    if (lc.tids.size() > 65535) return fail(FFT_OZAKI_ERR_INVALID, "more than 65535 transforms share one convolution length");
  int rc;
  if ((rc = dmalloc(p, (void**)&p->X, 4 * (size_t)xo))) return rc;
  if ((rc = dmalloc(p, (void**)&p->G, 4 * (size_t)go))) return rc;
  if ((rc = dmalloc(p, (void**)&p->Z, 4 * (size_t)zo))) return rc;
  if ((rc = dmalloc(p, (void**)&p->d_td, sizeof(TDesc) * count))) return rc;
  if ((rc = dmalloc(p, (void**)&p->d_ts, sizeof(TState) * count))) return rc;
  if ((rc = dmalloc(p, (void**)&p->d_tall, sizeof(int) * count))) return rc;
  if ((rc = dmalloc(p, (void**)&p->d_kd, sizeof(KernelDesc) * p->kernels.size()))) return rc;
  if ((rc = dmalloc(p, (void**)&p->d_io, sizeof(IoPtrs)))) return rc;
  HIPCHK(hipMemcpy(p->d_td, p->td.data(), sizeof(TDesc) * count, hipMemcpyHostToDevice));
  HIPCHK(hipMemset(p->d_ts, 0, sizeof(TState) * count));
  std::vector<int> all(count);
  for (int t = 0; t < count; ++t) all[t] = t;
  HIPCHK(hipMemcpy(p->d_tall, all.data(), sizeof(int) * count, hipMemcpyHostToDevice));
  std::vector<KernelDesc> kds;
  for (auto& kh : p->kernels) {
    KernelDesc k{};
    k.n = (int)kh.n;
    k.logN = kh.logN;
    k.N = 1 << kh.logN;
    k.alpha = kh.alpha;
    k.chirp = kh.chirp;
    k.W = kh.W;
    k.Wq = kh.Wq;
    for (int part = 0; part < 2; ++part) {
      k.kw[part] = kh.kw[part];
      for (int j = 0; j < KMAX; ++j) k.Ew[part][j] = kh.Ew[part][j];
    }
    kds.push_back(k);
  }
  HIPCHK(hipMemcpy(p->d_kd, kds.data(), sizeof(KernelDesc) * kds.size(), hipMemcpyHostToDevice));
  for (auto& lc : p->classes) {
    if ((rc = dmalloc(p, (void**)&lc.d_tlist, sizeof(int) * lc.tids.size()))) return rc;
    HIPCHK(hipMemcpy(lc.d_tlist, lc.tids.data(), sizeof(int) * lc.tids.size(), hipMemcpyHostToDevice));
  }
  if (!p->arena) HIPCHK(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
  HIPCHK(hipDeviceSynchronize());
  FO_LOG("plan: %d transforms, %zu distinct lengths, %zu length classes, K=%d L=%d mode=%d primes=%d, "
         "workspace %lld bytes%s",
         count, p->kernels.size(), p->classes.size(), K, p->L, p->mode, p->primes, (long long)p->bytes,
         p->arena ? " (static workspace)" : "");
  for (auto& lc : p->classes)
    FO_LOG("  class N=2^%d: %zu transforms, N1=2^%d N2=2^%d, column tile 2^%d, row tile 2^%d%s%s", lc.logN,
           lc.tids.size(), lc.geom.m1, lc.geom.m2, lc.geom.lc, lc.geom.lrows,
           fused_rows_ok(lc.geom, K) ? ", forward rows folded into the pipelined row pass" : "",
           fused_cols_ok(lc.geom) ? ", CRT fused into the column pass" : "");
  return FFT_OZAKI_OK;
}

// 1 when the plan's transforms read and write complex64 (binary32 target).
static inline int io32_of(const fft_ozaki_plan_s* p) { return p->precision == FFT_OZAKI_PREC_FP32 ? 1 : 0; }

// The batched launch sequence (also what gets captured into the graph), for
// two or three moduli alike.
// Stage boundary i of the batched sequence (stage timing only): 0 start,
// 1 after the split, 2 + c after class c's forward NTTs, 2 + C + 3c (+1, +2)
// after its inverse row pass (column pass, recombination).
// Stage-timed executions are not captured (see fft_ozaki_stage_timing).
static hipError_t mark(fft_ozaki_plan_s* p, size_t i, hipStream_t s) {
  return p->stage_timing ? hipEventRecord(p->tev[i], s) : hipSuccess;
}

static int enqueue_batched(fft_ozaki_plan_s* p, int dir, hipStream_t s, const void* in, void* out) {
  const int K = p->K, np = p->primes, count = (int)p->td.size();
  const size_t C = p->classes.size();
  HIPCHK(mark(p, 0, s));
  HIPCHK(launch_reset_io(p->d_ts, p->d_tall, count, p->d_io, in, out, s));
  // the premultiply and the extraction passes: one launch each over all
  // transforms (each workgroup stops at its transform's length), so the
  // length classes' work overlaps
  int nmax = 0;
  for (auto& lc : p->classes) nmax = std::max(nmax, lc.nmax);
  HIPCHK(launch_premul(p->d_io, nullptr, p->d_td, p->d_kd, p->d_ts, p->d_tall, count, nmax, dir, false, io32_of(p), s));
  HIPCHK(launch_split_plan(p->d_td, p->d_ts, p->d_kd, p->d_tall, count, K, s));
  for (int r = 0; r < K; ++r) {
    HIPCHK(launch_split_extract(p->d_io, p->d_kd, p->X, p->d_td, p->d_ts, p->d_tall, count, nmax, K, dir, false,
                                io32_of(p), np, s));
    HIPCHK(launch_split_check(p->d_td, p->d_ts, p->d_tall, count, K, s));
  }
  HIPCHK(mark(p, 1, s));
  for (size_t c = 0; c < C; ++c) {
    // forward NTTs; where the forward row pass is folded into the inverse
    // row pass, only the column pass here.  The accumulation schedule of the
    // class's transforms is computed inside the same launch.
    auto& lc = p->classes[c];
    const int which = fused_rows_ok(lc.geom, K) ? 1 : 0;
    HIPCHK(launch_fwd_stage(p->X, p->d_td, p->d_ts, lc.d_tlist, (int)lc.tids.size(), K, np, false, 0, 2 * np * K,
                            lc.geom, p->tb, step_for(p, lc.logN), which, s, p->d_ts, p->d_kd, p->L));
    HIPCHK(mark(p, 2 + c, s));
  }
  for (size_t c = 0; c < C; ++c) {
    auto& lc = p->classes[c];
    const int cnt = (int)lc.tids.size();
    const size_t b = 2 + C + 3 * c;
    // rows (with the forward rows where possible)
    HIPCHK(launch_inv_stage(p->X, p->G, p->Z, p->d_td, p->d_ts, p->d_kd, lc.d_tlist, cnt, K, np, 0, 4 * K * K, lc.geom,
                            p->tb, step_for(p, lc.logN), 1, s, fused_rows_ok(lc.geom, K)));
    HIPCHK(mark(p, b, s));
    if (fused_cols_ok(lc.geom)) {
      // fused columns + CRT + recombination (for transforms that need the
      // wide accumulator: the columns to the compact buffer, then the wide
      // recombination)
      HIPCHK(launch_inv_cols_rec(p->G, p->Z, p->d_io, p->d_td, p->d_ts, p->d_kd, lc.d_tlist, cnt, K, np, lc.geom, p->tb,
                                 dir, io32_of(p), s));
      HIPCHK(mark(p, b + 1, s));
      HIPCHK(launch_recombine_wide(p->Z, p->d_io, p->d_td, p->d_ts, p->d_kd, lc.d_tlist, cnt, lc.nmax, K, dir,
                                   io32_of(p), s, np));
    } else {
      HIPCHK(launch_inv_stage(p->X, p->G, p->Z, p->d_td, p->d_ts, p->d_kd, lc.d_tlist, cnt, K, np, 0, 4 * K * K,
                              lc.geom, p->tb, step_for(p, lc.logN), 2, s, fused_rows_ok(lc.geom, K)));
      HIPCHK(mark(p, b + 1, s));
      HIPCHK(launch_recombine(p->Z, p->d_io, p->d_td, p->d_ts, p->d_kd, lc.d_tlist, cnt, lc.nmax, K, dir, io32_of(p), s,
                              np));
    }
    HIPCHK(mark(p, b + 2, s));
  }
  return FFT_OZAKI_OK;
}

// Arguments of the descriptor-writing node for (in, out).
static hipError_t set_io_node(fft_ozaki_plan_s* p, GraphEntry& g, const void* in, void* out) {
  TState* ts = p->d_ts;
  const int* tl = p->d_tall;
  IoPtrs* io = p->d_io;
  void* args[5] = {&ts, &tl, &io, &in, &out};
  hipKernelNodeParams kp{};
  kp.func = const_cast<void*>(reset_io_kernel());
  kp.gridDim = dim3((unsigned)p->td.size());
  kp.blockDim = dim3(RESET_THREADS);
  kp.sharedMemBytes = 0;
  kp.kernelParams = args;
  kp.extra = nullptr;
  const hipError_t e = hipGraphExecKernelNodeSetParams(g.exec, g.io_node, &kp);
  if (e == hipSuccess) {
    g.in = in;
    g.out = out;
  }
  return e;
}

static int run_batched(fft_ozaki_plan_s* p, const void* in, void* out, int dir, hipStream_t s) {
  for (auto& lc : p->classes)
    if (fused_rows_ok(lc.geom, p->K)) p->x_rows_pending = true;
  // stage timing: the same launches in the same order, with the boundary
  // events, directly on the caller's stream
  if (p->stage_timing) return enqueue_batched(p, dir, s, in, out);
  for (size_t i = 0; i < p->graphs.size(); ++i) {
    GraphEntry& g = p->graphs[i];
    if (g.dir != dir) continue;
    if ((g.in != in || g.out != out) && set_io_node(p, g, in, out) != hipSuccess) {
      // the node could not be updated: capture this direction again below
      // (the graph may still run from an earlier call on another stream:
      // wait for the device before destroying it)
      (void)hipGetLastError();
      FO_LOG("graph argument update failed; capturing again");
      (void)hipDeviceSynchronize();
      (void)hipGraphExecDestroy(g.exec);
      (void)hipGraphDestroy(g.graph);
      p->graphs.erase(p->graphs.begin() + (long)i);
      break;
    }
    HIPCHK(hipGraphLaunch(g.exec, s));
    return FFT_OZAKI_OK;
  }
  // capture on the plan's private stream, after the caller's prior work
  hipEvent_t ev;
  HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  HIPCHK(hipEventRecord(ev, s));
  HIPCHK(hipStreamWaitEvent(p->cap, ev, 0));
  HIPCHK(hipStreamSynchronize(p->cap));
  (void)hipEventDestroy(ev);
  hipGraph_t graph;
  HIPCHK(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
  int rc = enqueue_batched(p, dir, p->cap, in, out);
  hipError_t ce = hipStreamEndCapture(p->cap, &graph);
  if (rc) {
    if (ce == hipSuccess) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (ce != hipSuccess) return fail(FFT_OZAKI_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
  // the descriptor-writing node: the graph's only launch of the reset kernel
  GraphEntry g{dir, graph, nullptr, nullptr, in, out};
  size_t nn = 0;
  HIPCHK(hipGraphGetNodes(graph, nullptr, &nn));
  std::vector<hipGraphNode_t> nodes(nn);
  HIPCHK(hipGraphGetNodes(graph, nodes.data(), &nn));
  for (hipGraphNode_t nd : nodes) {
    hipGraphNodeType ty;
    if (hipGraphNodeGetType(nd, &ty) != hipSuccess || ty != hipGraphNodeTypeKernel) continue;
    hipKernelNodeParams kp{};
    if (hipGraphKernelNodeGetParams(nd, &kp) == hipSuccess && kp.func == reset_io_kernel()) g.io_node = nd;
  }
  if (!g.io_node) {
    (void)hipGraphDestroy(graph);
    return fail(FFT_OZAKI_ERR_HIP, "captured graph has no descriptor node");
  }
  HIPCHK(hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0));
  FO_LOG("captured the batched schedule for direction %d (%zu kernel and other nodes)", dir, nn);
  p->graphs.push_back(g);
  HIPCHK(hipGraphLaunch(g.exec, s));
  return FFT_OZAKI_OK;
}

static int run_plain(fft_ozaki_plan_s* p, const void* in, void* out, int dir, hipStream_t s) {
  const int K = p->K, SL = 2 * K * K;   // slots per output component
  constexpr int np = 2;                 // the plain form serves two-modulus plans
  HIPCHK(launch_set_io(p->d_io, in, out, s));
  for (int t = 0; t < (int)p->td.size(); ++t) {
    const TDesc& d = p->td[t];
    const int* tl = p->d_tall + t;
    const NttGeom g = p->classes.empty() ? ntt_geom(d.logN) : [&] {
      for (auto& lc : p->classes)
        if (lc.logN == d.logN) return lc.geom;
      return ntt_geom(d.logN);
    }();
    const TwStep& st = step_for(p, d.logN);
    Range rt("transform");
    std::unique_ptr<Range> stage(new Range("premultiply + split"));
    HIPCHK(launch_reset_io(p->d_ts, tl, 1, nullptr, nullptr, nullptr, s));
    HIPCHK(launch_premul(p->d_io, nullptr, p->d_td, p->d_kd, p->d_ts, tl, 1, d.n, dir, false, io32_of(p), s));
    HIPCHK(launch_split_plan(p->d_td, p->d_ts, p->d_kd, tl, 1, K, s));
    for (int r = 0; r < K; ++r) {
      HIPCHK(launch_split_extract(p->d_io, p->d_kd, p->X, p->d_td, p->d_ts, tl, 1, d.n, K, dir, false, io32_of(p), np,
                                  s));
      HIPCHK(launch_split_check(p->d_td, p->d_ts, tl, 1, K, s));
      int act[2];
      HIPCHK(hipMemcpyAsync(act, &p->d_ts[t].active, sizeof act, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (!act[0] && !act[1]) break;
    }
    stage.reset(new Range("accumulation schedule"));
    HIPCHK(launch_groups(p->d_td, p->d_ts, p->d_kd, tl, 1, K, p->L, s));
    TState hs;
    HIPCHK(hipMemcpyAsync(&hs, &p->d_ts[t], sizeof hs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (!hs.status) {
      stage.reset(new Range("forward NTTs"));
      for (int part = 0; part < 2; ++part)
        for (int k = 0; k < hs.kx[part]; ++k)
          for (int prime = 0; prime < np; ++prime) {
            const int vi = (part * K + k) * np + prime;
            HIPCHK(launch_fwd_pipeline(p->X, p->d_td, p->d_ts, tl, 1, K, np, false, vi, vi + 1, g, p->tb, st, s));
          }
      stage.reset(new Range("NTT-domain multiply-accumulate + inverse NTTs"));
      for (int tg = 0; tg < 2; ++tg)
        for (int gi = 0; gi < hs.ngroups[tg]; ++gi) {
          const int slot = tg * SL + gi;
          HIPCHK(launch_inv_pipeline(p->X, p->G, p->Z, p->d_td, p->d_ts, p->d_kd, tl, 1, K, np, slot, slot + 1, g,
                                     p->tb, st, s));
        }
    }
    stage.reset(new Range("CRT + recombination + postmultiply"));
    HIPCHK(launch_recombine(p->Z, p->d_io, p->d_td, p->d_ts, p->d_kd, tl, 1, d.n, K, dir, io32_of(p), s, np));
  }
  HIPCHK(hipStreamSynchronize(s));
  return FFT_OZAKI_OK;
}

// One stage of the batched sequence for all transforms (measurement hook).
static const char* const kStageNames[9] = {"", "stage 1: premultiply + split", "stage 2: accumulation schedule",
                                            "stage 3: forward NTTs", "stage 4: forward column pass",
                                            "stage 5: forward row pass", "stage 6: row pass (fused MAC)",
                                            "stage 7: column pass (fused CRT)", "stage 8: recombination"};
static int enqueue_stage(fft_ozaki_plan_s* p, int stage, hipStream_t s) {
  const int K = p->K, np = p->primes, count = (int)p->td.size();
  Range range(stage >= 1 && stage <= 8 ? kStageNames[stage] : "stage");
  // the plan's descriptor still holds the last execution's in / out
  const int dir = p->last_dir;
  switch (stage) {
    case 1:   // split: premultiply, maxima and the K extraction/check passes
    {
      HIPCHK(launch_reset_io(p->d_ts, p->d_tall, count, nullptr, nullptr, nullptr, s));
      int nmax = 0;
      for (auto& lc : p->classes) nmax = std::max(nmax, lc.nmax);
      HIPCHK(launch_premul(p->d_io, nullptr, p->d_td, p->d_kd, p->d_ts, p->d_tall, count, nmax, dir, false,
                           io32_of(p), s));
      HIPCHK(launch_split_plan(p->d_td, p->d_ts, p->d_kd, p->d_tall, count, K, s));
      for (int r = 0; r < K; ++r) {
        HIPCHK(launch_split_extract(p->d_io, p->d_kd, p->X, p->d_td, p->d_ts, p->d_tall, count, nmax, K, dir, false,
                                    io32_of(p), np, s));
        HIPCHK(launch_split_check(p->d_td, p->d_ts, p->d_tall, count, K, s));
      }
      return FFT_OZAKI_OK;
    }
    case 2:
      HIPCHK(launch_groups(p->d_td, p->d_ts, p->d_kd, p->d_tall, count, K, p->L, s));
      return FFT_OZAKI_OK;
    case 3:
    case 4:
    case 5:
      for (auto& lc : p->classes) {
        NttGeom g = lc.geom;
        if (stage != 3 && !g.two_pass()) continue;
        const bool rows_folded = fused_rows_ok(g, K);   // the forward rows run inside stage 6
        if (stage == 5 && rows_folded) continue;
        const int which = stage == 3 ? (rows_folded ? 1 : 0) : stage - 3;
        HIPCHK(launch_fwd_stage(p->X, p->d_td, p->d_ts, lc.d_tlist, (int)lc.tids.size(), K, np, false, 0, 2 * np * K, g,
                                p->tb, step_for(p, lc.logN), which, s));
      }
      return FFT_OZAKI_OK;
    case 6:
      for (auto& lc : p->classes)
        HIPCHK(launch_inv_stage(p->X, p->G, p->Z, p->d_td, p->d_ts, p->d_kd, lc.d_tlist, (int)lc.tids.size(), K, np, 0,
                                4 * K * K, lc.geom, p->tb, step_for(p, lc.logN), 1, s, fused_rows_ok(lc.geom, K)));
      return FFT_OZAKI_OK;
    case 7:   // column pass (fused with CRT and recombination where the length allows)
      for (auto& lc : p->classes) {
        const int cnt = (int)lc.tids.size();
        if (fused_cols_ok(lc.geom))
          HIPCHK(launch_inv_cols_rec(p->G, p->Z, p->d_io, p->d_td, p->d_ts, p->d_kd, lc.d_tlist, cnt, K, np, lc.geom,
                                     p->tb, dir, io32_of(p), s));
        else
          HIPCHK(launch_inv_stage(p->X, p->G, p->Z, p->d_td, p->d_ts, p->d_kd, lc.d_tlist, cnt, K, np, 0, 4 * K * K,
                                  lc.geom, p->tb, step_for(p, lc.logN), 2, s));
      }
      return FFT_OZAKI_OK;
    case 8:   // recombination (for fused lengths: the wide-accumulator fallback only)
      for (auto& lc : p->classes) {
        const int cnt = (int)lc.tids.size();
        if (fused_cols_ok(lc.geom)) {
          HIPCHK(launch_recombine_wide(p->Z, p->d_io, p->d_td, p->d_ts, p->d_kd, lc.d_tlist, cnt, lc.nmax, K, dir,
                                       io32_of(p), s, np));
        } else {
          HIPCHK(launch_recombine(p->Z, p->d_io, p->d_td, p->d_ts, p->d_kd, lc.d_tlist, cnt, lc.nmax, K, dir, io32_of(p),
                                  s, np));
        }
      }
      return FFT_OZAKI_OK;
    default:
      return fail(FFT_OZAKI_ERR_INVALID, "unknown stage");
  }
}

// --- allocation-free execution ---------------------------------------------
// One region of device memory reserved by the library itself (a static
// device array, one copy per device, held until the process ends) holds the
// tables and buffers of a default-options plan of the last (n, batch) seen on
// that device.  Host code reaches the region only through the device address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[FFT_OZAKI_STATIC_WORKSPACE_BYTES];
constexpr int STATIC_DEVICES = 64;
struct StaticSlot {
  void* ptr = nullptr;                 // this device's address of `scratch`
  DevArena arena;
  fft_ozaki_plan_s* plan = nullptr;    // host description of what the region holds
};
static std::mutex g_static_mu;
static StaticSlot g_static[STATIC_DEVICES];

// Upper bound of the region an arena plan of `batch` transforms of length n
// takes with the default options (K = L = 3, N = n for a power-of-two n, two
// moduli): the carves of build_plan and prepare_kernel, each counted with
// its largest alignment padding.
static size_t static_bytes(i64 n, i64 batch) {
  const int K = 3, np = 2;
  const int logN = conv_log2(n, true);
  const size_t N = (size_t)1 << logN, B = (size_t)batch;
  const bool two = ntt_geom(logN).two_pass();
  size_t b = 0;
  auto add = [&](size_t x) { b += (x ? x : 16) + 255; };
  for (int i = 0; i < 2 * NPRIME_MAX; ++i) add(sizeof(uint2) * (BLOCK_MAX / 2));
  if (two)
    for (int i = 0; i < 2 * NPRIME_MAX; ++i) {
      add(sizeof(uint2) * 4096);
      add(sizeof(uint2) * (N > 4096 ? N >> 12 : 1));
    }
  add(sizeof(double2) * (size_t)n);                        // chirp
  add(4 * (size_t)(2 * np * K) * N);                       // W
  add(4 * (size_t)(2 * np * K) * N);                       // Wq
  add(sizeof(int));                                        // split temporaries
  add(sizeof(TState));
  add(sizeof(TDesc));
  add(sizeof(KernelDesc));
  add(sizeof(int));
  const size_t SL = (size_t)K * K, zs = (size_t)((n + 3) & ~(i64)3);
  add(4 * ((size_t)(4 * K) << logN) * B);                  // slice spectra
  add(two ? 4 * ((8 * SL) << logN) * B : 0);               // group rows
  add(4 * 8 * SL * zs * B);                                // compact outputs
  add(sizeof(TDesc) * B);
  add(sizeof(TState) * B);
  add(sizeof(int) * B);
  add(sizeof(KernelDesc));
  add(sizeof(int) * B);                                    // the class's transform list
  add(sizeof(IoPtrs));                                     // execution descriptor
  return b;
}

// Global tables for the standalone NTT entry point, per device.
struct StdTables {
  TwBlock tb{};
  std::map<int, TwStep> steps;
};
static std::mutex g_std_mu;
static std::map<int, StdTables> g_std;

}  // namespace fo

using namespace fo;

extern "C" {

int fft_ozaki_default_options(fft_ozaki_options* opt) {
  if (!opt) return fail(FFT_OZAKI_ERR_INVALID, "opt is NULL");
  opt->K = 3;
  opt->L = 3;
  opt->mode = FFT_OZAKI_MODE_BATCHED;
  opt->autotune = 0;
  opt->tune_cache = nullptr;
  opt->embedding = FFT_OZAKI_EMBED_AUTO;
  opt->accumulation = FFT_OZAKI_ACCUM_COMPLEX;
  opt->precision = FFT_OZAKI_PREC_FP64;
  opt->primes = 2;
  return FFT_OZAKI_OK;
}

int fft_ozaki_plan_ex(fft_ozaki_plan_t* plan, const int64_t* lengths, int64_t count, const fft_ozaki_options* opt) {
  g_err.clear();
  if (!plan) return fail(FFT_OZAKI_ERR_INVALID, "plan is NULL");
  *plan = nullptr;
  if (!lengths || count < 1) return fail(FFT_OZAKI_ERR_INVALID, "need count >= 1 and a lengths array");
  if (count > (1 << 24)) return fail(FFT_OZAKI_ERR_INVALID, "too many transforms");
  fft_ozaki_options o;
  fft_ozaki_default_options(&o);
  if (opt) o = *opt;
  if (o.K < 1 || o.K > KMAX) return fail(FFT_OZAKI_ERR_INVALID, "K must be in [1, 8]");
  if (o.L < 1 || o.L > (1 << 20)) return fail(FFT_OZAKI_ERR_INVALID, "L must be in [1, 2^20]");
  if (o.mode != FFT_OZAKI_MODE_PLAIN && o.mode != FFT_OZAKI_MODE_BATCHED)
    return fail(FFT_OZAKI_ERR_INVALID, "mode must be 0 (plain) or 1 (batched)");
  if (o.embedding != FFT_OZAKI_EMBED_PADDED && o.embedding != FFT_OZAKI_EMBED_AUTO)
    return fail(FFT_OZAKI_ERR_INVALID, "embedding must be 0 (padded) or 1 (auto)");
  const bool cyclic = o.embedding == FFT_OZAKI_EMBED_AUTO;
  if (o.accumulation != FFT_OZAKI_ACCUM_PER_CONV && o.accumulation != FFT_OZAKI_ACCUM_COMPLEX)
    return fail(FFT_OZAKI_ERR_INVALID, "accumulation must be 0 (per convolution) or 1 (complex)");
  if (o.precision != FFT_OZAKI_PREC_FP64 && o.precision != FFT_OZAKI_PREC_FP32)
    return fail(FFT_OZAKI_ERR_INVALID, "precision must be 0 (binary64) or 1 (binary32)");
  if (o.primes != 2 && o.primes != 3) return fail(FFT_OZAKI_ERR_INVALID, "primes must be 2 or 3");
  if (o.primes == 3 && o.mode != FFT_OZAKI_MODE_BATCHED)
    return fail(FFT_OZAKI_ERR_UNSUPPORTED, "three moduli are served by the batched mode only");
  i64 total = 0;
  for (int64_t i = 0; i < count; ++i) {
    const i64 n = lengths[i];
    if (n < 1) return fail(FFT_OZAKI_ERR_INVALID, "lengths must be >= 1");
    if (conv_log2(n, cyclic) > MAX_LOG2_N) return fail(FFT_OZAKI_ERR_INVALID, "convolution length exceeds 2^24");
    const int a = alpha_for(n, o.L, o.primes);
    if (a < 1 || a > (o.primes == 3 ? 46 : 30))
      return fail(FFT_OZAKI_ERR_INVALID, "split width alpha < 1 for this n and L");
    total += n;
  }
  if (total > ((i64)1 << 31)) return fail(FFT_OZAKI_ERR_INVALID, "total length too large");
  fft_ozaki_plan_s* p = new (std::nothrow) fft_ozaki_plan_s();
  if (!p) return fail(FFT_OZAKI_ERR_NOMEM, "host allocation");
  p->K = o.K;
  p->L = o.L;
  p->mode = o.mode;
  p->autotune = o.autotune;
  p->cyclic = cyclic;
  p->accumulation = o.accumulation;
  p->precision = o.precision;
  p->primes = o.primes;
  p->tune_cache = o.tune_cache ? o.tune_cache : "";
  p->lengths.assign(lengths, lengths + count);
  int rc = build_plan(p);
  if (rc) {
    std::string keep = g_err;
    destroy_plan(p);
    g_err = keep;
    return rc;
  }
  *plan = p;
  return FFT_OZAKI_OK;
}

int fft_ozaki_plan(fft_ozaki_plan_t* plan, int64_t n, int64_t batch) {
  if (batch < 1) return fail(FFT_OZAKI_ERR_INVALID, "batch must be >= 1");
  if (batch > (1 << 24)) return fail(FFT_OZAKI_ERR_INVALID, "batch too large");
  std::vector<int64_t> l((size_t)batch, n);
  return fft_ozaki_plan_ex(plan, l.data(), batch, nullptr);
}

int fft_ozaki_execute(fft_ozaki_plan_t plan, const void* in, void* out, int direction, void* stream) {
  g_err.clear();
  if (!plan) return fail(FFT_OZAKI_ERR_INVALID, "plan is NULL");
  if (!in || !out) return fail(FFT_OZAKI_ERR_INVALID, "in/out is NULL");
  if (direction < 0 || direction > 2) return fail(FFT_OZAKI_ERR_INVALID, "direction must be 0, 1 or 2");
  if (((uintptr_t)in | (uintptr_t)out) & (plan->precision == FFT_OZAKI_PREC_FP32 ? 7 : 15))
    return fail(FFT_OZAKI_ERR_INVALID, "in/out must be aligned to their element size");
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  if (cur != plan->device) HIPCHK(hipSetDevice(plan->device));
  hipStream_t s = (hipStream_t)stream;
  plan->last_in = in;
  plan->last_out = out;
  plan->last_dir = direction;
  Range range(plan->mode == FFT_OZAKI_MODE_PLAIN ? "fft_ozaki_execute (plain)" : "fft_ozaki_execute (batched)");
  int rc = plan->mode == FFT_OZAKI_MODE_PLAIN ? run_plain(plan, in, out, direction, s)
                                              : run_batched(plan, in, out, direction, s);
  plan->timed_last = rc == FFT_OZAKI_OK && plan->stage_timing && plan->mode == FFT_OZAKI_MODE_BATCHED;
  if (cur != plan->device) (void)hipSetDevice(cur);
  return rc;
}

int fft_ozaki_forward(fft_ozaki_plan_t plan, const void* in, void* out, void* stream) {
  return fft_ozaki_execute(plan, in, out, FFT_OZAKI_FORWARD, stream);
}

int fft_ozaki_inverse(fft_ozaki_plan_t plan, const void* in, void* out, void* stream) {
  return fft_ozaki_execute(plan, in, out, FFT_OZAKI_INVERSE, stream);
}

int fft_ozaki_query(fft_ozaki_plan_t plan, fft_ozaki_info* info) {
  if (!plan || !info) return fail(FFT_OZAKI_ERR_INVALID, "plan/info is NULL");
  info->count = (int64_t)plan->td.size();
  info->total_length = plan->total;
  info->K = plan->K;
  info->L = plan->L;
  info->mode = plan->mode;
  info->num_length_classes = (int)plan->classes.size();
  info->workspace_bytes = plan->bytes;
  info->embedding = plan->cyclic ? FFT_OZAKI_EMBED_AUTO : FFT_OZAKI_EMBED_PADDED;
  info->accumulation = plan->accumulation;
  info->precision = plan->precision;
  info->primes = plan->primes;
  return FFT_OZAKI_OK;
}

int fft_ozaki_query_transform(fft_ozaki_plan_t plan, int64_t index, fft_ozaki_transform_info* info) {
  if (!plan || !info) return fail(FFT_OZAKI_ERR_INVALID, "plan/info is NULL");
  if (index < 0 || index >= (int64_t)plan->td.size()) return fail(FFT_OZAKI_ERR_INVALID, "index out of range");
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  HIPCHK(hipSetDevice(plan->device));
  HIPCHK(hipDeviceSynchronize());
  TState hs;
  HIPCHK(hipMemcpy(&hs, &plan->d_ts[index], sizeof hs, hipMemcpyDeviceToHost));
  (void)hipSetDevice(cur);
  const TDesc& d = plan->td[index];
  const KernelHost& kh = plan->kernels[d.kd];
  memset(info, 0, sizeof *info);
  info->n = d.n;
  info->N = d.N;
  info->alpha = d.alpha;
  info->status = hs.status;
  int fr = 0, fo_ = 0, iv = 0;
  for (int part = 0; part < 2; ++part) {
    info->kx[part] = hs.kx[part];
    info->kw[part] = kh.kw[part];
    for (int k = 0; k < 8; ++k) {
      info->Ex[part][k] = k < hs.kx[part] ? hs.E[part][k] : 0;
      info->Ew[part][k] = kh.Ew[part][k];
    }
    fr += plan->primes * hs.kx[part];
    fo_ += plan->primes * kh.kw[part];
  }
  for (int tg = 0; tg < 2; ++tg) {
    info->ngroups[tg] = hs.ngroups[tg];
    iv += plan->primes * hs.ngroups[tg];
  }
  info->acc_limit = d.acc_limit;
  info->xsh[0] = hs.xsh[0];
  info->xsh[1] = hs.xsh[1];
  info->forward_runtime = fr;
  info->forward_offline = fo_;
  info->inverse = iv;
  info->ntt_log2N1 = ntt_geom(d.logN).m1;
  for (auto& lc : plan->classes)
    if (lc.logN == d.logN) {
      info->tile_cols_log2 = lc.geom.lc;
      info->tile_rows_log2 = lc.geom.lrows;
    }
  return FFT_OZAKI_OK;
}

int fft_ozaki_debug_dump(fft_ozaki_plan_t plan, int stage, int64_t index, void* host_dst, size_t bytes,
                         size_t* needed) {
  if (!plan) return fail(FFT_OZAKI_ERR_INVALID, "plan is NULL");
  if (index < 0 || index >= (int64_t)plan->td.size()) return fail(FFT_OZAKI_ERR_INVALID, "index out of range");
  const TDesc& d = plan->td[index];
  const KernelHost& kh = plan->kernels[d.kd];
  const int K = plan->K, np = plan->primes;
  const void* src = nullptr;
  size_t sz = 0;
  switch (stage) {
    case 1: sz = sizeof(double2) * (size_t)d.n; break;   // recomputed below
    case 2: src = plan->X + d.X_off; sz = 4 * ((size_t)(2 * np * K) << d.logN); break;
    case 3: src = plan->Z + d.Z_off; sz = 4 * (size_t)(4 * K * K * np) * (size_t)d.zs; break;
    case 4: src = kh.W; sz = 4 * ((size_t)(2 * np * K) << d.logN); break;
    case 5: src = kh.chirp; sz = sizeof(double2) * (size_t)d.n; break;
    default: return fail(FFT_OZAKI_ERR_INVALID, "unknown stage");
  }
  if (needed) *needed = sz;
  if (!host_dst) return FFT_OZAKI_OK;
  if (bytes < sz) return fail(FFT_OZAKI_ERR_INVALID, "buffer too small");
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  HIPCHK(hipSetDevice(plan->device));
  HIPCHK(hipDeviceSynchronize());
  if (stage == 1) {
    // x' is not kept by the execution: recompute it from the last
    // execution's input, which must still hold the same values
    if (!plan->last_in) return fail(FFT_OZAKI_ERR_INVALID, "no execution to copy x' from");
    if (plan->last_in == plan->last_out)
      return fail(FFT_OZAKI_ERR_UNSUPPORTED, "x' is rebuilt from the input, which the in-place execution overwrote");
    if (!plan->xp) {     // a test hook's buffer: not part of the execution's workspace
      const hipError_t e = hipMalloc((void**)&plan->xp, sizeof(double2) * (size_t)plan->total);
      if (e != hipSuccess) return fail(FFT_OZAKI_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
      plan->allocs.push_back(plan->xp);
    }
    int nmax = 0;
    for (const TDesc& e : plan->td) nmax = std::max(nmax, e.n);
    HIPCHK(launch_premul(plan->d_io, plan->xp, plan->d_td, plan->d_kd, plan->d_ts, plan->d_tall, (int)plan->td.size(),
                         nmax, plan->last_dir, false, io32_of(plan), nullptr));
    HIPCHK(hipDeviceSynchronize());
    src = plan->xp + d.xp_off;
  }
  if (stage == 2 && plan->mode == FFT_OZAKI_MODE_BATCHED && plan->x_rows_pending) {
    // the batched form folds the forward row pass into the inverse row pass;
    // complete the stored slice spectra with it (once per execution)
    for (auto& lc : plan->classes) {
      if (!fused_rows_ok(lc.geom, K)) continue;
      HIPCHK(launch_fwd_stage(plan->X, plan->d_td, plan->d_ts, lc.d_tlist, (int)lc.tids.size(), K, np, false, 0,
                              2 * np * K, lc.geom, plan->tb, step_for(plan, lc.logN), 2, nullptr));
    }
    HIPCHK(hipDeviceSynchronize());
    plan->x_rows_pending = false;
  }
  if (stage == 3 && plan->mode == FFT_OZAKI_MODE_BATCHED) {
    // the fused column pass keeps the group residues in registers; rebuild
    // them for this transform's length class from the stored row-pass output
    for (auto& lc : plan->classes) {
      if (lc.logN != d.logN || !fused_cols_ok(lc.geom)) continue;
      HIPCHK(launch_inv_stage(plan->X, plan->G, plan->Z, plan->d_td, plan->d_ts, plan->d_kd, lc.d_tlist,
                              (int)lc.tids.size(), K, np, 0, 4 * K * K, lc.geom, plan->tb, step_for(plan, lc.logN), 2,
                              nullptr));
      HIPCHK(hipDeviceSynchronize());
    }
  }
  HIPCHK(hipMemcpy(host_dst, src, sz, hipMemcpyDeviceToHost));
  (void)hipSetDevice(cur);
  return FFT_OZAKI_OK;
}

int fft_ozaki_profile_stage(fft_ozaki_plan_t plan, int stage, int reps, void* stream) {
  g_err.clear();
  if (!plan) return fail(FFT_OZAKI_ERR_INVALID, "plan is NULL");
  if (plan->mode != FFT_OZAKI_MODE_BATCHED) return fail(FFT_OZAKI_ERR_INVALID, "stage profiling needs the batched mode");
  if (!plan->last_in) return fail(FFT_OZAKI_ERR_INVALID, "execute the plan once before profiling");
  if (reps < 1) return fail(FFT_OZAKI_ERR_INVALID, "reps must be >= 1");
  for (int r = 0; r < reps; ++r) {
    int rc = enqueue_stage(plan, stage, (hipStream_t)stream);
    if (rc) return rc;
  }
  return FFT_OZAKI_OK;
}

int fft_ozaki_stage_timing(fft_ozaki_plan_t plan, int enable) {
  g_err.clear();
  if (!plan) return fail(FFT_OZAKI_ERR_INVALID, "plan is NULL");
  if (plan->mode != FFT_OZAKI_MODE_BATCHED) return fail(FFT_OZAKI_ERR_INVALID, "stage timing needs the batched mode");
  const bool on = enable != 0;
  if (on == plan->stage_timing) return FFT_OZAKI_OK;
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  if (cur != plan->device) HIPCHK(hipSetDevice(plan->device));
  const size_t need = 2 + 4 * plan->classes.size();
  while (on && plan->tev.size() < need) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    plan->tev.push_back(e);
  }
  plan->stage_timing = on;
  plan->timed_last = false;
  if (cur != plan->device) (void)hipSetDevice(cur);
  return FFT_OZAKI_OK;
}

int fft_ozaki_stage_times(fft_ozaki_plan_t plan, float* ms, int capacity, int* count) {
  g_err.clear();
  if (!plan) return fail(FFT_OZAKI_ERR_INVALID, "plan is NULL");
  const int C = (int)plan->classes.size(), n = 1 + 4 * C;
  if (count) *count = n;
  if (!ms || capacity < n) return fail(FFT_OZAKI_ERR_INVALID, "times array too small (" + std::to_string(n) + " needed)");
  if (!plan->timed_last) return fail(FFT_OZAKI_ERR_INVALID, "the last execution recorded no stage times");
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  if (cur != plan->device) HIPCHK(hipSetDevice(plan->device));
  const std::vector<hipEvent_t>& e = plan->tev;
  HIPCHK(hipEventSynchronize(e[1 + 4 * (size_t)C]));
  auto span = [&](size_t a, size_t b, float* out) { return hipEventElapsedTime(out, e[a], e[b]); };
  HIPCHK(span(0, 1, &ms[0]));
  for (int c = 0; c < C; ++c) {
    const size_t f = 2 + c, r = 2 + C + 3 * (size_t)c;
    HIPCHK(span(c == 0 ? 1 : f - 1, f, &ms[1 + 4 * c]));                    // forward NTTs
    HIPCHK(span(c == 0 ? 1 + (size_t)C : r - 1, r, &ms[1 + 4 * c + 1]));   // inverse row pass
    HIPCHK(span(r, r + 1, &ms[1 + 4 * c + 2]));                           // inverse column pass
    HIPCHK(span(r + 1, r + 2, &ms[1 + 4 * c + 3]));                       // recombination
  }
  if (cur != plan->device) (void)hipSetDevice(cur);
  return FFT_OZAKI_OK;
}

int fft_ozaki_destroy(fft_ozaki_plan_t plan) {
  if (!plan) return fail(FFT_OZAKI_ERR_INVALID, "plan is NULL");
  destroy_plan(plan);
  return FFT_OZAKI_OK;
}

const char* fft_ozaki_error_string(int status) {
  switch (status) {
    case FFT_OZAKI_OK: return "success";
    case FFT_OZAKI_ERR_INVALID: return "invalid argument";
    case FFT_OZAKI_ERR_NOMEM: return "out of memory";
    case FFT_OZAKI_ERR_HIP: return "HIP runtime error";
    case FFT_OZAKI_ERR_UNSUPPORTED: return "unsupported request";
    default: return "unknown status";
  }
}

const char* fft_ozaki_last_error_message(void) { return g_err.c_str(); }

int fft_ozaki_ntt_layout(int log2N, int* log2N1) {
  if (log2N < 0 || log2N > MAX_LOG2_N || !log2N1) return fail(FFT_OZAKI_ERR_INVALID, "log2N out of range");
  *log2N1 = ntt_geom(log2N).m1;
  return FFT_OZAKI_OK;
}

int fft_ozaki_ntt(int prime, int log2N, int64_t count, void* data, int inverse, void* stream) {
  g_err.clear();
  if (prime < 0 || prime > 2) return fail(FFT_OZAKI_ERR_INVALID, "prime must be 0, 1 or 2");
  if (log2N < 0 || log2N > MAX_LOG2_N) return fail(FFT_OZAKI_ERR_INVALID, "log2N out of range");
  if (count < 0 || count > 65535) return fail(FFT_OZAKI_ERR_INVALID, "count must be in [0, 65535]");
  if (!data && count) return fail(FFT_OZAKI_ERR_INVALID, "data is NULL");
  if (count == 0) return FFT_OZAKI_OK;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  TwBlock tb;
  TwStep st{};
  {
    std::lock_guard<std::mutex> lk(g_std_mu);
    StdTables& T = g_std[dev];
    if (!T.tb.fwd[0]) {
      void* a[2 * NPRIME_MAX];
      if (build_block_twiddles(&T.tb, a)) return fail(FFT_OZAKI_ERR_NOMEM, "twiddle tables");
    }
    NttGeom g = ntt_geom(log2N);
    if (g.two_pass() && !T.steps.count(log2N)) {
      void* a[4 * NPRIME_MAX];
      TwStep s{};
      if (build_step_twiddles(log2N, &s, a)) return fail(FFT_OZAKI_ERR_NOMEM, "step twiddles");
      T.steps[log2N] = s;
    }
    tb = T.tb;
    if (g.two_pass()) st = T.steps[log2N];
  }
  HIPCHK(launch_ntt_standalone((u32*)data, log2N, prime, (int)count, inverse != 0, ntt_geom(log2N), tb, st,
                               (hipStream_t)stream));
  return FFT_OZAKI_OK;
}

int fft_ozaki_execute_static(int64_t n, int64_t batch, const void* in, void* out, int direction, void* stream) {
  g_err.clear();
  if (n < 1 || batch < 1) return fail(FFT_OZAKI_ERR_INVALID, "need n >= 1 and batch >= 1");
  if (n > (1 << 24) || batch > (1 << 24)) return fail(FFT_OZAKI_ERR_INVALID, "n or batch too large");
  if (!in || !out) return fail(FFT_OZAKI_ERR_INVALID, "in/out is NULL");
  if (direction < 0 || direction > 2) return fail(FFT_OZAKI_ERR_INVALID, "direction must be 0, 1 or 2");
  if (((uintptr_t)in | (uintptr_t)out) & 15) return fail(FFT_OZAKI_ERR_INVALID, "in/out must be 16-byte aligned");
  if (conv_log2(n, true) > MAX_LOG2_N) return fail(FFT_OZAKI_ERR_INVALID, "convolution length exceeds 2^24");
  if (alpha_for(n, 3) < 1) return fail(FFT_OZAKI_ERR_INVALID, "split width alpha < 1 for this n");
  const size_t need = static_bytes(n, batch);
  if (need > (size_t)FFT_OZAKI_STATIC_WORKSPACE_BYTES)
    return fail(FFT_OZAKI_ERR_INVALID, "n = " + std::to_string(n) + ", batch = " + std::to_string(batch) +
                                           " needs up to " + std::to_string(need) +
                                           " bytes of workspace; the static workspace holds " +
                                           std::to_string((size_t)FFT_OZAKI_STATIC_WORKSPACE_BYTES));
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= STATIC_DEVICES) return fail(FFT_OZAKI_ERR_UNSUPPORTED, "device index too large");
  std::lock_guard<std::mutex> lk(g_static_mu);
  StaticSlot& sl = g_static[dev];
  if (!sl.ptr) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(FFT_OZAKI_ERR_HIP, "hipGetSymbolAddress returned NULL");
    sl.ptr = ptr;
  }
  hipStream_t s = (hipStream_t)stream;
  fft_ozaki_plan_s* p = sl.plan;
  if (!p || p->lengths.size() != (size_t)batch || p->lengths[0] != n) {
    // the region holds another size's tables: rebuild them once the work
    // already queued on this stream (which may still read them) is done
    HIPCHK(hipStreamSynchronize(s));
    delete sl.plan;
    sl.plan = nullptr;
    p = new (std::nothrow) fft_ozaki_plan_s();
    if (!p) return fail(FFT_OZAKI_ERR_NOMEM, "host allocation");
    sl.arena = DevArena{};
    sl.arena.base = static_cast<char*>(sl.ptr);
    sl.arena.size = (size_t)FFT_OZAKI_STATIC_WORKSPACE_BYTES;
    p->arena = &sl.arena;
    p->lengths.assign((size_t)batch, n);
    const int rc = build_plan(p);
    if (rc) {
      delete p;
      return rc;
    }
    sl.plan = p;
  }
  return enqueue_batched(p, direction, s, in, out);
}

}  // extern "C"
