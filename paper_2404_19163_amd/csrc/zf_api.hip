// Host driver and C ABI of libzf (see include/zf.h).
//
// One call of zf_refine_ex runs
//   setup:   split / pad S, form Z0 (given or I/sqrt(g), g the Gershgorin bound)
//   phase L: low-precision sweeps under the stop test of Algorithm 2 (Sec. IV.A)
//   phase H: FP64 residual sweeps (Sec. IV.B, Algorithm 3), ratio-stopped in FP64
//   output:  Z (FP64, unpadded)
// A sweep is: residual evaluation (GEMM1 A^T = Z^T S, GEMM2 delta = I - Z^T A,
// both with Frobenius-norm partials) -> one double to the host -> stop test ->
// correction Q = sum_{k>=1} c_k delta^k (m - 1 symmetric GEMMs, Horner) ->
// GEMM4 Z_new = Z + Z Q into the other half of a ping-pong pair.
//
// All internal matrices are zero-padded to a multiple of the GEMM tile; the
// identity of delta = I - X is restricted to the valid block, so the padding
// stays exactly zero through every sweep (the zero padding of Sec. V.E without
// its singular pad block).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "zf.h"
#include "zf_index.h"
#include "zf_internal.h"

namespace zf {

static thread_local std::string g_err;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

void clear_error() { g_err.clear(); }

// ---------------------------------------------------------------------------
// tracing: JSON lines (ZF_LOG) and roctx ranges
// ---------------------------------------------------------------------------
static FILE* g_log = nullptr;
static std::string g_log_path;

bool log_on() {
  const char* v = getenv("ZF_LOG");
  if (!v || !*v || strcmp(v, "0") == 0) return false;
  if (strcmp(v, "1") == 0) {
    if (g_log && g_log != stderr) fclose(g_log);
    g_log = stderr;
    g_log_path.clear();
    return true;
  }
  if (g_log && g_log != stderr && g_log_path == v) return true;
  if (g_log && g_log != stderr) fclose(g_log);
  g_log = fopen(v, "a");
  g_log_path = g_log ? v : "";
  return g_log != nullptr;
}

void log_line(const char* fmt, ...) {
  if (!g_log) return;
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  fprintf(g_log, "{%s}\n", buf);
  fflush(g_log);
}

TraceRange::TraceRange(const char* name) { roctxRangePushA(name); }
void TraceRange::end() {
  if (live) roctxRangePop();
  live = false;
}

#define fail set_error

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess)                                                                   \
      return fail(ZF_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__,    \
                  __LINE__);                                                                \
  } while (0)

#define ZF_TRY(expr)        \
  do {                      \
    int _r = (expr);        \
    if (_r < 0) return _r;  \
  } while (0)

static int round_up(int n, int g) { return (n + g - 1) / g * g; }

// Padded order: a multiple of 256 from n = 1024 on (the 256-wide BF16x3 tiles), else
// of 128 (every kernel's minimum tile).
static int pad_order(int n) { return n >= 1024 ? round_up(n, 256) : round_up(n, kTile); }

// ---------------------------------------------------------------------------
// per-kernel timing (HIP events on the caller's stream)
// ---------------------------------------------------------------------------
enum KClass {
  K_X3 = 0, K_X3_SYM, K_F64, K_F64_SYM, K_HH, K_HH_SYM, K_F32, K_F32_SYM, K_X3F16, K_X3F16_SYM,
  K_HHF16, K_HHF16_SYM, K_OZ, K_OZ_SYM, K_CRT, K_CRT_SYM, K_COUNT
};
static const char* kClassName[K_COUNT] = {
    "gemm_x3", "gemm_x3_sym", "gemm_f64", "gemm_f64_sym", "gemm_hh", "gemm_hh_sym",
    "gemm_f32", "gemm_f32_sym", "gemm_x3f16", "gemm_x3f16_sym", "gemm_hhf16", "gemm_hhf16_sym",
    "gemm_oz", "gemm_oz_sym", "gemm_crt", "gemm_crt_sym"};

struct PendingEvent {
  hipEvent_t a, b;
  int cls;
  double flops;
  bool skip;  // a launch the stop test's gate turned into a no-op: not counted
};

struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<PendingEvent> pending;
  long long launches[K_COUNT] = {};
  double ms[K_COUNT] = {};
  double flops[K_COUNT] = {};
};
static Profiler g_prof;

static hipEvent_t take_event() {
  if (!g_prof.pool.empty()) {
    hipEvent_t e = g_prof.pool.back();
    g_prof.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Harvest finished events (the caller has synchronized the stream).
static void prof_harvest() {
  for (auto& p : g_prof.pending) {
    float t = 0.f;
    if (!p.skip && hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
      g_prof.launches[p.cls] += 1;
      g_prof.ms[p.cls] += t;
      g_prof.flops[p.cls] += p.flops;
    }
    g_prof.pool.push_back(p.a);
    g_prof.pool.push_back(p.b);
  }
  g_prof.pending.clear();
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
struct Workspace {
  int device = -1;
  int np = 0;
  bool has_x3 = false, has_f64 = false;
  std::vector<void*> allocs;
  // x3 operands (BF16 hi/lo pairs)
  u16 *s_hi = nullptr, *s_lo = nullptr;
  // Z's pair row-major (zr) and transposed (zc).  Every pair of the workspace is
  // K-blocked (kb_offset): a K step of a GEMM tile reads one contiguous run, and
  // the transposed epilogue writes one per strip.
  u16 *zr_hi[2] = {}, *zr_lo[2] = {}, *zc_hi[2] = {}, *zc_lo[2] = {};
  u16 *at_hi = nullptr, *at_lo = nullptr, *d_hi = nullptr, *d_lo = nullptr;
  u16 *q_hi = nullptr, *q_lo = nullptr, *u_hi = nullptr, *u_lo = nullptr;
  float* z32[2] = {};  // FP32 master Z, row-major (BF16 and FP32 arithmetic)
  // FP32 operands ("single", Table I)
  bool has_f32 = false;
  float *s32 = nullptr, *zc32[2] = {}, *a32t = nullptr, *dl32 = nullptr, *q32 = nullptr,
        *u32 = nullptr;
  // FP64
  double *s64 = nullptr, *z64r[2] = {}, *z64c[2] = {}, *a64t = nullptr, *d64 = nullptr;
  double *q64 = nullptr, *u64 = nullptr;
  // emulated FP64 (integer slices): planes of S, Z^T and A^T = Z^T S, row exponents
  bool has_oz = false;
  signed char *oz_s = nullptr, *oz_z = nullptr, *oz_a = nullptr;
  int *oz_es = nullptr, *oz_ez = nullptr, *oz_ea = nullptr;
  // emulated FP64 (residues): planes of S, Z^T and A^T, row exponents, product residues
  bool has_crt = false;
  signed char *cr_s = nullptr, *cr_z = nullptr, *cr_a = nullptr;
  int *cr_es = nullptr, *cr_ez = nullptr, *cr_ea = nullptr;
  unsigned char* cr_rho = nullptr;
  // scalars
  double *partials = nullptr, *err_dev = nullptr, *rowsum = nullptr, *g_dev = nullptr;
  double *gscr = nullptr, *cg = nullptr;  // learned-guess scratch (8192) and coefficients (8)
  float* feats = nullptr;
  double* host_err = nullptr;  // pinned
  // device-side stop test: the phase's gate (nonzero once it stopped), the previous
  // Err, and a ring of kBoxSlots {Err, decision} pairs the host reads (pinned, coherent,
  // written by the device; box_dev is its device address)
  int* gate = nullptr;
  double* prev_dev = nullptr;
  double *box = nullptr, *box_dev = nullptr;
};
constexpr int kBoxSlots = 8;

static Workspace g_ws;

static void ws_free(Workspace& w) {
  for (void* p : w.allocs) hipFree(p);
  w.allocs.clear();
  if (w.host_err) hipHostFree(w.host_err);
  if (w.box) hipHostFree(w.box);
  int dev = w.device;
  w = Workspace();
  w.device = dev;
}

template <typename T>
static int ws_alloc(Workspace& w, T** out, size_t elems) {
  void* p = nullptr;
  const char* inject = getenv("ZF_FAULT_INJECT");
  if (inject && strcmp(inject, "alloc") == 0)
    return fail(ZF_ERR_NOMEM, "allocation of %zu bytes refused (ZF_FAULT_INJECT=alloc)",
                elems * sizeof(T));
  hipError_t e = hipMalloc(&p, elems * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(ZF_ERR_NOMEM, "hipMalloc(%zu bytes): %s", elems * sizeof(T), hipGetErrorString(e));
  }
  w.allocs.push_back(p);
  *out = (T*)p;
  return 0;
}

// Allocate every buffer of a workspace for order np with the given parts.  On any
// failure the partly built workspace is freed again and the error returned.
static int ws_build(Workspace& w, int dev, int np, bool x3, bool f64, bool f32, bool oz,
                    bool crt) {
  w.device = dev;
  w.np = np;
  w.has_x3 = x3;
  w.has_f64 = f64;
  w.has_f32 = f32;
  w.has_oz = oz;
  w.has_crt = crt;
  const size_t m = (size_t)np * np;
  const int tiles = max_blocks(np, np);
  ZF_TRY(ws_alloc(w, &w.partials, tiles));
  ZF_TRY(ws_alloc(w, &w.err_dev, 8));
  ZF_TRY(ws_alloc(w, &w.rowsum, np));
  ZF_TRY(ws_alloc(w, &w.g_dev, 8));
  ZF_TRY(ws_alloc(w, &w.gscr, 8192));
  ZF_TRY(ws_alloc(w, &w.cg, 8));
  ZF_TRY(ws_alloc(w, &w.feats, 64));
  if (hipHostMalloc((void**)&w.host_err, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    w.host_err = nullptr;
    return fail(ZF_ERR_NOMEM, "hipHostMalloc of the pinned norm word failed");
  }
  ZF_TRY(ws_alloc(w, &w.gate, 2));
  ZF_TRY(ws_alloc(w, &w.prev_dev, 1));
  if (hipHostMalloc((void**)&w.box, 2 * kBoxSlots * sizeof(double),
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer((void**)&w.box_dev, w.box, 0) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ZF_ERR_NOMEM, "hipHostMalloc of the stop-test mailbox failed");
  }
  // the BF16 pairs of delta and Q and the row-major Z pair serve both phases
  ZF_TRY(ws_alloc(w, &w.d_hi, m));
  ZF_TRY(ws_alloc(w, &w.d_lo, m));
  ZF_TRY(ws_alloc(w, &w.q_hi, m));
  ZF_TRY(ws_alloc(w, &w.q_lo, m));
  ZF_TRY(ws_alloc(w, &w.u_hi, m));
  ZF_TRY(ws_alloc(w, &w.u_lo, m));
  for (int b = 0; b < 2; ++b) {
    ZF_TRY(ws_alloc(w, &w.zr_hi[b], m));
    ZF_TRY(ws_alloc(w, &w.zr_lo[b], m));
  }
  if (x3) {
    ZF_TRY(ws_alloc(w, &w.s_hi, m));
    ZF_TRY(ws_alloc(w, &w.s_lo, m));
    ZF_TRY(ws_alloc(w, &w.at_hi, m));
    ZF_TRY(ws_alloc(w, &w.at_lo, m));
    for (int b = 0; b < 2; ++b) {
      ZF_TRY(ws_alloc(w, &w.zc_hi[b], m));
      ZF_TRY(ws_alloc(w, &w.zc_lo[b], m));
    }
  }
  if (x3 || f32)
    for (int b = 0; b < 2; ++b) ZF_TRY(ws_alloc(w, &w.z32[b], m));
  if (f32) {
    ZF_TRY(ws_alloc(w, &w.s32, m));
    ZF_TRY(ws_alloc(w, &w.a32t, m));
    ZF_TRY(ws_alloc(w, &w.dl32, m));
    ZF_TRY(ws_alloc(w, &w.q32, m));
    ZF_TRY(ws_alloc(w, &w.u32, m));
    for (int b = 0; b < 2; ++b) ZF_TRY(ws_alloc(w, &w.zc32[b], m));
  }
  if (f64) {
    ZF_TRY(ws_alloc(w, &w.s64, m));
    ZF_TRY(ws_alloc(w, &w.a64t, m));
    ZF_TRY(ws_alloc(w, &w.d64, m));
    ZF_TRY(ws_alloc(w, &w.q64, m));
    ZF_TRY(ws_alloc(w, &w.u64, m));
    for (int b = 0; b < 2; ++b) {
      ZF_TRY(ws_alloc(w, &w.z64r[b], m));
      ZF_TRY(ws_alloc(w, &w.z64c[b], m));
    }
  }
  if (oz) {
    ZF_TRY(ws_alloc(w, &w.oz_s, m * kOzMaxSlices));
    ZF_TRY(ws_alloc(w, &w.oz_z, m * kOzMaxSlices));
    ZF_TRY(ws_alloc(w, &w.oz_a, m * kOzMaxSlices));
    ZF_TRY(ws_alloc(w, &w.oz_es, np));
    ZF_TRY(ws_alloc(w, &w.oz_ez, np));
    ZF_TRY(ws_alloc(w, &w.oz_ea, np));
  }
  if (crt) {
    ZF_TRY(ws_alloc(w, &w.cr_s, m * kCrtMaxModuli));
    ZF_TRY(ws_alloc(w, &w.cr_z, m * kCrtMaxModuli));
    ZF_TRY(ws_alloc(w, &w.cr_a, m * kCrtMaxModuli));
    ZF_TRY(ws_alloc(w, &w.cr_rho, m * kCrtMaxModuli));
    ZF_TRY(ws_alloc(w, &w.cr_es, np));
    ZF_TRY(ws_alloc(w, &w.cr_ez, np));
    ZF_TRY(ws_alloc(w, &w.cr_ea, np));
  }
  return 0;
}

// The cached workspace of the current device, grown (never shrunk) to order np and
// the requested parts.  The old buffers are released before the new ones are
// allocated (at large n both would not fit).  If an allocation fails, every buffer
// of the new workspace is released and the cache is left empty (np = 0, no parts),
// so the next call allocates afresh instead of reusing null pointers.
static int ws_get(int np, bool need_x3, bool need_f64, Workspace** out, bool need_f32 = false,
                  bool need_oz = false, bool need_crt = false) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  Workspace& w = g_ws;
  if (w.device != dev || w.np < np || (need_x3 && !w.has_x3) || (need_f64 && !w.has_f64) ||
      (need_f32 && !w.has_f32) || (need_oz && !w.has_oz) || (need_crt && !w.has_crt)) {
    const bool same = w.device == dev;
    const bool x3 = need_x3 || (same && w.has_x3);
    const bool f64 = need_f64 || (same && w.has_f64);
    const bool f32 = need_f32 || (same && w.has_f32);
    const bool oz = need_oz || (same && w.has_oz);
    const bool crt = need_crt || (same && w.has_crt);
    const int np_new = (same && w.np > np) ? w.np : np;
    ws_free(w);
    w.device = -1;
    Workspace nw;
    const int rc = ws_build(nw, dev, np_new, x3, f64, f32, oz, crt);
    if (rc < 0) {
      ws_free(nw);
      return rc;
    }
    w = nw;
  }
  *out = &w;
  return 0;
}

// ---------------------------------------------------------------------------
// GEMM wrappers (timing + flop accounting)
// ---------------------------------------------------------------------------
static EpiParams epi0(int np, int n_valid) {
  EpiParams e;
  memset(&e, 0, sizeof e);
  e.alpha = 0.0;
  e.beta = 1.0;
  e.gamma = 0.0;
  e.ld = np;
  e.n_valid = n_valid;
  e.kb = 1;  // the workspace's 16-bit pairs are K-blocked
  return e;
}

// Operands are workspace pairs (np x np), all in the K-blocked layout (kb_offset).
static int gemm_x3(const u16* Ah, const u16* Al, const u16* Bh, const u16* Bl, int np, bool sym,
                   const EpiParams& ep, hipStream_t st, int pm = PM_X3) {
  PendingEvent pe{};
  const bool prof = g_prof.on;
  if (prof) {
    static const int cls[4][2] = {{K_X3, K_X3_SYM}, {K_HH, K_HH_SYM}, {K_X3F16, K_X3F16_SYM},
                                  {K_HHF16, K_HHF16_SYM}};
    pe.a = take_event();
    pe.b = take_event();
    pe.cls = cls[pm][sym ? 1 : 0];
    // executed MFMA flops: 3 (or 1) products of 2 * tile^2 * K per launched tile
    const double t = (double)x3_tile_edge(np, np, sym);
    pe.flops = ((pm & PM_HH) ? 1.0 : 3.0) * 2.0 * (double)x3_blocks(np, np, sym) * t * t * (double)np;
    HIP_TRY(hipEventRecord(pe.a, st));
  }
  HIP_TRY(launch_gemm_x3(Ah, Al, 32, Bh, Bl, 32, np, np, np, sym, ep, st, pm, 32 * np, 32 * np));
  if (prof) {
    HIP_TRY(hipEventRecord(pe.b, st));
    g_prof.pending.push_back(pe);
  }
  return 0;
}

static int gemm_f32(const float* A, const float* B, int np, bool sym, const EpiParams& ep,
                    hipStream_t st) {
  PendingEvent pe{};
  const bool prof = g_prof.on;
  if (prof) {
    pe.a = take_event();
    pe.b = take_event();
    pe.cls = sym ? K_F32_SYM : K_F32;
    const double t = (double)f32_tile_edge(np, np, sym);
    pe.flops = 2.0 * (double)f32_blocks(np, np, sym) * t * t * (double)np;
    HIP_TRY(hipEventRecord(pe.a, st));
  }
  HIP_TRY(launch_gemm_f32(A, np, B, np, np, np, np, sym, ep, st));
  if (prof) {
    HIP_TRY(hipEventRecord(pe.b, st));
    g_prof.pending.push_back(pe);
  }
  return 0;
}

static int gemm_f64(const double* A, const double* B, int np, bool sym, const EpiParams& ep,
                    hipStream_t st) {
  PendingEvent pe{};
  const bool prof = g_prof.on;
  if (prof) {
    pe.a = take_event();
    pe.b = take_event();
    pe.cls = sym ? K_F64_SYM : K_F64;
    const double t = (double)f64_tile_edge(np, np, sym);
    pe.flops = 2.0 * (double)f64_blocks(np, np, sym) * t * t * (double)np;
    HIP_TRY(hipEventRecord(pe.a, st));
  }
  HIP_TRY(launch_gemm_f64(A, np, B, np, np, np, np, sym, ep, st));
  if (prof) {
    HIP_TRY(hipEventRecord(pe.b, st));
    g_prof.pending.push_back(pe);
  }
  return 0;
}

// Emulated FP64 product of two sliced matrices (s slices each).
static int gemm_oz(const signed char* A, const int* ea, const signed char* B, const int* eb,
                   int np, int s, bool sym, const EpiParams& ep, hipStream_t st) {
  PendingEvent pe{};
  const bool prof = g_prof.on;
  if (prof) {
    pe.a = take_event();
    pe.b = take_event();
    pe.cls = sym ? K_OZ_SYM : K_OZ;
    // executed int8 matrix-core operations: s (s + 1) / 2 slice products per tile
    const double t = (double)oz_tile_edge(np, sym);
    pe.flops = 0.5 * s * (s + 1) * 2.0 * (double)oz_blocks(np, sym) * t * t * (double)np;
    HIP_TRY(hipEventRecord(pe.a, st));
  }
  HIP_TRY(launch_gemm_oz(A, ea, B, eb, np, s, sym, ep, st));
  if (prof) {
    HIP_TRY(hipEventRecord(pe.b, st));
    g_prof.pending.push_back(pe);
  }
  return 0;
}

// Emulated FP64 product through residues (L moduli, K valid terms).
static int gemm_crt(const signed char* A, const int* ea, const signed char* B, const int* eb,
                    int np, int L, int K, bool sym, unsigned char* rho, const EpiParams& ep,
                    hipStream_t st) {
  PendingEvent pe{};
  const bool prof = g_prof.on;
  if (prof) {
    pe.a = take_event();
    pe.b = take_event();
    pe.cls = sym ? K_CRT_SYM : K_CRT;
    // executed int8 matrix-core operations: L products of 2 * 256^2 * np per launched tile
    const double t = np / 256;
    pe.flops = (double)L * 2.0 * (sym ? t * (t + 1) / 2 : t * t) * 65536.0 * (double)np;
    HIP_TRY(hipEventRecord(pe.a, st));
  }
  HIP_TRY(launch_crt_product(A, ea, B, eb, np, L, K, sym, rho, ep, st));
  if (prof) {
    HIP_TRY(hipEventRecord(pe.b, st));
    g_prof.pending.push_back(pe);
  }
  return 0;
}

// ---------------------------------------------------------------------------
// the sweep
// ---------------------------------------------------------------------------
// Arithmetic of a sweep's residual evaluation or correction: BF16 pairs with the
// (h)(h)+(h)(l)+(l)(h) scheme (X3) or the (h)(h) scheme (HH), FP32 ("single") or
// FP64 matrix-core GEMMs (Table I).
// AR_EMU: FP64 residual emulated with integer slices on the int8 matrix cores.
// AR_CRT: FP64 residual emulated through residues on the int8 matrix cores.
enum Arith { AR_X3 = 0, AR_HH, AR_F32, AR_F64, AR_X3F16, AR_HHF16, AR_EMU, AR_CRT };

static bool ar_pairs(Arith a) {
  return a == AR_X3 || a == AR_HH || a == AR_X3F16 || a == AR_HHF16;
}
static bool ar_f16(Arith a) { return a == AR_X3F16 || a == AR_HHF16; }
static int ar_pm(Arith a) {
  return a == AR_HH ? PM_HH : a == AR_X3F16 ? PM_X3F16 : a == AR_HHF16 ? PM_HHF16 : PM_X3;
}

struct Ctx {
  Workspace* w;
  int n, np, order;
  hipStream_t st;
  double c[8];      // c_k = C(2k,k)/4^k
  bool keep_pairs;  // FP32 updates also write the row-major BF16 pair (a later X3 correction)
  double sigma;     // power-of-two scale of the FP16 delta pairs (FP16 halves only)
  int oz_slices = 7;     // slices per operand of the emulated residual
  bool oz_s_ready = false;  // S's slices are in the workspace (once per call)
  int crt_moduli = 14;       // moduli of the residue-emulated residual
  bool crt_s_ready = false;  // S's residues are in the workspace (once per call)
  bool crt_first = false;    // only the refinement phase's first evaluation uses AR_CRT
  bool log = false;         // ZF_LOG: one JSON line per residual evaluation
};

static void series(int m, double* c) {
  // c_0 = 1, c_k = c_{k-1} (2k - 1) / (2k): the binomial series of (1 - d)^(-1/2)
  c[0] = 1.0;
  for (int k = 1; k <= m; ++k) c[k] = c[k - 1] * (2.0 * k - 1.0) / (2.0 * k);
}

// Frobenius norm from the partials of the last GEMM2 (count = its block count) -> host
static int fetch_err(Ctx& c, int count, double* err) {
  HIP_TRY(launch_norm_finalize(c.w->partials, count, c.w->err_dev, c.st));
  HIP_TRY(hipMemcpyAsync(c.w->host_err, c.w->err_dev, sizeof(double), hipMemcpyDeviceToHost, c.st));
  HIP_TRY(hipStreamSynchronize(c.st));
  *err = c.w->host_err[0];
  return 0;
}

// Residual products of Z[cur] in arithmetic `da`, leaving delta where the correction
// in arithmetic `ca` reads it (BF16 pair, FP32 or FP64) and its norm partials (their
// count in *blocks).  Every launch reads `gate` (nullptr: none).
static int delta_products(Ctx& c, Arith da, Arith ca, int cur, const int* gate, int* blocks_out) {
  Workspace& w = *c.w;
  const int np = c.np;
  EpiParams e1 = epi0(np, c.n), e2 = epi0(np, c.n);
  e1.gate = e2.gate = gate;
  e2.beta = -1.0;
  e2.gamma = 1.0;
  e2.partials = w.partials;
  if (ca != da && ar_pairs(ca)) {  // FP64 delta, BF16-pair correction
    e2.ohi = e2.othi = w.d_hi;
    e2.olo = e2.otlo = w.d_lo;
  }
  int blocks = 0;
  if (ar_pairs(da)) {
    const int pm = ar_pm(da);
    const int fmt = ar_f16(da) ? PAIR_F16 : PAIR_BF16;
    e1.ohi = w.at_hi;
    e1.olo = w.at_lo;
    e1.pair_fmt = fmt;
    ZF_TRY(gemm_x3(w.zc_hi[cur], w.zc_lo[cur], w.s_hi, w.s_lo, np, false, e1, c.st, pm));
    if (ar_f16(da)) {
      e2.o32 = e2.ot32 = w.dl32;
    } else {
      e2.ohi = e2.othi = w.d_hi;
      e2.olo = e2.otlo = w.d_lo;
    }
    ZF_TRY(gemm_x3(w.zc_hi[cur], w.zc_lo[cur], w.at_hi, w.at_lo, np, true, e2, c.st, pm));
    blocks = x3_blocks(np, np, true);
  } else if (da == AR_EMU) {  // A^T = Z^T S and Z^T A, both emulated, A^T kept in FP64
    const int s = c.oz_slices;
    if (!c.oz_s_ready) {
      HIP_TRY(launch_oz_slice(w.s64, np, s, w.oz_s, w.oz_es, c.st));
      c.oz_s_ready = true;
    }
    HIP_TRY(launch_oz_slice(w.z64c[cur], np, s, w.oz_z, w.oz_ez, c.st, gate));
    e1.o64 = w.a64t;
    ZF_TRY(gemm_oz(w.oz_z, w.oz_ez, w.oz_s, w.oz_es, np, s, false, e1, c.st));
    HIP_TRY(launch_oz_slice(w.a64t, np, s, w.oz_a, w.oz_ea, c.st, gate));
    e2.o64 = e2.ot64 = w.d64;
    ZF_TRY(gemm_oz(w.oz_z, w.oz_ez, w.oz_a, w.oz_ea, np, s, true, e2, c.st));
    blocks = oz_blocks(np, true);
  } else if (da == AR_CRT) {  // the same two products through residues, A^T kept in FP64
    const int L = c.crt_moduli;
    if (!c.crt_s_ready) {
      HIP_TRY(launch_crt_residues(w.s64, np, L, c.n, w.cr_s, w.cr_es, c.st));
      c.crt_s_ready = true;
    }
    HIP_TRY(launch_crt_residues(w.z64c[cur], np, L, c.n, w.cr_z, w.cr_ez, c.st, gate));
    e1.o64 = w.a64t;
    ZF_TRY(gemm_crt(w.cr_z, w.cr_ez, w.cr_s, w.cr_es, np, L, c.n, false, w.cr_rho, e1, c.st));
    HIP_TRY(launch_crt_residues(w.a64t, np, L, c.n, w.cr_a, w.cr_ea, c.st, gate));
    e2.o64 = e2.ot64 = w.d64;
    ZF_TRY(gemm_crt(w.cr_z, w.cr_ez, w.cr_a, w.cr_ea, np, L, c.n, true, w.cr_rho, e2, c.st));
    blocks = crt_blocks(np, true);
  } else if (da == AR_F32) {
    e1.o32 = w.a32t;
    ZF_TRY(gemm_f32(w.zc32[cur], w.s32, np, false, e1, c.st));
    e2.o32 = e2.ot32 = w.dl32;
    ZF_TRY(gemm_f32(w.zc32[cur], w.a32t, np, true, e2, c.st));
    blocks = f32_blocks(np, np, true);
  } else {
    e1.o64 = w.a64t;
    ZF_TRY(gemm_f64(w.z64c[cur], w.s64, np, false, e1, c.st));
    e2.o64 = e2.ot64 = w.d64;
    ZF_TRY(gemm_f64(w.z64c[cur], w.a64t, np, true, e2, c.st));
    blocks = f64_blocks(np, np, true);
  }
  *blocks_out = blocks;
  return 0;
}

// With FP16 halves delta is formed in FP32 and, once Err is known, split into FP16
// pairs of sigma * delta with sigma = 2^-floor(log2 Err) (|sigma delta_ij| <= 2:
// delta's entries fall below FP16's normal range as Z converges).
static int delta_f16_split(Ctx& c, Arith da, double err) {
  if (!ar_f16(da) || !isfinite(err)) return 0;
  Workspace& w = *c.w;
  c.sigma = (err > 0.0) ? ldexp(1.0, -(int)floor(log2(err))) : 1.0;
  HIP_TRY(launch_widen(w.dl32, c.np, nullptr, nullptr, c.st, nullptr, w.d_hi, w.d_lo, nullptr,
                       nullptr, (float)c.sigma, PAIR_F16));
  return 0;
}

// Residual evaluation of Z[cur] with Err returned to the host (one synchronization).
static int delta_eval(Ctx& c, Arith da, Arith ca, int cur, double* err) {
  int blocks = 0;
  ZF_TRY(delta_products(c, da, ca, cur, nullptr, &blocks));
  ZF_TRY(fetch_err(c, blocks, err));
  return delta_f16_split(c, da, *err);
}

// Q = sum_{k=1..m} c_k delta^k by Horner over symmetric GEMMs (m >= 2) in arithmetic
// `ca`; delta came from arithmetic `da` (its D term in the first Horner step is read
// from there).  Returns the buffer holding Q in the correction's representation.
struct QRef {
  const u16 *hi, *lo;
  const float* f32;
  const double* f64;
};

static int build_q(Ctx& c, Arith da, Arith ca, QRef* q, const int* gate) {
  Workspace& w = *c.w;
  const int np = c.np, m = c.order;
  const u16 *bh = w.d_hi, *bl = w.d_lo;
  const float* b32 = w.dl32;
  const double* b64 = w.d64;
  // FP16 halves carry sigma * Q: U~_k = c_k sigma delta + (1/sigma) delta~ U~_{k+1}
  const bool f16 = ar_f16(ca);
  const double sg = f16 ? c.sigma : 1.0;
  for (int k = m - 1; k >= 1; --k) {
    EpiParams e = epi0(np, c.n);
    e.gate = gate;
    e.alpha = c.c[k] * sg;
    e.beta = ((k == m - 1) ? c.c[m] : 1.0) / sg;
    if (da == AR_F64 || da == AR_EMU || da == AR_CRT) e.d64 = w.d64;
    else if (da == AR_F32 || f16) e.d32 = w.dl32;
    else {
      e.dhi = w.d_hi;
      e.dlo = w.d_lo;
    }
    const bool to_q = (k % 2) == 1;
    if (ar_pairs(ca)) {
      u16* oh = to_q ? w.q_hi : w.u_hi;
      u16* ol = to_q ? w.q_lo : w.u_lo;
      e.ohi = e.othi = oh;
      e.olo = e.otlo = ol;
      e.pair_fmt = f16 ? PAIR_F16 : PAIR_BF16;
      ZF_TRY(gemm_x3(w.d_hi, w.d_lo, bh, bl, np, true, e, c.st, ar_pm(ca)));
      bh = oh;
      bl = ol;
    } else if (ca == AR_F32) {
      float* o = to_q ? w.q32 : w.u32;
      e.o32 = e.ot32 = o;
      ZF_TRY(gemm_f32(w.dl32, b32, np, true, e, c.st));
      b32 = o;
    } else {
      double* o = to_q ? w.q64 : w.u64;
      e.o64 = e.ot64 = o;
      ZF_TRY(gemm_f64(w.d64, b64, np, true, e, c.st));
      b64 = o;
    }
  }
  q->hi = bh;
  q->lo = bl;
  q->f32 = b32;
  q->f64 = b64;
  return 0;
}

// Z[cur] -> Z[cur ^ 1] = Z + Z Q, Q in arithmetic `ca`; the master Z is FP64 when
// `high` (refinement phase after an FP64 residual), else FP32.  Every launch reads
// `gate` (nullptr: none).
static int update(Ctx& c, Arith da, Arith ca, bool high, int cur, const int* gate) {
  Workspace& w = *c.w;
  const int np = c.np, nxt = cur ^ 1;
  QRef q{w.d_hi, w.d_lo, w.dl32, w.d64};
  double beta = 1.0;
  if (c.order == 1) beta = c.c[1];  // Q = c_1 delta: fold the scale into GEMM4
  else ZF_TRY(build_q(c, da, ca, &q, gate));
  if (ar_f16(ca)) beta /= c.sigma;  // the pairs hold sigma * Q
  EpiParams e = epi0(np, c.n);
  e.gate = gate;
  e.alpha = 1.0;
  e.beta = beta;
  e.pair_fmt = ar_f16(ca) ? PAIR_F16 : PAIR_BF16;
  if (high) {  // FP64 master
    e.d64 = w.z64r[cur];
    e.o64 = w.z64r[nxt];
    e.ot64 = w.z64c[nxt];
    if (ar_pairs(ca)) {
      e.ohi = w.zr_hi[nxt];
      e.olo = w.zr_lo[nxt];
      return gemm_x3(w.zr_hi[cur], w.zr_lo[cur], q.hi, q.lo, np, false, e, c.st, ar_pm(ca));
    }
    return gemm_f64(w.z64r[cur], q.f64, np, false, e, c.st);
  }
  e.d32 = w.z32[cur];
  e.o32 = w.z32[nxt];
  if (ar_pairs(ca)) {
    e.ohi = w.zr_hi[nxt];
    e.olo = w.zr_lo[nxt];
    e.othi = w.zc_hi[nxt];
    e.otlo = w.zc_lo[nxt];
    return gemm_x3(w.zr_hi[cur], w.zr_lo[cur], q.hi, q.lo, np, false, e, c.st, ar_pm(ca));
  }
  e.ot32 = w.zc32[nxt];
  if (c.keep_pairs) {
    e.ohi = w.zr_hi[nxt];
    e.olo = w.zr_lo[nxt];
  }
  return gemm_f32(w.z32[cur], q.f32, np, false, e, c.st);
}

struct PhaseOut {
  int updates = 0;   // updates contained in the chosen iterate
  int evals = 0;
  double err = 0.0;  // Err of the chosen iterate
  bool capped = false;
};

// One phase of Algorithm 2: evaluate, stop test, update, ping-pong.  The stop test
// runs on the device (launch_norm_decide) and the host queues one sweep ahead: the
// update of sweep it and the evaluation of sweep it + 1 are launched before the host
// reads sweep it's decision, and if that decision was to stop, the gate it set makes
// every one of those launches return at once (the buffer of the previous iterate is
// therefore never overwritten).  The GPU thus never waits for the host between
// sweeps.  With FP16 halves the next products need Err on the host (the scale of
// delta's split), so that phase reads each decision before it goes on.
static int run_phase(Ctx& c, Arith da, Arith ca, bool high, int stop_rule, int max_updates,
                     int& cur, std::vector<double>& hist, PhaseOut& out) {
  static const char* kName[8] = {"BF16x3", "BF16", "FP32",          "FP64",
                                 "FP16x3", "FP16", "emulated FP64", "residue-emulated FP64"};
  TraceRange phase_range(high ? "zf.phase_high" : "zf.phase_low");
  Workspace& w = *c.w;
  const bool ahead = !ar_f16(da);
  const int pw = c.order + 1;
  auto eval_arith = [&](int it) { return (high && it == 0 && c.crt_first) ? AR_CRT : da; };
  // residual products of sweep it on buffer b, then its device-side stop test
  auto enqueue_eval = [&](int it, int b) -> int {
    TraceRange r("zf.residual_eval");
    int blocks = 0;
    ZF_TRY(delta_products(c, eval_arith(it), ca, b, w.gate, &blocks));
    HIP_TRY(launch_norm_decide(w.partials, blocks, it, stop_rule == ZF_STOP_MONOTONE ? 1 : 0, pw,
                               w.gate, w.prev_dev, w.box_dev + 2 * (it % kBoxSlots), c.st));
    return 0;
  };
  HIP_TRY(hipMemsetAsync(w.gate, 0, sizeof(int), c.st));
  hipEvent_t ev[2] = {nullptr, nullptr};
  HIP_TRY(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  if (hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return fail(ZF_ERR_HIP, "hipEventCreate failed");
  }
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      (void)hipEventDestroy(e[0]);
      (void)hipEventDestroy(e[1]);
    }
  } guard{ev};
  double prev = 0.0;
  ZF_TRY(enqueue_eval(0, cur));
  HIP_TRY(hipEventRecord(ev[0], c.st));
  for (int it = 0;; ++it) {
    const bool capped = it >= max_updates;
    const size_t spec = g_prof.pending.size();  // timed launches queued ahead start here
    if (ahead && !capped) {  // queued before the decision of sweep it is known
      TraceRange r("zf.update");
      ZF_TRY(update(c, da, ca, high, cur, w.gate));
      ZF_TRY(enqueue_eval(it + 1, cur ^ 1));
      HIP_TRY(hipEventRecord(ev[(it + 1) & 1], c.st));
    }
    HIP_TRY(hipEventSynchronize(ev[it & 1]));
    const volatile double* box = w.box + 2 * (it % kBoxSlots);
    const double err = box[0];
    const int code = (int)box[1];
    out.evals++;
    hist.push_back(err);
    if (c.log)
      log_line("\"event\": \"eval\", \"n\": %d, \"arith\": \"%s\", \"phase\": \"%s\", \"it\": %d, "
               "\"err_f\": %.17g, \"rms\": %.6e, \"stop\": %s",
               c.n, kName[eval_arith(it)], high ? "high" : "low", it, err, err / sqrt((double)c.n),
               code == 1 ? "true" : "false");
    if (code != 0)  // the launches queued ahead were gated off
      for (size_t k = spec; k < g_prof.pending.size(); ++k) g_prof.pending[k].skip = true;
    if (code == 2)
      return fail(ZF_ERR_NONFINITE, "residual norm is not finite at %s sweep %d", kName[da], it);
    if (code == 1) {
      if (err > prev) {  // the previous iterate is still in the other buffer
        cur ^= 1;
        out.updates = it - 1;
        out.err = prev;
      } else {
        out.updates = it;
        out.err = err;
      }
      return 0;
    }
    if (capped) {
      out.updates = it;
      out.err = err;
      out.capped = true;
      return 0;
    }
    if (!ahead) {  // FP16 halves: delta's scaled split, then the update and next evaluation
      ZF_TRY(delta_f16_split(c, eval_arith(it), err));
      TraceRange r("zf.update");
      ZF_TRY(update(c, da, ca, high, cur, w.gate));
      ZF_TRY(enqueue_eval(it + 1, cur ^ 1));
      HIP_TRY(hipEventRecord(ev[(it + 1) & 1], c.st));
    }
    cur ^= 1;
    prev = err;
  }
}

// Learned guess into buffer 0 (every layout the first phase reads): S^2 by the
// symmetric matrix-core GEMM (BF16x3 when the BF16 pairs of S exist, else FP64),
// features, network, acceptance on the host.  Returns 1 when the guess was written,
// 0 to fall back to the scaled identity.  mixed: write the FP32 master and the BF16
// pairs; use_h: write the FP64 master.
static int learned_guess(Ctx& c, const double* S, bool mixed, bool use_h, bool pairs, int pm,
                         hipStream_t st) {
  Workspace& w = *c.w;
  const int n = c.n, np = c.np;
  if (!net_ready()) return 0;
  const double* S2d = nullptr;
  const float* S2f = nullptr;
  if (pairs) {  // BF16x3 S^2 into the second FP32 master (free until the first update)
    EpiParams e = epi0(np, n);
    e.o32 = e.ot32 = w.z32[1];
    ZF_TRY(gemm_x3(w.s_hi, w.s_lo, w.s_hi, w.s_lo, np, true, e, st, pm));
    S2f = w.z32[1];
  } else {  // FP64 S^2 into A^T's buffer (free until the first residual)
    EpiParams e = epi0(np, n);
    e.o64 = e.ot64 = w.a64t;
    ZF_TRY(gemm_f64(w.s64, w.s64, np, true, e, st));
    S2d = w.a64t;
  }
  ZF_TRY(guess_features(S, n, S2d, S2f, np, w.s64, w.feats, w.gscr, st));
  ZF_TRY(guess_infer(w.feats, w.cg, st));
  double hv[8];
  HIP_TRY(hipMemcpyAsync(hv, w.cg, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(hv + 3, w.gscr, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double cf[3] = {hv[0], hv[1], hv[2]};
  const double g = hv[3], glo = hv[4];
  if (!(g > 0.0) || !isfinite(cf[0]) || !isfinite(cf[1]) || !isfinite(cf[2])) return 0;
  if (!guess_accept(cf, glo > 0.0 ? glo / g : 0.0)) return 0;
  double cgh[4] = {cf[0], cf[1], cf[2], g};
  HIP_TRY(hipMemcpyAsync(w.cg + 4, cgh, sizeof cgh, hipMemcpyHostToDevice, st));
  HIP_TRY(launch_guess_write(S, n, S2d, S2f, np, w.cg + 4, mixed ? w.z32[0] : nullptr,
                             use_h ? w.z64r[0] : nullptr, use_h ? w.z64c[0] : nullptr, w.zr_hi[0],
                             w.zr_lo[0], pairs ? w.zc_hi[0] : nullptr, pairs ? w.zc_lo[0] : nullptr,
                             st));
  // the host copy cgh must outlive the asynchronous copy
  HIP_TRY(hipStreamSynchronize(st));
  return 1;
}

// Slices per operand of the emulated residual: 7 (56 bits; the product's error is
// below 8 2^-49 K 2^{e_i + f_j}); ZF_EMU_SLICES (3..8) overrides (tuning).
static int oz_slices_env() {
  const char* env = getenv("ZF_EMU_SLICES");
  const int v = env ? atoi(env) : 7;
  return (v >= 3 && v <= kOzMaxSlices) ? v : 7;
}

// Moduli of the residue-emulated residual: 14 (beta = 48 at K = 4096, 47 at 16384);
// ZF_EMU_MODULI (8..15) overrides (tuning).
static int crt_moduli_env() {
  const char* env = getenv("ZF_EMU_MODULI");
  const int v = env ? atoi(env) : 14;
  return (v >= 8 && v <= kCrtMaxModuli) ? v : 14;
}

static int refine_core(const double* S, const double* Z0, int n, const zf_opts& o, double* Z,
                       zf_result* res, double* hist, int hist_cap, hipStream_t st, bool log) {
  if (!S || !Z) return fail(ZF_ERR_ARG, "S and Z must be non-NULL device pointers");
  if (n <= 0) return fail(ZF_ERR_ARG, "n must be >= 1 (got %d)", n);
  if (o.order < 1 || o.order > 5) return fail(ZF_ERR_ARG, "order must be in 1..5 (got %d)", o.order);
  if (o.precision < ZF_FP64 || o.precision > ZF_FP16)
    return fail(ZF_ERR_ARG, "precision %d is not supported", o.precision);
  if (o.stop != ZF_STOP_RATIO && o.stop != ZF_STOP_MONOTONE)
    return fail(ZF_ERR_ARG, "unknown stop rule %d", o.stop);
  if (o.refine < ZF_REFINE_OFF || o.refine > ZF_REFINE_CRT_FIRST)
    return fail(ZF_ERR_ARG, "unknown refine mode %d", o.refine);
  if (o.refine == ZF_REFINE_EMU && o.precision != ZF_FP64 && pad_order(n) > kOzMaxOrder)
    return fail(ZF_ERR_ARG, "the emulated FP64 residual supports n <= %d (got %d)", kOzMaxOrder, n);
  const bool crt_mode = o.precision != ZF_FP64 &&
                        (o.refine == ZF_REFINE_CRT || o.refine == ZF_REFINE_CRT_FIRST);
  if (crt_mode && round_up(n, 256) > kCrtMaxOrder)
    return fail(ZF_ERR_ARG, "the residue-emulated residual supports n <= %d (got %d)",
                kCrtMaxOrder, n);
  if (hist_cap < 0 || (hist_cap > 0 && !hist)) return fail(ZF_ERR_ARG, "bad hist buffer");
  if (n > 46000) return fail(ZF_ERR_ARG, "n = %d exceeds the supported maximum 46000", n);
  if (o.z0 != ZF_Z0_GIVEN && o.z0 != ZF_Z0_SCALED_IDENTITY && o.z0 != ZF_Z0_LEARNED)
    return fail(ZF_ERR_ARG, "unknown guess kind %d", o.z0);
  if (o.z0 == ZF_Z0_GIVEN && !Z0) return fail(ZF_ERR_ARG, "opts.z0 = ZF_Z0_GIVEN needs a Z0");

  // arithmetic of the two phases (Table I): the first phase in the requested
  // precision; the refinement phase (Sec. IV.B) with an FP64 residual and a BF16x3
  // (F64_DELTA) or FP64 (F64_FULL) correction, or entirely in FP32 (F32)
  const bool fp64_only = o.precision == ZF_FP64;
  const Arith la = fp64_only ? AR_F64
                   : o.precision == ZF_BF16X3 ? AR_X3
                   : o.precision == ZF_BF16   ? AR_HH
                   : o.precision == ZF_FP16X3 ? AR_X3F16
                   : o.precision == ZF_FP16   ? AR_HHF16
                                              : AR_F32;
  const bool refine = !fp64_only && o.refine != ZF_REFINE_OFF;
  const Arith hd = o.refine == ZF_REFINE_F32   ? AR_F32
                   : o.refine == ZF_REFINE_EMU ? AR_EMU
                   : o.refine == ZF_REFINE_CRT ? AR_CRT
                                               : AR_F64;  // CRT_FIRST: AR_CRT on the first only
  const Arith hc = (o.refine == ZF_REFINE_F64_DELTA || o.refine == ZF_REFINE_EMU || crt_mode)
                       ? AR_X3
                       : hd;
  const bool high = refine && (hd == AR_F64 || hd == AR_EMU || hd == AR_CRT);  // FP64 master
  const bool learned = !Z0 && o.z0 == ZF_Z0_LEARNED;
  const bool need_pairs = ar_pairs(la) || (refine && ar_pairs(hc));
  const bool need_f32 = la == AR_F32 || ar_f16(la) || (refine && hd == AR_F32);
  const bool use_h = fp64_only || high;
  const bool mixed = !fp64_only;  // FP32 master Z in the first phase
  const bool s_pairs = ar_pairs(la);
  // the residue products run 256-wide tiles only
  const int np = crt_mode ? round_up(n, 256) : pad_order(n);
  Workspace* w = nullptr;
  ZF_TRY(ws_get(np, need_pairs, use_h || learned, &w, need_f32, refine && hd == AR_EMU,
                crt_mode));

  Ctx c;
  c.w = w;
  c.n = n;
  c.np = np;
  c.order = o.order;
  c.st = st;
  c.keep_pairs = la == AR_F32 && refine && ar_pairs(hc);
  c.sigma = 1.0;
  c.oz_slices = oz_slices_env();
  c.oz_s_ready = false;
  c.crt_moduli = crt_moduli_env();
  c.crt_s_ready = false;
  c.crt_first = o.refine == ZF_REFINE_CRT_FIRST;
  c.log = log;
  const int s_fmt = ar_f16(la) ? 2 : 1;  // split format of S: FP16 or BF16 halves
  series(o.order, c.c);
  const int max_l = o.max_sweeps > 0 ? o.max_sweeps : 100;
  const int max_h = o.max_refine > 0 ? o.max_refine : 10;

  // setup: operands of S, then Z0
  TraceRange setup_range("zf.setup");
  HIP_TRY(launch_split_pad(S, n, n, np, s_pairs ? w->s_hi : nullptr, s_pairs ? w->s_lo : nullptr,
                           (use_h || learned) ? w->s64 : nullptr,
                           need_f32 ? w->s32 : nullptr, false, s_fmt, st));
  int z0_used = Z0 ? ZF_Z0_GIVEN : ZF_Z0_SCALED_IDENTITY;
  int guess_flags = 0;
  if (learned) {
    int lr = learned_guess(c, S, mixed, fp64_only, s_pairs, ar_pm(la), st);
    if (lr < 0) return lr;
    if (lr == 1) z0_used = ZF_Z0_LEARNED;
    else guess_flags |= ZF_WARN_Z0_FALLBACK;
  }
  if (Z0) {
    HIP_TRY(launch_init_given(Z0, n, np, mixed ? w->z32[0] : nullptr,
                              fp64_only ? w->z64r[0] : nullptr, fp64_only ? w->z64c[0] : nullptr,
                              w->zr_hi[0], w->zr_lo[0], s_pairs ? w->zc_hi[0] : nullptr,
                              s_pairs ? w->zc_lo[0] : nullptr, st));
  } else if (z0_used == ZF_Z0_LEARNED) {
    // written by learned_guess
  } else {
    HIP_TRY(launch_row_abs_max(S, n, n, w->rowsum, w->g_dev, st));
    HIP_TRY(launch_init_identity(w->g_dev, n, np, mixed ? w->z32[0] : nullptr,
                                 fp64_only ? w->z64r[0] : nullptr,
                                 fp64_only ? w->z64c[0] : nullptr, w->zr_hi[0], w->zr_lo[0],
                                 s_pairs ? w->zc_hi[0] : nullptr, s_pairs ? w->zc_lo[0] : nullptr,
                                 st));
  }
  if (la == AR_F32) HIP_TRY(launch_widen(w->z32[0], np, nullptr, nullptr, st, w->zc32[0]));
  if (ar_f16(la))  // the initializers write BF16 pairs; the FP16 halves replace them
    HIP_TRY(launch_widen(w->z32[0], np, nullptr, nullptr, st, nullptr, w->zr_hi[0], w->zr_lo[0],
                         w->zc_hi[0], w->zc_lo[0], 1.0f, PAIR_F16));
  setup_range.end();

  std::vector<double> h;
  int cur = 0;
  PhaseOut pl, ph;
  int flags = guess_flags;
  int rc = 0;
  if (mixed) {
    rc = run_phase(c, la, la, false, o.stop, max_l, cur, h, pl);
    if (rc < 0) goto done;
    if (pl.capped) flags |= ZF_WARN_MAXSWEEPS;
    if (refine) {
      // Algorithm 3: Z into the refinement arithmetic, then its own ratio-stopped loop
      // (a BF16x3 correction after FP16 halves needs Z's BF16 pair too)
      const bool bf16_pairs = ar_pairs(hc) && ar_f16(la);
      if (high)
        HIP_TRY(launch_widen(w->z32[cur], np, w->z64r[cur], w->z64c[cur], st, nullptr,
                             bf16_pairs ? w->zr_hi[cur] : nullptr,
                             bf16_pairs ? w->zr_lo[cur] : nullptr, nullptr, nullptr, 1.0f,
                             PAIR_BF16));
      else if (la != AR_F32) HIP_TRY(launch_widen(w->z32[cur], np, nullptr, nullptr, st, w->zc32[cur]));
      rc = run_phase(c, hd, hc, high, o.stop, max_h, cur, h, ph);
      if (rc < 0) goto done;
      if (ph.capped) flags |= ZF_WARN_MAXSWEEPS;
    }
  } else {
    rc = run_phase(c, AR_F64, AR_F64, true, o.stop, max_l, cur, h, ph);
    if (rc < 0) goto done;
    if (ph.capped) flags |= ZF_WARN_MAXSWEEPS;
  }
  if (use_h) HIP_TRY(launch_unpad_f64(w->z64r[cur], np, n, Z, st));
  else HIP_TRY(launch_unpad_f32(w->z32[cur], np, n, Z, st));
  HIP_TRY(hipStreamSynchronize(st));

done:
  if (g_prof.on) prof_harvest();
  {
    const int len = (int)h.size() < hist_cap ? (int)h.size() : hist_cap;
    for (int i = 0; i < len; ++i) hist[i] = h[i];
    if ((int)h.size() > hist_cap && hist_cap >= 0 && rc >= 0) flags |= ZF_WARN_HIST_TRUNC;
    if (res) {
      res->iters = pl.updates + ph.updates;
      res->low_evals = pl.evals;
      res->high_evals = ph.evals;
      res->hist_len = len;
      res->flags = flags;
      res->final_err = (fp64_only || refine) ? ph.err : pl.err;
      res->final_rms = res->final_err / sqrt((double)n);
      res->status = rc < 0 ? rc : 0;
      res->z0_used = z0_used;
    }
  }
  if (rc < 0) return rc;
  const double fe = (fp64_only || refine) ? ph.err : pl.err;
  if (!(fe < 1.0)) {
    if (res) res->status = ZF_ERR_NOT_CONVERGED;
    return fail(ZF_ERR_NOT_CONVERGED,
                "||Z^T S Z - I||_F = %g >= 1: the guess violates ||X0 - I||_2 < 1 or S is not SPD",
                fe);
  }
  g_err.clear();
  return flags;
}

// refine_core under a roctx range, with one ZF_LOG line for the call's result.
static int refine_impl(const double* S, const double* Z0, int n, const zf_opts& o, double* Z,
                       zf_result* res, double* hist, int hist_cap, hipStream_t st) {
  TraceRange range("zf_refine");
  const bool log = log_on();
  zf_result r;
  memset(&r, 0, sizeof r);
  const auto t0 = std::chrono::steady_clock::now();
  const int rc = refine_core(S, Z0, n, o, Z, &r, hist, hist_cap, st, log);
  if (res) *res = r;
  if (log) {
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    log_line("\"event\": \"refine\", \"n\": %d, \"order\": %d, \"precision\": %d, \"refine\": %d, "
             "\"stop\": %d, \"rc\": %d, \"iters\": %d, \"low_evals\": %d, \"high_evals\": %d, "
             "\"final_rms\": %.6e, \"z0_used\": %d, \"flags\": %d, \"ms\": %.3f",
             n, o.order, o.precision, o.refine, o.stop, rc, r.iters, r.low_evals, r.high_evals,
             r.final_rms, r.z0_used, r.flags, ms);
  }
  return rc;
}

}  // namespace zf

using namespace zf;

extern "C" {

void zf_default_opts(zf_opts* o) {
  if (!o) return;
  o->order = 2;
  o->precision = ZF_BF16X3;
  o->stop = ZF_STOP_RATIO;
  o->max_sweeps = 100;
  o->refine = ZF_REFINE_F64_DELTA;
  o->max_refine = 10;
  o->z0 = ZF_Z0_SCALED_IDENTITY;
}

int zf_refine_ex(const double* S, const double* Z0, int n, const zf_opts* opts, double* Z,
                 zf_result* res, double* hist, int hist_cap, void* stream) {
  zf_opts o;
  zf_default_opts(&o);
  if (opts) o = *opts;
  return refine_impl(S, Z0, n, o, Z, res, hist, hist_cap, (hipStream_t)stream);
}

int zf_refine(const double* S, const double* Z0, int n, int order, int precision, double* Z,
              int* iters, double* hist, int hist_cap, int* hist_len, void* stream) {
  zf_opts o;
  zf_default_opts(&o);
  o.order = order;
  o.precision = precision;
  zf_result r;
  memset(&r, 0, sizeof r);
  const int rc = refine_impl(S, Z0, n, o, Z, &r, hist, hist_cap, (hipStream_t)stream);
  if (iters) *iters = r.iters;
  if (hist_len) *hist_len = r.hist_len;
  return rc;
}

int zf_residual(const double* S, const double* Z, int n, double* rms, void* stream) {
  if (!S || !Z || !rms) return fail(ZF_ERR_ARG, "NULL argument");
  if (n <= 0) return fail(ZF_ERR_ARG, "n must be >= 1 (got %d)", n);
  hipStream_t st = (hipStream_t)stream;
  const int np = pad_order(n);
  Workspace* w = nullptr;
  ZF_TRY(ws_get(np, false, true, &w));
  Ctx c;
  c.w = w;
  c.n = n;
  c.np = np;
  c.order = 2;
  c.st = st;
  c.keep_pairs = false;
  series(2, c.c);
  HIP_TRY(launch_split_pad(S, n, n, np, nullptr, nullptr, w->s64, nullptr, false, 1, st));
  HIP_TRY(launch_init_given(Z, n, np, nullptr, w->z64r[0], w->z64c[0], w->zr_hi[0], w->zr_lo[0],
                            nullptr, nullptr, st));
  double e = 0.0;
  ZF_TRY(delta_eval(c, AR_F64, AR_F64, 0, &e));
  if (g_prof.on) prof_harvest();
  *rms = e / sqrt((double)n);
  g_err.clear();
  return 0;
}

// ---------------------------------------------------------------------------
// zf_residual_noalloc: zf_residual's products on a fixed device array
// ---------------------------------------------------------------------------
// Layout (doubles): padded S | Z^T | A^T = Z^T S (each kNoAllocNp^2, row-major with
// ld = np for the padded order np of the call) | norm partials.  Every call
// overwrites what it reads before reading it, so nothing needs clearing; calls that
// overlap on one GPU share the array and race.
constexpr int kNoAllocMaxN = 1024;
constexpr int kNoAllocNp = 1024;  // pad_order(kNoAllocMaxN)
constexpr size_t kNoAllocMat = (size_t)kNoAllocNp * kNoAllocNp;
constexpr int kNoAllocParts = (kNoAllocNp / 64) * (kNoAllocNp / 64);  // max_blocks(np, np)
static __device__ __align__(256) double scratch[3 * kNoAllocMat + kNoAllocParts];

// Device address of `scratch` on each device, looked up once per device with that
// device current (host code uses these, never the array's own name).
constexpr int kNoAllocMaxDevices = 64;
static double* g_scratch_dev[kNoAllocMaxDevices] = {};
static std::mutex g_scratch_mu;

static int scratch_ptr(double** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices)
    return fail(ZF_ERR_ARG, "device %d outside 0..%d", dev, kNoAllocMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(ZF_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    }
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return 0;
}

int zf_residual_noalloc(const double* S, const double* Z, int n, double* rms_dev, void* stream) {
  if (!S || !Z || !rms_dev) return fail(ZF_ERR_ARG, "NULL argument");
  if (n <= 0 || n > kNoAllocMaxN)
    return fail(ZF_ERR_ARG, "n must be in 1..%d (got %d)", kNoAllocMaxN, n);
  hipStream_t st = (hipStream_t)stream;
  double* base = nullptr;
  ZF_TRY(scratch_ptr(&base));
  const int np = pad_order(n);
  double* s64 = base;
  double* zc = base + kNoAllocMat;
  double* at = base + 2 * kNoAllocMat;
  double* parts = base + 3 * kNoAllocMat;
  HIP_TRY(launch_split_pad(S, n, n, np, nullptr, nullptr, s64, nullptr, false, 1, st));
  HIP_TRY(launch_init_given(Z, n, np, nullptr, nullptr, zc, nullptr, nullptr, nullptr, nullptr, st));
  EpiParams e1 = epi0(np, n), e2 = epi0(np, n);
  e1.o64 = at;  // A^T = Z^T S
  e2.beta = -1.0;  // delta = I - Z^T A, only its norm partials are kept
  e2.gamma = 1.0;
  e2.partials = parts;
  HIP_TRY(launch_gemm_f64(zc, np, s64, np, np, np, np, false, e1, st));
  HIP_TRY(launch_gemm_f64(zc, np, at, np, np, np, np, true, e2, st));
  HIP_TRY(launch_norm_finalize(parts, f64_blocks(np, np, true), rms_dev, st, sqrt((double)n)));
  g_err.clear();
  return 0;
}

// H_perp = Z^T H Z (Sec. II.A, Eq. standard_form) with the residual's two matrix-core
// products: first A^T = Z^T H (H symmetric, so the NT kernel reads it row-major), then
// the symmetric product Z^T A written in FP64.  Both inputs are staged into the
// workspace before the first product, so Hp may alias H or Z.
int zf_congruence(const double* H, const double* Z, int n, int precision, double* Hp,
                  void* stream) {
  if (!H || !Z || !Hp) return fail(ZF_ERR_ARG, "H, Z and Hp must be non-NULL device pointers");
  if (n <= 0) return fail(ZF_ERR_ARG, "n must be >= 1 (got %d)", n);
  if (n > 46000) return fail(ZF_ERR_ARG, "n = %d exceeds the supported maximum 46000", n);
  if (precision < ZF_FP64 || precision > ZF_FP16)
    return fail(ZF_ERR_ARG, "precision %d is not supported", precision);
  hipStream_t st = (hipStream_t)stream;
  const Arith ar = precision == ZF_FP64     ? AR_F64
                   : precision == ZF_BF16X3 ? AR_X3
                   : precision == ZF_BF16   ? AR_HH
                   : precision == ZF_FP16X3 ? AR_X3F16
                   : precision == ZF_FP16   ? AR_HHF16
                                            : AR_F32;
  const bool pairs = ar_pairs(ar);
  const bool f16 = ar_f16(ar);
  const int np = pad_order(n);
  Workspace* w = nullptr;
  ZF_TRY(ws_get(np, pairs, true, &w, ar == AR_F32 || f16));
  EpiParams e1 = epi0(np, n), e2 = epi0(np, n);
  e2.o64 = e2.ot64 = w->d64;
  int rc = 0;
  if (pairs) {
    HIP_TRY(launch_split_pad(H, n, n, np, w->s_hi, w->s_lo, nullptr, nullptr, false, f16 ? 2 : 1,
                             st));
    if (f16) {  // Z through its FP32 copy into FP16 halves (transposed layout)
      HIP_TRY(launch_init_given(Z, n, np, w->z32[0], nullptr, nullptr, nullptr, nullptr, nullptr,
                                nullptr, st));
      HIP_TRY(launch_widen(w->z32[0], np, nullptr, nullptr, st, nullptr, nullptr, nullptr,
                           w->zc_hi[0], w->zc_lo[0], 1.0f, PAIR_F16));
    } else {
      HIP_TRY(launch_init_given(Z, n, np, nullptr, nullptr, nullptr, nullptr, nullptr, w->zc_hi[0],
                                w->zc_lo[0], st));
    }
    e1.ohi = w->at_hi;
    e1.olo = w->at_lo;
    e1.pair_fmt = f16 ? PAIR_F16 : PAIR_BF16;
    e2.pair_fmt = e1.pair_fmt;
    rc = gemm_x3(w->zc_hi[0], w->zc_lo[0], w->s_hi, w->s_lo, np, false, e1, st, ar_pm(ar));
    if (!rc) rc = gemm_x3(w->zc_hi[0], w->zc_lo[0], w->at_hi, w->at_lo, np, true, e2, st, ar_pm(ar));
  } else if (ar == AR_F32) {
    HIP_TRY(launch_split_pad(H, n, n, np, nullptr, nullptr, nullptr, w->s32, false, 1, st));
    HIP_TRY(launch_init_given(Z, n, np, w->z32[0], nullptr, nullptr, nullptr, nullptr, nullptr,
                              nullptr, st));
    HIP_TRY(launch_widen(w->z32[0], np, nullptr, nullptr, st, w->zc32[0]));
    e1.o32 = w->a32t;
    rc = gemm_f32(w->zc32[0], w->s32, np, false, e1, st);
    if (!rc) rc = gemm_f32(w->zc32[0], w->a32t, np, true, e2, st);
  } else {
    HIP_TRY(launch_split_pad(H, n, n, np, nullptr, nullptr, w->s64, nullptr, false, 1, st));
    HIP_TRY(launch_init_given(Z, n, np, nullptr, nullptr, w->z64c[0], nullptr, nullptr, nullptr,
                              nullptr, st));
    e1.o64 = w->a64t;
    rc = gemm_f64(w->z64c[0], w->s64, np, false, e1, st);
    if (!rc) rc = gemm_f64(w->z64c[0], w->a64t, np, true, e2, st);
  }
  if (rc) return rc;
  HIP_TRY(launch_unpad_f64(w->d64, np, n, Hp, st));
  if (g_prof.on) prof_harvest();
  g_err.clear();
  return 0;
}

void zf_release(void) {
  batch_release_all();
  if (g_ws.device >= 0) ws_free(g_ws);
  g_ws.device = -1;
  for (auto& p : g_prof.pending) {
    hipEventDestroy(p.a);
    hipEventDestroy(p.b);
  }
  g_prof.pending.clear();
  for (auto e : g_prof.pool) hipEventDestroy(e);
  g_prof.pool.clear();
}

const char* zf_last_error(void) { return g_err.c_str(); }

int zf_version(void) { return 4; }

// ---- per-kernel timing ------------------------------------------------------
void zf_profile_enable(int on) { g_prof.on = on != 0; }

void zf_profile_reset(void) {
  for (int k = 0; k < K_COUNT; ++k) {
    g_prof.launches[k] = 0;
    g_prof.ms[k] = 0.0;
    g_prof.flops[k] = 0.0;
  }
}

int zf_profile_read(int cls, const char** name, long long* launches, double* total_ms,
                    double* flops) {
  if (cls < 0 || cls >= K_COUNT) return fail(ZF_ERR_ARG, "kernel class %d out of range", cls);
  if (name) *name = kClassName[cls];
  if (launches) *launches = g_prof.launches[cls];
  if (total_ms) *total_ms = g_prof.ms[cls];
  if (flops) *flops = g_prof.flops[cls];
  return 0;
}

// ---- learned-guess helpers -----------------------------------------------------
int zf_features(const double* S, int n, float* feats, void* stream) {
  if (!S || !feats || n <= 0) return fail(ZF_ERR_ARG, "bad feature arguments");
  hipStream_t st = (hipStream_t)stream;
  const int np = pad_order(n);
  Workspace* w = nullptr;
  ZF_TRY(ws_get(np, false, true, &w));
  HIP_TRY(launch_split_pad(S, n, n, np, nullptr, nullptr, w->s64, nullptr, false, 1, st));
  EpiParams e = epi0(np, n);
  e.o64 = e.ot64 = w->a64t;
  ZF_TRY(gemm_f64(w->s64, w->s64, np, true, e, st));
  ZF_TRY(guess_features(S, n, w->a64t, nullptr, np, w->s64, feats, w->gscr, st));
  HIP_TRY(hipStreamSynchronize(st));
  g_err.clear();
  return 0;
}

int zf_guess_label(const double* S, const double* Z, int n, double* c, void* stream) {
  if (!S || !Z || !c || n <= 0) return fail(ZF_ERR_ARG, "bad label arguments");
  hipStream_t st = (hipStream_t)stream;
  const int np = pad_order(n);
  Workspace* w = nullptr;
  ZF_TRY(ws_get(np, false, true, &w));
  // S, Z padded; S^2 in a64t, S^3 in d64 (both symmetric)
  HIP_TRY(launch_split_pad(S, n, n, np, nullptr, nullptr, w->s64, nullptr, false, 1, st));
  HIP_TRY(launch_init_given(Z, n, np, nullptr, w->z64r[0], w->z64c[0], w->zr_hi[0], w->zr_lo[0],
                            nullptr, nullptr, st));
  EpiParams e = epi0(np, n);
  e.o64 = e.ot64 = w->a64t;
  ZF_TRY(gemm_f64(w->s64, w->s64, np, true, e, st));
  EpiParams e3 = epi0(np, n);
  e3.o64 = e3.ot64 = w->d64;
  ZF_TRY(gemm_f64(w->a64t, w->s64, np, true, e3, st));
  const double* a[7] = {w->s64, w->s64, w->a64t, w->a64t, w->s64, w->a64t, w->d64};
  const double* b[7] = {w->s64, w->a64t, w->a64t, w->d64, w->z64r[0], w->z64r[0], w->z64r[0]};
  ZF_TRY(gersh_stats(S, n, w->gscr, w->gscr + 4608, st));
  ZF_TRY(dots8(a, b, 7, n, np, w->gscr + 8, w->gscr + 16, st));
  double hv[16];
  HIP_TRY(hipMemcpyAsync(hv, w->gscr, 16 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const double g = hv[0];
  // t[k] = tr(S^k) for k = 1..5; u[j] = <S^j, Z> = tr(S^j Z) for j = 1..3
  const double t[6] = {0.0, hv[3], hv[8], hv[9], hv[10], hv[11]};
  const double u[4] = {0.0, hv[12], hv[13], hv[14]};
  double A[3][3], r[3], x[3];
  for (int j = 0; j < 3; ++j) {
    for (int k = 0; k < 3; ++k) A[j][k] = t[j + k + 1] / pow(g, j + k + 1);
    r[j] = sqrt(g) * u[j + 1] / pow(g, j + 1);
  }
  if (!solve3(A, r, x)) return fail(ZF_ERR_NONFINITE, "singular label system");
  for (int k = 0; k < 3; ++k) c[k] = x[k];
  g_err.clear();
  return 0;
}

// ---- kernel-level test entry points -----------------------------------------
int zf_t_split(const double* a, int64_t count, uint16_t* hi, uint16_t* lo, int fmt, void* stream) {
  if (count < 0) return fail(ZF_ERR_ARG, "negative count");
  if (fmt != 1 && fmt != 2) return fail(ZF_ERR_ARG, "fmt must be 1 (BF16) or 2 (FP16)");
  if (count == 0) return 0;
  if (!a || !hi || !lo) return fail(ZF_ERR_ARG, "NULL split buffer");
  HIP_TRY(launch_split_flat(a, count, hi, lo, fmt, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return 0;
}

// precision -1: the emulated product with oz_slices slices (zf_t_ozaki); precision -2:
// the residue-emulated product with oz_slices moduli (zf_t_crt)
static int t_gemm_impl(int precision, int oz_slices, int sym, int m, int nn, int k,
                       const double* A, const double* B, double alpha, const double* D,
                       double beta, double gamma, double* C, double* norm_sq, void* stream,
                       bool kb = false) {
  if (!A || !B || !C || m <= 0 || nn <= 0 || k <= 0) return fail(ZF_ERR_ARG, "bad gemm arguments");
  if (sym && m != nn) return fail(ZF_ERR_ARG, "symmetric mode needs m == nn");
  const bool crt = precision == -2;
  const bool oz = precision == -1;
  if (!oz && !crt && (precision < 0 || precision > ZF_FP16))
    return fail(ZF_ERR_ARG, "precision %d not supported", precision);
  if (oz && (oz_slices < 1 || oz_slices > kOzMaxSlices))
    return fail(ZF_ERR_ARG, "slices must be in 1..%d (got %d)", kOzMaxSlices, oz_slices);
  if (crt && (oz_slices < 2 || oz_slices > kCrtMaxModuli))
    return fail(ZF_ERR_ARG, "moduli must be in 2..%d (got %d)", kCrtMaxModuli, oz_slices);
  hipStream_t st = (hipStream_t)stream;
  // pad every operand to a common square tile multiple
  int np = m > nn ? m : nn;
  if (k > np) np = k;
  np = round_up(np, 256);
  if ((oz && np > kOzMaxOrder) || (crt && np > kCrtMaxOrder))
    return fail(ZF_ERR_ARG, "emulated products support dimensions up to %d", kOzMaxOrder);
  const size_t e = (size_t)np * np;
  std::vector<void*> tmp;
  auto alloc = [&](size_t bytes, void** p) -> int {
    if (hipMalloc(p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ZF_ERR_NOMEM, "hipMalloc(%zu) failed", bytes);
    }
    tmp.push_back(*p);
    return 0;
  };
  auto cleanup = [&]() {
    for (void* p : tmp) hipFree(p);
  };
  double *a64, *b64, *c64, *d64 = nullptr, *part;
  int rc = 0;
  if ((rc = alloc(e * 8, (void**)&a64)) || (rc = alloc(e * 8, (void**)&b64)) ||
      (rc = alloc(e * 8, (void**)&c64)) || (rc = alloc(max_blocks(np, np) * 8, (void**)&part)) ||
      (D && (rc = alloc(e * 8, (void**)&d64)))) {
    cleanup();
    return rc;
  }
  hipError_t he = hipSuccess;
  auto pad_in = [&](const double* src, int rows, int cols, double* dst) {
    if (he != hipSuccess) return;
    he = hipMemsetAsync(dst, 0, e * 8, st);
    if (he == hipSuccess)
      he = hipMemcpy2DAsync(dst, (size_t)np * 8, src, (size_t)cols * 8, (size_t)cols * 8, rows,
                            hipMemcpyDeviceToDevice, st);
  };
  pad_in(A, m, k, a64);
  pad_in(B, nn, k, b64);
  if (D) pad_in(D, m, nn, d64);
  if (he == hipSuccess) he = hipMemsetAsync(c64, 0, e * 8, st);
  EpiParams ep = epi0(np, m < nn ? m : nn);
  ep.kb = 0;  // this entry's operands and outputs are row-major
  ep.alpha = alpha;
  ep.beta = beta;
  ep.gamma = gamma;
  ep.d64 = d64;
  ep.o64 = c64;
  if (sym) ep.ot64 = c64;
  ep.partials = part;
  u16 *ah = nullptr, *al = nullptr, *bh = nullptr, *bl = nullptr;
  const bool pairs = precision == ZF_BF16X3 || precision == ZF_BF16 ||
                     precision == ZF_FP16X3 || precision == ZF_FP16;
  const bool f16 = precision == ZF_FP16X3 || precision == ZF_FP16;
  const int pm = precision == ZF_BF16 ? PM_HH
                 : precision == ZF_FP16X3 ? PM_X3F16
                 : precision == ZF_FP16   ? PM_HHF16
                                          : PM_X3;
  if (he == hipSuccess && crt) {
    signed char *as, *bs;
    unsigned char* rho;
    int *ea, *eb;
    if ((rc = alloc(e * oz_slices, (void**)&as)) || (rc = alloc(e * oz_slices, (void**)&bs)) ||
        (rc = alloc(e * oz_slices, (void**)&rho)) || (rc = alloc((size_t)np * 4, (void**)&ea)) ||
        (rc = alloc((size_t)np * 4, (void**)&eb))) {
      cleanup();
      return rc;
    }
    he = launch_crt_residues(a64, np, oz_slices, k, as, ea, st);
    if (he == hipSuccess) he = launch_crt_residues(b64, np, oz_slices, k, bs, eb, st);
    if (he == hipSuccess)
      he = launch_crt_product(as, ea, bs, eb, np, oz_slices, k, sym != 0, rho, ep, st);
  } else if (he == hipSuccess && oz) {
    signed char *as, *bs;
    int *ea, *eb;
    if ((rc = alloc(e * oz_slices, (void**)&as)) || (rc = alloc(e * oz_slices, (void**)&bs)) ||
        (rc = alloc((size_t)np * 4, (void**)&ea)) || (rc = alloc((size_t)np * 4, (void**)&eb))) {
      cleanup();
      return rc;
    }
    he = launch_oz_slice(a64, np, oz_slices, as, ea, st);
    if (he == hipSuccess) he = launch_oz_slice(b64, np, oz_slices, bs, eb, st);
    if (he == hipSuccess) he = launch_gemm_oz(as, ea, bs, eb, np, oz_slices, sym != 0, ep, st);
  } else if (he == hipSuccess && precision == ZF_FP32) {
    float *a32, *b32;
    if ((rc = alloc(e * 4, (void**)&a32)) || (rc = alloc(e * 4, (void**)&b32))) {
      cleanup();
      return rc;
    }
    he = launch_split_pad(a64, np, np, np, nullptr, nullptr, nullptr, a32, false, 1, st);
    if (he == hipSuccess)
      he = launch_split_pad(b64, np, np, np, nullptr, nullptr, nullptr, b32, false, 1, st);
    if (he == hipSuccess) he = launch_gemm_f32(a32, np, b32, np, np, np, np, sym != 0, ep, st);
  } else if (he == hipSuccess && pairs) {
    if ((rc = alloc(e * 2, (void**)&ah)) || (rc = alloc(e * 2, (void**)&al)) ||
        (rc = alloc(e * 2, (void**)&bh)) || (rc = alloc(e * 2, (void**)&bl))) {
      cleanup();
      return rc;
    }
    if (kb) {  // the solver's K-blocked pairs (split_pad writes that layout)
      he = launch_split_pad(a64, np, np, np, ah, al, nullptr, nullptr, false, f16 ? 2 : 1, st);
      if (he == hipSuccess)
        he = launch_split_pad(b64, np, np, np, bh, bl, nullptr, nullptr, false, f16 ? 2 : 1, st);
      if (he == hipSuccess)
        he = launch_gemm_x3(ah, al, 32, bh, bl, 32, np, np, np, sym != 0, ep, st, pm, 32 * np,
                            32 * np);
    } else {
      he = launch_split_flat(a64, (int64_t)e, ah, al, f16 ? 2 : 1, st);
      if (he == hipSuccess) he = launch_split_flat(b64, (int64_t)e, bh, bl, f16 ? 2 : 1, st);
      if (he == hipSuccess)
        he = launch_gemm_x3(ah, al, np, bh, bl, np, np, np, np, sym != 0, ep, st, pm);
    }
  } else if (he == hipSuccess) {
    he = launch_gemm_f64(a64, np, b64, np, np, np, np, sym != 0, ep, st);
  }
  double* nrm = nullptr;
  if (he == hipSuccess && norm_sq) {
    if ((rc = alloc(8, (void**)&nrm))) {
      cleanup();
      return rc;
    }
    const int nb = crt     ? crt_blocks(np, sym != 0)
                   : oz    ? oz_blocks(np, sym != 0)
                   : pairs ? x3_blocks(np, np, sym != 0)
                   : precision == ZF_FP32 ? f32_blocks(np, np, sym != 0)
                                          : f64_blocks(np, np, sym != 0);
    he = launch_norm_finalize(part, nb, nrm, st);
  }
  if (he == hipSuccess)
    he = hipMemcpy2DAsync(C, (size_t)nn * 8, c64, (size_t)np * 8, (size_t)nn * 8, m,
                          hipMemcpyDeviceToDevice, st);
  double nv = 0.0;
  if (he == hipSuccess && norm_sq) he = hipMemcpyAsync(&nv, nrm, 8, hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  cleanup();
  if (he != hipSuccess) return fail(ZF_ERR_HIP, "zf_t_gemm: %s", hipGetErrorString(he));
  if (norm_sq) *norm_sq = nv * nv;
  return 0;
}

int zf_t_gemm(int precision, int sym, int m, int nn, int k, const double* A, const double* B,
              double alpha, const double* D, double beta, double gamma, double* C, double* norm_sq,
              void* stream) {
  if (precision < ZF_FP64) return fail(ZF_ERR_ARG, "precision %d not supported", precision);
  return t_gemm_impl(precision, 0, sym, m, nn, k, A, B, alpha, D, beta, gamma, C, norm_sq, stream);
}

int zf_t_gemm_kb(int precision, int sym, int m, int nn, int k, const double* A, const double* B,
                 double alpha, const double* D, double beta, double gamma, double* C,
                 double* norm_sq, void* stream) {
  if (precision != ZF_BF16X3 && precision != ZF_BF16 && precision != ZF_FP16X3 &&
      precision != ZF_FP16)
    return fail(ZF_ERR_ARG, "precision %d has no 16-bit pairs", precision);
  return t_gemm_impl(precision, 0, sym, m, nn, k, A, B, alpha, D, beta, gamma, C, norm_sq, stream,
                     true);
}

int zf_t_crt(int moduli, int sym, int m, int nn, int k, const double* A, const double* B,
             double alpha, const double* D, double beta, double gamma, double* C,
             double* norm_sq, void* stream) {
  return t_gemm_impl(-2, moduli, sym, m, nn, k, A, B, alpha, D, beta, gamma, C, norm_sq, stream);
}

int zf_t_ozaki(int slices, int sym, int m, int nn, int k, const double* A, const double* B,
               double alpha, const double* D, double beta, double gamma, double* C,
               double* norm_sq, void* stream) {
  return t_gemm_impl(-1, slices, sym, m, nn, k, A, B, alpha, D, beta, gamma, C, norm_sq, stream);
}

int zf_t_gershgorin(const double* S, int n, double* g, void* stream) {
  if (!S || !g || n <= 0) return fail(ZF_ERR_ARG, "bad gershgorin arguments");
  hipStream_t st = (hipStream_t)stream;
  double *rs = nullptr, *gd = nullptr;
  if (hipMalloc((void**)&rs, (size_t)n * 8) != hipSuccess) return fail(ZF_ERR_NOMEM, "hipMalloc");
  if (hipMalloc((void**)&gd, 8) != hipSuccess) {
    hipFree(rs);
    return fail(ZF_ERR_NOMEM, "hipMalloc");
  }
  hipError_t he = launch_row_abs_max(S, n, n, rs, gd, st);
  double v = 0.0;
  if (he == hipSuccess) he = hipMemcpyAsync(&v, gd, 8, hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  hipFree(rs);
  hipFree(gd);
  if (he != hipSuccess) return fail(ZF_ERR_HIP, "zf_t_gershgorin: %s", hipGetErrorString(he));
  *g = v;
  return 0;
}

}  // extern "C"
