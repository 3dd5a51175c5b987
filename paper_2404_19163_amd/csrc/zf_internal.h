// Internal declarations shared by the libzf translation units (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zf {

typedef uint16_t u16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// Product modes of the 16-bit-halves GEMM: bit 0 = hi halves only ((h)(h)),
// bit 1 = FP16 halves (else BF16).
// PM_I8: one product of signed 8-bit slices (16 per 16-byte chunk) with exact int32
// accumulation, the accumulator registers holding the int32 bits
enum { PM_X3 = 0, PM_HH = 1, PM_X3F16 = 2, PM_HHF16 = 3, PM_I8 = 4 };
// Format of a 16-bit pair in memory (EpiParams::pair_fmt, element-wise kernels).
enum { PAIR_BF16 = 0, PAIR_F16 = 1 };
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// FP32 -> BF16 with round to nearest, ties to even (NaN kept quiet).
// ---------------------------------------------------------------------------
__device__ __forceinline__ u16 f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u16)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(u16 h) { return __uint_as_float(((uint32_t)h) << 16); }

// FP32 -> FP16 (IEEE binary16) with round to nearest even, via the hardware convert.
__device__ __forceinline__ u16 f32_to_f16_rne(float f) {
  _Float16 h = (_Float16)f;
  return *reinterpret_cast<u16*>(&h);
}
__device__ __forceinline__ float f16_to_f32(u16 b) {
  _Float16 h;
  *reinterpret_cast<u16*>(&h) = b;
  return (float)h;
}

// Two-term split of Sec. III.A: hi = LP[x], lo = LP[x - hi]; x - hi is exact in FP32.
__device__ __forceinline__ void split_bf16(float x, u16& hi, u16& lo) {
  hi = f32_to_bf16_rne(x);
  lo = f32_to_bf16_rne(x - bf16_to_f32(hi));
}
__device__ __forceinline__ void split_f16(float x, u16& hi, u16& lo) {
  hi = f32_to_f16_rne(x);
  lo = f32_to_f16_rne(x - f16_to_f32(hi));
}
__device__ __forceinline__ void split_pair(float x, u16& hi, u16& lo, int fmt) {
  if (fmt == PAIR_F16) split_f16(x, hi, lo);
  else split_bf16(x, hi, lo);
}
__device__ __forceinline__ float pair_sum(u16 hi, u16 lo, int fmt) {
  return fmt == PAIR_F16 ? f16_to_f32(hi) + f16_to_f32(lo) : bf16_to_f32(hi) + bf16_to_f32(lo);
}

// ---------------------------------------------------------------------------
// Learned guess helpers shared by the single-matrix and batched paths.
// ---------------------------------------------------------------------------
// The 8 network features from the Gershgorin statistics (g = max r_i, g_lo, mean r_i),
// tr S and the Frobenius products ||S||^2, <S, S^2>, ||S^2||^2 (= N times the mean
// of the k-th power of the spectrum of S/g for k = 1..4).
__host__ __device__ inline void finish_features(double g, double glo, double rmean, double trS,
                                                double d0, double d1, double d2, int n,
                                                float* f) {
  f[0] = (float)log((double)n);
  f[1] = (float)(trS / g / n);
  f[2] = (float)(d0 / (g * g) / n);
  f[3] = (float)(d1 / (g * g * g) / n);
  f[4] = (float)(d2 / (g * g * g * g) / n);
  f[5] = (float)(fmax(glo, 0.0) / g);
  f[6] = (float)(glo / g);
  f[7] = (float)(rmean / g);
}

// Acceptance of p(x) = c0 + c1 x + c2 x^2 on the Gershgorin interval [x_lo, 1]: the
// eigenvalues of X0 = Z0^T S Z0 are x p(x)^2 (x = lambda / g), and convergence needs
// them in (0, 2) (||X0 - I||_2 < 1, Sec. III).  Rejects if p <= 0 at a sampled x > 0,
// else rescales c so that the sampled maximum of x p(x)^2 is at most 1.9.
__host__ __device__ inline bool accept_poly(double c[3], double x_lo) {
  const int K = 1024;
  if (x_lo < 0.0) x_lo = 0.0;
  double mx = 0.0;
  for (int k = 0; k <= K; ++k) {
    const double x = x_lo + (1.0 - x_lo) * k / K;
    const double p = c[0] + c[1] * x + c[2] * x * x;
    if (p <= 0.0 && (x > 0.0)) return false;
    mx = fmax(mx, x * p * p);
  }
  if (!(mx > 0.0)) return false;
  if (mx > 1.9) {
    const double s = sqrt(1.9 / mx);
    for (int k = 0; k < 3; ++k) c[k] *= s;
  }
  return true;
}

// ---------------------------------------------------------------------------
// K-blocked layout of a 16-bit operand with ld rows of stride 32: element (r, k)
// of an (rows x K) operand at kb_offset(r, k, ld), i.e. K cut into blocks of 32
// and each block stored as a row-major (ld x 32) panel.  One K step of a GEMM
// tile then reads a contiguous run of 64-byte rows, and a producer that forms 32
// consecutive k of many rows (a transposed epilogue strip) writes one contiguous
// run instead of 64-byte pieces one ld apart.
// ---------------------------------------------------------------------------
__host__ __device__ inline size_t kb_offset(int r, int k, int ld) {
  return (size_t)(k >> 5) * ((size_t)ld << 5) + ((size_t)r << 5) + (size_t)(k & 31);
}

// ---------------------------------------------------------------------------
// GEMM epilogue: out = alpha * D + beta * acc + gamma * I  (I restricted to the
// valid n_valid x n_valid block so that zero padding stays exactly zero).
// Every output pointer is optional.  Normal outputs are written at
// [row * ld + col]; transposed outputs at [col * ld + row].  With kb set, every
// 16-bit pair read or written (dhi/dlo, ohi/olo, othi/otlo) is K-blocked instead:
// (row, col) at kb_offset(row, col, ld), the transposed one at kb_offset(col, row,
// ld); FP32 and FP64 matrices stay row-major.  In symmetric mode the caller passes
// the same matrices for both, and the kernel writes the upper triangle normally
// and mirrors it.
// ---------------------------------------------------------------------------
struct EpiParams {
  double alpha, beta, gamma;
  int n_valid;
  int ld;
  const float* d32;
  const double* d64;
  const u16* dhi;
  const u16* dlo;
  float* o32;
  double* o64;
  u16* ohi;
  u16* olo;
  float* ot32;
  double* ot64;
  u16* othi;
  u16* otlo;
  double* partials;  // per-tile sum of out^2 (FP64), or nullptr
  int pair_fmt;      // PAIR_BF16 / PAIR_F16: format of dhi/dlo and of every pair output
  int kb;            // 16-bit pairs in the K-blocked layout (kb_offset)
  const int* gate;   // non-null and nonzero: the launch does nothing (a stopped phase)
};

// Launchers (return hipSuccess or the launch error).  All dimensions must be
// multiples of kTile; the caller pads.  Symmetric mode requires M == N.
constexpr int kTile = 128;
int x3_tile_edge(int M, int N, bool sym);  // tile edge the BF16x3 launch will use
int x3_blocks(int M, int N, bool sym);   // blocks (= norm partials) of that launch
int f64_tile_edge(int M, int N, bool sym);
int f64_blocks(int M, int N, bool sym);
int max_blocks(int M, int N);            // upper bound of the above (smallest tile edge)

// pm: product mode PM_* (BF16 or FP16 halves; all three products or (h)(h) only).
// Operand element (r, k) sits at r * ld + (k / 32) * ks + k % 32: ks = 32 for a
// row-major operand, ld = 32 and ks = 32 * rows for a K-blocked one (kb_offset).
hipError_t launch_gemm_x3(const u16* Ahi, const u16* Alo, int lda, const u16* Bhi, const u16* Blo,
                          int ldb, int M, int N, int K, bool sym, const EpiParams& ep,
                          hipStream_t st, int pm = PM_X3, int ksa = 32, int ksb = 32);
int f32_tile_edge(int M, int N, bool sym);
int f32_blocks(int M, int N, bool sym);
hipError_t launch_gemm_f32(const float* A, int lda, const float* B, int ldb, int M, int N, int K,
                           bool sym, const EpiParams& ep, hipStream_t st);
hipError_t launch_gemm_f64(const double* A, int lda, const double* B, int ldb, int M, int N, int K,
                           bool sym, const EpiParams& ep, hipStream_t st);

// FP64 products emulated with 7-bit integer slices on the int8 matrix cores
// (ozaki.hip).  Slices of M (np x np FP64, row-major): s planes of np x np signed
// bytes (plane stride np^2) and a per-row exponent.  The GEMM forms the NT product
// A B^T of two sliced matrices (np % 128 == 0, np <= kOzMaxOrder) with the
// EpiParams epilogue; its norm partials number oz_blocks(np, sym).
constexpr int kOzMaxSlices = 8;
constexpr int kOzMaxOrder = 16384;  // s K 127^2 < 2^31 for every s <= 8
hipError_t launch_oz_slice(const double* M, int np, int s, signed char* out, int* ex,
                           hipStream_t st, const int* gate = nullptr);
hipError_t launch_gemm_oz(const signed char* A, const int* ea, const signed char* B, const int* eb,
                          int np, int s, bool sym, const EpiParams& ep, hipStream_t st);
int oz_tile_edge(int np, bool sym);
int oz_blocks(int np, bool sym);

// FP64 products emulated through residues (crt.hip): rows scaled by 2^(beta - e_i)
// and truncated to integers, the exact integer product recovered from one int8
// product per modulus (L pairwise coprime moduli <= 256) by the Chinese remainder
// theorem.  beta depends on L and on K, the number of valid (unpadded) terms of the
// contraction.  Residue planes: L planes of np x np signed bytes (plane stride np^2)
// and a per-row exponent.  The product runs the EpiParams epilogue on C = A B^T; its
// norm partials number crt_blocks(np, sym).  np % 256 == 0, np <= kCrtMaxOrder;
// rho is scratch for L byte planes.
constexpr int kCrtMaxModuli = 15;
constexpr int kCrtMaxOrder = 16384;
int crt_beta(int L, long long K);  // -1 for an unsupported L
hipError_t launch_crt_residues(const double* M, int np, int L, long long K, signed char* out,
                               int* ex, hipStream_t st, const int* gate = nullptr);
hipError_t launch_crt_product(const signed char* A, const int* ea, const signed char* B,
                              const int* eb, int np, int L, long long K, bool sym,
                              unsigned char* rho, const EpiParams& ep, hipStream_t st);
int crt_blocks(int np, bool sym);

// Elementwise / reduction kernels (elementwise.hip)
hipError_t launch_split_pad(const double* src, int n, int ld_src, int np, u16* hi, u16* lo,
                            double* copy64, float* copy32, bool transpose_copy, int fmt,
                            hipStream_t st);
hipError_t launch_split_flat(const double* src, int64_t count, u16* hi, u16* lo, int fmt,
                             hipStream_t st);
hipError_t launch_row_abs_max(const double* S, int n, int ld, double* row_sums, double* g_out,
                              hipStream_t st);
hipError_t launch_init_identity(const double* g, int n, int np, float* z32, double* z64r,
                                double* z64c, u16* zr_hi, u16* zr_lo, u16* zc_hi, u16* zc_lo,
                                hipStream_t st);
hipError_t launch_init_given(const double* Z0, int n, int np, float* z32, double* z64r,
                             double* z64c, u16* zr_hi, u16* zr_lo, u16* zc_hi, u16* zc_lo,
                             hipStream_t st);
// FP32 X -> FP64 row-major / FP64 transposed / FP32 transposed / 16-bit pairs of
// scale * X (row-major and transposed, format fmt); each optional; np % 64 == 0
hipError_t launch_widen(const float* z32, int np, double* z64r, double* z64c, hipStream_t st,
                        float* zc32 = nullptr, u16* prh = nullptr, u16* prl = nullptr,
                        u16* pch = nullptr, u16* pcl = nullptr, float scale = 1.0f,
                        int fmt = PAIR_BF16);
hipError_t launch_unpad_f64(const double* src, int np, int n, double* dst, hipStream_t st);
hipError_t launch_unpad_f32(const float* src, int np, int n, double* dst, hipStream_t st);
// out[0] = sqrt(sum of the partials) / div (div = 1: the Frobenius norm itself)
hipError_t launch_norm_finalize(const double* partials, int count, double* out, hipStream_t st,
                                double div = 1.0);
// The stop test of one sweep on the device: Err from the partials, then the rule of
// Algorithm 2 against the previous Err (state[0]): rule 1 (monotone) stops when Err >=
// prev, rule 0 (ratio) when Err > prev^pw.  box[0] = Err, box[1] = 0 (go on), 1 (stop)
// or 2 (Err not finite); a stop or a non-finite Err sets *gate, which every later
// launch of the phase reads and then does nothing, this one included.  box may be
// host memory (mapped, coherent).
hipError_t launch_norm_decide(const double* partials, int count, int it, int rule, int pw,
                              int* gate, double* state, double* box, hipStream_t st);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st);

// Tracing (zf_api.hip).
// ZF_LOG=1 writes one JSON object per line to stderr for every call, residual
// evaluation and result; ZF_LOG=<path> appends the same lines to that file.
// log_on() reads the variable (once per API call is enough); log_line formats one
// line (the caller passes the JSON body without braces) and flushes it.
bool log_on();
void log_line(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
// roctx ranges around the stages of a call (rocprofv3 --marker-trace shows them;
// without a profiler attached they cost a function call).
struct TraceRange {
  explicit TraceRange(const char* name);
  ~TraceRange() { end(); }
  void end();  // close the range before the scope ends (idempotent)
  bool live = true;
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

// Error reporting shared by the translation units (zf_api.hip): set the thread's
// message and return code; clear_error() empties it.
int set_error(int code, const char* fmt, ...);
void clear_error();
void batch_release_all();  // frees the batched path's cached state (batched.hip)

// learned guess (guess.hip)
int guess_features(const double* S, int n, const double* S2, const float* S2f, int np,
                   const double* S64pad, float* feats, double* scratch, hipStream_t st);
int guess_infer(const float* feats, double* coef, hipStream_t st);
// count feature vectors (8 floats each) -> count x {c0, c1, c2, .} (stride 4 doubles)
int guess_infer_batch(const float* feats, int count, double* coef, hipStream_t st);
bool net_ready();
bool guess_accept(double c[3], double x_lo);
hipError_t launch_guess_write(const double* S, int n, const double* S2, const float* S2f, int np,
                              const double* cg, float* z32, double* z64r, double* z64c, u16* zr_hi,
                              u16* zr_lo, u16* zc_hi, u16* zc_lo, hipStream_t st);
int dots8(const double* const* a, const double* const* b, int count, int n, int np, double* out_dev,
          double* partial, hipStream_t st);
int gersh_stats(const double* S, int n, double* out_dev, double* part, hipStream_t st);

}  // namespace zf
