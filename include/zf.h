/*
 * zf.h -- C ABI of libzf: iterative refinement of an inverse overlap factor Z
 * with Z^T S Z = I (equivalently Z Z^T = S^-1) for a dense symmetric
 * positive-definite overlap matrix S, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Habib, Finkelstein & Niklasson, "Efficient Mixed-Precision Matrix
 * Factorization of the Inverse Overlap Matrix in Electronic Structure
 * Calculations with AI-Hardware and GPUs" (LA-UR-24-24032):
 *   - recursion Z_{n+1} = Z_n sum_k c_k delta_n^k with delta_n = I - Z_n^T S Z_n
 *     (Sec. III, Eq. np1 and its delta form), c_k = C(2k,k)/4^k;
 *   - parameter-free stop test (Sec. IV.A, Algorithm 2, Eq. stopL2);
 *   - two-term split A = A^(h) + A^(l) with the (h)(h)+(h)(l)+(l)(h) products
 *     (Sec. III.A-B, Eqs. dualRep, splitStyle, SZn, Xn, Xsq);
 *   - a refinement phase in higher precision after the low-precision stop
 *     (Sec. IV.B, Algorithm 3).
 *
 * Conventions for every entry point:
 *   - Matrices are dense, row-major, leading dimension n, FP64, in DEVICE
 *     memory (hipMalloc'd or a torch CUDA tensor).  S must be symmetric; only
 *     its values are read, never written.
 *   - `stream` is a hipStream_t passed as void* (NULL = the legacy default
 *     stream).  Work is ordered on that stream.  Calls that report scalars to
 *     the host (iteration counts, histories, norms) synchronize the stream
 *     before returning.
 *   - Ownership: the caller owns every pointer it passes.  The library owns a
 *     per-device workspace cache sized for the largest n seen, allocated on
 *     first use and freed by zf_release().
 *   - Return value: 0 on success; a positive value is a bitmask of ZF_WARN_*;
 *     a negative value is a ZF_ERR_* code and zf_last_error() describes it.
 *     Nothing throws or aborts across this ABI.
 *   - Calls are not reentrant: do not run two calls concurrently from
 *     different host threads on one device.
 */
#ifndef ZF_H
#define ZF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ZF_OK 0
/* warnings (bitmask, positive) */
#define ZF_WARN_MAXSWEEPS 1   /* a phase ended at its sweep cap, not at the stop test */
#define ZF_WARN_Z0_FALLBACK 2 /* the learned guess was unavailable or rejected: scaled identity */
#define ZF_WARN_HIST_TRUNC 4  /* more residuals than hist_cap; the rest were dropped */
/* errors (negative) */
#define ZF_ERR_ARG -1            /* invalid argument (n <= 0, order out of range, NULL, ...) */
#define ZF_ERR_NOMEM -2          /* device or pinned allocation failed */
#define ZF_ERR_HIP -3            /* a HIP runtime call failed (message has hipGetErrorString) */
#define ZF_ERR_NONFINITE -4      /* a residual norm was NaN or Inf (S or Z0 not finite, or overflow) */
#define ZF_ERR_NOT_CONVERGED -5  /* returned Z has ||Z^T S Z - I||_F >= 1: the convergence
                                    condition ||X0 - I||_2 < 1 of Sec. III was not met */

/* Arithmetic of the low-precision phase (Sec. III, Table I). */
enum zf_precision {
  ZF_FP64 = 0,    /* "double": every product in FP64 on the FP64 matrix cores      */
  ZF_BF16X3 = 1,  /* (h)(h)+(h)(l)+(l)(h) with BF16 halves, FP32 accumulation       */
  ZF_FP16X3 = 2,  /* (h)(h)+(h)(l)+(l)(h) with FP16 halves (the paper's Eq. splitStyle);
                     delta and Q are split after a power-of-two scale to FP16's range;
                     S and Z entries must stay within FP16's range (|x| < 65504)       */
  ZF_BF16 = 3,    /* (h)(h): the hi halves' product only, FP32 accumulation         */
  ZF_FP32 = 4,    /* "single": FP32 operands on the FP32 matrix cores               */
  ZF_FP16 = 5     /* (h)(h) with FP16 halves                                        */
};

/* Stop rule (Sec. IV.A). */
enum zf_stop {
  ZF_STOP_RATIO = 0,    /* Algorithm 2: stop at n > 0 once Err_n > Err_{n-1}^(m+1)  */
  ZF_STOP_MONOTONE = 1  /* stop at n > 0 once Err_n >= Err_{n-1}                    */
};

/* The initial guess a run started from (zf_result.z0_used). */
enum zf_z0_kind {
  ZF_Z0_GIVEN = 0,           /* the caller's Z0                                        */
  ZF_Z0_SCALED_IDENTITY = 1, /* I / sqrt(g), g = max_i sum_j |S_ij| (Gershgorin bound)  */
  ZF_Z0_LEARNED = 2          /* (c0 I + c1 S/g + c2 (S/g)^2) / sqrt(g) from the network  */
};

/* Refinement phase after a low-precision stop (Sec. IV.B, Algorithm 3). */
enum zf_refine_mode {
  ZF_REFINE_OFF = 0,       /* return the first phase's result                         */
  ZF_REFINE_F64_DELTA = 1, /* FP64 delta and stop norm, BF16x3 correction              */
  ZF_REFINE_F64_FULL = 2,  /* FP64 delta and FP64 correction                          */
  ZF_REFINE_F32 = 3,       /* FP32 delta, stop norm and correction (Algorithm 3 with
                              FP32[Z], the "+refi" of Table I in single precision)    */
  ZF_REFINE_EMU = 4,       /* delta and stop norm from FP64 products emulated on the
                              int8 matrix cores (7-bit integer slices, Ozaki scheme;
                              ZF_EMU_SLICES = 3..8 slices, default 7), BF16x3
                              correction.  Each product's error is below
                              (s+1) 2^-7s n 2^(e_i+f_j), e_i, f_j the exponents of the
                              largest entries of the operand rows; n <= 16384.       */
  ZF_REFINE_CRT = 5,       /* delta and stop norm from FP64 products emulated through
                              residues on the int8 matrix cores (rows truncated to
                              beta-bit integers, one int8 product per modulus, Chinese
                              remainder theorem; Ozaki, Uchino & Imamura's scheme II;
                              ZF_EMU_MODULI = 8..15 moduli, default 14, beta = 48 at
                              n = 4096), BF16x3 correction.  Each product's error is
                              below 2^(1-beta) n 2^(e_i+f_j) plus a rounding;
                              n <= 16384.                                             */
  ZF_REFINE_CRT_FIRST = 6  /* as ZF_REFINE_F64_DELTA, but the refinement phase's first
                              delta comes from the residue-emulated products of
                              ZF_REFINE_CRT; every later evaluation, so the stopping
                              norm and the final residual, is FP64.  n <= 16384.      */
};

typedef struct {
  int order;      /* m, number of series terms after I; 1..5 (the paper uses 2)          */
  int precision;  /* enum zf_precision                                                   */
  int stop;       /* enum zf_stop                                                        */
  int max_sweeps; /* cap on Z updates in the first phase; <= 0 means 100                */
  int refine;     /* enum zf_refine_mode; ignored for ZF_FP64                            */
  int max_refine; /* cap on Z updates in the refinement phase; <= 0 means 10             */
  int z0;         /* enum zf_z0_kind: the guess when Z0 is NULL.  ZF_Z0_SCALED_IDENTITY
                     (default) or ZF_Z0_LEARNED (zf_mlp_*, scaled identity as fallback).
                     A non-NULL Z0 is always used as given; ZF_Z0_GIVEN with Z0 == NULL
                     is ZF_ERR_ARG.                                                       */
} zf_opts;

typedef struct {
  int iters;       /* Z updates contained in the returned Z (both phases)               */
  int low_evals;   /* residual evaluations in the low-precision phase                   */
  int high_evals;  /* FP64 residual evaluations (refinement phase or ZF_FP64 runs)     */
  int hist_len;    /* entries written to hist                                           */
  int flags;       /* ZF_WARN_* bits                                                    */
  double final_err;/* ||I - Z^T S Z||_F of the returned Z as last evaluated (FP64 when a
                      FP64 evaluation ran, else the low-precision value)               */
  double final_rms;/* final_err / sqrt(n)                                              */
  int status;      /* 0, or the ZF_ERR_* code of this matrix (batched calls report each)  */
  int z0_used;     /* enum zf_z0_kind                                                     */
} zf_result;

/* Fill *opts with the defaults: order 2, ZF_BF16X3, ZF_STOP_RATIO, 100 sweeps,
 * ZF_REFINE_F64_DELTA, 10 refinement sweeps, scaled-identity guess. */
void zf_default_opts(zf_opts* opts);

/*
 * zf_refine -- refine Z0 to Z with Z^T S Z = I (Sec. III-IV).
 *   S     [in]  device, n x n FP64 symmetric positive definite.
 *   Z0    [in]  device, n x n FP64 initial guess with ||Z0^T S Z0 - I||_2 < 1 (Sec. III),
 *               or NULL for the scaled identity I / sqrt(max_i sum_j |S_ij|).
 *   n     [in]  order of S, >= 1.
 *   order [in]  m in 1..5.
 *   precision [in] enum zf_precision; mixed precisions run ZF_REFINE_F64_DELTA.
 *   Z     [out] device, n x n FP64; may alias Z0.
 *   iters [out] host, Z updates in the returned Z (may be NULL).
 *   hist  [out] host, hist_cap doubles: unnormalized ||delta||_F per residual
 *               evaluation, first phase then refinement phase (may be NULL if
 *               hist_cap is 0).
 *   hist_len [out] host, entries written (may be NULL).
 * Stop rule ZF_STOP_RATIO; see zf_refine_ex for every option.
 */
int zf_refine(const double* S, const double* Z0, int n, int order, int precision, double* Z,
              int* iters, double* hist, int hist_cap, int* hist_len, void* stream);

/* zf_refine_ex -- as zf_refine with explicit options (opts NULL = defaults) and a result
 * record (res may be NULL). */
int zf_refine_ex(const double* S, const double* Z0, int n, const zf_opts* opts, double* Z,
                 zf_result* res, double* hist, int hist_cap, void* stream);

/*
 * zf_refine_batched -- refine count independent matrices of uneven order together.
 *   count       1..65535 matrices.
 *   S[m], Z[m]  device pointers (host arrays of count pointers), n[m] x n[m] FP64, n[m] in
 *               1..8192; Z0 may be NULL (all scaled identity) or hold NULL entries.
 *   opts        order must be 2, precision ZF_BF16X3, refine ZF_REFINE_OFF or
 *               ZF_REFINE_F64_DELTA (opts NULL = defaults).  opts.z0 = ZF_Z0_LEARNED
 *               gives every matrix without a Z0 the learned guess (per-matrix
 *               acceptance on the device, scaled-identity fallback flagged in its
 *               result); ZF_Z0_GIVEN requires a Z0 for every matrix.
 *   res         host[count] or NULL: per-matrix result including status.
 *   hist        host[count * hist_cap]: matrix m's residual history at m * hist_cap.
 * Every matrix runs the recursion and stop test of zf_refine_ex; the matrices advance
 * in lockstep macro-sweeps of grouped matrix-core GEMMs (one persistent launch per
 * stage), with the stop state kept on the device.  Runs of macro-sweeps (8 by
 * default, see zf_batched_set_graph_sweeps) are captured in one HIP graph; the host
 * launches it and reads the live count once per launch, and kernels of macro-sweeps
 * after every matrix has stopped return at once.  The tile edge per matrix comes from
 * the table of
 * zf_batched_set_tiles / zf_batched_autotune.  Returns the OR of the warnings, or the
 * first failing matrix's error (every result is still filled).
 */
int zf_refine_batched(int count, const double* const* S, const double* const* Z0, const int* n,
                      const zf_opts* opts, double* const* Z, zf_result* res, double* hist,
                      int hist_cap, void* stream);

/* zf_batched_set_tiles -- tile table: orders n <= max_n[k] use tile[k] (64 or 128); the
 * last entry covers every larger order.  1 <= count <= 16. */
int zf_batched_set_tiles(const int* max_n, const int* tile, int count);

/* zf_batched_get_tiles -- copy the table out (cap entries); returns its length. */
int zf_batched_get_tiles(int* max_n, int* tile, int cap);

/* zf_batched_autotune -- for each bucket order bucket_n[b], time the grouped BF16x3
 * residual GEMMs of batch matrices with 64 and 128 tiles (reps repetitions), store the
 * faster edge in best_tile[b] and the times in ms[2 b], ms[2 b + 1] (ms may be NULL),
 * and install the table (bucket b covers orders up to bucket_n[b]). */
int zf_batched_autotune(const int* bucket_n, int nbuckets, int batch, int reps, int* best_tile,
                        double* ms, void* stream);

/* zf_batched_use_graph -- 1 (default): replay the captured macro-sweep graph; 0: launch
 * the same kernels eagerly (for checking the graph). */
void zf_batched_use_graph(int on);

/* zf_batched_set_graph_sweeps -- macro-sweeps per graph launch: k > 0 (default 8)
 * launches graphs of k macro-sweeps until no matrix is live, reading the live count
 * after each launch; 0 captures every macro-sweep the sweep caps allow (one launch and
 * one synchronization per call, but each macro-sweep after the last stop still costs
 * its launches).  Returns ZF_ERR_ARG for k < 0. */
int zf_batched_set_graph_sweeps(int sweeps);

/* zf_batched_last_stats -- of the last zf_refine_batched call: the macro-sweeps in which
 * some matrix was still live, and the number of graph launches (either pointer may be
 * NULL). */
int zf_batched_last_stats(int* macro_sweeps, int* graph_launches);

/* zf_batched_release -- free the batched path's cached arena, graph and stream. */
void zf_batched_release(void);

/*
 * Learned initial guess Z0 = (c0 I + c1 S/g + c2 (S/g)^2) / sqrt(g), g = max_i sum_j |S_ij|.
 * The recursion converges from any Z0 with ||Z0^T S Z0 - I||_2 < 1 (Sec. III); good guesses
 * save sweeps (Sec. VI).  Features (8 floats): log N, tr((S/g)^k)/N for k = 1..4,
 * max(g_lo,0)/g, g_lo/g, mean_i sum_j |S_ij| / g, with g_lo the Gershgorin lower bound.
 * Network: 8 -> 64 -> 64 -> 3, tanh, FP32, 4931 parameters in the order W1 (64x8), b1,
 * W2 (64x64), b2, W3 (3x64), b3; inputs and outputs standardized by zf_mlp_set_norm.
 * With opts.z0 = ZF_Z0_LEARNED and Z0 == NULL, zf_refine_ex predicts (c0, c1, c2), rescales them so
 * that max x p(x)^2 <= 1.9 on the Gershgorin interval [max(g_lo,0)/g, 1], and falls back
 * to the scaled identity (ZF_WARN_Z0_FALLBACK) if p <= 0 there or no network is loaded.
 */
/* zf_features -- the 8 features of device S (n x n) into device feats (8 floats). */
int zf_features(const double* S, int n, float* feats, void* stream);
/* zf_guess_label -- training label: c (host, 3 doubles) minimizing
 * ||S^(1/2) (p(S/g)/sqrt(g) - Z)||_F for device S, Z (n x n), by FP64 GEMMs. */
int zf_guess_label(const double* S, const double* Z, int n, double* c, void* stream);
int zf_mlp_set_params(const float* host_params, int count);  /* count must be 4931 */
int zf_mlp_get_params(float* host_params, int count);
/* standardization: x' = (x - mu_x) / sd_x (8 each), y = y' sd_y + mu_y (3 each) */
int zf_mlp_set_norm(const float* mu_x, const float* sd_x, const float* mu_y, const float* sd_y);
/* zf_mlp_save / zf_mlp_load -- the loaded network (normalization and parameters) to / from
 * a file at path (host string): magic "ZFMLP\0\0\1", int32 {8, 64, 3, 4931}, float32
 * mu_x[8], sd_x[8], mu_y[3], sd_y[3], float32 parameters[4931], little-endian.  Save
 * needs a loaded network; load validates the magic, shape, size and finiteness and
 * leaves the current network untouched on any error (ZF_ERR_ARG). */
int zf_mlp_save(const char* path);
int zf_mlp_load(const char* path);
/* one Adam step (beta 0.9 / 0.999, eps 1e-8) on the mean squared error of the standardized
 * labels; feats (batch x 8) and labels (batch x 3, raw c) are device FP32; loss (host) may
 * be NULL (then the call does not synchronize). */
int zf_mlp_train_step(const float* feats, const float* labels, int batch, float lr, float* loss,
                      void* stream);
/* gradient of that loss (host, 4931 floats) and the loss, without updating (for checks) */
int zf_mlp_grad(const float* feats, const float* labels, int batch, float* grad_host,
                float* loss_host, void* stream);
/* raw coefficients (host, 3 doubles) predicted for one device feature vector */
int zf_mlp_predict(const float* feats, double* coef_host, void* stream);

/* zf_congruence -- Hp = Z^T H Z, the congruence transform that turns the generalized
 * eigenproblem H C = S C eps into the standard one Hp C' = C' eps once Z^T S Z = I
 * (Sec. II.A, Eq. standard_form, with C' = Z^{-1} C).
 *   H:  device, n x n FP64, row-major, symmetric (only its symmetry is assumed: the
 *       first product reads H's rows as its columns).
 *   Z:  device, n x n FP64, row-major (typically the Z returned by zf_refine).
 *   Hp: device, n x n FP64, row-major, written in full and exactly symmetric (the upper
 *       triangle is computed and mirrored).  Hp may alias H or Z: both are copied into
 *       the library's workspace before anything is written.
 *   precision: the arithmetic of both products, as for zf_refine's first phase:
 *       ZF_FP64 (FP64 matrix cores), ZF_BF16X3 / ZF_FP16X3 (split halves, three
 *       products, FP32 accumulation), ZF_BF16 / ZF_FP16 ((h)(h) only), ZF_FP32.  With
 *       FP16 halves the entries of H, Z and Z^T H must stay below 65504 in magnitude.
 *   Stream-ordered; does not synchronize.  Errors: ZF_ERR_ARG (NULL pointer, n < 1 or
 *   n > 46000, unknown precision), ZF_ERR_NOMEM, ZF_ERR_HIP; on error Hp is undefined. */
int zf_congruence(const double* H, const double* Z, int n, int precision, double* Hp,
                  void* stream);

/* zf_residual -- rms = ||Z^T S Z - I||_F / sqrt(n), the residual every result is judged
 * by, evaluated with the FP64 matrix-core products of the refinement phase (Sec. IV.B:
 * S Z, then the symmetric Z^T (S Z), and a fixed-order FP64 sum of squares).
 *   S, Z: device n x n FP64 (S symmetric), read only.  rms: host double.
 * Synchronizes the stream.  Errors: ZF_ERR_ARG (NULL pointer, n < 1), ZF_ERR_NOMEM,
 * ZF_ERR_HIP. */
int zf_residual(const double* S, const double* Z, int n, double* rms, void* stream);

/* zf_residual_noalloc -- zf_residual for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * The same FP64 products and the same fixed-order norm, on a device array of the
 * library (24 MiB per GPU, held until the process ends), for n <= 1024.
 *   S, Z:    device n x n FP64 (S symmetric), read only.
 *   rms_dev: device pointer to one double, receives ||Z^T S Z - I||_F / sqrt(n),
 *            bitwise equal to zf_residual's value for the same inputs.
 * Stream-ordered: enqueues its kernels on stream and returns without synchronizing.
 * Allocates nothing.  Every call on one GPU uses that GPU's array: calls that overlap
 * on one GPU (other streams or threads) race.  Errors: ZF_ERR_ARG (NULL pointer, n
 * outside 1..1024), ZF_ERR_HIP. */
int zf_residual_noalloc(const double* S, const double* Z, int n, double* rms_dev, void* stream);

/* zf_release -- free every cached workspace of the current device. */
void zf_release(void);

/* zf_last_error -- message for the last nonzero return on this host thread ("" if none). */
const char* zf_last_error(void);

/* zf_version -- ABI version (increases when an entry point changes). */
int zf_version(void);

/*
 * Per-kernel timing with HIP events recorded on the caller's stream around each
 * matrix-core GEMM launch (for roofline accounting).  Kernel classes:
 *   0 gemm_x3, 1 gemm_x3_sym, 2 gemm_f64, 3 gemm_f64_sym.
 * zf_profile_enable(1) starts recording (events add a few microseconds per
 * launch); totals accumulate until zf_profile_reset().  zf_profile_read fills
 * the class name (static string), launch count, summed milliseconds and
 * executed matrix-core flops (2 * tile^3 per tile step, three products per step
 * for gemm_x3).  Returns ZF_ERR_ARG for an unknown class.
 */
void zf_profile_enable(int on);
void zf_profile_reset(void);
int zf_profile_read(int cls, const char** name, long long* launches, double* total_ms,
                    double* flops);

/*
 * Kernel-level entry points, exported for unit tests.  They run one library
 * kernel on caller data through padded internal buffers.
 *
 * zf_t_split -- two-term split of Sec. III.A (Eq. splitStyle): for each of the
 *   count FP64 values a (device), x = FP32[a] (round to nearest even), hi = LP[x],
 *   lo = LP[x - hi], LP = BF16 (fmt 1) or FP16 (fmt 2), round to nearest even.
 *   hi, lo: device arrays of count raw 16-bit patterns.
 */
int zf_t_split(const double* a, int64_t count, uint16_t* hi, uint16_t* lo, int fmt,
               void* stream);

/*
 * zf_t_gemm -- one GEMM with its epilogue:
 *   C = alpha * D + beta * (A B^T) + gamma * I      (all device, FP64, row-major)
 *   A: m x k (ld k), B: nn x k (ld k), D: m x nn (ld nn) or NULL, C: m x nn (ld nn).
 *   precision ZF_FP64 runs the FP64 matrix-core kernel; ZF_BF16X3 splits A and B
 *   (as zf_t_split) and runs the (h)(h)+(h)(l)+(l)(h) kernel with FP32 accumulation
 *   (Sec. III.B); ZF_BF16 the (h)(h) product of the same split; ZF_FP32 rounds A
 *   and B to FP32 and runs the FP32 matrix-core kernel (the "single" of Table I).
 *   sym != 0 requires m == nn, computes only tiles on or above the
 *   diagonal and mirrors them (valid when A B^T is symmetric).
 *   norm_sq (host, may be NULL) receives the sum of C_ij^2 in FP64.
 */
int zf_t_gemm(int precision, int sym, int m, int nn, int k, const double* A, const double* B,
              double alpha, const double* D, double beta, double gamma, double* C,
              double* norm_sq, void* stream);

/*
 * zf_t_gemm_kb -- zf_t_gemm for the 16-bit-pair precisions (ZF_BF16X3, ZF_BF16,
 * ZF_FP16X3, ZF_FP16) with both operands split into the K-blocked layout that the
 * solver keeps its pairs in: with r rows (padded), element (i, k) at
 * (k / 32) * 32 r + 32 i + k % 32, i.e. 32-wide blocks of the contracted index, each
 * a row-major panel.  The products and their summation order are those of
 * zf_t_gemm, so C and norm_sq equal its results bit for bit.  Other precisions
 * return ZF_ERR_ARG.
 */
int zf_t_gemm_kb(int precision, int sym, int m, int nn, int k, const double* A, const double* B,
                 double alpha, const double* D, double beta, double gamma, double* C,
                 double* norm_sq, void* stream);

/*
 * zf_t_ozaki -- zf_t_gemm's product and epilogue with A B^T emulated from `slices`
 * (1..8) 7-bit integer slices per operand row on the int8 matrix cores (the
 * refinement residual's arithmetic under ZF_REFINE_EMU): row i of A is scaled by
 * 2^-e_i (e_i the frexp exponent of its largest magnitude) and cut into slices
 * a_p (|a_p| <= 127) by repeated truncation of 128 times the rest; the products
 * a_p b_q^T with p + q <= slices + 1 are summed exactly in int32 per weight 2^-7(p+q)
 * and the weights combined in FP64 from the smallest.  max(m, nn, k) <= 16384.
 * A row holding a non-finite entry gives NaN products.
 */
int zf_t_ozaki(int slices, int sym, int m, int nn, int k, const double* A, const double* B,
               double alpha, const double* D, double beta, double gamma, double* C,
               double* norm_sq, void* stream);

/*
 * zf_t_crt -- zf_t_gemm's product and epilogue with A B^T emulated through residues
 * (the refinement residual's arithmetic under ZF_REFINE_CRT): row i of A is scaled
 * by 2^(beta - e_i) (e_i the frexp exponent of its largest magnitude) and truncated
 * toward zero to an integer; with M the product of the first `moduli` (2..15) of the
 * pairwise coprime moduli 256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223,
 * 217, 211, 199, 197, beta is the largest value with 4 k 4^beta <= M (at most 52).
 * The exact integer product of the truncated rows is formed from one int8 product
 * per modulus and the Chinese remainder theorem, then scaled by 2^(e_i + f_j -
 * 2 beta).  max(m, nn, k) <= 16384.  A row holding a non-finite entry gives NaN
 * products.
 */
int zf_t_crt(int moduli, int sym, int m, int nn, int k, const double* A, const double* B,
             double alpha, const double* D, double beta, double gamma, double* C,
             double* norm_sq, void* stream);

/* zf_t_gershgorin -- g = max_i sum_j |S_ij| (host double) for device S (n x n). */
int zf_t_gershgorin(const double* S, int n, double* g, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* ZF_H */
