// Batched refinement: many overlap matrices of uneven order refined together.
//
// Every matrix runs the same recursion as zf_refine_ex (Sec. III, Algorithm 2 in
// the low-precision phase, the FP64 refinement phase of Sec. IV.B), but the
// matrices advance in lockstep "macro-sweeps".  One macro-sweep is
//
//   L1  grouped BF16x3 GEMM  A^T = Z^T S           (matrices in the low phase)
//   L2  grouped BF16x3 GEMM  delta = I - Z^T A     (symmetric, norm partials)
//   H1  grouped FP64 GEMM    A^T = Z^T S           (matrices in the FP64 phase)
//   H2  grouped FP64 GEMM    delta = I - Z^T A     (symmetric, norm partials)
//   DECIDE  per matrix: Err, history, stop test, next action (device-side); a
//           matrix whose low phase stops waits (parked) until every low phase has
//           stopped, then all enter the FP64 phase together, so that the FP64
//           stages run once per macro-sweep with every matrix in them
//   WIDEN   FP32 -> FP64 Z for matrices that just entered the FP64 phase
//   U3  grouped BF16x3 GEMM  Q = c1 delta + c2 delta^2  (matrices updating)
//   U4  grouped BF16x3 GEMM  Z_new = Z + Z Q           (matrices updating)
//
// Each grouped GEMM is one persistent launch over a static table of (matrix,
// tile) tasks; a task whose matrix is not in that stage is skipped on the device,
// so the macro-sweep is a fixed sequence of launches.  A run of macro-sweeps is
// captured once in a HIP graph; every kernel of a macro-sweep first reads the
// device-side count of live matrices and returns at once when it is zero, so
// macro-sweeps past the last matrix's stop cost only their launches (about 50 us
// each for the 512-matrix batch).  The graph holds 8 macro-sweeps by default and is
// launched until the live count, read after each launch, is zero: one host
// synchronization per 8 macro-sweeps and at most 7 idle ones.  (The 512-matrix batch
// takes 13 macro-sweeps: 51.2-51.9 ms with 1, 2, 4 or 8 per graph, 56.5 ms with all
// 113 that the caps allow in one graph.)  The tile edge of each
// matrix (64 or 128) comes from a table indexed by its order, filled by
// zf_batched_autotune or left at its defaults.
//
// Set-up (once, before the graph): split S; for matrices taking the learned guess
// the grouped BF16x3 S^2 (stage S2), then per-matrix statistics and features, one
// network inference per matrix and the acceptance test on the device; Z0 last.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "zf.h"
#include "zf_internal.h"
#include "gemm_tiles.inc"

namespace zf {

#define BHIP_TRY(expr)                                                                       \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess)                                                                    \
      return set_error(ZF_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                       __LINE__);                                                            \
  } while (0)

enum { PH_LOW = 0, PH_HIGH = 1 };
// ACT_PARKED: the low phase has stopped and the FP64 phase waits for every other
// matrix's low phase to stop, so that the FP64 stages run with all matrices at once.
enum { ACT_EVAL = 0, ACT_UPDATE = 1, ACT_TRANSITION = 2, ACT_DONE = 3, ACT_PARKED = 4 };
enum { OP_L1 = 0, OP_L2, OP_H1, OP_H2, OP_U3, OP_U4, OP_S2 };

// Per-matrix record: buffers (carved from one arena) and the device-side state of
// the recursion.  Only the DECIDE kernel writes the state.
struct BMat {
  int n, np, tile, tiles_sym;  // BF16x3 tile edge and its upper-triangle tile count
  int ftiles_sym;              // upper-triangle count of the 64-wide FP64 tiles
  long long pbase;  // first norm partial of this matrix (room for the larger count)
  int phase, action, it, cur, src;
  int upd_l, upd_h, evals_l, evals_h, flags, status, hist_len;
  int learn, z0_used;  // learned guess requested; guess taken (ZF_Z0_*)
  double prev, err_l, err_h;
  double* hist;
  u16 *s_hi, *s_lo, *zr_hi[2], *zr_lo[2], *zc_hi[2], *zc_lo[2];
  u16 *at_hi, *at_lo, *d_hi, *d_lo, *q_hi, *q_lo;
  float* z32[2];
  double *s64, *z64r[2], *z64c[2], *a64t, *d64;
};

// ---------------------------------------------------------------------------
// grouped GEMMs
// ---------------------------------------------------------------------------
// BF16x3 tiles: 64- or 128-wide, 4 waves, 2-stage load ring, two blocks per CU (in
// grouped launches this beat 8 waves with a 3-stage ring: 55.6 vs 60 ms for the
// 512-matrix batch); one grouped launch per tile edge.  FP64 tiles: 64 wide for every
// matrix, 4 waves.
template <int T>
using X3G = X3Cfg<T, T, 32, 2, 2>;
using F64_64 = F64Cfg<64, 64, 16, 2, 2>;
static_assert(F64_64::NT == 256, "the grouped FP64 kernel runs 256-thread blocks");

__device__ __forceinline__ bool op_applies(int op, const BMat& M) {
  const int phase = M.phase, action = M.action;
  switch (op) {
    case OP_S2:
      return M.learn != 0;
    case OP_L1:
    case OP_L2:
      return phase == PH_LOW && action != ACT_DONE && action != ACT_PARKED;
    case OP_H1:
    case OP_H2:
      return phase == PH_HIGH && action != ACT_DONE;
    default:
      return action == ACT_UPDATE;
  }
}

// Task tables are XCD-major: seg[0..16] bounds 16 runs of tasks, runs 0-7 with
// 128-wide tiles and runs 8-15 with 64-wide ones, run 8 p + x for XCD x.  Blocks are
// dispatched round-robin over the 8 XCDs (block b on XCD b % 8), so block b walks
// run x = b % 8 of its tile edge with stride gridDim.x / 8: the tiles of one matrix
// run together on one XCD and share its L2 (the grid is a multiple of 8).
__device__ __forceinline__ void xcd_run(const int* seg, int part, int& t0, int& t1, int& step) {
  const int x = blockIdx.x & 7;
  t0 = seg[8 * part + x] + (int)(blockIdx.x >> 3);
  t1 = seg[8 * part + x + 1];
  step = gridDim.x >> 3;
}

template <int T>
__global__ void __launch_bounds__(X3G<T>::NT, 2)
    grouped_x3_kernel(const TileTask* __restrict__ tasks, const int* __restrict__ seg,
                      const BMat* __restrict__ mats, int op, double c1, double c2,
                      double* partials, const int* __restrict__ live) {
  using CF = X3G<T>;
  __shared__ __attribute__((aligned(16))) u16 lds[2 * CF::STAGE_ELEMS];
  __shared__ double red[CF::NT / 64];
  if (live && *live == 0) return;  // no matrix in this stage
  int t0, t1, step;
  xcd_run(seg, T == 128 ? 0 : 1, t0, t1, step);
  for (int t = t0; t < t1; t += step) {
    const TileTask tk = tasks[t];
    const BMat& M = mats[tk.m];
    if (!op_applies(op, M)) continue;
    const int np = M.np;
    EpiParams ep;
    memset(&ep, 0, sizeof ep);
    ep.beta = 1.0;
    ep.ld = np;
    ep.n_valid = M.n;
    ep.kb = 1;  // the arena's pairs are K-blocked (kb_offset)
    const u16 *ah, *al, *bh, *bl;
    int mode = 0, pidx = 0;
    if (op == OP_L1) {
      ah = M.zc_hi[M.cur];
      al = M.zc_lo[M.cur];
      bh = M.s_hi;
      bl = M.s_lo;
      ep.ohi = M.at_hi;
      ep.olo = M.at_lo;
    } else if (op == OP_L2) {
      ah = M.zc_hi[M.cur];
      al = M.zc_lo[M.cur];
      bh = M.at_hi;
      bl = M.at_lo;
      ep.beta = -1.0;
      ep.gamma = 1.0;
      ep.ohi = ep.othi = M.d_hi;
      ep.olo = ep.otlo = M.d_lo;
      ep.partials = partials + M.pbase;
    } else if (op == OP_S2) {  // S^2 (symmetric) into the second FP32 master
      ah = bh = M.s_hi;
      al = bl = M.s_lo;
      ep.o32 = ep.ot32 = M.z32[1];
    } else if (op == OP_U3) {
      ah = bh = M.d_hi;
      al = bl = M.d_lo;
      ep.alpha = c1;
      ep.beta = c2;
      if (M.phase == PH_HIGH) ep.d64 = M.d64;
      else {
        ep.dhi = M.d_hi;
        ep.dlo = M.d_lo;
      }
      ep.ohi = ep.othi = M.q_hi;
      ep.olo = ep.otlo = M.q_lo;
    } else {  // OP_U4: Z[cur] = Z[src] + Z[src] Q
      ah = M.zr_hi[M.src];
      al = M.zr_lo[M.src];
      bh = M.q_hi;
      bl = M.q_lo;
      ep.alpha = 1.0;
      ep.ohi = M.zr_hi[M.cur];
      ep.olo = M.zr_lo[M.cur];
      if (M.phase == PH_HIGH) {
        ep.d64 = M.z64r[M.src];
        ep.o64 = M.z64r[M.cur];
        ep.ot64 = M.z64c[M.cur];
      } else {
        ep.d32 = M.z32[M.src];
        ep.o32 = M.z32[M.cur];
        ep.othi = M.zc_hi[M.cur];
        ep.otlo = M.zc_lo[M.cur];
      }
    }
    const bool sym = (op == OP_L2 || op == OP_U3 || op == OP_S2);
    if (sym) {
      mode = (tk.ti == tk.tj) ? 2 : 1;
      // index of (ti, tj) in the row-major upper triangle of a T x T tile grid
      const int tiles = np / T;
      pidx = tk.ti * tiles - tk.ti * (tk.ti - 1) / 2 + (tk.tj - tk.ti);
    }
    x3_tile<T, T, 32, 2, 2>(ah, al, 32, bh, bl, 32, np, tk.ti * T, tk.tj * T, mode, ep, pidx, lds,
                            red, 32 * np, 32 * np);
    __syncthreads();
  }
}

// FP64 stages use 64-wide tiles for every matrix (their own task tables, all in the
// 64-wide runs): four blocks per CU, the single path's choice.
__global__ void __launch_bounds__(256, 4)
    grouped_f64_kernel(const TileTask* __restrict__ tasks, const int* __restrict__ seg,
                       const BMat* __restrict__ mats, int op, double* partials,
                       const int* __restrict__ live) {
  __shared__ double lds[2 * F64_64::STAGE];
  __shared__ double red[4];
  if (*live == 0) return;  // no matrix in this stage
  int t0, t1, step;
  xcd_run(seg, 1, t0, t1, step);
  for (int t = t0; t < t1; t += step) {
    const TileTask tk = tasks[t];
    const BMat& M = mats[tk.m];
    if (!op_applies(op, M)) continue;
    const int np = M.np;
    constexpr int T = 64;
    EpiParams ep;
    memset(&ep, 0, sizeof ep);
    ep.beta = 1.0;
    ep.ld = np;
    ep.n_valid = M.n;
    ep.kb = 1;  // the delta pair it writes is K-blocked
    const double *a, *b;
    int mode = 0, pidx = 0;
    if (op == OP_H1) {
      a = M.z64c[M.cur];
      b = M.s64;
      ep.o64 = M.a64t;
    } else {  // OP_H2
      a = M.z64c[M.cur];
      b = M.a64t;
      ep.beta = -1.0;
      ep.gamma = 1.0;
      ep.o64 = ep.ot64 = M.d64;
      ep.ohi = ep.othi = M.d_hi;
      ep.olo = ep.otlo = M.d_lo;
      ep.partials = partials + M.pbase;
      mode = (tk.ti == tk.tj) ? 2 : 1;
      const int tiles = np / T;
      pidx = tk.ti * tiles - tk.ti * (tk.ti - 1) / 2 + (tk.tj - tk.ti);
    }
    f64_tile<64, 64, 16, 2, 2>(a, np, b, np, np, tk.ti * 64, tk.tj * 64, mode, ep, pidx, lds, red);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// device-side stop test (Algorithm 2, Sec. IV.A) and phase changes
// ---------------------------------------------------------------------------
__global__ void decide_kernel(BMat* mats, int count, const double* __restrict__ partials, int order,
                              int rule, int max_l, int max_h, int refine_on, int hist_cap,
                              int* remaining) {
  // remaining[0]: matrices not yet done; remaining[1]: macro-sweeps that had any;
  // the matrices each stage will find: [2] low-phase evaluations of the next
  // macro-sweep, [3] FP64 evaluations of the next macro-sweep, [4] updates of this
  // macro-sweep, [5] widenings of this macro-sweep (each stage returns at once on 0)
  if (remaining[0] == 0) return;
  __shared__ int live, low_running, n_high, n_upd, n_trans;
  if (threadIdx.x == 0) {
    live = 0;
    low_running = 0;
    n_high = 0;
    n_upd = 0;
    n_trans = 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    BMat& M = mats[i];
    if (M.action == ACT_DONE) continue;
    if (M.action == ACT_PARKED) {  // not evaluated: waiting for the other low phases
      atomicAdd(&live, 1);
      continue;
    }
    // every matrix not yet done was evaluated in this macro-sweep
    double s = 0.0;
    const int parts = (M.phase == PH_HIGH) ? M.ftiles_sym : M.tiles_sym;  // phase just evaluated
    for (int t = 0; t < parts; ++t) s += partials[M.pbase + t];
    const double err = sqrt(s);
    if (M.hist_len < hist_cap) M.hist[M.hist_len] = err;
    M.hist_len++;
    if (M.phase == PH_LOW) M.evals_l++;
    else M.evals_h++;
    if (!isfinite(err)) {
      M.status = ZF_ERR_NONFINITE;
      M.action = ACT_DONE;
      continue;
    }
    const int it = M.it;
    bool stop = false;
    if (it > 0) stop = (rule == ZF_STOP_MONOTONE) ? (err >= M.prev) : (err > pow(M.prev, (double)(order + 1)));
    const int cap = (M.phase == PH_LOW) ? max_l : max_h;
    bool finish = false;
    int upd = it;
    double chosen = err;
    if (stop) {
      finish = true;
      if (err > M.prev) {  // the previous iterate is still in the other buffer
        M.cur ^= 1;
        upd = it - 1;
        chosen = M.prev;
      }
    } else if (it >= cap) {
      finish = true;
      M.flags |= ZF_WARN_MAXSWEEPS;
    }
    if (finish) {
      if (M.phase == PH_LOW) {
        M.upd_l = upd;
        M.err_l = chosen;
        if (refine_on) {
          M.action = ACT_PARKED;
        } else {
          M.action = ACT_DONE;
        }
      } else {
        M.upd_h = upd;
        M.err_h = chosen;
        M.action = ACT_DONE;
      }
    } else {
      M.prev = err;
      M.it = it + 1;
      M.src = M.cur;
      M.cur ^= 1;
      M.action = ACT_UPDATE;
    }
    if (M.action != ACT_DONE) atomicAdd(&live, 1);
    if (M.phase == PH_LOW && M.action != ACT_DONE && M.action != ACT_PARKED)
      atomicAdd(&low_running, 1);
    if (M.phase == PH_HIGH && M.action != ACT_DONE) atomicAdd(&n_high, 1);
    if (M.action == ACT_UPDATE) atomicAdd(&n_upd, 1);
  }
  __syncthreads();
  // once no low phase is running, every parked matrix enters the FP64 phase together
  if (low_running == 0) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) {
      BMat& M = mats[i];
      if (M.action != ACT_PARKED) continue;
      M.phase = PH_HIGH;
      M.it = 0;
      M.action = ACT_TRANSITION;
      atomicAdd(&n_high, 1);
      atomicAdd(&n_trans, 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    remaining[0] = live;
    remaining[1] += 1;
    remaining[2] = low_running;
    remaining[3] = n_high;
    remaining[4] = n_upd;
    remaining[5] = n_trans;
  }
}

// remaining[0] = count (every matrix live), remaining[1] = 0 macro-sweeps, every
// matrix starting in the low phase, no update, FP64 evaluation or widening pending
__global__ void b_reset_kernel(int* remaining, int count) {
  if (threadIdx.x == 0) {
    remaining[0] = count;
    remaining[1] = 0;
    remaining[2] = count;
    remaining[3] = 0;
    remaining[4] = 0;
    remaining[5] = 0;
  }
}

// ---------------------------------------------------------------------------
// element-wise batched kernels: grid (tiles, count); block (x, m) handles the 64 x 64
// tile x of matrix m's padded np x np layout (row-major tile order) and exits at
// once when m has fewer tiles or is not in the kernel's stage.  Transposed copies
// go through a padded LDS tile so that both layouts are written coalesced.
// ---------------------------------------------------------------------------
constexpr int kET = 64;  // element-wise tile edge (np is a multiple of it)

__device__ __forceinline__ bool tile_of(const BMat& M, int& i0, int& j0) {
  const int T = M.np / kET;
  if ((int)blockIdx.x >= T * T) return false;
  i0 = ((int)blockIdx.x / T) * kET;
  j0 = ((int)blockIdx.x % T) * kET;
  return true;
}

// S_m (n x n) -> BF16 pair (K-blocked, kb_offset) and (optionally) FP64 copy,
// zero-padded to np x np
__global__ void __launch_bounds__(256) b_split_kernel(const BMat* __restrict__ mats,
                                                      const double* const* S, int with64) {
  const BMat& M = mats[blockIdx.y];
  int i0, j0;
  if (!tile_of(M, i0, j0)) return;
  const double* Sm = S[blockIdx.y];
  for (int e = threadIdx.x; e < kET * kET; e += 256) {
    const int i = i0 + e / kET, j = j0 + e % kET;
    const double a = (i < M.n && j < M.n) ? Sm[(size_t)i * M.n + j] : 0.0;
    const size_t le = (size_t)i * M.np + j;
    u16 h, l;
    split_bf16((float)a, h, l);
    const size_t ke = kb_offset(i, j, M.np);
    M.s_hi[ke] = h;
    M.s_lo[ke] = l;
    if (with64) M.s64[le] = a;
  }
}

// Per-matrix statistics: stats[4m..] = {g = max r_i, g_lo = min (S_ii - (r_i - |S_ii|)),
// mean r_i, tr S}, r_i = sum_j |S_ij|.  Matrices taking the learned guess also get
// the Frobenius products ||S||^2, <S, S^2>, ||S^2||^2 (S^2 from stage S2, FP32 in
// z32[1]) and their 8 features.  Pass 1: one block per chunk of kStatRows rows (one
// wave per row), 7 partial values per chunk; pass 2: one thread per matrix folds its
// chunks in order.  Fixed-order reductions: repeatable bit for bit.
constexpr int kStatRows = 32;

__global__ void __launch_bounds__(256) b_stats_rows_kernel(const BMat* __restrict__ mats,
                                                           const double* const* S, int chunks,
                                                           double* __restrict__ part) {
  const int m = blockIdx.y, c = blockIdx.x;
  const BMat& M = mats[m];
  const int n = M.n, np = M.np;
  const int r0 = c * kStatRows;
  if (r0 >= n) return;
  const int r1 = r0 + kStatRows < n ? r0 + kStatRows : n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double* Sm = S[m];
  const float* S2 = M.z32[1];
  const bool learn = M.learn != 0;
  __shared__ double red[4][7];
  double mx = 0.0, mn = 1e300, sm = 0.0, tr = 0.0, a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int i = r0 + wave; i < r1; i += 4) {
    const double* row = Sm + (size_t)i * n;
    double r = 0.0;
    for (int j = lane; j < n; j += 64) {
      const double v = row[j];
      r += fabs(v);
      if (learn) {
        const double q = (double)S2[(size_t)i * np + j];
        a0 += v * v;
        a1 += v * q;
        a2 += q * q;
      }
    }
    for (int o = 32; o > 0; o >>= 1) r += __shfl_xor(r, o, 64);
    const double d = row[i];
    mx = fmax(mx, r);
    mn = fmin(mn, d - (r - fabs(d)));
    sm += r;
    tr += d;
  }
  for (int o = 32; o > 0; o >>= 1) {
    a0 += __shfl_xor(a0, o, 64);
    a1 += __shfl_xor(a1, o, 64);
    a2 += __shfl_xor(a2, o, 64);
  }
  if (lane == 0) {
    red[wave][0] = mx;
    red[wave][1] = mn;
    red[wave][2] = sm;
    red[wave][3] = tr;
    red[wave][4] = a0;
    red[wave][5] = a1;
    red[wave][6] = a2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      red[0][0] = fmax(red[0][0], red[w][0]);
      red[0][1] = fmin(red[0][1], red[w][1]);
      for (int k = 2; k < 7; ++k) red[0][k] += red[w][k];
    }
    double* o = part + ((size_t)m * chunks + c) * 7;
    for (int k = 0; k < 7; ++k) o[k] = red[0][k];
  }
}

__global__ void b_stats_final_kernel(const BMat* __restrict__ mats, int count, int chunks,
                                     const double* __restrict__ part, double* g, double* stats,
                                     float* feats) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= count) return;
  const BMat& M = mats[m];
  const int n = M.n;
  const int used = (n + kStatRows - 1) / kStatRows;
  const double* p = part + (size_t)m * chunks * 7;
  double v[7] = {p[0], p[1], p[2], p[3], p[4], p[5], p[6]};
  for (int c = 1; c < used; ++c) {
    const double* q = p + 7 * c;
    v[0] = fmax(v[0], q[0]);
    v[1] = fmin(v[1], q[1]);
    for (int k = 2; k < 7; ++k) v[k] += q[k];
  }
  g[m] = v[0];
  stats[4 * m + 0] = v[0];
  stats[4 * m + 1] = v[1];
  stats[4 * m + 2] = v[2] / n;
  stats[4 * m + 3] = v[3];
  float* f = feats + 8 * (size_t)m;
  if (M.learn)
    finish_features(v[0], v[1], v[2] / n, v[3], v[4], v[5], v[6], n, f);
  else
    for (int k = 0; k < 8; ++k) f[k] = 0.f;
}

// Acceptance of the predicted coefficients (one thread per matrix); on success
// coef[4m + 3] = g and the guess is marked learned, else the scaled identity with
// ZF_WARN_Z0_FALLBACK.
__global__ void b_accept_kernel(BMat* mats, int count, const double* __restrict__ stats,
                                double* coef) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= count) return;
  BMat& M = mats[m];
  if (!M.learn) return;
  double c[3] = {coef[4 * m], coef[4 * m + 1], coef[4 * m + 2]};
  const double g = stats[4 * m], glo = stats[4 * m + 1];
  bool ok = (g > 0.0) && isfinite(c[0]) && isfinite(c[1]) && isfinite(c[2]);
  if (ok) ok = accept_poly(c, glo > 0.0 ? glo / g : 0.0);
  if (ok) {
    coef[4 * m] = c[0];
    coef[4 * m + 1] = c[1];
    coef[4 * m + 2] = c[2];
    coef[4 * m + 3] = g;
    M.z0_used = ZF_Z0_LEARNED;
  } else {
    M.z0_used = ZF_Z0_SCALED_IDENTITY;
    M.flags |= ZF_WARN_Z0_FALLBACK;
  }
}

// Z0 into Z32, Zr and Zc of buffer 0 (the pairs K-blocked): given, learned (c0 I +
// c1 S/g + c2 (S/g)^2) / sqrt(g) with S^2 from z32[1], or I / sqrt(g)
__global__ void __launch_bounds__(256) b_init_kernel(const BMat* __restrict__ mats,
                                                     const double* const* Z0, const double* const* S,
                                                     const double* __restrict__ g,
                                                     const double* __restrict__ coef) {
  __shared__ u16 th[kET][kET + 1], tl[kET][kET + 1];
  const int m = blockIdx.y;
  const BMat& M = mats[m];
  int i0, j0;
  if (!tile_of(M, i0, j0)) return;
  const int n = M.n, np = M.np;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (M.z0_used == ZF_Z0_LEARNED) {
    const double* cg = coef + 4 * (size_t)m;
    const double gg = cg[3], sg = 1.0 / sqrt(gg);
    a0 = cg[0] * sg;
    a1 = cg[1] * sg / gg;
    a2 = cg[2] * sg / (gg * gg);
  } else if (M.z0_used == ZF_Z0_SCALED_IDENTITY) {
    a0 = 1.0 / sqrt(g[m]);
  }
  for (int e = threadIdx.x; e < kET * kET; e += 256) {
    const int r = e / kET, c = e % kET;
    const int i = i0 + r, j = j0 + c;
    const size_t le = (size_t)i * np + j;
    double v = 0.0;
    if (i < n && j < n) {
      if (M.z0_used == ZF_Z0_GIVEN)
        v = Z0[m][(size_t)i * n + j];
      else if (M.z0_used == ZF_Z0_LEARNED)
        v = a1 * S[m][(size_t)i * n + j] + a2 * (double)M.z32[1][le] + (i == j ? a0 : 0.0);
      else
        v = (i == j) ? a0 : 0.0;
    }
    const float f = (float)v;
    u16 h, l;
    split_bf16(f, h, l);
    M.z32[0][le] = f;
    const size_t ke = kb_offset(i, j, np);
    M.zr_hi[0][ke] = h;
    M.zr_lo[0][ke] = l;
    th[r][c] = h;
    tl[r][c] = l;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kET * kET; e += 256) {
    const int r = e / kET, c = e % kET;  // transposed row j0 + r, column i0 + c
    const size_t t = kb_offset(j0 + r, i0 + c, np);
    M.zc_hi[0][t] = th[c][r];
    M.zc_lo[0][t] = tl[c][r];
  }
}

// FP32 master -> FP64 row-major and transposed for matrices entering the FP64 phase.
// It runs in every macro-sweep but has work in one, so it is a fixed grid walking the
// (matrix, 64 x 64 tile) pairs with a stride rather than a grid of every pair: the
// launches without work cost one read of the count.
__global__ void __launch_bounds__(256) b_widen_kernel(const BMat* __restrict__ mats, int count,
                                                      int etiles, const int* __restrict__ live) {
  __shared__ float tv[kET][kET + 1];
  if (*live == 0) return;
  const long long total = (long long)count * etiles;
  for (long long w = blockIdx.x; w < total; w += gridDim.x) {
    const int m = (int)(w / etiles), et = (int)(w - (long long)m * etiles);
    const BMat& M = mats[m];
    if (M.action != ACT_TRANSITION) continue;  // uniform over the block
    const int T = M.np / kET;
    if (et >= T * T) continue;
    const int i0 = (et / T) * kET, j0 = (et % T) * kET;
    const int np = M.np, cur = M.cur;
    const float* __restrict__ src = M.z32[cur];
    double* __restrict__ dr = M.z64r[cur];
    double* __restrict__ dc = M.z64c[cur];
    constexpr int PER = kET * kET / 256;
    float f[PER];  // every load of the tile requested before any store
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + 256 * q, r = e / kET, c = e % kET;
      f[q] = src[(size_t)(i0 + r) * np + j0 + c];
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + 256 * q, r = e / kET, c = e % kET;
      dr[(size_t)(i0 + r) * np + j0 + c] = (double)f[q];
      tv[r][c] = f[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + 256 * q, r = e / kET, c = e % kET;
      dc[(size_t)(j0 + r) * np + i0 + c] = (double)tv[c][r];
    }
    __syncthreads();  // tv is rewritten by the next pair
  }
}

// unpadded result: FP64 iterate if the FP64 phase ran, else the FP32 master
__global__ void __launch_bounds__(256) b_output_kernel(const BMat* __restrict__ mats,
                                                       double* const* Z, int from64) {
  const BMat& M = mats[blockIdx.y];
  int i0, j0;
  if (!tile_of(M, i0, j0)) return;
  double* Zm = Z[blockIdx.y];
  for (int e = threadIdx.x; e < kET * kET; e += 256) {
    const int i = i0 + e / kET, j = j0 + e % kET;
    if (i >= M.n || j >= M.n) continue;
    const size_t src = (size_t)i * M.np + j;
    Zm[(size_t)i * M.n + j] = from64 ? M.z64r[M.cur][src] : (double)M.z32[M.cur][src];
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// tile edge per order bucket: n <= g_tile_max[k] uses g_tile_edge[k]
static int g_tile_nb = 4;
static int g_tile_max[16] = {128, 256, 512, 1 << 30};
static int g_tile_edge[16] = {64, 64, 128, 128};
static bool g_use_graph = true;
static int g_graph_sweeps = 8;  // macro-sweeps per graph; 0 = every one the caps allow
static int g_last_sweeps = 0, g_last_launches = 0;  // of the last call (zf_batched_last_stats)

static int tile_for(int n) {
  for (int k = 0; k < g_tile_nb; ++k)
    if (n <= g_tile_max[k]) return g_tile_edge[k];
  return 128;
}

static int rup(long long n, int g) { return (int)((n + g - 1) / g * g); }
static inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct BatchState {
  int device = -1;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  void* meta = nullptr;  // device: mats, tasks, offsets, pointer tables, partials, hist, scalars
  size_t meta_bytes = 0;
  int* pinned = nullptr;
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<char> key;  // layout the captured graph was built for
};
static BatchState g_b;

static void batch_release() {
  if (g_b.exec) (void)hipGraphExecDestroy(g_b.exec);
  if (g_b.arena) (void)hipFree(g_b.arena);
  if (g_b.meta) (void)hipFree(g_b.meta);
  if (g_b.pinned) (void)hipHostFree(g_b.pinned);
  if (g_b.cap) (void)hipStreamDestroy(g_b.cap);
  g_b = BatchState();
}

static int grow(void** p, size_t* cap, size_t need) {
  if (*cap >= need) return 0;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  const char* inject = getenv("ZF_FAULT_INJECT");
  if (inject && strcmp(inject, "alloc") == 0)
    return set_error(ZF_ERR_NOMEM, "allocation of %zu bytes refused (ZF_FAULT_INJECT=alloc)", need);
  if (hipMalloc(p, need) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return set_error(ZF_ERR_NOMEM, "hipMalloc(%zu bytes) for the batch failed", need);
  }
  *cap = need;
  return 0;
}


struct Plan {
  std::vector<BMat> mats;
  std::vector<TileTask> full, sym;
  int fseg[17] = {}, sseg[17] = {};  // XCD-major run bounds of the two tables
  std::vector<TileTask> ffull, fsym;   // FP64 tables (64-wide tiles for every matrix)
  int ffseg[17] = {}, fsseg[17] = {};
  long long partials = 0;
  int max_etiles = 1;  // largest (np / 64)^2 of the batch: x extent of element-wise grids
  size_t arena = 0;
};

// XCD-major task tables (see xcd_run) of the matrices' padded orders and tile edges.
static void build_tables(const std::vector<BMat>& mats, std::vector<TileTask>& full,
                         std::vector<TileTask>& sym, int* fseg, int* sseg) {
  std::vector<int> np(mats.size()), tile(mats.size());
  for (size_t m = 0; m < mats.size(); ++m) {
    np[m] = mats[m].np;
    tile[m] = mats[m].tile;
  }
  build_task_tables((int)mats.size(), np.data(), tile.data(), full, sym, fseg, sseg);
}

// Buffer sizes for every matrix and the task tables.
static void make_plan(int count, const int* n, bool with64, Plan& P) {
  P.mats.resize(count);
  size_t bytes = 0;
  for (int m = 0; m < count; ++m) {
    BMat& M = P.mats[m];
    memset(&M, 0, sizeof M);
    M.n = n[m];
    M.tile = tile_for(n[m]);
    M.np = rup(n[m], M.tile);
    const int T = M.np / M.tile;
    M.tiles_sym = T * (T + 1) / 2;
    const int T64 = M.np / 64;
    M.ftiles_sym = T64 * (T64 + 1) / 2;
    M.pbase = P.partials;
    P.partials += std::max(M.tiles_sym, M.ftiles_sym);
    P.max_etiles = std::max(P.max_etiles, (M.np / kET) * (M.np / kET));
    const size_t e = (size_t)M.np * M.np;
    bytes += 16 * align256(e * 2) + 2 * align256(e * 4) + (with64 ? 7 * align256(e * 8) : 0);
  }
  P.arena = bytes;
  build_tables(P.mats, P.full, P.sym, P.fseg, P.sseg);
  if (with64) {
    std::vector<BMat> m64 = P.mats;
    for (BMat& M : m64) M.tile = 64;
    build_tables(m64, P.ffull, P.fsym, P.ffseg, P.fsseg);
  }
}

static void carve(Plan& P, char* base, bool with64) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char* p = base + o;
    o += align256(bytes);
    return p;
  };
  for (BMat& M : P.mats) {
    const size_t e = (size_t)M.np * M.np;
    M.s_hi = (u16*)take(e * 2);
    M.s_lo = (u16*)take(e * 2);
    for (int b = 0; b < 2; ++b) {
      M.zr_hi[b] = (u16*)take(e * 2);
      M.zr_lo[b] = (u16*)take(e * 2);
      M.zc_hi[b] = (u16*)take(e * 2);
      M.zc_lo[b] = (u16*)take(e * 2);
    }
    M.at_hi = (u16*)take(e * 2);
    M.at_lo = (u16*)take(e * 2);
    M.d_hi = (u16*)take(e * 2);
    M.d_lo = (u16*)take(e * 2);
    M.q_hi = (u16*)take(e * 2);
    M.q_lo = (u16*)take(e * 2);
    M.z32[0] = (float*)take(e * 4);
    M.z32[1] = (float*)take(e * 4);
    if (with64) {
      M.s64 = (double*)take(e * 8);
      M.z64r[0] = (double*)take(e * 8);
      M.z64r[1] = (double*)take(e * 8);
      M.z64c[0] = (double*)take(e * 8);
      M.z64c[1] = (double*)take(e * 8);
      M.a64t = (double*)take(e * 8);
      M.d64 = (double*)take(e * 8);
    }
  }
}

struct Launch {
  BMat* mats;
  TileTask *full, *sym;
  int nfull, nsym;
  const int *fseg, *sseg;   // XCD-major run bounds (17 each), device
  int hfseg[17], hsseg[17];  // the same on the host (which launches a stage makes)
  TileTask *ffull, *fsym;    // FP64 tables and their run bounds (device)
  const int *ffseg, *fsseg;
  int etiles;
  double* partials;
  int* remaining;
  int count, grid, order, rule, max_l, max_h, refine_on, hist_cap;
  int graph_sweeps;  // macro-sweeps captured in one graph
  double c1, c2;
};

// Grouped BF16x3 stage: one launch per tile edge present (host copy hseg of the run
// bounds decides which); grid is a multiple of 8.
// live: the device-side count of live matrices (the kernels return at once when it
// is zero), or nullptr outside the macro-sweep.
static void x3_group(const TileTask* tasks, const int* seg, const int* hseg, const BMat* mats,
                     int op, double c1, double c2, double* partials, int grid, hipStream_t st,
                     const int* live = nullptr) {
  if (hseg[8] > hseg[0])
    hipLaunchKernelGGL(grouped_x3_kernel<128>, dim3(grid), dim3(X3G<128>::NT), 0, st, tasks, seg,
                       mats, op, c1, c2, partials, live);
  if (hseg[16] > hseg[8])
    hipLaunchKernelGGL(grouped_x3_kernel<64>, dim3(grid), dim3(X3G<64>::NT), 0, st, tasks, seg,
                       mats, op, c1, c2, partials, live);
}

// one macro-sweep on stream st (captured into the graph, or run eagerly)
static hipError_t macro_sweep(const Launch& L, hipStream_t st) {
  // each stage reads the count of matrices it will find (written by DECIDE) and
  // returns at once when it is zero
  const int* low = L.remaining + 2;
  const int* high = L.remaining + 3;
  const int* upd = L.remaining + 4;
  const int* trans = L.remaining + 5;
  x3_group(L.full, L.fseg, L.hfseg, L.mats, OP_L1, 0.0, 0.0, L.partials, L.grid, st, low);
  x3_group(L.sym, L.sseg, L.hsseg, L.mats, OP_L2, 0.0, 0.0, L.partials, L.grid, st, low);
  if (L.refine_on) {
    // 64-wide FP64 tiles fit four blocks per CU: twice the grid
    hipLaunchKernelGGL(grouped_f64_kernel, dim3(2 * L.grid), dim3(256), 0, st, L.ffull, L.ffseg,
                       L.mats, (int)OP_H1, L.partials, high);
    hipLaunchKernelGGL(grouped_f64_kernel, dim3(2 * L.grid), dim3(256), 0, st, L.fsym, L.fsseg,
                       L.mats, (int)OP_H2, L.partials, high);
  }
  hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(256), 0, st, L.mats, L.count, L.partials, L.order,
                     L.rule, L.max_l, L.max_h, L.refine_on, L.hist_cap, L.remaining);
  if (L.refine_on)
    hipLaunchKernelGGL(b_widen_kernel, dim3(8 * L.grid), dim3(256), 0, st, L.mats, L.count,
                       L.etiles, trans);
  x3_group(L.sym, L.sseg, L.hsseg, L.mats, OP_U3, L.c1, L.c2, L.partials, L.grid, st, upd);
  x3_group(L.full, L.fseg, L.hfseg, L.mats, OP_U4, 0.0, 0.0, L.partials, L.grid, st, upd);
  return hipGetLastError();
}

static int batched_impl(int count, const double* const* S, const double* const* Z0, const int* n,
                        const zf_opts& o, double* const* Z, zf_result* res, double* hist,
                        int hist_cap, hipStream_t st) {
  if (count <= 0 || count > 65535 || !S || !Z || !n)
    return set_error(ZF_ERR_ARG, "bad batch arguments (count must be in 1..65535)");
  if (o.order != 2) return set_error(ZF_ERR_ARG, "the batched path supports order 2 (got %d)", o.order);
  if (o.precision != ZF_BF16X3)
    return set_error(ZF_ERR_ARG, "the batched path runs ZF_BF16X3 (got %d)", o.precision);
  if (o.refine != ZF_REFINE_OFF && o.refine != ZF_REFINE_F64_DELTA)
    return set_error(ZF_ERR_ARG, "the batched path supports refine off or F64_DELTA");
  if (o.stop != ZF_STOP_RATIO && o.stop != ZF_STOP_MONOTONE)
    return set_error(ZF_ERR_ARG, "unknown stop rule %d", o.stop);
  if (hist_cap < 0 || (hist_cap > 0 && !hist)) return set_error(ZF_ERR_ARG, "bad hist buffer");
  if (o.z0 != ZF_Z0_GIVEN && o.z0 != ZF_Z0_SCALED_IDENTITY && o.z0 != ZF_Z0_LEARNED)
    return set_error(ZF_ERR_ARG, "unknown guess kind %d", o.z0);
  for (int m = 0; m < count; ++m) {
    if (n[m] <= 0 || n[m] > 8192)
      return set_error(ZF_ERR_ARG, "matrix %d: order %d outside 1..8192", m, n[m]);
    if (!S[m] || !Z[m]) return set_error(ZF_ERR_ARG, "matrix %d: NULL S or Z", m);
    if (o.z0 == ZF_Z0_GIVEN && !(Z0 && Z0[m]))
      return set_error(ZF_ERR_ARG, "matrix %d: opts.z0 = ZF_Z0_GIVEN needs its Z0", m);
  }
  const bool with64 = o.refine == ZF_REFINE_F64_DELTA;
  const int max_l = o.max_sweeps > 0 ? o.max_sweeps : 100;
  const int max_h = o.max_refine > 0 ? o.max_refine : 10;
  const int hcap = std::max(hist_cap, 1);

  int dev = 0;
  BHIP_TRY(hipGetDevice(&dev));
  if (g_b.device != dev) {
    batch_release();
    g_b.device = dev;
  }
  if (!g_b.cap) BHIP_TRY(hipStreamCreateWithFlags(&g_b.cap, hipStreamNonBlocking));
  if (!g_b.pinned) BHIP_TRY(hipHostMalloc((void**)&g_b.pinned, 64, hipHostMallocDefault));

  Plan P;
  make_plan(count, n, with64, P);
  // guesses: given where Z0[m] is set, else learned (opts.z0 = ZF_Z0_LEARNED, network loaded; the
  // device may still fall back) or the scaled identity
  const bool have_net = net_ready();
  int n_learn = 0;
  for (int m = 0; m < count; ++m) {
    BMat& M = P.mats[m];
    if (Z0 && Z0[m]) {
      M.z0_used = ZF_Z0_GIVEN;
    } else if (o.z0 == ZF_Z0_LEARNED && have_net) {
      M.learn = 1;
      M.z0_used = ZF_Z0_LEARNED;
      ++n_learn;
    } else {
      M.z0_used = ZF_Z0_SCALED_IDENTITY;
      if (o.z0 == ZF_Z0_LEARNED) M.flags |= ZF_WARN_Z0_FALLBACK;
    }
  }
  int rc = grow(&g_b.arena, &g_b.arena_bytes, std::max<size_t>(P.arena, 256));
  if (rc < 0) return rc;
  carve(P, (char*)g_b.arena, with64);

  // metadata block: mats | full tasks | sym tasks | S, Z0, Z pointer
  // tables | partials | hist | g | remaining | stats | coef | feats
  size_t o_mats = 0;
  size_t o_full = align256(o_mats + sizeof(BMat) * count);
  size_t o_sym = align256(o_full + sizeof(TileTask) * P.full.size());
  size_t o_ps = align256(o_sym + sizeof(TileTask) * P.sym.size());
  size_t o_pz0 = align256(o_ps + 8 * count);
  size_t o_pz = align256(o_pz0 + 8 * count);
  size_t o_part = align256(o_pz + 8 * count);
  size_t o_hist = align256(o_part + 8 * P.partials);
  size_t o_g = align256(o_hist + 8 * (size_t)count * hcap);
  size_t o_rem = align256(o_g + 8 * count);
  size_t o_stats = align256(o_rem + 64);
  size_t o_coef = align256(o_stats + 32 * (size_t)count);
  size_t o_feat = align256(o_coef + 32 * (size_t)count);
  int max_n = 1;
  for (int m = 0; m < count; ++m) max_n = std::max(max_n, n[m]);
  const int stat_chunks = (max_n + kStatRows - 1) / kStatRows;
  size_t o_spart = align256(o_feat + 32 * (size_t)count);
  size_t o_fseg = align256(o_spart + 56 * (size_t)count * stat_chunks);
  size_t o_sseg = align256(o_fseg + sizeof P.fseg);
  size_t o_ffull = align256(o_sseg + sizeof P.sseg);
  size_t o_fsym = align256(o_ffull + sizeof(TileTask) * P.ffull.size());
  size_t o_ffseg = align256(o_fsym + sizeof(TileTask) * P.fsym.size());
  size_t o_fsseg = align256(o_ffseg + sizeof P.ffseg);
  size_t total_meta = align256(o_fsseg + sizeof P.fsseg);
  rc = grow(&g_b.meta, &g_b.meta_bytes, total_meta);
  if (rc < 0) return rc;
  char* mb = (char*)g_b.meta;
  for (int m = 0; m < count; ++m) P.mats[m].hist = (double*)(mb + o_hist) + (size_t)m * hcap;

  std::vector<const void*> ps(count), pz0(count), pz(count);
  for (int m = 0; m < count; ++m) {
    ps[m] = S[m];
    pz0[m] = Z0 ? Z0[m] : nullptr;
    pz[m] = Z[m];
  }
  // host -> device metadata (the host vectors outlive the synchronizing copies)
  BHIP_TRY(hipMemcpyAsync(mb + o_mats, P.mats.data(), sizeof(BMat) * count, hipMemcpyHostToDevice, st));
  BHIP_TRY(hipMemcpyAsync(mb + o_full, P.full.data(), sizeof(TileTask) * P.full.size(), hipMemcpyHostToDevice, st));
  BHIP_TRY(hipMemcpyAsync(mb + o_sym, P.sym.data(), sizeof(TileTask) * P.sym.size(), hipMemcpyHostToDevice, st));
  BHIP_TRY(hipMemcpyAsync(mb + o_fseg, P.fseg, sizeof P.fseg, hipMemcpyHostToDevice, st));
  BHIP_TRY(hipMemcpyAsync(mb + o_sseg, P.sseg, sizeof P.sseg, hipMemcpyHostToDevice, st));
  if (with64) {
    BHIP_TRY(hipMemcpyAsync(mb + o_ffull, P.ffull.data(), sizeof(TileTask) * P.ffull.size(),
                            hipMemcpyHostToDevice, st));
    BHIP_TRY(hipMemcpyAsync(mb + o_fsym, P.fsym.data(), sizeof(TileTask) * P.fsym.size(),
                            hipMemcpyHostToDevice, st));
    BHIP_TRY(hipMemcpyAsync(mb + o_ffseg, P.ffseg, sizeof P.ffseg, hipMemcpyHostToDevice, st));
    BHIP_TRY(hipMemcpyAsync(mb + o_fsseg, P.fsseg, sizeof P.fsseg, hipMemcpyHostToDevice, st));
  }
  BHIP_TRY(hipMemcpyAsync(mb + o_ps, ps.data(), 8 * count, hipMemcpyHostToDevice, st));
  BHIP_TRY(hipMemcpyAsync(mb + o_pz0, pz0.data(), 8 * count, hipMemcpyHostToDevice, st));
  BHIP_TRY(hipMemcpyAsync(mb + o_pz, pz.data(), 8 * count, hipMemcpyHostToDevice, st));

  BMat* d_mats = (BMat*)(mb + o_mats);
  const double* const* d_S = (const double* const*)(mb + o_ps);
  const double* const* d_Z0 = (const double* const*)(mb + o_pz0);
  double* const* d_Z = (double* const*)(mb + o_pz);
  double* d_g = (double*)(mb + o_g);
  double* d_stats = (double*)(mb + o_stats);
  double* d_coef = (double*)(mb + o_coef);
  float* d_feat = (float*)(mb + o_feat);

  // setup: operands of S and Z0
  const dim3 eg(P.max_etiles, count);
  hipLaunchKernelGGL(b_split_kernel, eg, dim3(256), 0, st, d_mats, d_S, with64 ? 1 : 0);
  int cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
    cus = prop.multiProcessorCount;
  if (n_learn > 0)
    x3_group((const TileTask*)(mb + o_sym), (const int*)(mb + o_sseg), P.sseg, d_mats, OP_S2, 0.0, 0.0,
             nullptr, 2 * cus, st);
  double* d_spart = (double*)(mb + o_spart);
  hipLaunchKernelGGL(b_stats_rows_kernel, dim3(stat_chunks, count), dim3(256), 0, st, d_mats, d_S,
                     stat_chunks, d_spart);
  hipLaunchKernelGGL(b_stats_final_kernel, dim3((count + 255) / 256), dim3(256), 0, st, d_mats,
                     count, stat_chunks, d_spart, d_g, d_stats, d_feat);
  BHIP_TRY(hipGetLastError());
  if (n_learn > 0) {
    rc = guess_infer_batch(d_feat, count, d_coef, st);
    if (rc < 0) return rc;
    hipLaunchKernelGGL(b_accept_kernel, dim3((count + 255) / 256), dim3(256), 0, st, d_mats, count,
                       d_stats, d_coef);
  }
  hipLaunchKernelGGL(b_init_kernel, eg, dim3(256), 0, st, d_mats, d_Z0, d_S, d_g, d_coef);
  hipLaunchKernelGGL(b_reset_kernel, dim3(1), dim3(64), 0, st, (int*)(mb + o_rem), count);
  BHIP_TRY(hipGetLastError());

  Launch L;
  memset(&L, 0, sizeof L);  // the struct's bytes are the graph's key
  L.mats = d_mats;
  L.full = (TileTask*)(mb + o_full);
  L.sym = (TileTask*)(mb + o_sym);
  L.nfull = (int)P.full.size();
  L.nsym = (int)P.sym.size();
  L.fseg = (const int*)(mb + o_fseg);
  L.sseg = (const int*)(mb + o_sseg);
  memcpy(L.hfseg, P.fseg, sizeof L.hfseg);
  memcpy(L.hsseg, P.sseg, sizeof L.hsseg);
  L.ffull = (TileTask*)(mb + o_ffull);
  L.fsym = (TileTask*)(mb + o_fsym);
  L.ffseg = (const int*)(mb + o_ffseg);
  L.fsseg = (const int*)(mb + o_fsseg);
  L.etiles = P.max_etiles;
  L.partials = (double*)(mb + o_part);
  L.remaining = (int*)(mb + o_rem);
  L.count = count;
  L.grid = (2 * cus + 7) / 8 * 8;  // a multiple of the 8 XCDs
  L.order = o.order;
  L.rule = o.stop;
  L.max_l = max_l;
  L.max_h = max_h;
  L.refine_on = with64 ? 1 : 0;
  L.hist_cap = hcap;
  L.c1 = 0.5;
  L.c2 = 0.375;
  // every macro-sweep the caps allow: max_l low-phase evaluations after the first,
  // the phase change, max_h FP64 evaluations after the first, and one to spare
  const int max_macro = max_l + (with64 ? max_h + 1 : 0) + 2;
  L.graph_sweeps = (g_graph_sweeps > 0 && g_graph_sweeps < max_macro) ? g_graph_sweeps : max_macro;

  // graph of graph_sweeps macro-sweeps, rebuilt when the layout changes
  std::vector<char> key(sizeof(Launch));
  memcpy(key.data(), &L, sizeof(Launch));
  if (g_use_graph && (g_b.key != key || !g_b.exec)) {
    if (g_b.exec) {
      (void)hipGraphExecDestroy(g_b.exec);
      g_b.exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    BHIP_TRY(hipStreamBeginCapture(g_b.cap, hipStreamCaptureModeThreadLocal));
    hipError_t ce = hipSuccess;
    for (int k = 0; k < L.graph_sweeps && ce == hipSuccess; ++k) ce = macro_sweep(L, g_b.cap);
    hipError_t ee = hipStreamEndCapture(g_b.cap, &graph);
    if (ce != hipSuccess || ee != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return set_error(ZF_ERR_HIP, "graph capture failed: %s",
                       hipGetErrorString(ce != hipSuccess ? ce : ee));
    }
    hipError_t ie = hipGraphInstantiate(&g_b.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      g_b.exec = nullptr;
      return set_error(ZF_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
    }
    g_b.key = key;
  }

  // Graph: launches of graph_sweeps macro-sweeps each until the live count is zero
  // (graph_sweeps = every macro-sweep the caps allow: one launch, after which the
  // output kernel and the copies of the results follow on the stream, so the call
  // synchronizes once).  Eager: one macro-sweep at a time, the host reading the live
  // count after each.
  const int chunk = g_use_graph ? L.graph_sweeps : 1;
  int launched = 0, launches = 0;
  for (;;) {
    if (g_use_graph) BHIP_TRY(hipGraphLaunch(g_b.exec, st));
    else BHIP_TRY(macro_sweep(L, st));
    launched += chunk;
    ++launches;
    if (launched >= max_macro) break;
    BHIP_TRY(hipMemcpyAsync(g_b.pinned, L.remaining, sizeof(int), hipMemcpyDeviceToHost, st));
    BHIP_TRY(hipStreamSynchronize(st));
    if (g_b.pinned[0] == 0) break;
  }
  hipLaunchKernelGGL(b_output_kernel, eg, dim3(256), 0, st, d_mats, d_Z, with64 ? 1 : 0);
  BHIP_TRY(hipGetLastError());
  std::vector<BMat> out(count);
  BHIP_TRY(hipMemcpyAsync(out.data(), d_mats, sizeof(BMat) * count, hipMemcpyDeviceToHost, st));
  std::vector<double> h((size_t)count * hcap);
  BHIP_TRY(hipMemcpyAsync(h.data(), mb + o_hist, 8 * h.size(), hipMemcpyDeviceToHost, st));
  BHIP_TRY(hipMemcpyAsync(g_b.pinned, L.remaining, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  BHIP_TRY(hipStreamSynchronize(st));
  g_last_sweeps = g_b.pinned[1];
  g_last_launches = launches;
  if (g_b.pinned[0] != 0)
    return set_error(ZF_ERR_HIP, "batched refinement did not finish in %d macro-sweeps",
                     launched);

  int ret = 0, first_err = 0, first_m = -1;
  for (int m = 0; m < count; ++m) {
    const BMat& M = out[m];
    const int len = std::min(M.hist_len, hist_cap);
    for (int k = 0; k < len; ++k) hist[(size_t)m * hist_cap + k] = h[(size_t)m * hcap + k];
    int flags = M.flags;
    if (M.hist_len > hist_cap) flags |= ZF_WARN_HIST_TRUNC;
    const double fe = with64 ? M.err_h : M.err_l;
    int status = M.status;
    if (status == 0 && !(fe < 1.0)) status = ZF_ERR_NOT_CONVERGED;
    if (res) {
      res[m].iters = M.upd_l + M.upd_h;
      res[m].low_evals = M.evals_l;
      res[m].high_evals = M.evals_h;
      res[m].hist_len = len;
      res[m].flags = flags;
      res[m].final_err = fe;
      res[m].final_rms = fe / sqrt((double)M.n);
      res[m].status = status;
      res[m].z0_used = M.z0_used;
    }
    if (status < 0 && first_err == 0) {
      first_err = status;
      first_m = m;
    }
    ret |= flags;
  }
  if (first_err < 0)
    return set_error(first_err, "matrix %d of the batch failed (status %d); see the results",
                     first_m, first_err);
  clear_error();
  return ret;
}

// ---------------------------------------------------------------------------
// autotuner: time the grouped BF16x3 GEMM (plain + symmetric) per order bucket
// ---------------------------------------------------------------------------
static int autotune_impl(const int* bucket_n, int nb, int batch, int reps, int* best,
                         double* ms_out, hipStream_t st) {
  if (nb <= 0 || nb > 16 || !bucket_n || batch <= 0 || reps <= 0)
    return set_error(ZF_ERR_ARG, "bad autotune arguments");
  const int cand[2] = {64, 128};
  int dev = 0;
  BHIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  BHIP_TRY(hipGetDeviceProperties(&prop, dev));
  const int grid = (2 * prop.multiProcessorCount + 7) / 8 * 8;
  hipEvent_t e0, e1;
  BHIP_TRY(hipEventCreate(&e0));
  BHIP_TRY(hipEventCreate(&e1));
  int rc = 0;
  for (int b = 0; b < nb && rc == 0; ++b) {
    double best_ms = 1e30;
    best[b] = 128;
    for (int c = 0; c < 2 && rc == 0; ++c) {
      const int T = cand[c];
      const int np = rup(bucket_n[b], T);
      const int tiles = np / T;
      std::vector<BMat> mats(batch);
      std::vector<TileTask> full, sym;
      const size_t e = (size_t)np * np;
      void* buf = nullptr;
      // per matrix: the operands of L1 / L2 only (zero data; timing does not depend on values)
      const size_t per = 8 * align256(e * 2) + align256(8 * tiles * (tiles + 1) / 2);
      if (hipMalloc(&buf, per * batch + 256) != hipSuccess) {
        (void)hipGetLastError();
        rc = set_error(ZF_ERR_NOMEM, "autotune allocation failed");
        break;
      }
      (void)hipMemsetAsync(buf, 0, per * batch + 256, st);
      char* p = (char*)buf;
      for (int m = 0; m < batch; ++m) {
        BMat& M = mats[m];
        memset(&M, 0, sizeof M);
        M.n = bucket_n[b];
        M.np = np;
        M.tile = T;
        M.tiles_sym = tiles * (tiles + 1) / 2;
        u16* q[8];
        for (int k = 0; k < 8; ++k) {
          q[k] = (u16*)p;
          p += align256(e * 2);
        }
        M.zc_hi[0] = q[0];
        M.zc_lo[0] = q[1];
        M.s_hi = q[2];
        M.s_lo = q[3];
        M.at_hi = q[4];
        M.at_lo = q[5];
        M.d_hi = q[6];
        M.d_lo = q[7];
        M.pbase = 0;
        M.phase = PH_LOW;
        M.action = ACT_EVAL;
        p += align256(8 * tiles * (tiles + 1) / 2);
      }
      int fseg[17], sseg[17];
      build_tables(mats, full, sym, fseg, sseg);
      void* meta = nullptr;
      const size_t mbytes = align256(sizeof(BMat) * batch) + align256(sizeof(TileTask) * full.size()) +
                            align256(sizeof(TileTask) * sym.size()) + align256(8 * (size_t)tiles * tiles) +
                            2 * align256(sizeof fseg);
      if (hipMalloc(&meta, mbytes) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(buf);
        rc = set_error(ZF_ERR_NOMEM, "autotune allocation failed");
        break;
      }
      char* mp = (char*)meta;
      BMat* dm = (BMat*)mp;
      TileTask* df = (TileTask*)(mp + align256(sizeof(BMat) * batch));
      TileTask* ds = (TileTask*)((char*)df + align256(sizeof(TileTask) * full.size()));
      double* dpart = (double*)((char*)ds + align256(sizeof(TileTask) * sym.size()));
      int* dfseg = (int*)((char*)dpart + align256(8 * (size_t)tiles * tiles));
      int* dsseg = (int*)((char*)dfseg + align256(sizeof fseg));
      (void)hipMemcpyAsync(dm, mats.data(), sizeof(BMat) * batch, hipMemcpyHostToDevice, st);
      (void)hipMemcpyAsync(df, full.data(), sizeof(TileTask) * full.size(), hipMemcpyHostToDevice, st);
      (void)hipMemcpyAsync(ds, sym.data(), sizeof(TileTask) * sym.size(), hipMemcpyHostToDevice, st);
      (void)hipMemcpyAsync(dfseg, fseg, sizeof fseg, hipMemcpyHostToDevice, st);
      (void)hipMemcpyAsync(dsseg, sseg, sizeof sseg, hipMemcpyHostToDevice, st);
      // every matrix uses partial base 0: timing only, the sums are discarded
      for (int r = 0; r <= reps; ++r) {
        if (r == 1) (void)hipEventRecord(e0, st);
        x3_group(df, dfseg, fseg, dm, OP_L1, 0.0, 0.0, dpart, grid, st);
        x3_group(ds, dsseg, sseg, dm, OP_L2, 0.0, 0.0, dpart, grid, st);
      }
      (void)hipEventRecord(e1, st);
      hipError_t he = hipEventSynchronize(e1);
      float t = 0.f;
      if (he == hipSuccess) he = hipEventElapsedTime(&t, e0, e1);
      (void)hipFree(meta);
      (void)hipFree(buf);
      if (he != hipSuccess) {
        rc = set_error(ZF_ERR_HIP, "autotune timing: %s", hipGetErrorString(he));
        break;
      }
      const double ms = t / reps;
      if (ms_out) ms_out[2 * b + c] = ms;
      if (ms < best_ms) {
        best_ms = ms;
        best[b] = T;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc < 0) return rc;
  g_tile_nb = nb;
  for (int b = 0; b < nb; ++b) {
    g_tile_max[b] = (b == nb - 1) ? (1 << 30) : bucket_n[b];
    g_tile_edge[b] = best[b];
  }
  g_b.key.clear();  // layouts change with the table
  clear_error();
  return 0;
}

void batch_release_all() { batch_release(); }

}  // namespace zf

using namespace zf;

extern "C" {

int zf_refine_batched(int count, const double* const* S, const double* const* Z0, const int* n,
                      const zf_opts* opts, double* const* Z, zf_result* res, double* hist,
                      int hist_cap, void* stream) {
  zf_opts o;
  zf_default_opts(&o);
  if (opts) o = *opts;
  return batched_impl(count, S, Z0, n, o, Z, res, hist, hist_cap, (hipStream_t)stream);
}

int zf_batched_set_tiles(const int* max_n, const int* tile, int count) {
  if (count <= 0 || count > 16 || !max_n || !tile)
    return set_error(ZF_ERR_ARG, "tile table needs 1..16 entries");
  for (int k = 0; k < count; ++k)
    if (tile[k] != 64 && tile[k] != 128) return set_error(ZF_ERR_ARG, "tile edges are 64 or 128");
  g_tile_nb = count;
  for (int k = 0; k < count; ++k) {
    g_tile_max[k] = (k == count - 1) ? (1 << 30) : max_n[k];
    g_tile_edge[k] = tile[k];
  }
  g_b.key.clear();
  return 0;
}

int zf_batched_get_tiles(int* max_n, int* tile, int cap) {
  if (!max_n || !tile || cap < g_tile_nb) return set_error(ZF_ERR_ARG, "table needs %d entries", g_tile_nb);
  for (int k = 0; k < g_tile_nb; ++k) {
    max_n[k] = g_tile_max[k];
    tile[k] = g_tile_edge[k];
  }
  return g_tile_nb;
}

int zf_batched_autotune(const int* bucket_n, int nbuckets, int batch, int reps, int* best_tile,
                        double* ms, void* stream) {
  return autotune_impl(bucket_n, nbuckets, batch, reps, best_tile, ms, (hipStream_t)stream);
}

void zf_batched_use_graph(int on) { g_use_graph = on != 0; }

int zf_batched_set_graph_sweeps(int sweeps) {
  if (sweeps < 0) return set_error(ZF_ERR_ARG, "sweeps per graph must be >= 0 (got %d)", sweeps);
  g_graph_sweeps = sweeps;
  g_b.key.clear();
  return 0;
}

int zf_batched_last_stats(int* macro_sweeps, int* graph_launches) {
  if (macro_sweeps) *macro_sweeps = g_last_sweeps;
  if (graph_launches) *graph_launches = g_last_launches;
  return 0;
}

void zf_batched_release(void) { batch_release(); }

}  // extern "C"
