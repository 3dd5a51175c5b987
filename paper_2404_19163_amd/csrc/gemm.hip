// Matrix-core GEMMs of the refinement sweep (gfx950).
//
// Both kernels compute an "NT" product C[i][j] = sum_k A[i][k] * B[j][k] with A
// (M x K) and B (N x K) row-major, i.e. both operands contiguous along the
// contracted index.  The sweep keeps every operand in that form: S and the
// iterates delta, Q are symmetric, and Z is stored both row-major and
// transposed, so no kernel ever needs a transposing load.  Z's transposed pair
// is K-blocked (kb_offset: 32-wide K blocks, each a row-major panel), which the
// BF16x3 main loop reads through its per-operand K-block stride and which the
// update's transposed epilogue writes as one contiguous run per strip.
//
//   gemm_x3  : (h)(h) + (h)(l) + (l)(h) of Sec. III.B (Eqs. SZn, Xn, Xsq): each
//              operand is a BF16 hi/lo pair, the three products accumulate into
//              one FP32 accumulator on v_mfma_f32_32x32x16_bf16.
//   gemm_f64 : FP64 products on v_mfma_f64_16x16x4_f64 (the "double" scheme).
//
// Symmetric mode computes only the tiles with tile_row <= tile_col of a product
// known to be symmetric (Z^T S Z, delta * delta and polynomials of delta) and
// mirrors them, which halves those GEMMs.  Inside a diagonal tile the upper
// triangle is written and mirrored, so the stored matrix is exactly symmetric.
//
// The epilogue forms out = alpha * D + beta * acc + gamma * I in FP64 and writes
// any of: FP32, FP64, a BF16 hi/lo split (Sec. III.A), each in normal and/or
// transposed layout, plus a per-tile FP64 sum of out^2 for the Frobenius norm
// of the stop test (Sec. IV.A).
#include <stdlib.h>

#include "zf_internal.h"
#include "gemm_tiles.inc"

namespace zf {
// SYM is a template parameter so that the two modes are distinct kernels (and show
// up separately in a kernel trace).
template <int BM, int BN, int BK, int WM, int WN, bool SYM, int PM, int NS>
__global__ void __launch_bounds__(WM* WN * 64)
    gemm_x3_kernel(const u16* __restrict__ Ahi, const u16* __restrict__ Alo, int lda,
                   const u16* __restrict__ Bhi, const u16* __restrict__ Blo, int ldb, int K,
                   int tiles_n, int gm, EpiParams ep, int ksa, int ksb) {
  using C = X3Cfg<BM, BN, BK, WM, WN>;
  __shared__ __attribute__((aligned(16))) u16 lds[NS * C::STAGE_ELEMS];
  __shared__ double red[C::NT / 64];
  if (ep.gate && *ep.gate) return;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  int ti, tj;
  tile_coords(bid, tiles_n, SYM, ti, tj, gm);
  const int mode = SYM ? (ti == tj ? 2 : 1) : 0;
  x3_tile<BM, BN, BK, WM, WN, PM, NS>(Ahi, Alo, lda, Bhi, Blo, ldb, K, ti * BM, tj * BN, mode, ep,
                                  tile_index(ti, tj, tiles_n, SYM), lds, red, ksa, ksb);
}

// FP32 matrix-core GEMM ("single"): f32_mainloop + the shared epilogue.
template <int BM, int BN, int WM, int WN, bool SYM>
__global__ void __launch_bounds__(WM* WN * 64)
    gemm_f32_kernel(const float* __restrict__ A, int lda, const float* __restrict__ B, int ldb,
                    int K, int tiles_n, int gm, EpiParams ep) {
  using C = X3Cfg<BM, BN, 32, WM, WN>;
  __shared__ __attribute__((aligned(16))) u16 lds[2 * C::STAGE_ELEMS];
  __shared__ double red[C::NT / 64];
  if (ep.gate && *ep.gate) return;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  int ti, tj;
  tile_coords(bid, tiles_n, SYM, ti, tj, gm);
  const int mode = SYM ? (ti == tj ? 2 : 1) : 0;
  X3Acc<BM, BN, 32, WM, WN> acc;
#pragma unroll
  for (int a = 0; a < C::FM; ++a)
#pragma unroll
    for (int b = 0; b < C::FN; ++b) acc[a][b] = f32x16{};
  f32_mainloop<BM, BN, WM, WN>(A, lda, B, ldb, 0, K, ti * BM, tj * BN, lds, acc);
  x3_epilogue<BM, BN, 32, WM, WN>(acc, ti * BM, tj * BN, mode, ep, tile_index(ti, tj, tiles_n, SYM),
                                  lds, red);
}

// ---------------------------------------------------------------------------
// FP64 kernel
// ---------------------------------------------------------------------------
template <int BM, int BN, int BK, int WM, int WN, bool SYM>
__global__ void __launch_bounds__(WM* WN * 64, 2)
    gemm_f64_kernel(const double* __restrict__ A, int lda, const double* __restrict__ B, int ldb,
                    int K, int tiles_n, int gm, EpiParams ep) {
  using C = F64Cfg<BM, BN, BK, WM, WN>;
  __shared__ double lds[2 * C::STAGE];
  __shared__ double red[C::NT / 64];
  if (ep.gate && *ep.gate) return;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  int ti, tj;
  tile_coords(bid, tiles_n, SYM, ti, tj, gm);
  const int mode = SYM ? (ti == tj ? 2 : 1) : 0;
  f64_tile<BM, BN, BK, WM, WN>(A, lda, B, ldb, K, ti * BM, tj * BN, mode, ep,
                               tile_index(ti, tj, tiles_n, SYM), lds, red);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static bool dims_ok(int M, int N, int K, bool sym) {
  return M > 0 && N > 0 && K > 0 && M % kTile == 0 && N % kTile == 0 && K % kTile == 0 &&
         (!sym || M == N);
}

static int grid_blocks(int M, int N, int t, bool sym) {
  const int tm = M / t, tn = N / t;
  return sym ? tm * (tm + 1) / 2 : tm * tn;
}

// Tile edge of a launch: 256 when it divides both output dimensions and yields at
// least 128 workgroups (half of the 256 CUs: fewer, larger tiles beat more, smaller
// ones down to that point), else 128 when that yields at least 192 workgroups (the
// 128-wide tile runs one 8-wave block per CU), else 64.  Measured on the mixed solve:
// 64-wide tiles beat 128-wide grids of 136-171 tiles (N = 1536, 2048, 2304) by 3-6%,
// 128-wide ones win from about 200 tiles on (N = 2560, 2816).  ZF_X3_TILE /
// ZF_X3_SYM_TILE (64, 128 or 256) force the BF16x3 edge when it divides (tuning).
int x3_tile_edge(int M, int N, bool sym) {
  const char* env = getenv(sym ? "ZF_X3_SYM_TILE" : "ZF_X3_TILE");
  if (env) {
    const int want = atoi(env);
    if ((want == 64 || want == 128 || want == 256) && M % want == 0 && N % want == 0) return want;
  }
  if (M % 256 == 0 && N % 256 == 0 && grid_blocks(M, N, 256, sym) >= 128) return 256;
  if (M % 128 == 0 && N % 128 == 0 && grid_blocks(M, N, 128, sym) >= 192) return 128;
  return 64;
}

int x3_blocks(int M, int N, bool sym) { return grid_blocks(M, N, x3_tile_edge(M, N, sym), sym); }


// FP64 tile edge: 64.  The 64-wide tile runs four blocks per CU at the same
// per-flop rate as the 128-wide one (both ~82% of FP64 peak on full N = 4096
// grids) and quantizes far better on triangular grids (N = 4096: 2080 blocks
// instead of 528 on 512 two-per-CU slots).  ZF_F64_TILE / ZF_F64_SYM_TILE = 128
// select the larger tile (tuning).
int f64_tile_edge(int M, int N, bool sym) {
  const char* env = getenv(sym ? "ZF_F64_SYM_TILE" : "ZF_F64_TILE");
  if (env && atoi(env) == 128 && M % 128 == 0 && N % 128 == 0) return 128;
  return 64;
}

// Row-group height of the full-grid tile order: 4 (a run of 32 tiles on one XCD then
// covers 4 x 8 tiles, 12 operand panels instead of 18); ZF_TILE_GROUP overrides.
static int tile_group(int M, int t) {
  const char* env = getenv("ZF_TILE_GROUP");
  const int gm = env ? atoi(env) : 4;
  return (gm > 1 && (M / t) % gm == 0) ? gm : 1;
}

// Band height of the symmetric-grid tile order: 4 (a run of 17 of the 136 tiles of
// an N = 4096 triangle then spans about 4 x 5 tiles instead of one tile row; the
// symmetric BF16x3 GEMM measured 308 -> 303 us); ZF_SYM_TILE_GROUP overrides (1: row
// by row).
static int sym_group() {
  const char* env = getenv("ZF_SYM_TILE_GROUP");
  const int g = env ? atoi(env) : 4;
  return g >= 1 ? g : 1;
}

int f64_blocks(int M, int N, bool sym) { return grid_blocks(M, N, f64_tile_edge(M, N, sym), sym); }

int max_blocks(int M, int N) { return grid_blocks(M, N, 64, false); }

template <int BM, int BN, int WM, int WN, int PM, int NS = 2>
static void x3_launch(const u16* Ahi, const u16* Alo, int lda, const u16* Bhi, const u16* Blo,
                      int ldb, int M, int N, int K, bool sym, int blocks, const EpiParams& ep,
                      hipStream_t st, int ksa, int ksb) {
  if (sym)
    hipLaunchKernelGGL((gemm_x3_kernel<BM, BN, 32, WM, WN, true, PM, NS>), dim3(blocks),
                       dim3(WM * WN * 64), 0, st, Ahi, Alo, lda, Bhi, Blo, ldb, K, N / BN, sym_group(), ep,
                       ksa, ksb);
  else
    hipLaunchKernelGGL((gemm_x3_kernel<BM, BN, 32, WM, WN, false, PM, NS>), dim3(blocks),
                       dim3(WM * WN * 64), 0, st, Ahi, Alo, lda, Bhi, Blo, ldb, K, N / BN,
                       tile_group(M, BM), ep, ksa, ksb);
}

template <int BM, int BN, int WM, int WN>
static void f32_launch(const float* A, int lda, const float* B, int ldb, int M, int N, int K,
                       bool sym, int blocks, const EpiParams& ep, hipStream_t st) {
  if (sym)
    hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, WM, WN, true>), dim3(blocks), dim3(WM * WN * 64),
                       0, st, A, lda, B, ldb, K, N / BN, sym_group(), ep);
  else
    hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, WM, WN, false>), dim3(blocks), dim3(WM * WN * 64),
                       0, st, A, lda, B, ldb, K, N / BN, tile_group(M, BM), ep);
}

template <int BM, int BN, int WM, int WN>
static void f64_launch(const double* A, int lda, const double* B, int ldb, int M, int N, int K,
                       bool sym, int blocks, const EpiParams& ep, hipStream_t st) {
  if (sym)
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, 16, WM, WN, true>), dim3(blocks),
                       dim3(WM * WN * 64), 0, st, A, lda, B, ldb, K, N / BN, sym_group(), ep);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, 16, WM, WN, false>), dim3(blocks),
                       dim3(WM * WN * 64), 0, st, A, lda, B, ldb, K, N / BN, tile_group(M, BM),
                       ep);
}

template <int PM>
static void x3_dispatch(const u16* Ahi, const u16* Alo, int lda, const u16* Bhi, const u16* Blo,
                        int ldb, int M, int N, int K, bool sym, int tile, int blocks,
                        const EpiParams& ep, hipStream_t st, int ksa, int ksb) {
  if (tile == 256)
    x3_launch<256, 256, 2, 4, PM>(Ahi, Alo, lda, Bhi, Blo, ldb, M, N, K, sym, blocks, ep, st, ksa,
                                  ksb);
  else if (tile == 128)  // 8 waves of 32 x 64 and a 3-stage ring (loads two stages ahead)
    x3_launch<128, 128, 4, 2, PM, 3>(Ahi, Alo, lda, Bhi, Blo, ldb, M, N, K, sym, blocks, ep, st,
                                     ksa, ksb);
  else
    x3_launch<64, 64, 2, 2, PM>(Ahi, Alo, lda, Bhi, Blo, ldb, M, N, K, sym, blocks, ep, st, ksa,
                                ksb);
}

hipError_t launch_gemm_x3(const u16* Ahi, const u16* Alo, int lda, const u16* Bhi, const u16* Blo,
                          int ldb, int M, int N, int K, bool sym, const EpiParams& ep,
                          hipStream_t st, int pm, int ksa, int ksb) {
  if (!dims_ok(M, N, K, sym) || pm < 0 || pm > 3) return hipErrorInvalidValue;
  if (ksa < 32 || ksa % 32 || ksb < 32 || ksb % 32) return hipErrorInvalidValue;
  const int tile = x3_tile_edge(M, N, sym);
  const int blocks = x3_blocks(M, N, sym);
  switch (pm) {
    case PM_X3:
      x3_dispatch<PM_X3>(Ahi, Alo, lda, Bhi, Blo, ldb, M, N, K, sym, tile, blocks, ep, st, ksa,
                          ksb);
      break;
    case PM_HH:
      x3_dispatch<PM_HH>(Ahi, Alo, lda, Bhi, Blo, ldb, M, N, K, sym, tile, blocks, ep, st, ksa,
                          ksb);
      break;
    case PM_X3F16:
      x3_dispatch<PM_X3F16>(Ahi, Alo, lda, Bhi, Blo, ldb, M, N, K, sym, tile, blocks, ep, st, ksa,
                          ksb);
      break;
    default:
      x3_dispatch<PM_HHF16>(Ahi, Alo, lda, Bhi, Blo, ldb, M, N, K, sym, tile, blocks, ep, st, ksa,
                          ksb);
  }
  return hipGetLastError();
}

// FP32 tiles follow the BF16x3 choice (same tile bodies and occupancy).
int f32_tile_edge(int M, int N, bool sym) { return x3_tile_edge(M, N, sym); }
int f32_blocks(int M, int N, bool sym) { return x3_blocks(M, N, sym); }

hipError_t launch_gemm_f32(const float* A, int lda, const float* B, int ldb, int M, int N, int K,
                           bool sym, const EpiParams& ep, hipStream_t st) {
  if (!dims_ok(M, N, K, sym)) return hipErrorInvalidValue;
  const int tile = f32_tile_edge(M, N, sym);
  const int blocks = f32_blocks(M, N, sym);
  if (tile == 256)
    f32_launch<256, 256, 2, 4>(A, lda, B, ldb, M, N, K, sym, blocks, ep, st);
  else if (tile == 128)
    f32_launch<128, 128, 2, 2>(A, lda, B, ldb, M, N, K, sym, blocks, ep, st);
  else
    f32_launch<64, 64, 2, 2>(A, lda, B, ldb, M, N, K, sym, blocks, ep, st);
  return hipGetLastError();
}

hipError_t launch_gemm_f64(const double* A, int lda, const double* B, int ldb, int M, int N, int K,
                           bool sym, const EpiParams& ep, hipStream_t st) {
  if (!dims_ok(M, N, K, sym)) return hipErrorInvalidValue;
  const int blocks = f64_blocks(M, N, sym);
  if (f64_tile_edge(M, N, sym) == 128)
    f64_launch<128, 128, 2, 2>(A, lda, B, ldb, M, N, K, sym, blocks, ep, st);
  else
    f64_launch<64, 64, 2, 2>(A, lda, B, ldb, M, N, K, sym, blocks, ep, st);
  return hipGetLastError();
}

}  // namespace zf
