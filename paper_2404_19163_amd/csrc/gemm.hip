// Matrix-core GEMMs of the refinement sweep (gfx950).
//
// Both kernels compute an "NT" product C[i][j] = sum_k A[i][k] * B[j][k] with A
// (M x K) and B (N x K) row-major, i.e. both operands contiguous along the
// contracted index.  The sweep keeps every operand in that form: S and the
// iterates delta, Q are symmetric, and Z is stored both row-major and
// transposed, so no kernel ever needs a transposing load.
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
template <int BM, int BN, int BK, int WM, int WN>
__global__ void __launch_bounds__(WM* WN * 64)
    gemm_x3_kernel(const u16* __restrict__ Ahi, const u16* __restrict__ Alo, int lda,
                   const u16* __restrict__ Bhi, const u16* __restrict__ Blo, int ldb, int K,
                   int tiles_n, int sym, EpiParams ep) {
  using C = X3Cfg<BM, BN, BK, WM, WN>;
  __shared__ __attribute__((aligned(16))) u16 lds[2 * C::STAGE_ELEMS];
  __shared__ double red[C::NT / 64];
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  int ti, tj;
  tile_coords(bid, tiles_n, sym, ti, tj);
  const int mode = sym ? (ti == tj ? 2 : 1) : 0;
  x3_tile<BM, BN, BK, WM, WN>(Ahi, Alo, lda, Bhi, Blo, ldb, K, ti * BM, tj * BN, mode, ep,
                              blockIdx.x, lds, red);
}

// ---------------------------------------------------------------------------
// FP64 kernel
// ---------------------------------------------------------------------------
template <int BM, int BN, int BK, int WM, int WN>
__global__ void __launch_bounds__(WM* WN * 64, 2)
    gemm_f64_kernel(const double* __restrict__ A, int lda, const double* __restrict__ B, int ldb,
                    int K, int tiles_n, int sym, EpiParams ep) {
  using C = F64Cfg<BM, BN, BK, WM, WN>;
  __shared__ double lds[2 * C::STAGE];
  __shared__ double red[C::NT / 64];
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  int ti, tj;
  tile_coords(bid, tiles_n, sym, ti, tj);
  const int mode = sym ? (ti == tj ? 2 : 1) : 0;
  f64_tile<BM, BN, BK, WM, WN>(A, lda, B, ldb, K, ti * BM, tj * BN, mode, ep, blockIdx.x, lds, red);
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

// Tile edge of a launch: the largest of 256 / 128 / 64 that divides both output
// dimensions and still yields at least 128 workgroups (half of the 256 CUs; fewer,
// larger tiles beat more, smaller ones down to that point).  ZF_X3_TILE /
// ZF_X3_SYM_TILE (64, 128 or 256) force the BF16x3 edge when it divides (tuning).
int x3_tile_edge(int M, int N, bool sym) {
  const char* env = getenv(sym ? "ZF_X3_SYM_TILE" : "ZF_X3_TILE");
  if (env) {
    const int want = atoi(env);
    if ((want == 64 || want == 128 || want == 256) && M % want == 0 && N % want == 0) return want;
  }
  if (M % 256 == 0 && N % 256 == 0 && grid_blocks(M, N, 256, sym) >= 128) return 256;
  if (grid_blocks(M, N, 128, sym) >= 128) return 128;
  return 64;
}

int x3_blocks(int M, int N, bool sym) { return grid_blocks(M, N, x3_tile_edge(M, N, sym), sym); }

int f64_tile_edge(int M, int N, bool sym) {
  return grid_blocks(M, N, 128, sym) >= 128 ? 128 : 64;
}

int f64_blocks(int M, int N, bool sym) { return grid_blocks(M, N, f64_tile_edge(M, N, sym), sym); }

int max_blocks(int M, int N) { return grid_blocks(M, N, 64, false); }

hipError_t launch_gemm_x3(const u16* Ahi, const u16* Alo, int lda, const u16* Bhi, const u16* Blo,
                          int ldb, int M, int N, int K, bool sym, const EpiParams& ep,
                          hipStream_t st) {
  if (!dims_ok(M, N, K, sym)) return hipErrorInvalidValue;
  const int tile = x3_tile_edge(M, N, sym);
  const int blocks = x3_blocks(M, N, sym);
  if (tile == 256) {
    constexpr int BM = 256, BN = 256, BK = 32, WM = 2, WN = 4;
    hipLaunchKernelGGL((gemm_x3_kernel<BM, BN, BK, WM, WN>), dim3(blocks), dim3(WM * WN * 64), 0,
                       st, Ahi, Alo, lda, Bhi, Blo, ldb, K, N / BN, sym ? 1 : 0, ep);
  } else if (tile == 128) {
    constexpr int BM = 128, BN = 128, BK = 32, WM = 2, WN = 2;
    hipLaunchKernelGGL((gemm_x3_kernel<BM, BN, BK, WM, WN>), dim3(blocks), dim3(WM * WN * 64), 0,
                       st, Ahi, Alo, lda, Bhi, Blo, ldb, K, N / BN, sym ? 1 : 0, ep);
  } else {
    constexpr int BM = 64, BN = 64, BK = 32, WM = 2, WN = 2;
    hipLaunchKernelGGL((gemm_x3_kernel<BM, BN, BK, WM, WN>), dim3(blocks), dim3(WM * WN * 64), 0,
                       st, Ahi, Alo, lda, Bhi, Blo, ldb, K, N / BN, sym ? 1 : 0, ep);
  }
  return hipGetLastError();
}

hipError_t launch_gemm_f64(const double* A, int lda, const double* B, int ldb, int M, int N, int K,
                           bool sym, const EpiParams& ep, hipStream_t st) {
  if (!dims_ok(M, N, K, sym)) return hipErrorInvalidValue;
  const int blocks = f64_blocks(M, N, sym);
  if (f64_tile_edge(M, N, sym) == 128) {
    constexpr int BM = 128, BN = 128, BK = 16, WM = 2, WN = 2;
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, WM, WN>), dim3(blocks), dim3(WM * WN * 64), 0,
                       st, A, lda, B, ldb, K, N / BN, sym ? 1 : 0, ep);
  } else {
    constexpr int BM = 64, BN = 64, BK = 16, WM = 2, WN = 2;
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, WM, WN>), dim3(blocks), dim3(WM * WN * 64), 0,
                       st, A, lda, B, ldb, K, N / BN, sym ? 1 : 0, ep);
  }
  return hipGetLastError();
}

}  // namespace zf
