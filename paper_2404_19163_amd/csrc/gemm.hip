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
                    int K, int tiles_n, int gm, EpiParams ep, int split_from) {
  using C = F64Cfg<BM, BN, BK, WM, WN>;
  __shared__ double lds[2 * C::STAGE];
  __shared__ double red[C::NT / 64];
  if (ep.gate && *ep.gate) return;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  int ti, tj;
  tile_coords(bid, tiles_n, SYM, ti, tj, gm);
  const int pidx = tile_index(ti, tj, tiles_n, SYM);
  if (pidx >= split_from) return;  // one of the tail kernel's tiles
  const int mode = SYM ? (ti == tj ? 2 : 1) : 0;
  f64_tile<BM, BN, BK, WM, WN>(A, lda, B, ldb, K, ti * BM, tj * BN, mode, ep, pidx, lds, red);
}

// The last tiles of an FP64 grid whose last round of blocks would run nearly alone
// (N = 4096 symmetric: 2080 tiles of 64 on 1024 four-per-CU block slots, 32 tiles
// left for a third round), launched right after the main grid as `pieces` K ranges
// per tile, one block each: the last round then holds 4 x 32 short blocks instead of
// 32 long ones.  The split tiles are those with norm-partial index split_from and
// above (the main grid skips them), the same tiles whatever order the main grid walks
// in, so results do not depend on the band height.  Block u takes piece u % pieces of
// tile split_from + u / pieces.  The block
// with a tile's last K range adds the other pieces' FP64 partial sums (part, one
// tile-sized slot per block, added in piece order) and runs the epilogue; it waits
// only on the tile's earlier pieces, blocks with smaller index that wait on nothing,
// and the wait is bounded (a block that gives up writes NaN for its tile, which the
// stop test reports).  flags[u / pieces] counts the finished pieces and is brought
// back to 0 by the last one.  A kernel of its own: the split's extra registers would
// cost the main grid a quarter of its block slots.
constexpr int kF64SpinLimit = 1 << 20;

template <int BM, int BN, int BK, int WM, int WN, bool SYM>
__global__ void __launch_bounds__(WM* WN * 64, 2)
    gemm_f64_tail_kernel(const double* __restrict__ A, int lda, const double* __restrict__ B,
                         int ldb, int K, int tiles_n, EpiParams ep, int split_from, int pieces,
                         double* __restrict__ part, int* __restrict__ flags) {
  using C = F64Cfg<BM, BN, BK, WM, WN>;
  __shared__ double lds[2 * C::STAGE];
  __shared__ double red[C::NT / 64];
  __shared__ int ok_s;
  if (ep.gate && *ep.gate) return;
  const int u = blockIdx.x, tt = u / pieces, pc = u % pieces;
  int ti, tj;
  tile_of_index(split_from + tt, tiles_n, SYM, ti, tj);
  const int mode = SYM ? (ti == tj ? 2 : 1) : 0;
  const int kp = K / pieces;
  F64Acc<BM, BN, BK, WM, WN> acc;
  f64_mainloop<BM, BN, BK, WM, WN>(A, lda, B, ldb, pc * kp, (pc + 1) * kp, ti * BM, tj * BN, lds,
                                   acc);
  // the accumulators as lane-contiguous 16-byte vectors: pair (a, b, h) of thread tid
  // at ((a FN + b) 2 + h) NT + tid
  constexpr int SLOT = BM * BN;
  if (pc < pieces - 1) {
    double2* dst = reinterpret_cast<double2*>(part + (size_t)u * SLOT);
#pragma unroll
    for (int a = 0; a < C::FM; ++a)
#pragma unroll
      for (int b = 0; b < C::FN; ++b)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          dst[((a * C::FN + b) * 2 + h) * C::NT + threadIdx.x] =
              make_double2(acc[a][b][2 * h], acc[a][b][2 * h + 1]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(flags + tt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  if (threadIdx.x == 0) {
    int ok = 1, polls = 0;
    while (__hip_atomic_load(flags + tt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < pieces - 1) {
      if (++polls > kF64SpinLimit) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __hip_atomic_fetch_add(flags + tt, -(pieces - 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ok_s = ok;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  // the last piece's own sum, then the earlier pieces in order
  for (int q = 0; q < pieces - 1; ++q) {
    const double2* src = reinterpret_cast<const double2*>(part + (size_t)(u - pc + q) * SLOT);
#pragma unroll
    for (int a = 0; a < C::FM; ++a)
#pragma unroll
      for (int b = 0; b < C::FN; ++b)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const double2 v = src[((a * C::FN + b) * 2 + h) * C::NT + threadIdx.x];
          acc[a][b][2 * h] += v.x;
          acc[a][b][2 * h + 1] += v.y;
        }
  }
  if (!ok_s) {
#pragma unroll
    for (int a = 0; a < C::FM; ++a)
#pragma unroll
      for (int b = 0; b < C::FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[a][b][r] = __builtin_nan("");
  }
  f64_epilogue<BM, BN, BK, WM, WN>(acc, ti * BM, tj * BN, mode, ep,
                                   tile_index(ti, tj, tiles_n, SYM), red);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// CUs of the current device (cached per device), 0 if unknown.
static int device_cus() {
  static int cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (!cached[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    cached[dev] = v;
  }
  return cached[dev];
}

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

// The FP64 tail split (gemm_f64_kernel) of a grid of T tiles of 64 with contracted
// dimension K: in a grid of at least one full round of the 4-per-CU block slots, the
// tiles left for a last round that is at most a quarter full, as 4 K pieces each
// (main = T - tail blocks first).  Grids smaller than one round keep one block per
// tile.  ZF_F64_TAIL = 0 turns the split off (tuning, tests).
static void f64_tail_plan(int T, int K, int& main_blocks, int& pieces) {
  main_blocks = T;
  pieces = 1;
  const char* env = getenv("ZF_F64_TAIL");
  if (env && atoi(env) == 0) return;
  const int slots = 4 * device_cus();
  if (slots <= 0 || T < slots || K % (4 * 16)) return;
  const int tail = T % slots;
  if (tail == 0 || 4 * tail > slots) return;
  main_blocks = T - tail;
  pieces = 4;
}

size_t f64_split_part_elems() { return (size_t)device_cus() * 4 * 64 * 64; }
int f64_split_flag_count() { return device_cus(); }

template <int BM, int BN, int WM, int WN>
static void f64_launch(const double* A, int lda, const double* B, int ldb, int M, int N, int K,
                       bool sym, int blocks, const EpiParams& ep, hipStream_t st,
                       const F64Split* sp) {
  int main_blocks = blocks, pieces = 1;
  if (BM == 64 && sp && sp->part && sp->flags) {
    f64_tail_plan(blocks, K, main_blocks, pieces);
    const int tail = blocks - main_blocks;
    if (pieces > 1 && ((size_t)tail * pieces * BM * BN > sp->part_elems || tail > sp->flag_count)) {
      main_blocks = blocks;
      pieces = 1;
    }
  }
  // the main grid walks every tile and leaves tiles main_blocks.. (by norm-partial
  // index) to the tail kernel
  if (sym)
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, 16, WM, WN, true>), dim3(blocks),
                       dim3(WM * WN * 64), 0, st, A, lda, B, ldb, K, N / BN, sym_group(), ep,
                       main_blocks);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, 16, WM, WN, false>), dim3(blocks),
                       dim3(WM * WN * 64), 0, st, A, lda, B, ldb, K, N / BN, tile_group(M, BM),
                       ep, main_blocks);
  if (main_blocks == blocks) return;
  const int grid = (blocks - main_blocks) * pieces;
  if (sym)
    hipLaunchKernelGGL((gemm_f64_tail_kernel<BM, BN, 16, WM, WN, true>), dim3(grid),
                       dim3(WM * WN * 64), 0, st, A, lda, B, ldb, K, N / BN, ep, main_blocks,
                       pieces, sp->part, sp->flags);
  else
    hipLaunchKernelGGL((gemm_f64_tail_kernel<BM, BN, 16, WM, WN, false>), dim3(grid),
                       dim3(WM * WN * 64), 0, st, A, lda, B, ldb, K, N / BN, ep, main_blocks,
                       pieces, sp->part, sp->flags);
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
                           bool sym, const EpiParams& ep, hipStream_t st, const F64Split* sp) {
  if (!dims_ok(M, N, K, sym)) return hipErrorInvalidValue;
  const int blocks = f64_blocks(M, N, sym);
  if (f64_tile_edge(M, N, sym) == 128)
    f64_launch<128, 128, 2, 2>(A, lda, B, ldb, M, N, K, sym, blocks, ep, st, nullptr);
  else
    f64_launch<64, 64, 2, 2>(A, lda, B, ldb, M, N, K, sym, blocks, ep, st, sp);
  return hipGetLastError();
}

}  // namespace zf
