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

namespace zf {

typedef __attribute__((address_space(3))) void* lds_ptr;

// 16 bytes per lane, global -> LDS, bypassing VGPRs: lane l's data lands at
// lds_dst + 16 l (lds_dst is wave-uniform, passed in M0).  Issued as inline asm so
// that the compiler does not serialize it against reads of the other pipeline
// stage; callers wait with s_waitcnt vmcnt(0) before the barrier that publishes it.
__device__ __forceinline__ void dma16(const u16* gsrc, u16* lds_dst) {
  const unsigned m0v = __builtin_amdgcn_readfirstlane((unsigned)(uintptr_t)(lds_ptr)lds_dst);
  asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
               :
               : "s"(m0v), "v"(gsrc)
               : "memory", "m0");
}

// ---------------------------------------------------------------------------
// tile index -> (tile_row, tile_col)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tile_coords(int bid, int tiles_n, int sym, int& ti, int& tj) {
  if (!sym) {
    ti = bid / tiles_n;
    tj = bid - ti * tiles_n;
    return;
  }
  // upper triangle in row-major order: row t holds tiles_n - t tiles
  int t = 0;
  int b = bid;
  while (b >= tiles_n - t) {
    b -= tiles_n - t;
    ++t;
  }
  ti = t;
  tj = t + b;
}

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD b % 8).
// Renumber so that each XCD receives a contiguous run of tiles, which then share
// operand rows in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  if (nblocks % 8 != 0) return bid;
  return (bid % 8) * (nblocks / 8) + bid / 8;
}

// ---------------------------------------------------------------------------
// epilogue for 4 consecutive rows (row0 .. row0+3) of one column
//   mode 0: plain; 1: symmetric, tile above the diagonal; 2: symmetric, diagonal tile
// ---------------------------------------------------------------------------
__device__ __forceinline__ void epi_group(const EpiParams& ep, int row0, int col, const double acc[4],
                                          int mode, double& nsum) {
  const int ld = ep.ld;
  double v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = row0 + q;
    const size_t idx = (size_t)row * ld + col;
    double x = ep.beta * acc[q];
    if (ep.d64) x += ep.alpha * ep.d64[idx];
    else if (ep.d32) x += ep.alpha * (double)ep.d32[idx];
    else if (ep.dhi) x += ep.alpha * ((double)bf16_to_f32(ep.dhi[idx]) + (double)bf16_to_f32(ep.dlo[idx]));
    if (row == col && row < ep.n_valid) x += ep.gamma;
    v[q] = x;
  }
  // normal layout
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = row0 + q;
    if (mode == 2 && row > col) continue;
    const size_t idx = (size_t)row * ld + col;
    const double w = (mode == 0) ? 1.0 : ((mode == 1 || row < col) ? 2.0 : 1.0);
    nsum += w * v[q] * v[q];
    if (ep.o64) ep.o64[idx] = v[q];
    const float f = (float)v[q];
    if (ep.o32) ep.o32[idx] = f;
    if (ep.ohi) {
      u16 h, l;
      split_bf16(f, h, l);
      ep.ohi[idx] = h;
      ep.olo[idx] = l;
    }
  }
  // transposed layout (the mirror in symmetric mode)
  const bool any_t = ep.ot64 || ep.ot32 || ep.othi;
  if (!any_t) return;
  const size_t tidx = (size_t)col * ld + row0;
  if (mode == 2) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = row0 + q;
      if (row >= col) continue;
      const float f = (float)v[q];
      if (ep.ot64) ep.ot64[tidx + q] = v[q];
      if (ep.ot32) ep.ot32[tidx + q] = f;
      if (ep.othi) {
        u16 h, l;
        split_bf16(f, h, l);
        ep.othi[tidx + q] = h;
        ep.otlo[tidx + q] = l;
      }
    }
    return;
  }
  if (ep.ot64) {
    double2* p = reinterpret_cast<double2*>(ep.ot64 + tidx);
    p[0] = make_double2(v[0], v[1]);
    p[1] = make_double2(v[2], v[3]);
  }
  float f[4] = {(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
  if (ep.ot32) *reinterpret_cast<float4*>(ep.ot32 + tidx) = make_float4(f[0], f[1], f[2], f[3]);
  if (ep.othi) {
    u16 h[4], l[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) split_bf16(f[q], h[q], l[q]);
    *reinterpret_cast<uint2*>(ep.othi + tidx) =
        make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16));
    *reinterpret_cast<uint2*>(ep.otlo + tidx) =
        make_uint2((uint32_t)l[0] | ((uint32_t)l[1] << 16), (uint32_t)l[2] | ((uint32_t)l[3] << 16));
  }
}

// One output element of the LDS-staged epilogue: value = alpha D + beta acc +
// gamma I in FP64.  normal != 0 writes the normal-layout outputs (and adds the
// element's weight to nsum); normal == 0 writes the transposed outputs.
__device__ __forceinline__ void epi_elem(const EpiParams& ep, int row, int col, float accv, int mode,
                                         int normal, double& nsum) {
  if (normal) {
    if (mode == 2 && row > col) return;
  } else {
    if (mode == 2 && row >= col) return;
  }
  const size_t idx = (size_t)row * ep.ld + col;
  double x = ep.beta * (double)accv;
  if (ep.d64) x += ep.alpha * ep.d64[idx];
  else if (ep.d32) x += ep.alpha * (double)ep.d32[idx];
  else if (ep.dhi) x += ep.alpha * ((double)bf16_to_f32(ep.dhi[idx]) + (double)bf16_to_f32(ep.dlo[idx]));
  if (row == col && row < ep.n_valid) x += ep.gamma;
  const float f = (float)x;
  if (normal) {
    const double w = (mode == 0) ? 1.0 : ((mode == 1 || row < col) ? 2.0 : 1.0);
    nsum += w * x * x;
    if (ep.o64) ep.o64[idx] = x;
    if (ep.o32) ep.o32[idx] = f;
    if (ep.ohi) {
      u16 h, l;
      split_bf16(f, h, l);
      ep.ohi[idx] = h;
      ep.olo[idx] = l;
    }
  } else {
    const size_t t = (size_t)col * ep.ld + row;
    if (ep.ot64) ep.ot64[t] = x;
    if (ep.ot32) ep.ot32[t] = f;
    if (ep.othi) {
      u16 h, l;
      split_bf16(f, h, l);
      ep.othi[t] = h;
      ep.otlo[t] = l;
    }
  }
}

template <int NT>
__device__ __forceinline__ void block_norm_store(double nsum, double* partials, int tile_id,
                                                 double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) nsum += __shfl_xor(nsum, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = nsum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += red[w];
    partials[tile_id] = s;
  }
}

// ---------------------------------------------------------------------------
// (h)(h)+(h)(l)+(l)(h) kernel, BF16 halves, FP32 accumulation
// ---------------------------------------------------------------------------
template <int BM, int BN, int BK, int WM, int WN>
struct X3Cfg {
  static constexpr int NT = WM * WN * 64;
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int FM = WTM / 32, FN = WTN / 32;
  static constexpr int VPR = BK / 8;  // 16-byte chunks per tile row
  static constexpr int A_PT = BM * VPR / NT, B_PT = BN * VPR / NT;
  static constexpr int STAGE = (BM + BN) * 2 * BK;  // 16-bit elements per pipeline stage
  static constexpr int SP = BN + 1;                  // epilogue strip pitch (floats)
  // a stage buffer also holds one 32-row epilogue strip
  static constexpr int STAGE_ELEMS = (STAGE > 32 * SP * 2) ? STAGE : 32 * SP * 2;
  static_assert(BK == 32, "the LDS swizzle assumes 64-byte tile rows");
  static_assert(BM % (WM * 32) == 0 && BN % (WN * 32) == 0, "wave tile");
  static_assert((BM * VPR) % NT == 0 && (BN * VPR) % NT == 0, "load split");
};

// Element offset of logical 16-byte chunk c of tile row r in an unpadded LDS tile
// with 64-byte rows.  Chunk c sits at c ^ f(r), f(r) = ((r >> 1) ^ (r >> 3)) & 3:
// one logical chunk of any 8 aligned consecutive rows (an 8-lane phase over 32
// banks) and of any 16 (a 16-lane phase over 64 banks) lands on distinct banks.
__device__ __forceinline__ int swz64(int r, int c) {
  return r * 32 + ((c ^ (((r >> 1) ^ (r >> 3)) & 3)) << 3);
}

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
  const int m0 = ti * BM, n0 = tj * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;

  // Operands go global -> LDS directly (global_load_lds_dwordx4), one K block
  // ahead, into the swizzled layout: a wave's 64 lanes fill one contiguous 1 KB
  // block (16 rows x 4 physical chunks), so lane l loads row 16 j + l / 4, logical
  // chunk (l % 4) ^ f(row), which is exactly where the reader looks for it.
  constexpr int NW = WM * WN;
  constexpr int ABL = BM / 16 / NW, BBL = BN / 16 / NW;  // 1 KB blocks per wave and matrix
  static_assert(ABL * 16 * NW == BM && BBL * 16 * NW == BN, "direct-load split");
  int a_goff[ABL], b_goff[BBL];
#pragma unroll
  for (int i = 0; i < ABL; ++i) {
    const int r = 16 * (wave + i * NW) + (lane >> 2);
    const int c = (lane & 3) ^ (((r >> 1) ^ (r >> 3)) & 3);
    a_goff[i] = (m0 + r) * lda + c * 8;
  }
#pragma unroll
  for (int i = 0; i < BBL; ++i) {
    const int r = 16 * (wave + i * NW) + (lane >> 2);
    const int c = (lane & 3) ^ (((r >> 1) ^ (r >> 3)) & 3);
    b_goff[i] = (n0 + r) * ldb + c * 8;
  }

  f32x16 acc[C::FM][C::FN];
#pragma unroll
  for (int a = 0; a < C::FM; ++a)
#pragma unroll
    for (int b = 0; b < C::FN; ++b) acc[a][b] = f32x16{};

  const int KT = K / BK;
#define ZF_X3_ISSUE(buf, k0)                                                                      \
  do {                                                                                            \
    u16* base_ = (buf);                                                                           \
    _Pragma("unroll") for (int i = 0; i < ABL; ++i) {                                             \
      const int j = wave + i * NW;                                                                \
      dma16(Ahi + a_goff[i] + (k0), base_ + j * 512);                                             \
      dma16(Alo + a_goff[i] + (k0), base_ + BM * BK + j * 512);                                   \
    }                                                                                             \
    _Pragma("unroll") for (int i = 0; i < BBL; ++i) {                                             \
      const int j = wave + i * NW;                                                                \
      dma16(Bhi + b_goff[i] + (k0), base_ + 2 * BM * BK + j * 512);                               \
      dma16(Blo + b_goff[i] + (k0), base_ + 2 * BM * BK + BN * BK + j * 512);                     \
    }                                                                                             \
  } while (0)

  // Fragment reads of one stage and the three MFMA passes of its K block.
  // Fragments are read per product pass (hh, hl, lh) so that only three of the
  // four operand halves are live at once; consecutive MFMAs never update the
  // same accumulator.
#define ZF_X3_COMPUTE(buf)                                                                        \
  do {                                                                                            \
    const u16* as_h = (buf);                                                                      \
    const u16* as_l = as_h + BM * BK;                                                             \
    const u16* bs_h = as_l + BM * BK;                                                             \
    const u16* bs_l = bs_h + BN * BK;                                                             \
    _Pragma("unroll") for (int kk = 0; kk < BK / 16; ++kk) {                                      \
      const int ch = kk * 2 + (lane >> 5);                                                        \
      int ao[C::FM], bo[C::FN];                                                                   \
      _Pragma("unroll") for (int a = 0; a < C::FM; ++a)                                           \
          ao[a] = swz64(wm * C::WTM + a * 32 + (lane & 31), ch);                                  \
      _Pragma("unroll") for (int b = 0; b < C::FN; ++b)                                           \
          bo[b] = swz64(wn * C::WTN + b * 32 + (lane & 31), ch);                                  \
      bf16x8 ah[C::FM], bx[C::FN], bl[C::FN];                                                     \
      _Pragma("unroll") for (int a = 0; a < C::FM; ++a)                                           \
          ah[a] = *reinterpret_cast<const bf16x8*>(as_h + ao[a]);                                 \
      _Pragma("unroll") for (int b = 0; b < C::FN; ++b)                                           \
          bx[b] = *reinterpret_cast<const bf16x8*>(bs_h + bo[b]);                                 \
      _Pragma("unroll") for (int a = 0; a < C::FM; ++a)                                           \
      _Pragma("unroll") for (int b = 0; b < C::FN; ++b)                                           \
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bx[b], acc[a][b], 0, 0, 0);  \
      _Pragma("unroll") for (int b = 0; b < C::FN; ++b)                                           \
          bl[b] = *reinterpret_cast<const bf16x8*>(bs_l + bo[b]);                                 \
      _Pragma("unroll") for (int a = 0; a < C::FM; ++a)                                           \
      _Pragma("unroll") for (int b = 0; b < C::FN; ++b)                                           \
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);  \
      _Pragma("unroll") for (int a = 0; a < C::FM; ++a)                                           \
          ah[a] = *reinterpret_cast<const bf16x8*>(as_l + ao[a]);                                 \
      _Pragma("unroll") for (int a = 0; a < C::FM; ++a)                                           \
      _Pragma("unroll") for (int b = 0; b < C::FN; ++b)                                           \
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bx[b], acc[a][b], 0, 0, 0);  \
    }                                                                                             \
  } while (0)

  ZF_X3_ISSUE(lds, 0);
  __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): this wave's direct loads have landed
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    u16* cur = lds + (kt & 1) * C::STAGE_ELEMS;
    u16* nxt = lds + ((kt & 1) ^ 1) * C::STAGE_ELEMS;
    // nxt was last read in iteration kt - 1, which every wave has left
    if (kt + 1 < KT) ZF_X3_ISSUE(nxt, (kt + 1) * BK);
    ZF_X3_COMPUTE(cur);
    __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
    __syncthreads();
  }
#undef ZF_X3_ISSUE
#undef ZF_X3_COMPUTE

  // Epilogue through LDS, one 32-row strip of the tile at a time.  A lane holds
  // rows 8 (r / 4) + 4 (lane / 32) + r % 4, column lane % 32 of each 32x32 block;
  // the strip is walked row-major (normal outputs, coalesced) and column-major
  // (transposed / mirrored outputs, coalesced).
  const int mode = sym ? (ti == tj ? 2 : 1) : 0;
  const bool any_t = ep.ot64 || ep.ot32 || ep.othi;
  float* strip = reinterpret_cast<float*>(lds);
  double nsum = 0.0;
  for (int wr = 0; wr < WM; ++wr) {
#pragma unroll
    for (int a = 0; a < C::FM; ++a) {
      __syncthreads();
      if (wm == wr) {
#pragma unroll
        for (int b = 0; b < C::FN; ++b)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int lr = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const int lc = wn * C::WTN + b * 32 + (lane & 31);
            strip[lr * C::SP + lc] = acc[a][b][r];
          }
      }
      __syncthreads();
      const int row0 = m0 + wr * C::WTM + a * 32;
      for (int e = tid; e < 32 * BN; e += C::NT) {
        const int lr = e / BN, lc = e % BN;
        epi_elem(ep, row0 + lr, n0 + lc, strip[lr * C::SP + lc], mode, 1, nsum);
      }
      if (any_t) {
        for (int e = tid; e < 32 * BN; e += C::NT) {
          const int lr = e & 31, lc = e >> 5;
          epi_elem(ep, row0 + lr, n0 + lc, strip[lr * C::SP + lc], mode, 0, nsum);
        }
      }
    }
  }
  if (ep.partials) block_norm_store<C::NT>(nsum, ep.partials, blockIdx.x, red);
}

// ---------------------------------------------------------------------------
// FP64 kernel
// ---------------------------------------------------------------------------
template <int BM, int BN, int BK, int WM, int WN>
struct F64Cfg {
  static constexpr int NT = WM * WN * 64;
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int FM = WTM / 16, FN = WTN / 16;
  static constexpr int LS = BK + 1;   // LDS row stride in doubles (odd: conflict-free columns)
  static constexpr int VPR = BK / 2;  // 16-byte vectors per tile row
  static constexpr int A_PT = BM * VPR / NT, B_PT = BN * VPR / NT;
  static constexpr int STAGE = (BM + BN) * LS;
  static_assert(BM % (WM * 16) == 0 && BN % (WN * 16) == 0, "wave tile");
  static_assert(BK % 4 == 0, "k step");
  static_assert((BM * VPR) % NT == 0 && (BN * VPR) % NT == 0, "load split");
};

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
  const int m0 = ti * BM, n0 = tj * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;

  double2 ra[C::A_PT], rb[C::B_PT];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < C::A_PT; ++i) {
      const int v = tid + i * C::NT, r = v / C::VPR, c = v % C::VPR;
      ra[i] = *reinterpret_cast<const double2*>(A + (size_t)(m0 + r) * lda + k0 + c * 2);
    }
#pragma unroll
    for (int i = 0; i < C::B_PT; ++i) {
      const int v = tid + i * C::NT, r = v / C::VPR, c = v % C::VPR;
      rb[i] = *reinterpret_cast<const double2*>(B + (size_t)(n0 + r) * ldb + k0 + c * 2);
    }
  };
  auto sstore = [&](int s) {
    double* as = lds + s * C::STAGE;
    double* bs = as + BM * C::LS;
#pragma unroll
    for (int i = 0; i < C::A_PT; ++i) {
      const int v = tid + i * C::NT, r = v / C::VPR, c = v % C::VPR;
      as[r * C::LS + c * 2] = ra[i].x;
      as[r * C::LS + c * 2 + 1] = ra[i].y;
    }
#pragma unroll
    for (int i = 0; i < C::B_PT; ++i) {
      const int v = tid + i * C::NT, r = v / C::VPR, c = v % C::VPR;
      bs[r * C::LS + c * 2] = rb[i].x;
      bs[r * C::LS + c * 2 + 1] = rb[i].y;
    }
  };

  f64x4 acc[C::FM][C::FN];
#pragma unroll
  for (int a = 0; a < C::FM; ++a)
#pragma unroll
    for (int b = 0; b < C::FN; ++b) acc[a][b] = f64x4{};

  const int KT = K / BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    const int s = kt & 1;
    if (kt + 1 < KT) gload((kt + 1) * BK);
    const double* as = lds + s * C::STAGE;
    const double* bs = as + BM * C::LS;
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kc = kk * 4 + (lane >> 4);
      double av[C::FM], bv[C::FN];
      // v_mfma_f64_16x16x4_f64 returns row (lane/16) + 4 r of its A operand in
      // accumulator item r; feeding A row 4 (s % 4) + s / 4 into row slot s makes
      // item r of lane group g hold row 4 g + r (4 consecutive rows per lane).
      const int s16 = lane & 15;
      const int arow = ((s16 & 3) << 2) | (s16 >> 2);
#pragma unroll
      for (int a = 0; a < C::FM; ++a) av[a] = as[(wm * C::WTM + a * 16 + arow) * C::LS + kc];
#pragma unroll
      for (int b = 0; b < C::FN; ++b) bv[b] = bs[(wn * C::WTN + b * 16 + (lane & 15)) * C::LS + kc];
#pragma unroll
      for (int a = 0; a < C::FM; ++a)
#pragma unroll
        for (int b = 0; b < C::FN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (kt + 1 < KT) sstore(s ^ 1);
    __syncthreads();
  }

  // epilogue: lane holds rows 4*(lane/16) + r, column lane%16 of each 16x16 block
  const int mode = sym ? (ti == tj ? 2 : 1) : 0;
  double nsum = 0.0;
#pragma unroll
  for (int a = 0; a < C::FM; ++a)
#pragma unroll
    for (int b = 0; b < C::FN; ++b) {
      const int col = n0 + wn * C::WTN + b * 16 + (lane & 15);
      const int row0 = m0 + wm * C::WTM + a * 16 + (lane >> 4) * 4;
      double v[4] = {acc[a][b][0], acc[a][b][1], acc[a][b][2], acc[a][b][3]};
      epi_group(ep, row0, col, v, mode, nsum);
    }
  if (ep.partials) block_norm_store<C::NT>(nsum, ep.partials, blockIdx.x, red);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int num_tiles(int M, int N, bool sym) {
  const int tm = M / kTile, tn = N / kTile;
  return sym ? tm * (tm + 1) / 2 : tm * tn;
}

static bool dims_ok(int M, int N, int K, bool sym) {
  return M > 0 && N > 0 && K > 0 && M % kTile == 0 && N % kTile == 0 && K % kTile == 0 &&
         (!sym || M == N);
}

// Tile edge for the (h)(h)+(h)(l)+(l)(h) kernel: 256 (8 waves) when both output
// dimensions allow it, else 128 (4 waves).  ZF_X3_TILE / ZF_X3_SYM_TILE = 128 or
// 256 override the choice for plain / symmetric launches (tuning only).
int x3_tile(int M, int N, bool sym) {
  const char* env = getenv(sym ? "ZF_X3_SYM_TILE" : "ZF_X3_TILE");
  const int want = env ? atoi(env) : 256;
  if (want == 256 && M % 256 == 0 && N % 256 == 0) return 256;
  return 128;
}

int x3_blocks(int M, int N, bool sym) {
  const int t = x3_tile(M, N, sym);
  const int tm = M / t, tn = N / t;
  return sym ? tm * (tm + 1) / 2 : tm * tn;
}

hipError_t launch_gemm_x3(const u16* Ahi, const u16* Alo, int lda, const u16* Bhi, const u16* Blo,
                          int ldb, int M, int N, int K, bool sym, const EpiParams& ep,
                          hipStream_t st) {
  if (!dims_ok(M, N, K, sym)) return hipErrorInvalidValue;
  const int tile = x3_tile(M, N, sym);
  const int blocks = x3_blocks(M, N, sym);
  if (tile == 256) {
    constexpr int BM = 256, BN = 256, BK = 32, WM = 2, WN = 4;
    hipLaunchKernelGGL((gemm_x3_kernel<BM, BN, BK, WM, WN>), dim3(blocks), dim3(WM * WN * 64), 0,
                       st, Ahi, Alo, lda, Bhi, Blo, ldb, K, N / BN, sym ? 1 : 0, ep);
  } else {
    constexpr int BM = 128, BN = 128, BK = 32, WM = 2, WN = 2;
    hipLaunchKernelGGL((gemm_x3_kernel<BM, BN, BK, WM, WN>), dim3(blocks), dim3(WM * WN * 64), 0,
                       st, Ahi, Alo, lda, Bhi, Blo, ldb, K, N / BN, sym ? 1 : 0, ep);
  }
  return hipGetLastError();
}

hipError_t launch_gemm_f64(const double* A, int lda, const double* B, int ldb, int M, int N, int K,
                           bool sym, const EpiParams& ep, hipStream_t st) {
  if (!dims_ok(M, N, K, sym)) return hipErrorInvalidValue;
  constexpr int BM = 128, BN = 128, BK = 16, WM = 2, WN = 2;
  static_assert(BM == kTile && BN == kTile, "padding granule");
  const int blocks = num_tiles(M, N, sym);
  hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, WM, WN>), dim3(blocks), dim3(WM * WN * 64), 0, st,
                     A, lda, B, ldb, K, N / BN, sym ? 1 : 0, ep);
  return hipGetLastError();
}

}  // namespace zf
