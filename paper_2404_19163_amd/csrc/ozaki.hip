// FP64 products emulated on the int8 matrix cores (v_mfma_i32_32x32x32_i8): the
// Ozaki scheme with 7-bit signed slices, for the residual of the refinement phase
// (Sec. IV.B).  The paper's splitting (Sec. III.A) turns one FP32 number into two
// FP16 words for the Tensor cores; the same idea carried to integer words gives
// near-FP64 products with exact integer accumulation.
//
// Each operand row i is scaled by 2^{-e_i} (e_i the frexp exponent of the row's
// largest magnitude, so every scaled entry lies in (-1, 1)) and cut into s slices
// of 7 bits plus sign: x = sum_p a_p 2^{-7p} + r, |a_p| <= 127, |r| < 2^{-7s}
// (each slice is the integer part of 128 times what is left, so every step is exact
// in FP64).  The NT product C = A B^T then keeps the slice products with
// p + q <= s + 1: products of one weight d = p + q are summed exactly in int32 over
// the whole K (at most s K 127^2 < 2^31 for K <= 16384, s <= 8), and the weights are
// combined in FP64 from the smallest to the largest before the 2^{e_i + f_j} scale.
// Error per entry: |C - A B^T|_ij < (s + 1) 2^{-7s} K 2^{e_i + f_j}.
//
// Slices are stored as s planes of np x np signed bytes; the GEMM reads each plane
// through the 16-bit-unit tile loader of the matrix-core mainloop (two bytes per
// unit, 64-byte rows per pipeline stage), with the int8 product mode.  The tile's
// FP64 accumulators then go through the shared FP64 epilogue (outputs in any
// format and layout, per-tile norm partials).
#include <limits.h>
#include <stdlib.h>

#include "zf_internal.h"
#include "gemm_tiles.inc"

namespace zf {

// Marker exponent of a row holding a non-finite entry: the products of that row
// come out NaN.
constexpr int kOzBad = INT_MIN;

// One block per row: the row's largest magnitude, its exponent, and the s slice
// planes (4 consecutive columns per thread: one 4-byte store per plane).
__global__ void __launch_bounds__(256) oz_slice_kernel(const double* __restrict__ M, int np,
                                                       int s, size_t plane,
                                                       signed char* __restrict__ out,
                                                       int* __restrict__ ex,
                                                       const int* __restrict__ gate) {
  __shared__ double red[4];
  if (gate && *gate) return;
  __shared__ int bad_s[4];
  const int row = blockIdx.x;
  const double* r = M + (size_t)row * np;
  double m = 0.0;
  int bad = 0;
  for (int k = threadIdx.x; k < np; k += 256) {
    const double v = r[k];
    bad |= !isfinite(v);
    m = fmax(m, fabs(v));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    m = fmax(m, __shfl_xor(m, off, 64));
    bad |= __shfl_xor(bad, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = m;
    bad_s[threadIdx.x >> 6] = bad;
  }
  __syncthreads();
  m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  bad = bad_s[0] | bad_s[1] | bad_s[2] | bad_s[3];
  int e = 0;
  if (m > 0.0 && !bad) (void)frexp(m, &e);
  if (threadIdx.x == 0) ex[row] = bad ? kOzBad : e;
  for (int k0 = threadIdx.x * 4; k0 < np; k0 += 1024) {
    double t[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) t[q] = bad ? 0.0 : ldexp(r[k0 + q], -e);
    for (int p = 0; p < s; ++p) {
      unsigned packed = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        t[q] *= 128.0;
        const double iq = trunc(t[q]);
        t[q] -= iq;
        packed |= ((unsigned)(int)iq & 0xffu) << (8 * q);
      }
      *reinterpret_cast<unsigned*>(out + p * plane + (size_t)row * np + k0) = packed;
    }
  }
}

hipError_t launch_oz_slice(const double* M, int np, int s, signed char* out, int* ex,
                           hipStream_t st, const int* gate) {
  if (np <= 0 || np % 128 != 0 || s < 1 || s > kOzMaxSlices) return hipErrorInvalidValue;
  hipLaunchKernelGGL(oz_slice_kernel, dim3(np), dim3(256), 0, st, M, np, s, (size_t)np * np, out,
                     ex, gate);
  return hipGetLastError();
}

// One BM x BN output tile of the emulated product, with the FP64 epilogue.
template <int BM, int BN, int WM, int WN, bool SYM>
__global__ void __launch_bounds__(WM* WN * 64, 2)
    gemm_oz_kernel(const u16* __restrict__ A, const int* __restrict__ ea,
                   const u16* __restrict__ B, const int* __restrict__ eb, int ld16,
                   size_t plane16, int K16, int s, int tiles_n, int gm, EpiParams ep) {
  using C = X3Cfg<BM, BN, 32, WM, WN>;
  __shared__ __attribute__((aligned(16))) u16 lds[2 * C::STAGE_ELEMS];
  __shared__ double red[C::NT / 64];
  if (ep.gate && *ep.gate) return;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  int ti, tj;
  tile_coords(bid, tiles_n, SYM, ti, tj, gm);
  const int mode = SYM ? (ti == tj ? 2 : 1) : 0;
  const int m0 = ti * BM, n0 = tj * BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WN, wn = wave % WN;

  double acc64[C::FM][C::FN][16];
#pragma unroll
  for (int a = 0; a < C::FM; ++a)
#pragma unroll
    for (int b = 0; b < C::FN; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc64[a][b][r] = 0.0;
  X3Acc<BM, BN, 32, WM, WN> acc;
  for (int d = s + 1; d >= 2; --d) {  // weights 2^{-7d}, smallest first
#pragma unroll
    for (int a = 0; a < C::FM; ++a)
#pragma unroll
      for (int b = 0; b < C::FN; ++b) acc[a][b] = f32x16{};
    for (int p = 1; p < d; ++p) {
      const int q = d - p;
      x3_mainloop<BM, BN, 32, WM, WN, PM_I8>(A + (size_t)(p - 1) * plane16, nullptr, ld16,
                                             B + (size_t)(q - 1) * plane16, nullptr, ld16, 0, K16,
                                             m0, n0, lds, acc);
    }
    const double w = ldexp(1.0, -7 * d);
#pragma unroll
    for (int a = 0; a < C::FM; ++a)
#pragma unroll
      for (int b = 0; b < C::FN; ++b) {
        // reinterpret the whole register block (a bit cast of one vector element
        // would read the block's first element)
        const i32x16 iv = __builtin_bit_cast(i32x16, acc[a][b]);
#pragma unroll
        for (int r = 0; r < 16; ++r) acc64[a][b][r] += (double)iv[r] * w;
      }
  }

  // A lane holds rows 8 (r / 4) + 4 (lane / 32) + r % 4, column lane % 32 of each
  // 32 x 32 block: groups of 4 consecutive rows of one column, as epi_group takes them.
  double nsum = 0.0;
#pragma unroll
  for (int a = 0; a < C::FM; ++a)
#pragma unroll
    for (int b = 0; b < C::FN; ++b) {
      const int col = n0 + wn * C::WTN + b * 32 + (lane & 31);
      const int ec = eb[col];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int row0 = m0 + wm * C::WTM + a * 32 + 8 * g + 4 * (lane >> 5);
        double v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int er = ea[row0 + q];
          v[q] = (er == kOzBad || ec == kOzBad) ? __builtin_nan("")
                                                 : ldexp(acc64[a][b][4 * g + q], er + ec);
        }
        epi_group(ep, row0, col, v, mode, nsum);
      }
    }
  if (ep.partials) block_norm_store<C::NT>(nsum, ep.partials, tile_index(ti, tj, tiles_n, SYM), red);
}

static int oz_grid(int np, int t, bool sym) {
  const int tm = np / t;
  return sym ? tm * (tm + 1) / 2 : tm * tm;
}

// Tile edge: 128 while that gives at least 128 workgroups, else 64.  ZF_OZ_TILE /
// ZF_OZ_SYM_TILE (64 or 128) force the edge (tuning).
int oz_tile_edge(int np, bool sym) {
  const char* env = getenv(sym ? "ZF_OZ_SYM_TILE" : "ZF_OZ_TILE");
  if (env && (atoi(env) == 64 || atoi(env) == 128)) return atoi(env);
  return oz_grid(np, 128, sym) >= 128 ? 128 : 64;
}
int oz_blocks(int np, bool sym) { return oz_grid(np, oz_tile_edge(np, sym), sym); }

template <int BM, int WM, int WN>
static void oz_launch(const signed char* A, const int* ea, const signed char* B, const int* eb,
                      int np, int s, bool sym, const EpiParams& ep, hipStream_t st) {
  const int blocks = oz_grid(np, BM, sym);
  const u16* a16 = reinterpret_cast<const u16*>(A);
  const u16* b16 = reinterpret_cast<const u16*>(B);
  const size_t plane16 = (size_t)np * np / 2;
  const int tiles = np / BM;
  const int gm = (!sym && tiles % 4 == 0) ? 4 : 1;
  if (sym)
    hipLaunchKernelGGL((gemm_oz_kernel<BM, BM, WM, WN, true>), dim3(blocks), dim3(WM * WN * 64), 0,
                       st, a16, ea, b16, eb, np / 2, plane16, np / 2, s, tiles, 1, ep);
  else
    hipLaunchKernelGGL((gemm_oz_kernel<BM, BM, WM, WN, false>), dim3(blocks), dim3(WM * WN * 64),
                       0, st, a16, ea, b16, eb, np / 2, plane16, np / 2, s, tiles, gm, ep);
}

hipError_t launch_gemm_oz(const signed char* A, const int* ea, const signed char* B, const int* eb,
                          int np, int s, bool sym, const EpiParams& ep, hipStream_t st) {
  if (np <= 0 || np % 128 != 0 || np > kOzMaxOrder || s < 1 || s > kOzMaxSlices)
    return hipErrorInvalidValue;
  if (oz_tile_edge(np, sym) == 128) oz_launch<128, 2, 2>(A, ea, B, eb, np, s, sym, ep, st);
  else oz_launch<64, 2, 2>(A, ea, B, eb, np, s, sym, ep, st);
  return hipGetLastError();
}

}  // namespace zf
