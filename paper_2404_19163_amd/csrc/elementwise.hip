// Bandwidth-bound helpers of the refinement path (gfx950): operand preparation
// (split, zero padding, layouts), the scaled-identity guess, the final copy-out
// and the deterministic reduction of the per-tile norm partials.
//
// Every matrix kernel here is a grid-stride loop over 4 consecutive elements of
// a row per thread, so reads and normal-layout writes are coalesced.
#include "zf_internal.h"

namespace zf {

static inline int grid_for(size_t work, int block) {
  size_t g = (work + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

// ---------------------------------------------------------------------------
// S (n x n, ld_src) -> padded np x np: BF16 hi/lo pair (Sec. III.A: the FP64
// value is first rounded to FP32, then split) in the K-blocked layout of the
// matrix-core operands (kb_offset), optionally an FP64 / FP32 row-major copy.
// ---------------------------------------------------------------------------
__global__ void split_pad_kernel(const double* __restrict__ src, int n, int ld_src, int np,
                                 u16* __restrict__ hi, u16* __restrict__ lo,
                                 double* __restrict__ c64, float* __restrict__ c32, int fmt) {
  const size_t total = (size_t)np * np;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / np), j = (int)(e % np);
    const double a = (i < n && j < n) ? src[(size_t)i * ld_src + j] : 0.0;
    const float x = (float)a;
    if (hi) {
      u16 h, l;
      if (fmt == 2) split_f16(x, h, l);
      else split_bf16(x, h, l);
      const size_t k = kb_offset(i, j, np);
      hi[k] = h;
      lo[k] = l;
    }
    if (c64) c64[e] = a;
    if (c32) c32[e] = x;
  }
}

hipError_t launch_split_pad(const double* src, int n, int ld_src, int np, u16* hi, u16* lo,
                            double* copy64, float* copy32, bool transpose_copy, int fmt,
                            hipStream_t st) {
  (void)transpose_copy;
  const size_t total = (size_t)np * np;
  hipLaunchKernelGGL(split_pad_kernel, dim3(grid_for(total, 256)), dim3(256), 0, st, src, n, ld_src,
                     np, hi, lo, copy64, copy32, fmt);
  return hipGetLastError();
}

__global__ void split_flat_kernel(const double* __restrict__ src, int64_t count, u16* __restrict__ hi,
                                  u16* __restrict__ lo, int fmt) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float x = (float)src[e];
    u16 h, l;
    if (fmt == 2) split_f16(x, h, l);
    else split_bf16(x, h, l);
    hi[e] = h;
    lo[e] = l;
  }
}

hipError_t launch_split_flat(const double* src, int64_t count, u16* hi, u16* lo, int fmt,
                             hipStream_t st) {
  hipLaunchKernelGGL(split_flat_kernel, dim3(grid_for((size_t)count, 256)), dim3(256), 0, st, src,
                     count, hi, lo, fmt);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gershgorin bound g = max_i sum_j |S_ij| (FP64).  One wave per row, then one
// block takes the maximum.
// ---------------------------------------------------------------------------
__global__ void row_abs_kernel(const double* __restrict__ S, int n, int ld, double* __restrict__ rs) {
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= n) return;
  const double* row = S + (size_t)wave * ld;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += fabs(row[j]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) rs[wave] = s;
}

__global__ void max_kernel(const double* __restrict__ v, int n, double* __restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, v[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

hipError_t launch_row_abs_max(const double* S, int n, int ld, double* row_sums, double* g_out,
                              hipStream_t st) {
  const int waves_per_block = 4;
  hipLaunchKernelGGL(row_abs_kernel, dim3((n + waves_per_block - 1) / waves_per_block),
                     dim3(64 * waves_per_block), 0, st, S, n, ld, row_sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(max_kernel, dim3(1), dim3(256), 0, st, row_sums, n, g_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Z0 = I / sqrt(g) in every layout the sweep reads (g read on the device).  The
// pairs are K-blocked (kb_offset), where the row-major and the transposed pair of
// the (symmetric) Z0 coincide; the loop walks them in storage order.
// ---------------------------------------------------------------------------
__global__ void init_identity_kernel(const double* __restrict__ g, int n, int np, float* z32,
                                     double* z64r, double* z64c, u16* zr_hi, u16* zr_lo,
                                     u16* zc_hi, u16* zc_lo) {
  const double c = 1.0 / sqrt(g[0]);
  const size_t total = (size_t)np * np;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / np), j = (int)(e % np);
    const double v = (i == j && i < n) ? c : 0.0;
    const float f = (float)v;
    if (z32) z32[e] = f;
    if (z64r) z64r[e] = v;
    if (z64c) z64c[e] = v;
    if (zr_hi || zc_hi) {  // storage element e of a K-blocked pair: k block e / (32 np), row, k % 32
      const size_t panel = (size_t)np << 5;
      const int kk = (int)(e / panel) * 32 + (int)(e & 31), rr = (int)((e % panel) >> 5);
      const float fc = (rr == kk && rr < n) ? (float)c : 0.0f;
      u16 hc, lc;
      split_bf16(fc, hc, lc);
      if (zr_hi) { zr_hi[e] = hc; zr_lo[e] = lc; }
      if (zc_hi) { zc_hi[e] = hc; zc_lo[e] = lc; }
    }
  }
}

hipError_t launch_init_identity(const double* g, int n, int np, float* z32, double* z64r,
                                double* z64c, u16* zr_hi, u16* zr_lo, u16* zc_hi, u16* zc_lo,
                                hipStream_t st) {
  const size_t total = (size_t)np * np;
  hipLaunchKernelGGL(init_identity_kernel, dim3(grid_for(total, 256)), dim3(256), 0, st, g, n, np,
                     z32, z64r, z64c, zr_hi, zr_lo, zc_hi, zc_lo);
  return hipGetLastError();
}

// Given Z0 (n x n, ld n): padded copies in row-major and transposed layouts (the
// pairs K-blocked, kb_offset).  One 64 x 64 tile per block; the transposed copies
// go through a padded LDS tile so that Z0 is read, and every layout written, in
// contiguous runs.  The pairs are the split of Z0's FP32 value.
__global__ void __launch_bounds__(256) init_given_kernel(const double* __restrict__ Z0, int n,
                                                         int np, float* __restrict__ z32,
                                                         double* __restrict__ z64r,
                                                         double* __restrict__ z64c,
                                                         u16* __restrict__ zr_hi,
                                                         u16* __restrict__ zr_lo,
                                                         u16* __restrict__ zc_hi,
                                                         u16* __restrict__ zc_lo) {
  __shared__ double t[64][65];
  const int T = np / 64;
  const int i0 = (blockIdx.x / T) * 64, j0 = (blockIdx.x % T) * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63, i = i0 + r, j = j0 + c;
    const double v = (i < n && j < n) ? Z0[(size_t)i * n + j] : 0.0;
    const size_t idx = (size_t)i * np + j;
    if (z32) z32[idx] = (float)v;
    if (z64r) z64r[idx] = v;
    if (zr_hi) {
      u16 h, l;
      split_bf16((float)v, h, l);
      const size_t kidx = kb_offset(i, j, np);
      zr_hi[kidx] = h;
      zr_lo[kidx] = l;
    }
    t[r][c] = v;
  }
  if (!z64c && !zc_hi) return;
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;  // transposed row j0 + r, column i0 + c
    const size_t idx = (size_t)(j0 + r) * np + i0 + c;
    const double v = t[c][r];
    if (z64c) z64c[idx] = v;
    if (zc_hi) {
      u16 h, l;
      split_bf16((float)v, h, l);
      const size_t kidx = kb_offset(j0 + r, i0 + c, np);
      zc_hi[kidx] = h;
      zc_lo[kidx] = l;
    }
  }
}

hipError_t launch_init_given(const double* Z0, int n, int np, float* z32, double* z64r,
                             double* z64c, u16* zr_hi, u16* zr_lo, u16* zc_hi, u16* zc_lo,
                             hipStream_t st) {
  if (np % 64 != 0 || n > np) return hipErrorInvalidValue;
  const int T = np / 64;
  hipLaunchKernelGGL(init_given_kernel, dim3(T * T), dim3(256), 0, st, Z0, n, np, z32, z64r, z64c,
                     zr_hi, zr_lo, zc_hi, zc_lo);
  return hipGetLastError();
}

// FP32 master -> FP64 row-major and transposed (start of the refinement phase).
// FP32 matrix X (np x np, row-major) -> any of: FP64 row-major, FP64 transposed,
// FP32 transposed, and 16-bit pairs (format fmt) of scale * X in the K-blocked
// layout of the matrix-core operands (kb_offset), of X and/or of its transpose.
// scale is a power of two (exact).  One 64 x 64 tile per block; the transposed
// copies go through a padded LDS tile so that both layouts are read and written in
// contiguous runs.
__global__ void __launch_bounds__(256) widen_kernel(const float* __restrict__ z32, int np,
                                                    double* __restrict__ z64r,
                                                    double* __restrict__ z64c,
                                                    float* __restrict__ zc32, u16* __restrict__ prh,
                                                    u16* __restrict__ prl, u16* __restrict__ pch,
                                                    u16* __restrict__ pcl, float scale, int fmt) {
  __shared__ float t[64][65];
  const int T = np / 64;
  const int i0 = (blockIdx.x / T) * 64, j0 = (blockIdx.x % T) * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    const size_t idx = (size_t)(i0 + r) * np + j0 + c;
    const float v = z32[idx];
    if (z64r) z64r[idx] = (double)v;
    if (prh) {
      u16 h, l;
      split_pair(v * scale, h, l, fmt);
      const size_t kidx = kb_offset(i0 + r, j0 + c, np);
      prh[kidx] = h;
      prl[kidx] = l;
    }
    t[r][c] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;  // transposed row j0 + r, column i0 + c
    const size_t idx = (size_t)(j0 + r) * np + i0 + c;
    const float v = t[c][r];
    if (z64c) z64c[idx] = (double)v;
    if (zc32) zc32[idx] = v;
    if (pch) {
      u16 h, l;
      split_pair(v * scale, h, l, fmt);
      const size_t kidx = kb_offset(j0 + r, i0 + c, np);
      pch[kidx] = h;
      pcl[kidx] = l;
    }
  }
}

hipError_t launch_widen(const float* z32, int np, double* z64r, double* z64c, hipStream_t st,
                        float* zc32, u16* prh, u16* prl, u16* pch, u16* pcl, float scale,
                        int fmt) {
  if (np % 64 != 0) return hipErrorInvalidValue;
  const int T = np / 64;
  hipLaunchKernelGGL(widen_kernel, dim3(T * T), dim3(256), 0, st, z32, np, z64r, z64c, zc32, prh,
                     prl, pch, pcl, scale, fmt);
  return hipGetLastError();
}

__global__ void unpad_f64_kernel(const double* __restrict__ src, int np, int n, double* __restrict__ dst) {
  const size_t total = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    dst[e] = src[(size_t)i * np + j];
  }
}

__global__ void unpad_f32_kernel(const float* __restrict__ src, int np, int n, double* __restrict__ dst) {
  const size_t total = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    dst[e] = (double)src[(size_t)i * np + j];
  }
}

hipError_t launch_unpad_f64(const double* src, int np, int n, double* dst, hipStream_t st) {
  hipLaunchKernelGGL(unpad_f64_kernel, dim3(grid_for((size_t)n * n, 256)), dim3(256), 0, st, src, np,
                     n, dst);
  return hipGetLastError();
}

hipError_t launch_unpad_f32(const float* src, int np, int n, double* dst, hipStream_t st) {
  hipLaunchKernelGGL(unpad_f32_kernel, dim3(grid_for((size_t)n * n, 256)), dim3(256), 0, st, src, np,
                     n, dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ||.||_F from per-tile partial sums: fixed summation order (bitwise repeatable).
// ---------------------------------------------------------------------------
__global__ void norm_finalize_kernel(const double* __restrict__ partials, int count, double* out,
                                     double div) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) s += partials[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(red[0]) / div;
}

hipError_t launch_norm_finalize(const double* partials, int count, double* out, hipStream_t st,
                                double div) {
  hipLaunchKernelGGL(norm_finalize_kernel, dim3(1), dim3(256), 0, st, partials, count, out, div);
  return hipGetLastError();
}

// Err of the sweep (the same fixed-order sum as norm_finalize_kernel), then the stop
// test of Algorithm 2 (Sec. IV.A) on the device; see launch_norm_decide.
__global__ void norm_decide_kernel(const double* __restrict__ partials, int count, int it,
                                   int rule, int pw, int* gate, double* state, double* box) {
  __shared__ double red[256];
  if (*gate) return;
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) s += partials[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double err = sqrt(red[0]);
  int code = 0;
  if (!isfinite(err)) {
    code = 2;
  } else if (it > 0) {
    const double prev = state[0];
    code = rule == 1 ? (err >= prev) : (err > pow(prev, (double)pw));
  }
  if (code) *gate = 1;
  else state[0] = err;
  box[0] = err;
  box[1] = (double)code;
}

hipError_t launch_norm_decide(const double* partials, int count, int it, int rule, int pw,
                              int* gate, double* state, double* box, hipStream_t st) {
  hipLaunchKernelGGL(norm_decide_kernel, dim3(1), dim3(256), 0, st, partials, count, it, rule, pw,
                     gate, state, box);
  return hipGetLastError();
}

__global__ void fill_zero_kernel(uint32_t* p, size_t words) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < words;
       e += (size_t)gridDim.x * blockDim.x)
    p[e] = 0u;
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t words = bytes / 4;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(words, 256)), dim3(256), 0, st, (uint32_t*)p, words);
  return hipGetLastError();
}

}  // namespace zf
