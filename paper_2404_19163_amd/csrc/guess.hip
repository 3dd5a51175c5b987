// Learned initial guess Z0 = p(S/g) / sqrt(g), p(x) = c0 + c1 x + c2 x^2.
//
// The recursion converges from any Z0 with ||Z0^T S Z0 - I||_2 < 1 (Sec. III) and
// costs fewer sweeps the closer X0 is to I (Sec. VI: good guesses from earlier
// steps).  A polynomial in S keeps Z0 commuting with S; its coefficients come from
// a small network on cheap spectral features of S:
//   f = [log N, tr(St^k)/N (k = 1..4), max(g_lo,0)/g, g_lo/g, mean_i r_i / g],
//   r_i = sum_j |S_ij|, g = max_i r_i, g_lo = min_i (S_ii - sum_{j != i} |S_ij|), St = S/g,
//   network 8 -> 64 -> 64 -> 3 in FP32 with tanh, on standardized features/labels.
// Training pairs are (features, least-squares fit of p to a converged Z in the
// S^(1/2)-weighted norm); the fit's normal equations need tr(St^k), k = 1..5, and
// <St^k, Z>, k = 1..3, which zf_guess_label evaluates with FP64 GEMMs.
// Training (forward, MSE, backward, Adam) and inference are the kernels below.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "zf.h"
#include "zf_internal.h"

namespace zf {

#define GHIP_TRY(expr)                                                                       \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess)                                                                    \
      return set_error(ZF_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                       __LINE__);                                                            \
  } while (0)

constexpr int NF = 8, NH = 64, NO = 3;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NF, OFF_W2 = OFF_B1 + NH,
              OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NO * NH,
              NPARAM = OFF_B3 + NO;
static_assert(NPARAM == 4931, "parameter layout");

// ---------------------------------------------------------------------------
// reductions over S (and S^2, S^3, Z): one block per row chunk, FP64 partials,
// a fixed-order final sum (bitwise repeatable)
// ---------------------------------------------------------------------------
// Gershgorin statistics and tr(S): out[0] = max r_i, out[1] = min (S_ii - (r_i - |S_ii|)),
// out[2] = mean r_i, out[3] = tr(S).  S: n x n, ld n.
// Gershgorin statistics of S (n x n, ld n) in two passes: one wave per row (coalesced
// row sums, a fixed-order shuffle tree), per-block partials {max r_i, min lo_i,
// sum r_i, sum S_ii}, then one thread folds the partials in block order, so the result
// depends on n only (deterministic).  lo_i = S_ii - (r_i - |S_ii|).
constexpr int kGershBlocks = 512;

__global__ void __launch_bounds__(256) gersh_rows_kernel(const double* __restrict__ S, int n,
                                                         double* __restrict__ part) {
  __shared__ double red[4][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double mx = 0.0, mn = 1e300, sm = 0.0, tr = 0.0;
  for (int i = blockIdx.x * 4 + wave; i < n; i += gridDim.x * 4) {
    const double* row = S + (size_t)i * n;
    double r = 0.0;
    for (int j = lane; j < n; j += 64) r += fabs(row[j]);
    for (int o = 32; o > 0; o >>= 1) r += __shfl_xor(r, o, 64);
    const double d = row[i];
    mx = fmax(mx, r);
    mn = fmin(mn, d - (r - fabs(d)));
    sm += r;
    tr += d;
  }
  if (lane == 0) {
    red[wave][0] = mx;
    red[wave][1] = mn;
    red[wave][2] = sm;
    red[wave][3] = tr;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      red[0][0] = fmax(red[0][0], red[w][0]);
      red[0][1] = fmin(red[0][1], red[w][1]);
      red[0][2] += red[w][2];
      red[0][3] += red[w][3];
    }
    for (int k = 0; k < 4; ++k) part[(size_t)blockIdx.x * 4 + k] = red[0][k];
  }
}

__global__ void gersh_final_kernel(const double* __restrict__ part, int blocks, int n,
                                   double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double mx = part[0], mn = part[1], sm = part[2], tr = part[3];
  for (int b = 1; b < blocks; ++b) {
    mx = fmax(mx, part[4 * b]);
    mn = fmin(mn, part[4 * b + 1]);
    sm += part[4 * b + 2];
    tr += part[4 * b + 3];
  }
  out[0] = mx;
  out[1] = mn;
  out[2] = sm / n;
  out[3] = tr;
}

static void launch_gersh(const double* S, int n, double* out, double* part, hipStream_t st) {
  const int rows4 = (n + 3) / 4;
  const int blocks = rows4 < kGershBlocks ? rows4 : kGershBlocks;
  hipLaunchKernelGGL(gersh_rows_kernel, dim3(blocks), dim3(256), 0, st, S, n, part);
  hipLaunchKernelGGL(gersh_final_kernel, dim3(1), dim3(64), 0, st, part, blocks, n, out);
}

// Up to 8 Frobenius inner products <A_k, B_k> over the valid n x n block of np x np
// matrices: partial sums per block (grid-stride rows), then finalize.
struct Dots {
  const double* a[8];
  const double* b[8];
  int count;
};

__global__ void dots_partial_kernel(Dots d, int n, int np, double* partial) {
  __shared__ double red[8][256];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = blockIdx.x; i < n; i += gridDim.x)
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      const size_t e = (size_t)i * np + j;
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (k < d.count) acc[k] += d.a[k][e] * d.b[k][e];
    }
#pragma unroll
  for (int k = 0; k < 8; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < 8; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 8) partial[(size_t)blockIdx.x * 8 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void dots_final_kernel(const double* __restrict__ partial, int blocks, double* out) {
  if (threadIdx.x < 8) {
    double s = 0.0;
    for (int b = 0; b < blocks; ++b) s += partial[(size_t)b * 8 + threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// the network (FP32)
// ---------------------------------------------------------------------------
struct Net {
  float* params = nullptr;  // NPARAM
  float* m = nullptr;       // Adam moments
  float* v = nullptr;
  float* norm = nullptr;    // mu_x[8], sd_x[8], mu_y[3], sd_y[3]
  float h_norm[32] = {0};   // host copy of norm (for zf_mlp_save)
  double* coef = nullptr;   // prediction output (3 doubles)
  int step = 0;
  bool has_params = false, has_norm = false;
  // training scratch (grown on demand)
  float *act = nullptr, *grad = nullptr, *lpart = nullptr;
  int act_cap = 0;
};
static Net g_net;

static int net_alloc() {
  if (g_net.params) return 0;
  if (hipMalloc((void**)&g_net.params, NPARAM * 4) != hipSuccess ||
      hipMalloc((void**)&g_net.m, NPARAM * 4) != hipSuccess ||
      hipMalloc((void**)&g_net.v, NPARAM * 4) != hipSuccess ||
      hipMalloc((void**)&g_net.norm, 32 * 4) != hipSuccess ||
      hipMalloc((void**)&g_net.grad, NPARAM * 4) != hipSuccess ||
      hipMalloc((void**)&g_net.coef, 64) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(ZF_ERR_NOMEM, "network allocation failed");
  }
  return 0;
}

// Forward for one sample per block (64 threads): standardize, two tanh layers, output.
// act layout per sample: x[8] | h1[64] | h2[64] | y[3].
constexpr int ACT = NF + NH + NH + NO;

__global__ void mlp_forward_kernel(const float* __restrict__ P, const float* __restrict__ norm,
                                   const float* __restrict__ feats, int B, float* __restrict__ act) {
  const int b = blockIdx.x, j = threadIdx.x;
  if (b >= B) return;
  __shared__ float x[NF], h1[NH], h2[NH];
  float* a = act + (size_t)b * ACT;
  if (j < NF) {
    x[j] = (feats[(size_t)b * NF + j] - norm[j]) / norm[NF + j];
    a[j] = x[j];
  }
  __syncthreads();
  float s = P[OFF_B1 + j];
  for (int k = 0; k < NF; ++k) s += P[OFF_W1 + j * NF + k] * x[k];
  h1[j] = tanhf(s);
  a[NF + j] = h1[j];
  __syncthreads();
  s = P[OFF_B2 + j];
  for (int k = 0; k < NH; ++k) s += P[OFF_W2 + j * NH + k] * h1[k];
  h2[j] = tanhf(s);
  a[NF + NH + j] = h2[j];
  __syncthreads();
  if (j < NO) {
    s = P[OFF_B3 + j];
    for (int k = 0; k < NH; ++k) s += P[OFF_W3 + j * NH + k] * h2[k];
    a[NF + 2 * NH + j] = s;
  }
}

// Per sample: dy = 2 (y - t) / (3 B) on standardized labels and the hidden deltas
// dz2 = (W3^T dy) (1 - h2^2), dz1 = (W2^T dz2) (1 - h1^2), written to dl as
// dy[3] | dz2[64] | dz1[64]; lpart[b] = sum of squared errors of the sample.
__global__ void mlp_backward_sample_kernel(const float* __restrict__ P, const float* __restrict__ norm,
                                           const float* __restrict__ labels, int B,
                                           const float* __restrict__ act, float* __restrict__ dl,
                                           float* __restrict__ lpart) {
  const int b = blockIdx.x, j = threadIdx.x;
  if (b >= B) return;
  __shared__ float dy[NO], dz2[NH], lsum[NO];
  const float* a = act + (size_t)b * ACT;
  float* d = dl + (size_t)b * (NO + NH + NH);
  if (j < NO) {
    const float t = (labels[(size_t)b * NO + j] - norm[2 * NF + j]) / norm[2 * NF + NO + j];
    const float e = a[NF + 2 * NH + j] - t;
    dy[j] = 2.f * e / (float)(NO * B);
    lsum[j] = e * e;
    d[j] = dy[j];
  }
  __syncthreads();
  const float h2 = a[NF + NH + j];
  float s = 0.f;
  for (int o = 0; o < NO; ++o) s += P[OFF_W3 + o * NH + j] * dy[o];
  dz2[j] = s * (1.f - h2 * h2);
  d[NO + j] = dz2[j];
  __syncthreads();
  const float h1 = a[NF + j];
  s = 0.f;
  for (int k = 0; k < NH; ++k) s += P[OFF_W2 + k * NH + j] * dz2[k];
  d[NO + NH + j] = s * (1.f - h1 * h1);
  if (j == 0) lpart[b] = lsum[0] + lsum[1] + lsum[2];
}

// One thread per parameter: the batch sum of its gradient in fixed sample order.
__global__ void mlp_param_grad_kernel(const float* __restrict__ act, const float* __restrict__ dl,
                                      int B, float* __restrict__ g) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  float s = 0.f;
  if (p < OFF_B1) {
    const int j = (p - OFF_W1) / NF, k = (p - OFF_W1) % NF;
    for (int b = 0; b < B; ++b) s += dl[(size_t)b * (NO + 2 * NH) + NO + NH + j] * act[(size_t)b * ACT + k];
  } else if (p < OFF_W2) {
    const int j = p - OFF_B1;
    for (int b = 0; b < B; ++b) s += dl[(size_t)b * (NO + 2 * NH) + NO + NH + j];
  } else if (p < OFF_B2) {
    const int j = (p - OFF_W2) / NH, k = (p - OFF_W2) % NH;
    for (int b = 0; b < B; ++b) s += dl[(size_t)b * (NO + 2 * NH) + NO + j] * act[(size_t)b * ACT + NF + k];
  } else if (p < OFF_W3) {
    const int j = p - OFF_B2;
    for (int b = 0; b < B; ++b) s += dl[(size_t)b * (NO + 2 * NH) + NO + j];
  } else if (p < OFF_B3) {
    const int o = (p - OFF_W3) / NH, k = (p - OFF_W3) % NH;
    for (int b = 0; b < B; ++b) s += dl[(size_t)b * (NO + 2 * NH) + o] * act[(size_t)b * ACT + NF + NH + k];
  } else {
    const int o = p - OFF_B3;
    for (int b = 0; b < B; ++b) s += dl[(size_t)b * (NO + 2 * NH) + o];
  }
  g[p] = s;
}

__global__ void adam_kernel(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, float lr, float bc1, float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float gp = g[p];
  const float mp = 0.9f * m[p] + 0.1f * gp;
  const float vp = 0.999f * v[p] + 0.001f * gp * gp;
  m[p] = mp;
  v[p] = vp;
  P[p] -= lr * (mp / bc1) / (sqrtf(vp / bc2) + 1e-8f);
}

__global__ void loss_sum_kernel(const float* __restrict__ lpart, int B, float* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += lpart[b];
    out[0] = (float)(s / (NO * B));
  }
}

// ---------------------------------------------------------------------------
// guess construction: Z0 = (c0 I + c1 S/g + c2 S2/g^2) / sqrt(g) into every layout
// ---------------------------------------------------------------------------
__global__ void guess_write_kernel(const double* __restrict__ S, int n, const double* __restrict__ S2,
                                   const float* __restrict__ S2f, int np, const double* __restrict__ cg,
                                   float* z32, double* z64r, double* z64c, u16* zr_hi, u16* zr_lo,
                                   u16* zc_hi, u16* zc_lo) {
  // cg = {c0, c1, c2, g}
  const double g = cg[3], sg = 1.0 / sqrt(g);
  const double a0 = cg[0] * sg, a1 = cg[1] * sg / g, a2 = cg[2] * sg / (g * g);
  const size_t total = (size_t)np * np;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / np), j = (int)(e % np);
    double v = 0.0;
    if (i < n && j < n) {
      const double s2 = S2 ? S2[e] : (double)S2f[e];
      v = a1 * S[(size_t)i * n + j] + a2 * s2 + (i == j ? a0 : 0.0);
    }
    const float f = (float)v;
    const size_t t = (size_t)j * np + i;
    u16 h, l;
    split_bf16(f, h, l);
    if (z32) z32[e] = f;
    if (z64r) z64r[e] = v;
    if (z64c) z64c[t] = v;
    if (zr_hi) {  // both pairs are K-blocked
      const size_t kr = kb_offset(i, j, np);
      zr_hi[kr] = h;
      zr_lo[kr] = l;
    }
    if (zc_hi) {
      const size_t kt = kb_offset(j, i, np);
      zc_hi[kt] = h;
      zc_lo[kt] = l;
    }
  }
}

// ---------------------------------------------------------------------------
// host helpers used by zf_api.hip
// ---------------------------------------------------------------------------
// features from S (n x n, ld n) and S^2 (np x np: FP64 S2 or FP32 S2f); writes 8 floats
// to feats (device); scratch (>= 6656 doubles) starts with {g, g_lo, mean r_i, tr S}.
int guess_features(const double* S, int n, const double* S2, const float* S2f, int np,
                   const double* S64pad, float* feats, double* scratch, hipStream_t st);

__global__ void features_finish_kernel(const double* __restrict__ gs, const double* __restrict__ dots,
                                       int n, float* feats) {
  if (threadIdx.x != 0) return;
  finish_features(gs[0], gs[1], gs[2], gs[3], dots[0], dots[1], dots[2], n, feats);
}

// ||S||^2, <S, S^2>, ||S^2||^2 over the valid block (S2 in FP64 or FP32)
__global__ void feat_dots_partial_kernel(const double* __restrict__ S, const double* __restrict__ S2d,
                                         const float* __restrict__ S2f, int n, int np,
                                         double* partial) {
  __shared__ double red[3][256];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int i = blockIdx.x; i < n; i += gridDim.x)
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      const size_t e = (size_t)i * np + j;
      const double s = S[e], q = S2d ? S2d[e] : (double)S2f[e];
      a0 += s * s;
      a1 += s * q;
      a2 += q * q;
    }
  red[0][threadIdx.x] = a0;
  red[1][threadIdx.x] = a1;
  red[2][threadIdx.x] = a2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) partial[(size_t)blockIdx.x * 8 + threadIdx.x] = red[threadIdx.x][0];
}

int guess_features(const double* S, int n, const double* S2, const float* S2f, int np,
                   const double* S64pad, float* feats, double* scratch, hipStream_t st) {
  // scratch: [0..3] Gershgorin statistics and tr(S), [8..15] dots, [16..16+8*512) dot
  // partials, [4608..4608+4*512) Gershgorin partials
  launch_gersh(S, n, scratch, scratch + 4608, st);
  const int blocks = n < 512 ? n : 512;
  hipLaunchKernelGGL(feat_dots_partial_kernel, dim3(blocks), dim3(256), 0, st, S64pad, S2, S2f, n,
                     np, scratch + 16);
  hipLaunchKernelGGL(dots_final_kernel, dim3(1), dim3(64), 0, st, scratch + 16, blocks, scratch + 8);
  hipLaunchKernelGGL(features_finish_kernel, dim3(1), dim3(64), 0, st, scratch, scratch + 8, n, feats);
  GHIP_TRY(hipGetLastError());
  return 0;
}

// network inference on one feature vector (device) -> standardized-back coefficients
// (device, 3 doubles); returns ZF_ERR_ARG when no parameters are loaded.
// one block of NH threads per feature vector; coefficients at coef + 4 * block
__global__ void mlp_infer_kernel(const float* __restrict__ P, const float* __restrict__ norm,
                                 const float* __restrict__ feats_all, double* coef_all) {
  __shared__ float x[NF], h1[NH], h2[NH];
  const int j = threadIdx.x;
  const float* feats = feats_all + (size_t)NF * blockIdx.x;
  double* coef = coef_all + (size_t)4 * blockIdx.x;
  if (j < NF) x[j] = (feats[j] - norm[j]) / norm[NF + j];
  __syncthreads();
  float s = P[OFF_B1 + j];
  for (int k = 0; k < NF; ++k) s += P[OFF_W1 + j * NF + k] * x[k];
  h1[j] = tanhf(s);
  __syncthreads();
  s = P[OFF_B2 + j];
  for (int k = 0; k < NH; ++k) s += P[OFF_W2 + j * NH + k] * h1[k];
  h2[j] = tanhf(s);
  __syncthreads();
  if (j < NO) {
    s = P[OFF_B3 + j];
    for (int k = 0; k < NH; ++k) s += P[OFF_W3 + j * NH + k] * h2[k];
    coef[j] = (double)(s * norm[2 * NF + NO + j] + norm[2 * NF + j]);
  }
}

bool net_ready() { return g_net.has_params && g_net.has_norm; }

int guess_infer(const float* feats, double* coef, hipStream_t st) {
  if (!net_ready()) return set_error(ZF_ERR_ARG, "no network parameters / normalization loaded");
  hipLaunchKernelGGL(mlp_infer_kernel, dim3(1), dim3(NH), 0, st, g_net.params, g_net.norm, feats, coef);
  GHIP_TRY(hipGetLastError());
  return 0;
}

int guess_infer_batch(const float* feats, int count, double* coef, hipStream_t st) {
  if (!net_ready()) return set_error(ZF_ERR_ARG, "no network parameters / normalization loaded");
  if (count <= 0) return 0;
  hipLaunchKernelGGL(mlp_infer_kernel, dim3(count), dim3(NH), 0, st, g_net.params, g_net.norm, feats,
                     coef);
  GHIP_TRY(hipGetLastError());
  return 0;
}

bool guess_accept(double c[3], double x_lo) { return accept_poly(c, x_lo); }

hipError_t launch_guess_write(const double* S, int n, const double* S2, const float* S2f, int np,
                              const double* cg, float* z32, double* z64r, double* z64c, u16* zr_hi,
                              u16* zr_lo, u16* zc_hi, u16* zc_lo, hipStream_t st) {
  size_t total = (size_t)np * np;
  size_t g = (total + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(guess_write_kernel, dim3((unsigned)g), dim3(256), 0, st, S, n, S2, S2f, np, cg,
                     z32, z64r, z64c, zr_hi, zr_lo, zc_hi, zc_lo);
  return hipGetLastError();
}

int dots8(const double* const* a, const double* const* b, int count, int n, int np, double* out_dev,
          double* partial, hipStream_t st) {
  Dots d;
  memset(&d, 0, sizeof d);
  for (int k = 0; k < count; ++k) {
    d.a[k] = a[k];
    d.b[k] = b[k];
  }
  d.count = count;
  const int blocks = n < 512 ? n : 512;
  hipLaunchKernelGGL(dots_partial_kernel, dim3(blocks), dim3(256), 0, st, d, n, np, partial);
  hipLaunchKernelGGL(dots_final_kernel, dim3(1), dim3(64), 0, st, partial, blocks, out_dev);
  GHIP_TRY(hipGetLastError());
  return 0;
}

int gersh_stats(const double* S, int n, double* out_dev, double* part, hipStream_t st) {
  launch_gersh(S, n, out_dev, part, st);
  GHIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace zf

using namespace zf;

extern "C" {

int zf_mlp_set_params(const float* host_params, int count) {
  if (!host_params || count != NPARAM) return set_error(ZF_ERR_ARG, "expected %d parameters", NPARAM);
  int rc = net_alloc();
  if (rc < 0) return rc;
  GHIP_TRY(hipMemcpy(g_net.params, host_params, NPARAM * 4, hipMemcpyHostToDevice));
  GHIP_TRY(hipMemset(g_net.m, 0, NPARAM * 4));
  GHIP_TRY(hipMemset(g_net.v, 0, NPARAM * 4));
  g_net.step = 0;
  g_net.has_params = true;
  return 0;
}

int zf_mlp_get_params(float* host_params, int count) {
  if (!host_params || count != NPARAM) return set_error(ZF_ERR_ARG, "expected %d parameters", NPARAM);
  if (!g_net.has_params) return set_error(ZF_ERR_ARG, "no parameters loaded");
  GHIP_TRY(hipMemcpy(host_params, g_net.params, NPARAM * 4, hipMemcpyDeviceToHost));
  return 0;
}

int zf_mlp_set_norm(const float* mu_x, const float* sd_x, const float* mu_y, const float* sd_y) {
  if (!mu_x || !sd_x || !mu_y || !sd_y) return set_error(ZF_ERR_ARG, "NULL normalization");
  for (int k = 0; k < NF; ++k)
    if (!(sd_x[k] > 0.f)) return set_error(ZF_ERR_ARG, "feature scale %d must be > 0", k);
  for (int k = 0; k < NO; ++k)
    if (!(sd_y[k] > 0.f)) return set_error(ZF_ERR_ARG, "label scale %d must be > 0", k);
  int rc = net_alloc();
  if (rc < 0) return rc;
  float h[32] = {0};
  memcpy(h, mu_x, NF * 4);
  memcpy(h + NF, sd_x, NF * 4);
  memcpy(h + 2 * NF, mu_y, NO * 4);
  memcpy(h + 2 * NF + NO, sd_y, NO * 4);
  GHIP_TRY(hipMemcpy(g_net.norm, h, 32 * 4, hipMemcpyHostToDevice));
  memcpy(g_net.h_norm, h, sizeof h);
  g_net.has_norm = true;
  return 0;
}

// File layout (little-endian): 8-byte magic "ZFMLP\0\0\1", int32 {8, 64, 3, 4931},
// float32 mu_x[8], sd_x[8], mu_y[3], sd_y[3], float32 parameters[4931].
static const char kMagic[8] = {'Z', 'F', 'M', 'L', 'P', 0, 0, 1};

int zf_mlp_save(const char* path) {
  if (!path) return set_error(ZF_ERR_ARG, "NULL path");
  if (!net_ready()) return set_error(ZF_ERR_ARG, "no network parameters / normalization loaded");
  std::vector<float> p(NPARAM);
  GHIP_TRY(hipMemcpy(p.data(), g_net.params, NPARAM * 4, hipMemcpyDeviceToHost));
  FILE* f = fopen(path, "wb");
  if (!f) return set_error(ZF_ERR_ARG, "cannot open %s for writing", path);
  const int32_t dims[4] = {NF, NH, NO, NPARAM};
  bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(dims, 4, 4, f) == 4 &&
            fwrite(g_net.h_norm, 4, 2 * NF + 2 * NO, f) == (size_t)(2 * NF + 2 * NO) &&
            fwrite(p.data(), 4, NPARAM, f) == (size_t)NPARAM;
  ok = (fclose(f) == 0) && ok;
  if (!ok) return set_error(ZF_ERR_ARG, "short write to %s", path);
  return 0;
}

int zf_mlp_load(const char* path) {
  if (!path) return set_error(ZF_ERR_ARG, "NULL path");
  FILE* f = fopen(path, "rb");
  if (!f) return set_error(ZF_ERR_ARG, "cannot open %s", path);
  char magic[8];
  int32_t dims[4];
  float nrm[2 * NF + 2 * NO];
  std::vector<float> p(NPARAM);
  const bool ok = fread(magic, 1, 8, f) == 8 && fread(dims, 4, 4, f) == 4 &&
                  fread(nrm, 4, 2 * NF + 2 * NO, f) == (size_t)(2 * NF + 2 * NO) &&
                  fread(p.data(), 4, NPARAM, f) == (size_t)NPARAM;
  const bool trailing = ok && fgetc(f) != EOF;
  fclose(f);
  if (!ok || trailing || memcmp(magic, kMagic, 8) != 0)
    return set_error(ZF_ERR_ARG, "%s is not a network file of this library", path);
  if (dims[0] != NF || dims[1] != NH || dims[2] != NO || dims[3] != NPARAM)
    return set_error(ZF_ERR_ARG, "%s: network shape %d-%d-%d (%d parameters) differs from 8-64-3",
                     path, dims[0], dims[1], dims[2], dims[3]);
  for (int k = 0; k < NPARAM; ++k)
    if (!isfinite(p[k])) return set_error(ZF_ERR_ARG, "%s: parameter %d is not finite", path, k);
  int rc = zf_mlp_set_norm(nrm, nrm + NF, nrm + 2 * NF, nrm + 2 * NF + NO);
  if (rc < 0) return rc;
  return zf_mlp_set_params(p.data(), NPARAM);
}

static int train_common(const float* feats, const float* labels, int batch, hipStream_t st,
                        float* loss_host) {
  if (!feats || !labels || batch <= 0 || batch > 1 << 20) return set_error(ZF_ERR_ARG, "bad batch");
  if (!net_ready()) return set_error(ZF_ERR_ARG, "set parameters and normalization first");
  if (g_net.act_cap < batch) {
    if (g_net.act) (void)hipFree(g_net.act);
    if (g_net.lpart) (void)hipFree(g_net.lpart);
    g_net.act = nullptr;
    g_net.lpart = nullptr;
    g_net.act_cap = 0;
    if (hipMalloc((void**)&g_net.act, (size_t)batch * (ACT + NO + 2 * NH) * 4) != hipSuccess ||
        hipMalloc((void**)&g_net.lpart, (size_t)batch * 4 + 64) != hipSuccess) {
      (void)hipGetLastError();
      return set_error(ZF_ERR_NOMEM, "training scratch allocation failed");
    }
    g_net.act_cap = batch;
  }
  float* act = g_net.act;
  float* dl = g_net.act + (size_t)batch * ACT;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(batch), dim3(NH), 0, st, g_net.params, g_net.norm,
                     feats, batch, act);
  hipLaunchKernelGGL(mlp_backward_sample_kernel, dim3(batch), dim3(NH), 0, st, g_net.params,
                     g_net.norm, labels, batch, act, dl, g_net.lpart);
  hipLaunchKernelGGL(mlp_param_grad_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, act, dl,
                     batch, g_net.grad);
  hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(64), 0, st, g_net.lpart, batch,
                     g_net.lpart + batch);
  GHIP_TRY(hipGetLastError());
  if (loss_host) {
    GHIP_TRY(hipMemcpyAsync(loss_host, g_net.lpart + batch, 4, hipMemcpyDeviceToHost, st));
  }
  return 0;
}

int zf_mlp_grad(const float* feats, const float* labels, int batch, float* grad_host,
                float* loss_host, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  int rc = train_common(feats, labels, batch, st, loss_host);
  if (rc < 0) return rc;
  if (grad_host) GHIP_TRY(hipMemcpyAsync(grad_host, g_net.grad, NPARAM * 4, hipMemcpyDeviceToHost, st));
  GHIP_TRY(hipStreamSynchronize(st));
  return 0;
}

int zf_mlp_train_step(const float* feats, const float* labels, int batch, float lr, float* loss,
                      void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (!(lr > 0.f)) return set_error(ZF_ERR_ARG, "learning rate must be > 0");
  int rc = train_common(feats, labels, batch, st, loss);
  if (rc < 0) return rc;
  g_net.step += 1;
  const float bc1 = 1.f - powf(0.9f, (float)g_net.step);
  const float bc2 = 1.f - powf(0.999f, (float)g_net.step);
  hipLaunchKernelGGL(adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, g_net.params,
                     g_net.m, g_net.v, g_net.grad, lr, bc1, bc2);
  GHIP_TRY(hipGetLastError());
  if (loss) GHIP_TRY(hipStreamSynchronize(st));
  return 0;
}

int zf_mlp_predict(const float* feats, double* coef_host, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (!feats || !coef_host) return set_error(ZF_ERR_ARG, "NULL argument");
  int rc = net_alloc();
  if (rc < 0) return rc;
  rc = guess_infer(feats, g_net.coef, st);
  if (rc < 0) return rc;
  GHIP_TRY(hipMemcpyAsync(coef_host, g_net.coef, 24, hipMemcpyDeviceToHost, st));
  GHIP_TRY(hipStreamSynchronize(st));
  return 0;
}

}  // extern "C"
