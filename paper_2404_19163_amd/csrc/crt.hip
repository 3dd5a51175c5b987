// FP64 products emulated through residues on the int8 matrix cores: the second
// scheme of Ozaki, Uchino & Imamura ("Ozaki scheme II", 2025), for the residual of
// the refinement phase (Sec. IV.B).
//
// Each operand row i is scaled by 2^(beta - e_i) (e_i the frexp exponent of the
// row's largest magnitude) and truncated toward zero to an integer a of at most
// beta bits.  The exact integer product C' = A' B'^T is recovered from its residues
// modulo L pairwise coprime moduli m_l <= 256:
//   residues: a mod m_l in the balanced range [-(m_l / 2), (m_l - 1) / 2] (int8);
//   products: one int8 GEMM per modulus on v_mfma_i32_32x32x32_i8, exact in int32
//             (K 128^2 < 2^31), reduced to rho_l = C'_l mod m_l in [0, m_l);
//   CRT:      T = sum_l rho_l w_l with w_l = (M / m_l) ((M / m_l)^-1 mod m_l) mod M,
//             C' = T - M round(T / M).
// beta is the largest value with 4 K 4^beta <= M (K the number of valid terms), so
// |C'| < M / 4: the quotient T / M is a quarter period away from a rounding tie and
// a double-precision estimate of it is exact after rounding.  T and M are held as
// three 41-bit limbs each (T_p = sum_l rho_l w_{l,p} < 15 * 2^8 * 2^41 < 2^53 is exact
// in FP64); C' = sum_p (T_p - q M_p) 2^(41 p) with every difference exact, summed
// with an error-free transformation, so the result is C' to within about one unit
// before the final 2^(e_i + f_j - 2 beta) scale.
#include <limits.h>
#include <math.h>
#include <stdlib.h>

#include "zf_internal.h"
#include "gemm_tiles.inc"

namespace zf {

// Marker exponent of a row holding a non-finite entry: its products come out NaN.
constexpr int kCrtBad = INT_MIN;
constexpr int kCrtLimbBits = 41;

// The moduli, largest first (pairwise coprime, each <= 256); the first L are used.
__host__ __device__ constexpr int crt_mod(int l) {
  constexpr int m[kCrtMaxModuli] = {256, 255, 253, 251, 247, 241, 239, 233,
                                    229, 227, 223, 217, 211, 199, 197};
  return m[l];
}

// Constants of one moduli set, passed by value to the kernels.
struct CrtConsts {
  int L, beta;
  int mod[kCrtMaxModuli];
  double w[kCrtMaxModuli][3];  // limbs of w_l, least significant first
  double M[3];                 // limbs of M
  double rq[3];                // 2^(41 p) / M
};

// ---------------------------------------------------------------------------
// residues of the truncated rows
// ---------------------------------------------------------------------------
// One block per row: the row's largest magnitude and exponent, then for 4
// consecutive columns per thread the integer a = trunc(x 2^(beta - e)) (|a| < 2^52,
// exact) and its balanced residue modulo each m_l (one 4-byte store per plane).
template <int L, int R>
__global__ void __launch_bounds__(256) crt_residue_kernel(const double* __restrict__ Mat, int np,
                                                          size_t plane, int beta,
                                                          signed char* __restrict__ out,
                                                          int* __restrict__ ex,
                                                          const int* __restrict__ gate) {
  if (gate && *gate) return;
  // R > 0: the row (np <= 1024 R) is read once, into registers, 4 consecutive values
  // per thread and 1024-element chunk; R = 0: read twice (maximum, then residues).
  __shared__ double red[4];
  __shared__ int bad_s[4];
  const int row = blockIdx.x;
  const double* r = Mat + (size_t)row * np;
  double m = 0.0;
  int bad = 0;
  double v[R > 0 ? R : 1][4];
  if constexpr (R > 0) {
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const int k0 = threadIdx.x * 4 + 1024 * c;
      if (k0 < np) {  // np is a multiple of 256, so all 4 are inside
        const double2 u = *reinterpret_cast<const double2*>(r + k0);
        const double2 w = *reinterpret_cast<const double2*>(r + k0 + 2);
        v[c][0] = u.x;
        v[c][1] = u.y;
        v[c][2] = w.x;
        v[c][3] = w.y;
      } else {
        v[c][0] = v[c][1] = v[c][2] = v[c][3] = 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        bad |= !isfinite(v[c][q]);
        m = fmax(m, fabs(v[c][q]));
      }
    }
  } else {
    for (int k = threadIdx.x; k < np; k += 256) {
      const double x = r[k];
      bad |= !isfinite(x);
      m = fmax(m, fabs(x));
    }
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
  if (threadIdx.x == 0) ex[row] = bad ? kCrtBad : e;
  // residues of the 4 values x at k0 .., one packed 4-byte word per modulus
  auto residues = [&](int k0, const double x[4]) __attribute__((always_inline)) {
    double a[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = bad ? 0.0 : trunc(ldexp(x[q], beta - e));
#pragma unroll
    for (int l = 0; l < L; ++l) {
      const int md = crt_mod(l);
      const double dm = (double)md, inv = 1.0 / dm;
      unsigned packed = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // a - m rint(a / m) is exact (both terms are integers below 2^53) and within
        // (-m, m); one step brings it into [0, m), a second into the balanced range
        int ri = (int)(a[q] - dm * rint(a[q] * inv));
        if (ri < 0) ri += md;
        if (ri > (md - 1) / 2) ri -= md;
        packed |= ((unsigned)ri & 0xffu) << (8 * q);
      }
      *reinterpret_cast<unsigned*>(out + l * plane + (size_t)row * np + k0) = packed;
    }
  };
  if constexpr (R > 0) {
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const int k0 = threadIdx.x * 4 + 1024 * c;
      if (k0 < np) residues(k0, v[c]);
    }
  } else {
    for (int k0 = threadIdx.x * 4; k0 < np; k0 += 1024) {
      const double x[4] = {r[k0], r[k0 + 1], r[k0 + 2], r[k0 + 3]};
      residues(k0, x);
    }
  }
}

// ---------------------------------------------------------------------------
// one int8 product per modulus, reduced to its residue
// ---------------------------------------------------------------------------
// 256 x 256 output tiles, 8 waves of 128 x 64, the BF16 tiles' direct-to-LDS
// mainloop in its int8 mode with a 3-stage ring.  One block per (tile, modulus): the products of the L
// moduli are independent, so a grid of L times the tile count fills the chip even
// when the tiles alone would not (the symmetric N = 4096 product: 136 tiles, 1904
// blocks).  The block's int32 sums are reduced to rho_l in [0, m_l) and stored as bytes
// of plane l.  Symmetric mode computes the tiles on or above the diagonal only (the
// reconstruction mirrors).  Blocks are numbered modulus-major, so consecutive blocks
// (renumbered to run together on one XCD) share that modulus's operand panels.
template <bool SYM>
__global__ void __launch_bounds__(512)
    crt_gemm_kernel(const u16* __restrict__ A, const u16* __restrict__ B, int ld16,
                    size_t plane16, int K16, int tiles_n, int gm, CrtConsts cc,
                    unsigned char* __restrict__ rho, size_t plane, int np,
                    const int* __restrict__ gate) {
  if (gate && *gate) return;
  constexpr int BM = 256, BN = 256, WM = 2, WN = 4, NS = 3;
  using C = X3Cfg<BM, BN, 32, WM, WN>;
  // single-product stages of (BM + BN) 32 elements: a 3-stage ring, two stages loading
  __shared__ __attribute__((aligned(16))) u16 lds[NS * (BM + BN) * 32];
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int ntiles = gridDim.x / cc.L;
  const int l = bid / ntiles;
  int ti, tj;
  tile_coords(bid - l * ntiles, tiles_n, SYM, ti, tj, gm);
  const int m0 = ti * BM, n0 = tj * BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WN, wn = wave % WN;
  X3Acc<BM, BN, 32, WM, WN> acc;
  {
#pragma unroll
    for (int a = 0; a < C::FM; ++a)
#pragma unroll
      for (int b = 0; b < C::FN; ++b) acc[a][b] = f32x16{};
    x3_mainloop<BM, BN, 32, WM, WN, PM_I8, NS>(A + (size_t)l * plane16, nullptr, ld16,
                                           B + (size_t)l * plane16, nullptr, ld16, 0, K16, m0,
                                           n0, lds, acc);
    const int md = cc.mod[l];
    const float inv = 1.0f / (float)md;
    // a lane holds rows 8 (r / 4) + 4 (lane / 32) + r % 4, column lane % 32 of each
    // 32 x 32 block
    unsigned char* out = rho + (size_t)l * plane + (size_t)(m0 + wm * C::WTM + 4 * (lane >> 5)) * np +
                         n0 + wn * C::WTN + (lane & 31);
#pragma unroll
    for (int a = 0; a < C::FM; ++a)
#pragma unroll
      for (int b = 0; b < C::FN; ++b) {
        const i32x16 iv = __builtin_bit_cast(i32x16, acc[a][b]);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          // |c| <= K 128^2 <= 2^28: the single-precision quotient is off by at most
          // one, so c - m q lies in (-m, m) and one step brings it into [0, m)
          const int c = iv[r];
          int ri = c - md * (int)rintf((float)c * inv);
          if (ri < 0) ri += md;
          out[(size_t)(a * 32 + 8 * (r >> 2) + (r & 3)) * np + b * 32] = (unsigned char)ri;
        }
      }
  }
}

// ---------------------------------------------------------------------------
// reconstruction and epilogue
// ---------------------------------------------------------------------------
// C' from the L residues of one element (see the file comment), in units of
// 2^(e_i + f_j - 2 beta).
template <int L>
__device__ __forceinline__ double crt_value(const unsigned char (&res)[L], const CrtConsts& cc) {
  double t0 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll
  for (int l = 0; l < L; ++l) {
    const double r = (double)res[l];
    t0 = fma(r, cc.w[l][0], t0);  // every partial sum is an integer below 2^53: exact
    t1 = fma(r, cc.w[l][1], t1);
    t2 = fma(r, cc.w[l][2], t2);
  }
  const double q = rint(t2 * cc.rq[2] + t1 * cc.rq[1] + t0 * cc.rq[0]);
  const double d0 = fma(-q, cc.M[0], t0);  // exact: q M_p < 2^53, both terms >= 0
  const double d1 = fma(-q, cc.M[1], t1);
  const double d2 = fma(-q, cc.M[2], t2);
  const double x = ldexp(d2, 2 * kCrtLimbBits), y = ldexp(d1, kCrtLimbBits);
  // x + y = s + err exactly (two-sum), then the small terms
  const double s = x + y;
  const double bp = s - x;
  const double err = (x - (s - bp)) + (y - bp);
  return s + (err + d0);
}

// One 64 x 64 element tile per block (symmetric mode: tiles on or above the
// diagonal, walked row by row, each element of the upper triangle formed once and
// mirrored by the epilogue); each thread takes groups of 4 consecutive rows of one
// column, the FP64 epilogue's unit, and requests the group's 4 L residues before
// using any of them.
template <int L>
__global__ void __launch_bounds__(256)
    crt_reconstruct_kernel(const unsigned char* __restrict__ rho, size_t plane, int np,
                           const int* __restrict__ ea, const int* __restrict__ eb, int sym,
                           CrtConsts cc, EpiParams ep) {
  __shared__ double red[4];
  if (ep.gate && *ep.gate) return;
  const int T = np / 64;
  int ti, tj;
  tile_coords(blockIdx.x, T, sym != 0, ti, tj, 1);
  const int mode = sym ? (ti == tj ? 2 : 1) : 0;
  const int col = tj * 64 + (threadIdx.x & 63);
  const int ec = eb[col];
  double nsum = 0.0;
#pragma unroll 1
  for (int g = 0; g < 4; ++g) {
    const int row0 = ti * 64 + 4 * ((threadIdx.x >> 6) + 4 * g);
    unsigned char res[4][L];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int l = 0; l < L; ++l) res[q][l] = rho[l * plane + (size_t)(row0 + q) * np + col];
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = row0 + q;
      const int er = ea[row];
      if (mode == 2 && row > col) {
        v[q] = 0.0;  // below the diagonal: formed from its mirror
      } else if (er == kCrtBad || ec == kCrtBad) {
        v[q] = __builtin_nan("");
      } else {
        v[q] = ldexp(crt_value<L>(res[q], cc), er + ec - 2 * cc.beta);
      }
    }
    epi_group(ep, row0, col, v, mode, nsum);
  }
  if (ep.partials) block_norm_store<256>(nsum, ep.partials, tile_index(ti, tj, T, sym != 0), red);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
typedef unsigned __int128 u128;

static long long inv_mod(long long a, long long m) {  // a^-1 mod m, gcd(a, m) = 1
  long long t = 0, nt = 1, r = m, nr = a % m;
  while (nr != 0) {
    const long long q = r / nr;
    long long x = t - q * nt;
    t = nt;
    nt = x;
    x = r - q * nr;
    r = nr;
    nr = x;
  }
  return t < 0 ? t + m : t;
}

// Moduli, limbs of w_l and M, and beta for L moduli and K valid terms.
static bool crt_consts(int L, long long K, CrtConsts& cc) {
  if (L < 2 || L > kCrtMaxModuli || K < 1) return false;
  u128 M = 1;
  for (int l = 0; l < L; ++l) M *= (u128)crt_mod(l);
  cc.L = L;
  int b = 0;  // largest beta with 4 K 4^beta <= M
  while (b < 52 && ((u128)4 * (u128)K << (2 * (b + 1))) <= M) ++b;
  cc.beta = b;
  const u128 mask = ((u128)1 << kCrtLimbBits) - 1;
  for (int l = 0; l < L; ++l) {
    const long long m = crt_mod(l);
    cc.mod[l] = (int)m;
    const u128 Ml = M / (u128)m;
    const u128 w = Ml * (u128)inv_mod((long long)(Ml % (u128)m), m) % M;
    for (int p = 0; p < 3; ++p) cc.w[l][p] = (double)(unsigned long long)((w >> (kCrtLimbBits * p)) & mask);
  }
  for (int l = L; l < kCrtMaxModuli; ++l) {
    cc.mod[l] = 1;
    cc.w[l][0] = cc.w[l][1] = cc.w[l][2] = 0.0;
  }
  const double Md = (double)M;
  for (int p = 0; p < 3; ++p) {
    cc.M[p] = (double)(unsigned long long)((M >> (kCrtLimbBits * p)) & mask);
    cc.rq[p] = ldexp(1.0, kCrtLimbBits * p) / Md;
  }
  return true;
}

int crt_beta(int L, long long K) {
  CrtConsts cc;
  return crt_consts(L, K, cc) ? cc.beta : -1;
}

hipError_t launch_crt_residues(const double* Mat, int np, int L, long long K, signed char* out,
                               int* ex, hipStream_t st, const int* gate) {
  CrtConsts cc;
  if (np <= 0 || np % 256 != 0 || !crt_consts(L, K, cc)) return hipErrorInvalidValue;
  const size_t plane = (size_t)np * np;
  // rows of up to 8192 values stay in registers between the maximum and the residues
#define ZF_CRT_RES(LL)                                                                        \
  case LL:                                                                                     \
    if (np <= 8192)                                                                            \
      hipLaunchKernelGGL((crt_residue_kernel<LL, 8>), dim3(np), dim3(256), 0, st, Mat, np,     \
                         plane, cc.beta, out, ex, gate);                                       \
    else                                                                                       \
      hipLaunchKernelGGL((crt_residue_kernel<LL, 0>), dim3(np), dim3(256), 0, st, Mat, np,     \
                         plane, cc.beta, out, ex, gate);                                       \
    break;
  switch (L) {
    ZF_CRT_RES(2) ZF_CRT_RES(3) ZF_CRT_RES(4) ZF_CRT_RES(5) ZF_CRT_RES(6) ZF_CRT_RES(7)
    ZF_CRT_RES(8) ZF_CRT_RES(9) ZF_CRT_RES(10) ZF_CRT_RES(11) ZF_CRT_RES(12) ZF_CRT_RES(13)
    ZF_CRT_RES(14) ZF_CRT_RES(15)
    default:
      return hipErrorInvalidValue;
  }
#undef ZF_CRT_RES
  return hipGetLastError();
}

int crt_blocks(int np, bool sym) {
  const int T = np / 64;
  return sym ? T * (T + 1) / 2 : T * T;
}

hipError_t launch_crt_product(const signed char* A, const int* ea, const signed char* B,
                              const int* eb, int np, int L, long long K, bool sym,
                              unsigned char* rho, const EpiParams& ep, hipStream_t st) {
  CrtConsts cc;
  if (np <= 0 || np % 256 != 0 || np > kCrtMaxOrder || !crt_consts(L, K, cc))
    return hipErrorInvalidValue;
  const int tiles = np / 256;
  const int blocks = (sym ? tiles * (tiles + 1) / 2 : tiles * tiles) * L;
  const u16* a16 = reinterpret_cast<const u16*>(A);
  const u16* b16 = reinterpret_cast<const u16*>(B);
  const size_t plane16 = (size_t)np * np / 2, plane = (size_t)np * np;
  if (sym)
    hipLaunchKernelGGL(crt_gemm_kernel<true>, dim3(blocks), dim3(512), 0, st, a16, b16, np / 2,
                       plane16, np / 2, tiles, 1, cc, rho, plane, np, ep.gate);
  else
    hipLaunchKernelGGL(crt_gemm_kernel<false>, dim3(blocks), dim3(512), 0, st, a16, b16, np / 2,
                       plane16, np / 2, tiles, tiles % 4 == 0 ? 4 : 1, cc, rho, plane, np,
                       ep.gate);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid(crt_blocks(np, sym));
  const int s = sym ? 1 : 0;
#define ZF_CRT_RECON(LL)                                                                       \
  case LL:                                                                                      \
    hipLaunchKernelGGL(crt_reconstruct_kernel<LL>, grid, dim3(256), 0, st, rho, plane, np, ea,  \
                       eb, s, cc, ep);                                                          \
    break;
  switch (L) {
    ZF_CRT_RECON(2) ZF_CRT_RECON(3) ZF_CRT_RECON(4) ZF_CRT_RECON(5) ZF_CRT_RECON(6)
    ZF_CRT_RECON(7) ZF_CRT_RECON(8) ZF_CRT_RECON(9) ZF_CRT_RECON(10) ZF_CRT_RECON(11)
    ZF_CRT_RECON(12) ZF_CRT_RECON(13) ZF_CRT_RECON(14) ZF_CRT_RECON(15)
    default:
      return hipErrorInvalidValue;
  }
#undef ZF_CRT_RECON
  return hipGetLastError();
}

}  // namespace zf
