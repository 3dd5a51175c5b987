// Per-tile GEMM bodies shared by the single-matrix kernels (gemm.hip) and the
// grouped batched kernels (batched.hip).  Defined in gemm_tiles.inc, included by
// both translation units.
#pragma once

#include "zf_internal.h"

namespace zf {

template <int BM, int BN, int BK, int WM, int WN>
struct X3Cfg {
  static constexpr int NT = WM * WN * 64;
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int FM = WTM / 32, FN = WTN / 32;
  static constexpr int STAGE = (BM + BN) * 2 * BK;  // 16-bit elements per pipeline stage
  static constexpr int SP = BN + 1;                  // epilogue strip pitch (elements)
  // the two stage buffers also hold the epilogue's 32-row strips: FP32 accumulators
  // then FP64 values, 32 SP (4 + 8) bytes = 192 SP 16-bit elements
  static constexpr int STAGE_ELEMS = (2 * STAGE > 192 * SP) ? STAGE : 96 * SP;
  static_assert(BK == 32, "the LDS swizzle assumes 64-byte tile rows");
  static_assert(BM % (WM * 32) == 0 && BN % (WN * 32) == 0, "wave tile");
};

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

}  // namespace zf
