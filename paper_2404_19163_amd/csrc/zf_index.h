// Index arithmetic shared by the device kernels and the host planners: the order in
// which a GEMM grid walks its output tiles, the norm-partial slot of a tile, the
// renumbering of blocks over the 8 XCDs, the task tables of the grouped (batched)
// GEMMs and the 3 x 3 solve of the learned guess's labels.  Everything here is plain
// integer / FP64 arithmetic, so the header also builds for the host alone, where a
// sanitizer test exercises it.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

namespace zf {

// ---------------------------------------------------------------------------
// tile index -> (tile_row, tile_col)
// ---------------------------------------------------------------------------
// Full grids are walked in groups of gm tile rows, column by column inside a
// group (gm = 1: row-major), so that a run of consecutive tiles covers a squarer
// block of the output and touches fewer operand panels; symmetric grids likewise in
// bands of gm rows of the upper triangle.  For full grids gm must divide tiles_m
// (the launchers fall back to 1 otherwise).
__host__ __device__ inline void tile_coords(int bid, int tiles_n, int sym, int& ti, int& tj,
                                            int gm = 1) {
  if (!sym) {
    if (gm > 1) {
      const int g = bid / (gm * tiles_n);
      const int r = bid - g * gm * tiles_n;
      ti = g * gm + r % gm;
      tj = r / gm;
      return;
    }
    ti = bid / tiles_n;
    tj = bid - ti * tiles_n;
    return;
  }
  // Upper triangle in bands of gm tile rows.  Inside a band, column by column: its
  // triangular head (column b0 + c holds rows b0 .. b0 + c), then full columns of
  // the band's rows, so that a run of consecutive tiles covers a squarer block.
  // gm = 1 walks the triangle row by row.
  ti = tj = 0;
  int r = bid;
  for (int b0 = 0; b0 < tiles_n;) {
    const int g = gm < tiles_n - b0 ? gm : tiles_n - b0;  // rows in this band
    const int head = g * (g + 1) / 2;
    const int cnt = head + g * (tiles_n - b0 - g);
    if (r < cnt) {
      if (r < head) {
        int c = 0;
        while ((c + 1) * (c + 2) / 2 <= r) ++c;
        tj = b0 + c;
        ti = b0 + (r - c * (c + 1) / 2);
      } else {
        const int q = r - head;
        tj = b0 + g + q / g;
        ti = b0 + q % g;
      }
      return;
    }
    r -= cnt;
    b0 += g;
  }
}

// Norm partial of tile (ti, tj): its row-major index in the grid (the upper triangle
// when sym), so the partials are summed in one order whatever order the blocks walk.
__host__ __device__ inline int tile_index(int ti, int tj, int tiles_n, bool sym) {
  return sym ? ti * tiles_n - ti * (ti - 1) / 2 + (tj - ti) : ti * tiles_n + tj;
}

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD b % 8).
// Renumber so that each XCD receives a contiguous run of tiles, which then share
// operand rows in that XCD's L2.  A permutation of [0, nblocks) when nblocks is a
// multiple of 8, the identity otherwise.
__host__ __device__ inline int xcd_remap(int bid, int nblocks) {
  if (nblocks % 8 != 0) return bid;
  return (bid % 8) * (nblocks / 8) + bid / 8;
}

// ---------------------------------------------------------------------------
// task tables of the grouped GEMMs
// ---------------------------------------------------------------------------
struct TileTask {
  int m;
  short ti, tj;
};

// XCD-major task tables for count matrices of padded order np[m] and tile edge
// tile[m] (64 or 128).  seg[0..16] bounds 16 runs: runs 0-7 hold the 128-wide
// matrices, runs 8-15 the 64-wide ones, run 8 p + x for XCD x.  Per tile edge the
// matrices go to the 8 XCDs in snake order of decreasing np (each XCD gets a like mix
// of sizes); within a run, matrices by decreasing np, each matrix's tiles consecutive
// in row-major order.  `full` holds every tile, `sym` the tiles with ti <= tj.
inline void build_task_tables(int count, const int* np, const int* tile,
                              std::vector<TileTask>& full, std::vector<TileTask>& sym, int* fseg,
                              int* sseg) {
  full.clear();
  sym.clear();
  for (int part = 0; part < 2; ++part) {
    const int edge = part == 0 ? 128 : 64;
    std::vector<int> ms;
    for (int m = 0; m < count; ++m)
      if (tile[m] == edge) ms.push_back(m);
    std::stable_sort(ms.begin(), ms.end(), [&](int a, int b) { return np[a] > np[b]; });
    std::vector<int> run[8];
    for (int i = 0; i < (int)ms.size(); ++i) {
      const int r = i / 8, pos = i % 8;
      run[(r % 2 == 0) ? pos : 7 - pos].push_back(ms[i]);
    }
    for (int x = 0; x < 8; ++x) {
      fseg[8 * part + x] = (int)full.size();
      sseg[8 * part + x] = (int)sym.size();
      for (int m : run[x]) {
        const int T = np[m] / tile[m];
        for (int i = 0; i < T; ++i)
          for (int j = 0; j < T; ++j) {
            full.push_back(TileTask{m, (short)i, (short)j});
            if (j >= i) sym.push_back(TileTask{m, (short)i, (short)j});
          }
      }
    }
  }
  fseg[16] = (int)full.size();
  sseg[16] = (int)sym.size();
}

// ---------------------------------------------------------------------------
// 3 x 3 linear solve (the normal equations of the learned guess's labels)
// ---------------------------------------------------------------------------
// Gaussian elimination with partial pivoting; A and b are overwritten.  Returns false
// (x untouched) when a pivot is exactly zero or a result is not finite.
inline bool solve3(double A[3][3], double b[3], double x[3]) {
  int p[3] = {0, 1, 2};
  for (int k = 0; k < 3; ++k) {
    int piv = k;
    for (int i = k + 1; i < 3; ++i)
      if (std::fabs(A[p[i]][k]) > std::fabs(A[p[piv]][k])) piv = i;
    std::swap(p[k], p[piv]);
    if (A[p[k]][k] == 0.0) return false;
    for (int i = k + 1; i < 3; ++i) {
      const double f = A[p[i]][k] / A[p[k]][k];
      for (int j = k; j < 3; ++j) A[p[i]][j] -= f * A[p[k]][j];
      b[p[i]] -= f * b[p[k]];
    }
  }
  double y[3];
  for (int k = 2; k >= 0; --k) {
    double s = b[p[k]];
    for (int j = k + 1; j < 3; ++j) s -= A[p[k]][j] * y[j];
    y[k] = s / A[p[k]][k];
  }
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(y[k])) return false;
  for (int k = 0; k < 3; ++k) x[k] = y[k];
  return true;
}

}  // namespace zf
