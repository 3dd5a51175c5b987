// Host-only check of the index arithmetic shared by the GEMM kernels and the batched
// planner (zf_index.h) and of the learned guess's acceptance rule (zf_internal.h).
// Built with hipcc --offload-host-only under AddressSanitizer and UBSan by
// tests/test_host_sanitize.py; no GPU is touched.  Prints "ok <checks>" or the first
// failure and exits non-zero.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "zf_index.h"
#include "zf_internal.h"

using namespace zf;

static long g_checks = 0;
#define CHECK(cond, ...)                                 \
  do {                                                   \
    ++g_checks;                                          \
    if (!(cond)) {                                       \
      fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      fprintf(stderr, __VA_ARGS__);                      \
      fprintf(stderr, "\n");                             \
      exit(1);                                           \
    }                                                    \
  } while (0)

// Every tile of a full T x T grid (group height gm dividing T, or 1) is visited once.
static void full_grid(int T, int gm) {
  std::vector<int> seen(T * T, 0);
  for (int b = 0; b < T * T; ++b) {
    int ti = -1, tj = -1;
    tile_coords(b, T, 0, ti, tj, gm);
    CHECK(ti >= 0 && ti < T && tj >= 0 && tj < T, "full T=%d gm=%d bid %d -> (%d,%d)", T, gm, b, ti, tj);
    const int idx = tile_index(ti, tj, T, false);
    CHECK(idx == ti * T + tj, "full index");
    CHECK(seen[idx]++ == 0, "full T=%d gm=%d tile (%d,%d) twice", T, gm, ti, tj);
  }
}

// Every upper-triangle tile of a T x T grid is visited once for every band height,
// and tile_index maps the triangle onto [0, T(T+1)/2) one to one.
static void sym_grid(int T, int gm) {
  const int cnt = T * (T + 1) / 2;
  std::vector<int> seen(cnt, 0);
  for (int b = 0; b < cnt; ++b) {
    int ti = -1, tj = -1;
    tile_coords(b, T, 1, ti, tj, gm);
    CHECK(ti >= 0 && ti <= tj && tj < T, "sym T=%d gm=%d bid %d -> (%d,%d)", T, gm, b, ti, tj);
    const int idx = tile_index(ti, tj, T, true);
    CHECK(idx >= 0 && idx < cnt, "sym index %d out of range", idx);
    CHECK(seen[idx]++ == 0, "sym T=%d gm=%d tile (%d,%d) twice", T, gm, ti, tj);
  }
  // the row-major triangle index itself: row ti starts after the rows above it
  int k = 0;
  for (int i = 0; i < T; ++i)
    for (int j = i; j < T; ++j) CHECK(tile_index(i, j, T, true) == k++, "row-major triangle order");
}

static void remap(int nb) {
  std::vector<int> seen(nb, 0);
  for (int b = 0; b < nb; ++b) {
    const int r = xcd_remap(b, nb);
    CHECK(r >= 0 && r < nb, "xcd_remap(%d, %d) = %d", b, nb, r);
    CHECK(seen[r]++ == 0, "xcd_remap(%d) hits %d twice", nb, r);
    if (nb % 8 == 0) CHECK(r / (nb / 8) == b % 8, "block %d not in its XCD's run", b);
  }
}

static void tables(std::mt19937& rng, int count) {
  std::vector<int> np(count), tile(count);
  std::uniform_int_distribution<int> dn(1, 1024);
  for (int m = 0; m < count; ++m) {
    const int n = dn(rng);
    tile[m] = n <= 256 ? 64 : 128;
    np[m] = (n + tile[m] - 1) / tile[m] * tile[m];
  }
  std::vector<TileTask> full, sym;
  int fseg[17], sseg[17];
  build_task_tables(count, np.data(), tile.data(), full, sym, fseg, sseg);
  for (int k = 0; k < 16; ++k) {
    CHECK(fseg[k] <= fseg[k + 1] && sseg[k] <= sseg[k + 1], "run bounds not monotone at %d", k);
  }
  CHECK(fseg[0] == 0 && sseg[0] == 0 && fseg[16] == (int)full.size() && sseg[16] == (int)sym.size(),
        "run bounds do not span the tables");
  // each matrix's tiles exactly once, inside one run of its tile edge's part
  std::vector<std::vector<int>> fcnt(count), scnt(count);
  std::vector<int> frun(count, -1), srun(count, -1);
  for (int m = 0; m < count; ++m) {
    const int T = np[m] / tile[m];
    fcnt[m].assign(T * T, 0);
    scnt[m].assign(T * T, 0);
  }
  for (int run = 0; run < 16; ++run) {
    for (int t = fseg[run]; t < fseg[run + 1]; ++t) {
      const TileTask& k = full[t];
      CHECK(k.m >= 0 && k.m < count, "task matrix %d", k.m);
      const int T = np[k.m] / tile[k.m];
      CHECK(k.ti >= 0 && k.ti < T && k.tj >= 0 && k.tj < T, "task tile out of grid");
      CHECK((run < 8) == (tile[k.m] == 128), "matrix %d in the wrong part", k.m);
      CHECK(frun[k.m] == -1 || frun[k.m] == run, "matrix %d split over runs", k.m);
      frun[k.m] = run;
      CHECK(fcnt[k.m][k.ti * T + k.tj]++ == 0, "full task twice");
    }
    for (int t = sseg[run]; t < sseg[run + 1]; ++t) {
      const TileTask& k = sym[t];
      const int T = np[k.m] / tile[k.m];
      CHECK(k.ti <= k.tj && k.tj < T, "sym task below the diagonal");
      CHECK(srun[k.m] == -1 || srun[k.m] == run, "matrix %d split over sym runs", k.m);
      srun[k.m] = run;
      CHECK(scnt[k.m][k.ti * T + k.tj]++ == 0, "sym task twice");
    }
  }
  for (int m = 0; m < count; ++m) {
    const int T = np[m] / tile[m];
    CHECK(frun[m] == srun[m] && frun[m] >= 0, "matrix %d runs differ", m);
    for (int i = 0; i < T; ++i)
      for (int j = 0; j < T; ++j) {
        CHECK(fcnt[m][i * T + j] == 1, "matrix %d full tile (%d,%d) missing", m, i, j);
        CHECK(scnt[m][i * T + j] == (j >= i ? 1 : 0), "matrix %d sym tile (%d,%d)", m, i, j);
      }
  }
}

// max of x p(x)^2 over K + 1 equally spaced points of [x_lo, 1]
static double max_phi(const double c[3], double x_lo, int K = 1024) {
  double mx = 0.0;
  for (int k = 0; k <= K; ++k) {
    const double x = x_lo + (1.0 - x_lo) * k / K;
    const double p = c[0] + c[1] * x + c[2] * x * x;
    mx = fmax(mx, x * p * p);
  }
  return mx;
}

static void acceptance() {
  double c1[3] = {1.0, 0.0, 0.0};  // the scaled identity: x p^2 = x <= 1, kept as is
  CHECK(accept_poly(c1, 0.0) && c1[0] == 1.0 && c1[1] == 0.0 && c1[2] == 0.0, "identity changed");
  double c2[3] = {2.0, 0.0, 0.0};  // max x p^2 = 4: scaled by sqrt(1.9 / 4)
  CHECK(accept_poly(c2, 0.0), "scaled guess rejected");
  CHECK(fabs(c2[0] - 2.0 * sqrt(1.9 / 4.0)) < 1e-15 && max_phi(c2, 0.0) <= 1.9 + 1e-12,
        "rescale to 1.9: c0 = %.17g", c2[0]);
  double c3[3] = {1.0, -2.0, 0.0};  // p changes sign at x = 1/2
  CHECK(!accept_poly(c3, 0.0), "sign change accepted");
  double c4[3] = {1.0, -2.0, 0.0};  // ... but not on [0.6, 1], where p < 0 throughout
  CHECK(!accept_poly(c4, 0.6), "negative p accepted");
  double c5[3] = {0.0, 0.0, 0.0};
  CHECK(!accept_poly(c5, 0.0), "zero polynomial accepted");
  // positive on [0, 1]; x p^2 peaks inside (about 2.38 near x = 0.7): rescaled so that
  // the sampled maximum is 1.9, and the maximum between samples stays well below 2
  double c6[3] = {3.0, -2.0, 0.5};
  CHECK(accept_poly(c6, 0.25), "quadratic guess rejected");
  CHECK(fabs(max_phi(c6, 0.25) - 1.9) < 1e-12, "sampled maximum %.17g", max_phi(c6, 0.25));
  CHECK(max_phi(c6, 0.25, 1 << 16) < 1.9 * (1.0 + 1e-5), "maximum between samples");
}

static void solves(std::mt19937& rng) {
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  for (int t = 0; t < 2000; ++t) {
    double A[3][3], A0[3][3], x[3], b[3], xs[3] = {7.0, 7.0, 7.0};
    for (int i = 0; i < 3; ++i) {
      x[i] = u(rng);
      for (int j = 0; j < 3; ++j) A[i][j] = A0[i][j] = u(rng) + (i == j ? 3.0 : 0.0);
    }
    for (int i = 0; i < 3; ++i) b[i] = A0[i][0] * x[0] + A0[i][1] * x[1] + A0[i][2] * x[2];
    CHECK(solve3(A, b, xs), "diagonally dominant system refused");
    for (int i = 0; i < 3; ++i) CHECK(fabs(xs[i] - x[i]) < 1e-12, "solve3 error %g", xs[i] - x[i]);
  }
  double P[3][3] = {{0, 1, 0}, {0, 0, 2}, {4, 0, 0}}, pb[3] = {1, 2, 3}, px[3];
  CHECK(solve3(P, pb, px) && px[0] == 0.75 && px[1] == 1.0 && px[2] == 1.0, "permutation system");
  double Sg[3][3] = {{1, 2, 3}, {2, 4, 6}, {1, 0, 1}}, sb[3] = {1, 2, 3}, sx[3] = {5, 5, 5};
  CHECK(!solve3(Sg, sb, sx) && sx[0] == 5 && sx[1] == 5 && sx[2] == 5, "singular system accepted");
  double Nn[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, nb[3] = {NAN, 0, 0}, nx[3] = {5, 5, 5};
  CHECK(!solve3(Nn, nb, nx) && nx[0] == 5, "non-finite solution accepted");
}

int main() {
  for (int T = 1; T <= 40; ++T)
    for (int gm = 1; gm <= 8; ++gm)
      if (gm == 1 || T % gm == 0) full_grid(T, gm);
  for (int T = 1; T <= 48; ++T)
    for (int gm = 1; gm <= 9; ++gm) sym_grid(T, gm);
  sym_grid(64, 4);  // N = 4096 at 64-wide tiles (the FP64 triangle)
  sym_grid(80, 4);  // N = 5120
  for (int nb = 1; nb <= 4096; ++nb) remap(nb);
  remap(32 * 33 / 2 * 8);
  std::mt19937 rng(12345);
  for (int count : {1, 2, 7, 8, 9, 16, 63, 512}) tables(rng, count);
  acceptance();
  solves(rng);
  printf("ok %ld\n", g_checks);
  return 0;
}
