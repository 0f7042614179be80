// tables.cpp -- host construction of the 1D tables, in float64.
//
// * Gauss-Legendre rule on (0,1): the N-point rule exact for degree 2N-1
//   that the staged quadrature uses in every direction (text after (2.22),
//   (2.23)-(2.25)).  Nodes by Newton's method on the Legendre three-term
//   recurrence, weights 2 / ((1 - x^2) P_N'(x)^2), mapped from (-1,1).
// * chi_k = L_k and chi'_k at the nodes: shifted Legendre recursion
//   (2.91)-(2.93), integrated Legendre (2.99)-(2.101), chi'_0 = -1,
//   chi'_k = P_{k-1} (2.98).
// * F^{rs}_ij = int_0^1 chi^<r>_i chi^<s>_j (2.90) from the closed-form chart
//   (2.103)-(2.114) (the j = i + 2 case of (2.103) by the stated symmetry).
#include <cmath>

#include "kernels.h"
#include "tables.h"

namespace dpg {

void gauss_legendre_01(int N, double* zeta, double* w) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < N; ++i) {
    double x = std::cos(pi * (i + 0.75) / (N + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= N; ++k) {
        const double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      if (N == 1) { p0 = 1.0; p1 = x; }
      dp = N * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) <= 1e-16 * std::fabs(x) + 1e-300) break;
    }
    // final derivative at the converged node
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= N; ++k) {
      const double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = pk;
    }
    if (N == 1) { p0 = 1.0; p1 = x; }
    dp = N * (x * p1 - p0) / (x * x - 1.0);
    // x runs from near +1 downwards; zeta = (1 - x)/2 increases with i
    zeta[i] = 0.5 * (1.0 - x);
    w[i] = 1.0 / ((1.0 - x * x) * dp * dp);   // (2 / ...) / 2
  }
}

void chi_tables(int L, const double* zeta, int kmax, double* chi, double* dchi) {
  for (int l = 0; l < L; ++l) {
    const double x = zeta[l], t = 2.0 * x - 1.0;
    double P[KT + 2];
    P[0] = 1.0;
    P[1] = t;
    for (int i = 2; i <= kmax + 1; ++i) P[i] = ((2.0 * i - 1.0) * t * P[i - 1] - (i - 1.0) * P[i - 2]) / i;
    for (int k = 0; k <= kmax; ++k) {
      double v, d;
      if (k == 0) { v = 1.0 - x; d = -1.0; }
      else if (k == 1) { v = x; d = 1.0; }
      else { v = (P[k] - P[k - 2]) / (2.0 * (2.0 * k - 1.0)); d = P[k - 1]; }
      chi[k * L + l] = v;
      dchi[k * L + l] = d;
    }
  }
}

static double F00(int i, int j) {
  if (i < j) { const int t = i; i = j; j = t; }
  if (j >= 2) {
    if (i == j) return (1.0 / (2 * j + 1) + 1.0 / (2 * j - 3)) / (4.0 * (2 * j - 1) * (2 * j - 1));
    if (i == j + 2) return -1.0 / (4.0 * (2 * j + 3) * (2 * j - 1) * (2 * j + 1));
    return 0.0;
  }
  if (j == 1) return i == 1 ? 1.0 / 3 : i == 2 ? -1.0 / 12 : i == 3 ? -1.0 / 60 : 0.0;
  if (i == 0) return 1.0 / 3;
  if (i == 1) return 1.0 / 6;
  return ((i & 1) ? -1.0 : 1.0) * F00(i, 1);
}

static double F01(int i, int j) {
  if (j == 0) return -F01(i, 1);
  if (i == 0) return j == 1 ? 0.5 : j == 2 ? -1.0 / 6 : 0.0;
  if (i == 1) return j == 1 ? 0.5 : j == 2 ? 1.0 / 6 : 0.0;
  if (i == 2) return j == 1 ? -1.0 / 6 : j == 3 ? 1.0 / 30 : 0.0;
  double v = 0.0;
  if (i == j - 1) v += 1.0 / (2 * i + 1);
  if (i - 1 == j) v -= 1.0 / (2 * i - 3);
  return v / (2.0 * (2 * i - 1));
}

static double F11(int i, int j) {
  if (i >= 1 && j >= 1) return i == j ? 1.0 / (2 * i - 1) : 0.0;
  if (i < j) { const int t = i; i = j; j = t; }
  return i == 0 ? 1.0 : i == 1 ? -1.0 : 0.0;
}

double ftable_entry(int r, int s, int i, int j) {
  if (r == 0 && s == 0) return F00(i, j);
  if (r == 0 && s == 1) return F01(i, j);
  if (r == 1 && s == 0) return F01(j, i);
  return F11(i, j);
}

void build_tables(double* tab64, float* tab32, double* f64, float* f32) {
  for (int L = 1; L <= LMAX; ++L) {
    double* blk = tab64 + table_offset(L);
    gauss_legendre_01(L, blk, blk + L);
    chi_tables(L, blk, KT - 1, blk + 2 * L, blk + 2 * L + KT * L);
  }
  for (int i = 0; i < TABLE_LEN; ++i) tab32[i] = static_cast<float>(tab64[i]);
  for (int r = 0; r < 2; ++r)
    for (int s = 0; s < 2; ++s)
      for (int i = 0; i < KT; ++i)
        for (int j = 0; j < KT; ++j) {
          const int o = ((2 * r + s) * KT + i) * KT + j;
          f64[o] = ftable_entry(r, s, i, j);
          f32[o] = static_cast<float>(f64[o]);
        }
}

}  // namespace dpg
