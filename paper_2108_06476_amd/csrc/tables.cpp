// tables.cpp -- LGL nodes, weights, differentiation matrix and the orthonormal-Legendre
// Vandermonde inverse for the nodal DGSEM (Section 2.1: DG on Gauss-Lobatto nodes).
//
// The LGL nodes are the zeros of q(x) = P_{N+1}(x) - P_{N-1}(x), which is proportional to
// (1 - x^2) P_N'(x) and has q'(x) = (2N+1) P_N(x); Newton's method on q from the
// Chebyshev-Gauss-Lobatto points.  Weights 2/(N(N+1) P_N(x_i)^2).  The differentiation
// matrix uses the closed form D_ij = P_N(x_i)/(P_N(x_j)(x_i - x_j)) off the diagonal and
// -N(N+1)/4, 0, ..., 0, N(N+1)/4 on it.
#include "tables.h"

#include <cmath>

#include "kernels.h"

namespace dgx {

static void legendre_all(int N, double x, double* P) {
  P[0] = 1.0;
  if (N >= 1) P[1] = x;
  for (int k = 1; k < N; ++k) P[k + 1] = ((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1);
}

bool lgl_tables(int N, double* x, double* w, double* D, double* Vinv) {
  if (N < 1 || N > 15) return false;
  const int n = N + 1;
  double P[18];
  for (int i = 0; i <= N; ++i) {
    double xi = -std::cos(M_PI * i / N);
    if (i > 0 && i < N) {
      for (int it = 0; it < 60; ++it) {
        legendre_all(N + 1, xi, P);
        const double q = P[N + 1] - P[N - 1];
        const double dq = (2 * N + 1) * P[N];
        const double step = q / dq;
        xi -= step;
        if (std::fabs(step) < 1e-17) break;
      }
    }
    x[i] = xi;
  }
  double PN[16];
  for (int i = 0; i < n; ++i) {
    legendre_all(N, x[i], P);
    PN[i] = P[N];
    w[i] = 2.0 / (N * (N + 1.0) * PN[i] * PN[i]);
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      if (i != j) D[i * n + j] = PN[i] / (PN[j] * (x[i] - x[j]));
      else if (i == 0) D[i * n + j] = -N * (N + 1) / 4.0;
      else if (i == N) D[i * n + j] = N * (N + 1) / 4.0;
      else D[i * n + j] = 0.0;
    }
  // V_ia = sqrt((2a+1)/2) P_a(x_i); invert [V | I] by Gauss-Jordan with row pivoting.
  double M[16][32];
  for (int i = 0; i < n; ++i) {
    legendre_all(N, x[i], P);
    for (int a = 0; a < n; ++a) {
      M[i][a] = std::sqrt((2 * a + 1) / 2.0) * P[a];
      M[i][n + a] = (i == a);
    }
  }
  for (int c = 0; c < n; ++c) {
    int best = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(M[r][c]) > std::fabs(M[best][c])) best = r;
    if (M[best][c] == 0.0) return false;
    for (int k = 0; k < 2 * n; ++k) std::swap(M[c][k], M[best][k]);
    const double piv = M[c][c];
    for (int k = 0; k < 2 * n; ++k) M[c][k] /= piv;
    for (int r = 0; r < n; ++r) {
      if (r == c || M[r][c] == 0.0) continue;
      const double f = M[r][c];
      for (int k = 0; k < 2 * n; ++k) M[r][k] -= f * M[c][k];
    }
  }
  for (int a = 0; a < n; ++a)
    for (int i = 0; i < n; ++i) Vinv[a * n + i] = M[a][n + i];
  return true;
}

bool stage_tables(int N, const double* h, double* T, bool weak) {
  double x[16], w[16], D[256], Vinv[256];
  if (N < 1 || N >= TMAX || !lgl_tables(N, x, w, D, Vinv)) return false;
  const int n = N + 1;
  for (int d = 0; d < 3; ++d) {
    const double jac = 2.0 / h[d];
    for (int i = 0; i < n; ++i)
      for (int m = 0; m < n; ++m)
        T[TAB_S + (d * TMAX + i) * TMAX + m] =
            weak ? jac * (w[m] / w[i]) * D[m * n + i] : ((i == m) ? 0.0 : -jac * 2.0 * D[i * n + m]);
    T[TAB_LIFT + d * 2 + 0] = jac / w[0];
    T[TAB_LIFT + d * 2 + 1] = -jac / w[N];
    for (int i = 0; i < n; ++i) T[TAB_FV + d * TMAX + i] = -jac / w[i];
    T[TAB_JAC + d] = jac;
  }
  for (int a = 0; a < n; ++a)
    for (int i = 0; i < n; ++i) T[TAB_VINV + a * TMAX + i] = Vinv[a * n + i];
  for (int i = 0; i < n; ++i) {
    T[TAB_W + i] = w[i];
    T[TAB_X + i] = x[i];
  }
  return true;
}

}  // namespace dgx
