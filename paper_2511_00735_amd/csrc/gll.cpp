// Host GLL reference tables (Sec. 3.1): nodes, weights, differentiation matrix
// and the reference stiffness Kr = D^T diag(w) D on [-1, 1].
#include <cmath>
#include <vector>

#include "host.h"

namespace hps {

// P_N(x) and P_{N-1}(x) by the Bonnet recurrence.
static void legendre_pair(int N, double x, double& pn, double& pnm1) {
  double a = 1.0, b = x;  // P_0, P_1
  if (N == 0) { pn = 1.0; pnm1 = 0.0; return; }
  for (int k = 1; k < N; ++k) {
    const double c = ((2.0 * k + 1.0) * x * b - k * a) / (k + 1.0);
    a = b;
    b = c;
  }
  pn = b;
  pnm1 = a;
}

// Interior GLL nodes are the zeros of q(x) = x P_N - P_{N-1} other than +-1, because
// (1 - x^2) P_N' = N (P_{N-1} - x P_N); since q' = (N+1) P_N, Newton's step is
// dx = q / ((N+1) P_N).  Start from the Chebyshev-Lobatto points.
GllTables gll_tables(int N) {
  GllTables t;
  t.N = N;
  t.xi.assign(N + 1, 0.0);
  t.w.assign(N + 1, 0.0);
  t.D.assign((N + 1) * (N + 1), 0.0);
  t.Kr.assign((N + 1) * (N + 1), 0.0);
  std::vector<double> pn(N + 1);
  for (int j = 0; j <= N; ++j) {
    double x = -std::cos(M_PI * j / N);
    if (j > 0 && j < N) {
      for (int it = 0; it < 100; ++it) {
        double p, q;
        legendre_pair(N, x, p, q);
        const double dx = (x * p - q) / ((N + 1.0) * p);
        x -= dx;
        if (std::fabs(dx) < 1e-16) break;
      }
    }
    t.xi[j] = (j == 0) ? -1.0 : (j == N ? 1.0 : x);
    double p, q;
    legendre_pair(N, t.xi[j], p, q);
    pn[j] = p;
    t.w[j] = 2.0 / (N * (N + 1.0) * p * p);
  }
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= N; ++j)
      t.D[i * (N + 1) + j] = (i == j) ? 0.0 : pn[i] / (pn[j] * (t.xi[i] - t.xi[j]));
  t.D[0] = -N * (N + 1.0) / 4.0;
  t.D[N * (N + 1) + N] = N * (N + 1.0) / 4.0;
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= N; ++j) {
      double s = 0.0;
      for (int k = 0; k <= N; ++k) s += t.D[k * (N + 1) + i] * t.w[k] * t.D[k * (N + 1) + j];
      t.Kr[i * (N + 1) + j] = s;
    }
  return t;
}

}  // namespace hps
