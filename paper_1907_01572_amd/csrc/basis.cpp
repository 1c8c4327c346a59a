// 1-D rules of the nodal DG basis: Gauss-Legendre quadrature (Sec. II.A.5), Legendre-
// Gauss-Lobatto collocation nodes (Sec. II.A.3, Eq. Lagrange_Basis) and barycentric
// Lagrange evaluation (values and first derivatives) at arbitrary points.
#include <cmath>

#include "host.hpp"

namespace hpdg {

namespace {
// P_n(x) with P_{n-1}(x)
void legendre_pair(int n, double x, double& pn, double& pnm1) {
  double a = 1.0, b = x;
  if (n == 0) { pn = 1.0; pnm1 = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double c = ((2.0 * k - 1.0) * x * b - (k - 1.0) * a) / k;
    a = b;
    b = c;
  }
  pn = b;
  pnm1 = a;
}
}  // namespace

void gauss_legendre(int q, double* x, double* w) {
  for (int i = 0; i < (q + 1) / 2; ++i) {
    // Newton from the Tricomi-type initial guess, largest roots first
    double z = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, pm;
      legendre_pair(q, z, p, pm);
      double dp = q * (z * p - pm) / (z * z - 1.0);
      double dz = p / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    double p, pm;
    legendre_pair(q, z, p, pm);
    double dp = q * (z * p - pm) / (z * z - 1.0);
    double wi = 2.0 / ((1.0 - z * z) * dp * dp);
    x[q - 1 - i] = z;
    x[i] = -z;
    w[i] = w[q - 1 - i] = wi;
  }
  if (q % 2 == 1) x[q / 2] = 0.0;
}

void gauss_lobatto(int n, double* x, double* w) {
  const int N = n - 1;
  x[0] = -1.0;
  x[N] = 1.0;
  for (int i = 1; i < (n + 1) / 2; ++i) {
    // interior nodes: roots of P_N'; Newton with P_N'' from Legendre's equation
    double z = -std::cos(M_PI * i / N);
    for (int it = 0; it < 100; ++it) {
      double p, pm;
      legendre_pair(N, z, p, pm);
      double dp = N * (z * p - pm) / (z * z - 1.0);
      double d2p = (2.0 * z * dp - N * (N + 1.0) * p) / (1.0 - z * z);
      double dz = dp / d2p;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    x[i] = z;
    x[N - i] = -z;
  }
  if (n % 2 == 1) x[N / 2] = 0.0;
  for (int i = 0; i < n; ++i) {
    double p, pm;
    legendre_pair(N, x[i], p, pm);
    w[i] = 2.0 / (N * (N + 1.0) * p * p);
  }
}

void lagrange_eval(int n, const double* x, int m, const double* y, double* L, double* D) {
  double bw[kMaxQ + 2];
  for (int i = 0; i < n; ++i) {
    double prod = 1.0;
    for (int j = 0; j < n; ++j)
      if (j != i) prod *= (x[i] - x[j]);
    bw[i] = 1.0 / prod;
  }
  for (int a = 0; a < m; ++a) {
    double t = y[a];
    int hit = -1;
    for (int i = 0; i < n; ++i)
      if (std::fabs(t - x[i]) < 1e-15) hit = i;
    if (hit >= 0) {
      // at a node: Kronecker values, derivative from the differentiation matrix
      double diag = 0.0;
      for (int i = 0; i < n; ++i) {
        L[a * n + i] = (i == hit) ? 1.0 : 0.0;
        if (i != hit) {
          D[a * n + i] = (bw[i] / bw[hit]) / (x[hit] - x[i]);
          diag += 1.0 / (x[hit] - x[i]);
        }
      }
      D[a * n + hit] = diag;
      continue;
    }
    double den = 0.0;
    for (int i = 0; i < n; ++i) den += bw[i] / (t - x[i]);
    double s_all = 0.0;
    for (int j = 0; j < n; ++j) s_all += 1.0 / (t - x[j]);
    for (int i = 0; i < n; ++i) {
      double li = (bw[i] / (t - x[i])) / den;
      L[a * n + i] = li;
      // l_i'(t) = l_i(t) sum_{j != i} 1 / (t - x_j)
      D[a * n + i] = li * (s_all - 1.0 / (t - x[i]));
    }
  }
}

}  // namespace hpdg
