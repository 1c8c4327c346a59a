// Analytic macro-element maps, their Jacobians and the manufactured sources, shared by the
// host tables and the device kernels that evaluate them at quadrature points (Sec. II.A.1,
// Eq. Phi_e; Sec. II.A.5, Eq. Jacobian; Sec. III.C, Eq. inverse_mapping and the cubed-sphere
// macro-mesh).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace hpdg {

// r = 1 / s with s linear in z between (x1, 1/r1) and (x2, 1/r2): the inverse radial map, free of
// cancellation; dr / dz
__host__ __device__ inline void inverse_radius(double z, double x1, double x2, double r1, double r2, double& r,
                                               double& dr) {
  const double s = ((x2 - z) / r1 + (z - x1) / r2) / (x2 - x1);
  r = 1.0 / s;
  dr = -r * r * (1.0 / r2 - 1.0 / r1) / (x2 - x1);
}

// radial coordinate r(z) and dr/dz of a shell patch: par[9] kind (0 linear, 1 inverse, 2 linear
// to zeta_break then inverse), par[10..13] r_in, r_out, zeta_break, r_break; zc (the cell
// centre's z) decides the branch of a point exactly at the break
__host__ __device__ inline void shell_radius(const double* par, double z, double zc, double& r, double& dr) {
  const int kind = static_cast<int>(par[9]);
  const double r_in = par[10], r_out = par[11], zb = par[12], rb = par[13];
  if (kind == 0) {
    r = r_in + 0.5 * (z + 1.0) * (r_out - r_in);
    dr = 0.5 * (r_out - r_in);
  } else if (kind == 1) {
    inverse_radius(z, -1.0, 1.0, r_in, r_out, r, dr);
  } else if (z < zb || (z == zb && zc <= zb)) {
    dr = (rb - r_in) / (zb + 1.0);
    r = r_in + (z + 1.0) * dr;
  } else {
    inverse_radius(z, zb, 1.0, rb, r_out, r, dr);
  }
}

// x(xi) and J[i][j] = dx_i / dxi_j of a macro of map ``kind`` with parameters P at macro
// coordinates xi: 0 affine (x = o + sum_j (xi_j + 1)/2 a_j), 1 cubed-sphere shell patch,
// 2 cube-to-sphere wedge
__host__ __device__ inline void macro_map(int kind, const double* P, const double xi[3], double zc, double x[3],
                                          double J[3][3]) {
  if (kind == 0) {
    for (int i = 0; i < 3; ++i) {
      x[i] = P[i];
      for (int j = 0; j < 3; ++j) {
        const double a = P[3 + 3 * j + i];
        x[i] += 0.5 * (xi[j] + 1.0) * a;
        J[i][j] = 0.5 * a;
      }
    }
    return;
  }
  // equiangular direction: X = tan(pi xi0 / 4), Y = tan(pi xi1 / 4), v = R (X, Y, 1)
  const double q = 0.25 * M_PI;
  const double X = tan(q * xi[0]), Y = tan(q * xi[1]);
  const double dXdxi = q * (1.0 + X * X), dYdxi = q * (1.0 + Y * Y);
  double v[3], Rc0[3], Rc1[3];
  for (int i = 0; i < 3; ++i) {
    Rc0[i] = P[3 * i + 0];
    Rc1[i] = P[3 * i + 1];
    v[i] = P[3 * i + 0] * X + P[3 * i + 1] * Y + P[3 * i + 2];
  }
  const double len = sqrt(X * X + Y * Y + 1.0);
  double u[3], duX[3], duY[3];
  for (int i = 0; i < 3; ++i) {
    u[i] = v[i] / len;
    // d(v/|v|)/dX = R e0 / |v| - v (v . R e0) / |v|^3, with v . R e0 = X (R orthogonal)
    duX[i] = Rc0[i] / len - v[i] * X / (len * len * len);
    duY[i] = Rc1[i] / len - v[i] * Y / (len * len * len);
  }
  if (kind == 1) {  // shell: x = r(xi2) u
    double r, dr;
    shell_radius(P, xi[2], zc, r, dr);
    for (int i = 0; i < 3; ++i) {
      x[i] = r * u[i];
      J[i][0] = r * dXdxi * duX[i];
      J[i][1] = r * dYdxi * duY[i];
      J[i][2] = dr * u[i];
    }
    return;
  }
  // cube-to-sphere wedge: (1 - s) a R (xi0, xi1, 1) + s r_s u, s = (xi2 + 1)/2
  const double a = P[10], rs = P[11], s = 0.5 * (xi[2] + 1.0);
  for (int i = 0; i < 3; ++i) {
    const double flat = a * (P[3 * i + 0] * xi[0] + P[3 * i + 1] * xi[1] + P[3 * i + 2]);
    const double sph = rs * u[i];
    x[i] = (1.0 - s) * flat + s * sph;
    J[i][0] = (1.0 - s) * a * Rc0[i] + s * rs * dXdxi * duX[i];
    J[i][1] = (1.0 - s) * a * Rc1[i] + s * rs * dYdxi * duY[i];
    J[i][2] = 0.5 * (sph - flat);
  }
}

// x and J of the octree cell (level, anchor a) of a macro at the cell's reference point xi: the
// cell covers macro coordinates -1 + (2 a + 1 + xi) / 2^level
__host__ __device__ inline void cell_map(int kind, const double* P, int level, const int a[3], const double xi[3],
                                         double x[3], double J[3][3]) {
  const double h = 1.0 / double(1 << level);
  double xm[3];
  for (int d = 0; d < 3; ++d) xm[d] = -1.0 + (2.0 * a[d] + 1.0 + xi[d]) * h;
  const double zc = -1.0 + (2.0 * a[2] + 1.0) * h;
  double Jm[3][3];
  macro_map(kind, P, xm, zc, x, Jm);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) J[i][j] = Jm[i][j] * h;
}

__host__ __device__ inline double det3x3(const double J[3][3]) {
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// the source g of the right-hand side kinds (HPDG_RHS_*) with parameters P[nP] at x:
// 0 sin sin sin (g = 3 pi^2 u), 2 the k-jump problem (-6), 3 a polynomial u (g = -lap u, P its
// K^3 coefficients C[a][b][c] of x^a y^b z^c), 4 a sum of Gaussians (rows amplitude, centre,
// width); the others have no source
__host__ __device__ inline double rhs_source(int kind, const double* P, int nP, const double x[3]) {
  const double X = x[0], Y = x[1], Z = x[2];
  switch (kind) {
    case 0: return 3.0 * M_PI * M_PI * sin(M_PI * X) * sin(M_PI * Y) * sin(M_PI * Z);
    case 2: return -6.0;
    case 3: {
      int K = 1;
      while ((K + 1) * (K + 1) * (K + 1) <= nP) ++K;
      double g = 0, px[16], py[16], pz[16];
      px[0] = py[0] = pz[0] = 1.0;
      for (int a = 1; a < K && a < 16; ++a) {
        px[a] = px[a - 1] * X;
        py[a] = py[a - 1] * Y;
        pz[a] = pz[a - 1] * Z;
      }
      for (int a = 0; a < K && a < 16; ++a)
        for (int b = 0; b < K && b < 16; ++b)
          for (int c = 0; c < K && c < 16; ++c) {
            const double C = P[(a * K + b) * K + c];
            if (a >= 2) g -= C * a * (a - 1) * px[a - 2] * py[b] * pz[c];
            if (b >= 2) g -= C * b * (b - 1) * px[a] * py[b - 2] * pz[c];
            if (c >= 2) g -= C * c * (c - 1) * px[a] * py[b] * pz[c - 2];
          }
      return g;
    }
    case 4: {
      double g = 0;
      for (int r = 0; r + 4 < nP; r += 5) {
        const double dx = X - P[r + 1], dy = Y - P[r + 2], dz = Z - P[r + 3], s = P[r + 4];
        g += P[r] * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * s * s));
      }
      return g;
    }
    default: return 0.0;
  }
}

}  // namespace hpdg
