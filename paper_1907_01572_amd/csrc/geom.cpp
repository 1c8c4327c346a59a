// Analytic macro-element maps and their Jacobians (Sec. II.A.1, Eq. Phi_e; Sec. II.A.5,
// Eq. Jacobian; Sec. III.C, Eq. inverse_mapping and the cubed-sphere macro-mesh).
#include <cmath>

#include "host.hpp"

namespace hpdg {

namespace {

// radial coordinate r(z) and dr/dz of a shell patch (zc: cell centre, see below)
void shell_radius(const double* par, double z, double zc, double& r, double& dr) {
  const int kind = static_cast<int>(par[9]);
  const double r_in = par[10], r_out = par[11], zb = par[12], rb = par[13];
  // 1/r interpolates 1/r1 and 1/r2 linearly in z (the inverse map, free of cancellation)
  auto inverse = [&](double x1, double x2, double r1, double r2) {
    double s = ((x2 - z) / r1 + (z - x1) / r2) / (x2 - x1);
    r = 1.0 / s;
    dr = -r * r * (1.0 / r2 - 1.0 / r1) / (x2 - x1);
  };
  if (kind == 0) {
    r = r_in + 0.5 * (z + 1.0) * (r_out - r_in);
    dr = 0.5 * (r_out - r_in);
  } else if (kind == 1) {
    inverse(-1.0, 1.0, r_in, r_out);
  } else {
    // branch of the point itself; exactly at the break, the element's cell centre decides
    if (z < zb || (z == zb && zc <= zb)) {
      dr = (rb - r_in) / (zb + 1.0);
      r = r_in + (z + 1.0) * dr;
    } else {
      inverse(zb, 1.0, rb, r_out);
    }
  }
}

}  // namespace

void macro_eval(const Macro& M, const double xi[3], double zc, double x[3], double J[3][3]) {
  const double* P = M.par;
  if (M.kind == 0) {  // affine: x = o + sum_j (xi_j + 1)/2 a_j
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
  const double X = std::tan(q * xi[0]), Y = std::tan(q * xi[1]);
  const double dXdxi = q * (1.0 + X * X), dYdxi = q * (1.0 + Y * Y);
  double v[3], Rc0[3], Rc1[3];
  for (int i = 0; i < 3; ++i) {
    Rc0[i] = P[3 * i + 0];
    Rc1[i] = P[3 * i + 1];
    v[i] = P[3 * i + 0] * X + P[3 * i + 1] * Y + P[3 * i + 2];
  }
  const double len = std::sqrt(X * X + Y * Y + 1.0);
  double u[3], duX[3], duY[3];
  for (int i = 0; i < 3; ++i) {
    u[i] = v[i] / len;
    // d(v/|v|)/dX = R e0 / |v| - v (v . R e0) / |v|^3, with v . R e0 = X (R orthogonal)
    duX[i] = Rc0[i] / len - v[i] * X / (len * len * len);
    duY[i] = Rc1[i] / len - v[i] * Y / (len * len * len);
  }
  if (M.kind == 1) {  // shell: x = r(xi2) u
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

}  // namespace hpdg
