// Geometry maps of the mapped spatial domains and the metric terms of the
// pulled-back operators (§2.2, the domains of §5), callable from host and
// device code.
//
//   quarter annulus: 1 < r < 2 in the first quadrant,
//     x = (1 + eta_1) cos(pi eta_2 / 2),  y = (1 + eta_1) sin(pi eta_2 / 2);
//   rotated quarter annulus: that domain (x0, y0) revolved by pi/2 about the
//     line y = -1, z = 0:  x = x0, y = -1 + rho cos(phi), z = rho sin(phi),
//     rho = y0 + 1, phi = (pi/2) eta_3.
//
// For v = v^ o G^{-1} the physical derivatives are
//   grad v . grad w = sum_ab g^ab d_a v^ d_b w^,   g^ab = grad eta_a . grad eta_b,
//   Lap v = sum_ab g^ab d_a d_b v^ + sum_j (Lap eta_j) d_j v^,
//   Lap eta_j = -sum_ab g^ab [J^{-1} d_a d_b G]_j.
#pragma once

#include <cmath>

#if defined(__HIP__)
#define STLS_HD __host__ __device__
#else
#define STLS_HD
#endif

namespace stls {

struct Metric {
  double det;      // |det J|
  double g[3][3];  // g^ab
  double lap[3];   // Lap eta_j
};

// Jacobian J[i][a] = d x_i / d eta_a and Hessian H[i][a][b] of the map.
STLS_HD inline void quarter_annulus(const double* e, double J[3][3], double H[3][3][3]) {
  const double A = 1.57079632679489661923, r = 1.0 + e[0], th = A * e[1];
  const double c = ::cos(th), s = ::sin(th);
  J[0][0] = c;
  J[0][1] = -A * r * s;
  J[1][0] = s;
  J[1][1] = A * r * c;
  for (int i = 0; i < 2; ++i)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) H[i][a][b] = 0.0;
  H[0][0][1] = H[0][1][0] = -A * s;
  H[0][1][1] = -A * A * r * c;
  H[1][0][1] = H[1][1][0] = A * c;
  H[1][1][1] = -A * A * r * s;
}

STLS_HD inline void rotated_quarter_annulus(const double* e, double J[3][3], double H[3][3][3]) {
  double J0[3][3], H0[3][3][3];
  quarter_annulus(e, J0, H0);
  const double A = 1.57079632679489661923, r = 1.0 + e[0], y0 = r * ::sin(A * e[1]);
  const double rho = y0 + 1.0, ph = A * e[2], c = ::cos(ph), s = ::sin(ph);
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < 3; ++a) {
      J[i][a] = 0.0;
      for (int b = 0; b < 3; ++b) H[i][a][b] = 0.0;
    }
  for (int a = 0; a < 2; ++a) {
    J[0][a] = J0[0][a];
    J[1][a] = J0[1][a] * c;
    J[2][a] = J0[1][a] * s;
    for (int b = 0; b < 2; ++b) {
      H[0][a][b] = H0[0][a][b];
      H[1][a][b] = H0[1][a][b] * c;
      H[2][a][b] = H0[1][a][b] * s;
    }
    H[1][a][2] = H[1][2][a] = -A * J0[1][a] * s;
    H[2][a][2] = H[2][2][a] = A * J0[1][a] * c;
  }
  J[1][2] = -A * rho * s;
  J[2][2] = A * rho * c;
  H[1][2][2] = -A * A * rho * c;
  H[2][2][2] = -A * A * rho * s;
}

// |det J|, g^ab and Lap eta_j at the parametric point e (geom 1: quarter
// annulus, d = 2; geom 2: rotated quarter annulus, d = 3).
STLS_HD inline void metric_at(int geom, int d, const double* e, Metric& m) {
  double J[3][3], H[3][3][3];
  if (geom == 1) quarter_annulus(e, J, H);
  else rotated_quarter_annulus(e, J, H);
  double Ji[3][3];  // Ji[a][i] = d eta_a / d x_i
  if (d == 2) {
    const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    m.det = ::fabs(det);
    Ji[0][0] = J[1][1] / det;
    Ji[0][1] = -J[0][1] / det;
    Ji[1][0] = -J[1][0] / det;
    Ji[1][1] = J[0][0] / det;
  } else {
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    m.det = ::fabs(det);
    Ji[0][0] = c00 / det;
    Ji[1][0] = c01 / det;
    Ji[2][0] = c02 / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  }
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double v = 0.0;
      for (int i = 0; i < d; ++i) v += Ji[a][i] * Ji[b][i];
      m.g[a][b] = v;
    }
  for (int j = 0; j < d; ++j) {
    double v = 0.0;
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        double t = 0.0;
        for (int i = 0; i < d; ++i) t += Ji[j][i] * H[i][a][b];
        v += m.g[a][b] * t;
      }
    m.lap[j] = -v;
  }
}

}  // namespace stls
