// Mapped spatial domains of the stls library (host side).
//
// Paper: Montardini, Negri, Sangalli, Tani, arXiv:1809.10026.  The discrete
// space on Omega = G((0,1)^d) is the restricted tensor B-spline space
// composed with G^{-1} (§2.2).  The least-squares matrix keeps the time
// Kronecker structure of §4.1,
//   A = K_t (x) M_s + kappa^2 M_t (x) J_s + kappa W_t (x) L_s,
// with sparse spatial factors M_s = int B_i B_j, L_s = int grad B_i . grad B_j
// and J_s = int Lap B_i Lap B_j over Omega.  They are assembled here by
// tensor Gauss quadrature in the parametric domain (p + 3 points per
// non-empty span: the integrands carry the geometry and are not
// polynomial) and stored as stencils: row i of the restricted tensor basis
// holds its prod_k (2 p_k + 1) entries at the column offsets o in
// [-p_k, p_k]^d, colexicographic in o (zero where the column leaves the
// box).  Physical derivatives of v = v^ o G^{-1}:
//   grad v . grad w = sum_ab g^ab d_a v^ d_b w^,   g^ab = grad eta_a . grad eta_b,
//   Lap v = sum_ab g^ab d_a d_b v^ + sum_j (Lap eta_j) d_j v^,
//   Lap eta_j = -sum_ab g^ab [J^{-1} d_a d_b G]_j.
//
// Preconditioner on the mapped domain (§4.4): either the parametric P of
// §4.2 (the unit-box factors; G ignored) or P^G = D^1/2 Pbar^G D^1/2 with
// Pbar^G = K^G_t (x) M^G_s + kappa^2 M^G_t (x) Jtilde^G_s built from the
// univariate matrices weighted by mu_k, omega_k: the separable
// approximation (Algorithm 2 of Appendix A.3, maxit = 2) of the coefficients
//   c_k = |grad eta_k|^4 |det J| T (k <= d),  c_{d+1} = |det J| / T
// interpolated at the element barycentres (eq. coefficients-c; |grad eta_k|
// is the norm of row k of J^{-1}, the factor of d^2/d eta_k^2 in the pulled
// back Laplacian), and D = diag(A) / diag(Pbar^G).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <thread>
#include <vector>

#include "stls_internal.h"

namespace stls {

namespace {

constexpr double kHalfPi = 1.57079632679489661923;

// Jacobian J[i][a] = d x_i / d eta_a and Hessian H[i][a][b] of the map.
void quarter_annulus(const double* e, double J[3][3], double H[3][3][3]) {
  const double A = kHalfPi, r = 1.0 + e[0], th = A * e[1];
  const double c = std::cos(th), s = std::sin(th);
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

// quarter annulus (x0, y0)(eta_1, eta_2) revolved by pi/2 about y = -1, z = 0:
// x = x0, y = -1 + rho cos(phi), z = rho sin(phi), rho = y0 + 1, phi = (pi/2) eta_3
void rotated_quarter_annulus(const double* e, double J[3][3], double H[3][3][3]) {
  double J0[3][3], H0[3][3][3];
  quarter_annulus(e, J0, H0);
  const double A = kHalfPi, r = 1.0 + e[0], y0 = r * std::sin(A * e[1]);
  const double rho = y0 + 1.0, ph = A * e[2], c = std::cos(ph), s = std::sin(ph);
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

struct Metric {
  double det;        // |det J|
  double g[3][3];    // g^ab
  double lap[3];     // Lap eta_j
};

void metric_at(int geom, int d, const double* e, Metric& m) {
  double J[3][3], H[3][3][3];
  if (geom == 1) quarter_annulus(e, J, H);
  else rotated_quarter_annulus(e, J, H);
  double Ji[3][3];  // Ji[a][i] = d eta_a / d x_i
  if (d == 2) {
    const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    m.det = std::fabs(det);
    Ji[0][0] = J[1][1] / det;
    Ji[0][1] = -J[0][1] / det;
    Ji[1][0] = -J[1][0] / det;
    Ji[1][1] = J[0][0] / det;
  } else {
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    m.det = std::fabs(det);
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

// Quadrature points of one direction: per non-empty span, q Gauss points
// with the values and first two derivatives of the span's p + 1 functions.
struct Quad1 {
  int p = 0, q = 0;
  std::vector<int> span;         // knot span index of each non-empty span
  std::vector<double> x, w;      // points and weights (span-major)
  std::vector<double> v;         // [point][3][p+1]
  std::vector<int> first_span;   // for each full function f: first non-empty span index (in span[]) with f in support
};

void build_quad(const Dir& D, int q, Quad1& Q) {
  const int p = D.p;
  Q.p = p;
  Q.q = q;
  std::vector<double> gx, gw;
  gauss_legendre(q, gx, gw);
  for (int s = p; s < D.m; ++s) {
    const double a = D.knots[s], b = D.knots[s + 1];
    if (!(b > a)) continue;
    Q.span.push_back(s);
    for (int g = 0; g < q; ++g) {
      const double u = 0.5 * (b - a) * gx[g] + 0.5 * (a + b);
      double t[3][16];
      span_basis(D.knots, p, s, u, t);
      Q.x.push_back(u);
      Q.w.push_back(0.5 * (b - a) * gw[g]);
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c <= p; ++c) Q.v.push_back(t[r][c]);
    }
  }
}

// Weighted banded matrix of one direction: int wgt b_i^(ord) b_j^(ord) with a
// weight constant on every non-empty span (p + 1 Gauss points: exact),
// restricted like the unweighted factors (space: drop the first and last
// function; time: drop the first).
std::vector<double> weighted_band(const Dir& D, const std::vector<double>& wgt, int ord) {
  const int p = D.p, m = D.m, n = D.n, bw = 2 * p + 1;
  std::vector<double> full((size_t)m * bw, 0.0);
  std::vector<double> gx, gw;
  gauss_legendre(p + 1, gx, gw);
  int e = 0;
  for (int s = p; s < m; ++s) {
    const double a = D.knots[s], b = D.knots[s + 1];
    if (!(b > a)) continue;
    for (int g = 0; g <= p; ++g) {
      const double u = 0.5 * (b - a) * gx[g] + 0.5 * (a + b);
      const double wq = 0.5 * (b - a) * gw[g] * wgt[e];
      double t[3][16];
      span_basis(D.knots, p, s, u, t);
      for (int r = 0; r <= p; ++r)
        for (int c = 0; c <= p; ++c) {
          const int i = s - p + r, j = s - p + c;
          full[(size_t)i * bw + (j - i + p)] += wq * t[ord][r] * t[ord][c];
        }
    }
    ++e;
  }
  std::vector<double> out((size_t)n * bw, 0.0);
  for (int ri = 0; ri < n; ++ri)
    for (int o = 0; o < bw; ++o) {
      const int rj = ri + o - p;
      if (rj < 0 || rj >= n) continue;
      out[(size_t)ri * bw + o] = full[(size_t)(ri + 1) * bw + o];
    }
  return out;
}

void band_to_dense(const std::vector<double>& band, int n, int p, std::vector<double>& dense) {
  const int bw = 2 * p + 1;
  dense.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int o = 0; o < bw; ++o) {
      const int j = i + o - p;
      if (j >= 0 && j < n) dense[(size_t)j * n + i] = band[(size_t)i * bw + o];
    }
}

// Separable approximation of positive tensors C[k] over the elements
// (D = d + 1 variables, colex, time slowest), Algorithm 2 of Appendix A.3:
//   C^(k) ~ mu^(1) .. omega^(k) .. mu^(D).
// A sweep sets each omega^(k)_j to the geometric midpoint of the values
// C^(k) implies for it on the slice i_k = j (others fixed), then each
// mu^(k)_j in turn to the geometric midpoint of the values that the other
// equations l != k imply for it on that slice.  (The appendix's listing
// writes the indices of its W^(k,l) the other way round; with the roles as
// here the two-variable case decouples into independent problems, as the
// appendix states.)
void separate(const std::vector<std::vector<double>>& C, const std::vector<int>& shape, int maxit,
              std::vector<std::vector<double>>& mu, std::vector<std::vector<double>>& om) {
  const int D = (int)shape.size();
  size_t total = 1;
  for (int n : shape) total *= (size_t)n;
  mu.assign(D, {});
  om.assign(D, {});
  for (int l = 0; l < D; ++l) {
    mu[l].assign(shape[l], 1.0);
    om[l].assign(shape[l], 1.0);
  }
  std::vector<int> idx(D);
  auto decode = [&](size_t e) {
    for (int l = 0; l < D; ++l) {
      idx[l] = (int)(e % shape[l]);
      e /= shape[l];
    }
  };
  for (int it = 0; it < maxit; ++it) {
    for (int k = 0; k < D; ++k) {
      std::vector<double> lo(shape[k], HUGE_VAL), hi(shape[k], -HUGE_VAL);
      for (size_t e = 0; e < total; ++e) {
        decode(e);
        double v = C[k][e];
        for (int l = 0; l < D; ++l)
          if (l != k) v /= mu[l][idx[l]];
        lo[idx[k]] = std::min(lo[idx[k]], v);
        hi[idx[k]] = std::max(hi[idx[k]], v);
      }
      for (int j = 0; j < shape[k]; ++j) om[k][j] = std::sqrt(lo[j] * hi[j]);
    }
    for (int k = 0; k < D; ++k) {
      std::vector<double> lo(shape[k], HUGE_VAL), hi(shape[k], -HUGE_VAL);
      for (size_t e = 0; e < total; ++e) {
        decode(e);
        for (int l = 0; l < D; ++l) {
          if (l == k) continue;
          // equation l: C^(l) = omega^(l) prod_{j != l} mu^(j), solved for mu^(k)
          double v = C[l][e] / om[l][idx[l]];
          for (int j = 0; j < D; ++j)
            if (j != k && j != l) v /= mu[j][idx[j]];
          lo[idx[k]] = std::min(lo[idx[k]], v);
          hi[idx[k]] = std::max(hi[idx[k]], v);
        }
      }
      for (int j = 0; j < shape[k]; ++j) mu[k][j] = std::sqrt(lo[j] * hi[j]);
    }
  }
}

}  // namespace

int mapped_host_setup(stls_ctx* h, int geometry, int prec) {
  const int d = h->d;
  if ((geometry == 1 && d != 2) || (geometry == 2 && d != 3)) {
    set_error("the quarter annulus is a 2-D domain, the rotated quarter annulus a 3-D one");
    return STLS_EINVAL;
  }
  h->geometry = geometry;
  h->geo_prec = prec;
  // --- quadrature of the spatial factors
  Quad1 Q[kMaxDim];
  size_t npts = 1;
  int ncol[kMaxDim], bwk[kMaxDim], n[kMaxDim];
  for (int k = 0; k < d; ++k) {
    build_quad(h->dir[k], h->dir[k].p + 3, Q[k]);
    ncol[k] = (int)Q[k].x.size();
    npts *= (size_t)ncol[k];
    bwk[k] = 2 * h->dir[k].p + 1;
    n[k] = h->dir[k].n;
  }
  if (npts > ((size_t)1 << 26)) {
    set_error("mapped domain too large for the host assembly of its spatial factors (quadrature points > 2^26)");
    return STLS_EINVAL;
  }
  // metric at every tensor point (colex, direction 1 fastest), weight folded in
  std::vector<Metric> met(npts);
  {
    const int nth = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (int t = 0; t < nth; ++t)
      pool.emplace_back([&, t]() {
        for (size_t e = t; e < npts; e += nth) {
          double eta[3];
          double w = 1.0;
          size_t rem = e;
          for (int k = 0; k < d; ++k) {
            const int i = (int)(rem % ncol[k]);
            rem /= ncol[k];
            eta[k] = Q[k].x[i];
            w *= Q[k].w[i];
          }
          metric_at(geometry, d, eta, met[e]);
          met[e].det *= w;  // quadrature weight x |det J|
        }
      });
    for (auto& th : pool) th.join();
  }
  int S = 1;
  for (int k = 0; k < d; ++k) S *= bwk[k];
  h->stencil = S;
  const int64_t ns = h->ns;
  std::vector<double> Ms((size_t)S * ns, 0.0), Js((size_t)S * ns, 0.0), Ls((size_t)S * ns, 0.0);
  // --- assembly by rows (test functions): every row is owned by one thread
  {
    const int nth = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (int t = 0; t < nth; ++t)
      pool.emplace_back([&, t]() {
        for (int64_t row = t; row < ns; row += nth) {
          int ir[3] = {0, 0, 0};
          {
            int64_t rem = row;
            for (int k = 0; k < d; ++k) {
              ir[k] = (int)(rem % n[k]);
              rem /= n[k];
            }
          }
          // support spans per direction: spans s with s - p <= f <= s, f = ir + 1
          std::vector<int> sp[3];
          for (int k = 0; k < d; ++k) {
            const int f = ir[k] + 1, p = Q[k].p;
            for (int e = 0; e < (int)Q[k].span.size(); ++e)
              if (Q[k].span[e] - p <= f && f <= Q[k].span[e]) sp[k].push_back(e);
          }
          // loop over the support's points
          int ce[3] = {0, 0, 0}, cg[3] = {0, 0, 0};
          const int ne0 = (int)sp[0].size(), ne1 = d > 1 ? (int)sp[1].size() : 1, ne2 = d > 2 ? (int)sp[2].size() : 1;
          for (ce[2] = 0; ce[2] < ne2; ++ce[2])
            for (ce[1] = 0; ce[1] < ne1; ++ce[1])
              for (ce[0] = 0; ce[0] < ne0; ++ce[0]) {
                int el[3] = {0, 0, 0};
                for (int k = 0; k < d; ++k) el[k] = sp[k][ce[k]];
                const int q0 = Q[0].q, q1 = d > 1 ? Q[1].q : 1, q2 = d > 2 ? Q[2].q : 1;
                for (cg[2] = 0; cg[2] < q2; ++cg[2])
                  for (cg[1] = 0; cg[1] < q1; ++cg[1])
                    for (cg[0] = 0; cg[0] < q0; ++cg[0]) {
                      // 1-D data of this point per direction: values of the
                      // span's functions and the position of the row's function
                      const double* v1[3];
                      int rpos[3];
                      size_t pidx = 0, stride = 1;
                      for (int k = 0; k < d; ++k) {
                        const int pi = el[k] * Q[k].q + cg[k];
                        v1[k] = &Q[k].v[(size_t)pi * 3 * (Q[k].p + 1)];
                        rpos[k] = ir[k] + 1 - (Q[k].span[el[k]] - Q[k].p);
                        pidx += (size_t)pi * stride;
                        stride *= (size_t)ncol[k];
                      }
                      const Metric& mt = met[pidx];
                      // test function: value, gradient, second derivatives
                      auto val = [&](const int* c, int da, int db, double* out_v) {
                        // derivative orders per direction from (da, db): -1 = none
                        double prod = 1.0;
                        for (int k = 0; k < d; ++k) {
                          const int ord = (k == da) + (k == db);
                          prod *= v1[k][ord * (Q[k].p + 1) + c[k]];
                        }
                        *out_v = prod;
                      };
                      double Bt, gt[3], Ht[3][3];
                      val(rpos, -1, -1, &Bt);
                      for (int a = 0; a < d; ++a) val(rpos, a, -1, &gt[a]);
                      double lapt = 0.0;
                      for (int a = 0; a < d; ++a)
                        for (int b = 0; b < d; ++b) {
                          val(rpos, a, b, &Ht[a][b]);
                          lapt += mt.g[a][b] * Ht[a][b];
                        }
                      for (int a = 0; a < d; ++a) lapt += mt.lap[a] * gt[a];
                      const double W = mt.det;
                      // trial functions of this point's span
                      int c[3] = {0, 0, 0};
                      const int pc0 = Q[0].p + 1, pc1 = d > 1 ? Q[1].p + 1 : 1, pc2 = d > 2 ? Q[2].p + 1 : 1;
                      for (c[2] = 0; c[2] < pc2; ++c[2])
                        for (c[1] = 0; c[1] < pc1; ++c[1])
                          for (c[0] = 0; c[0] < pc0; ++c[0]) {
                            int o = 0, ostride = 1;
                            bool ok = true;
                            for (int k = 0; k < d; ++k) {
                              const int jr = Q[k].span[el[k]] - Q[k].p + c[k] - 1;  // restricted column
                              if (jr < 0 || jr >= n[k]) { ok = false; break; }
                              o += (jr - ir[k] + Q[k].p) * ostride;
                              ostride *= bwk[k];
                            }
                            if (!ok) continue;
                            double Bc, gc[3];
                            val(c, -1, -1, &Bc);
                            for (int a = 0; a < d; ++a) val(c, a, -1, &gc[a]);
                            double lapc = 0.0, gg = 0.0;
                            for (int a = 0; a < d; ++a)
                              for (int b = 0; b < d; ++b) {
                                double hcb;
                                val(c, a, b, &hcb);
                                lapc += mt.g[a][b] * hcb;
                                gg += mt.g[a][b] * gt[a] * gc[b];
                              }
                            for (int a = 0; a < d; ++a) lapc += mt.lap[a] * gc[a];
                            const size_t at = (size_t)o * ns + (size_t)row;
                            Ms[at] += W * Bt * Bc;
                            Ls[at] += W * gg;
                            Js[at] += W * lapt * lapc;
                          }
                    }
              }
        }
      });
    for (auto& th : pool) th.join();
  }
  // centre entries: the diagonals of M_s, J_s, L_s
  int centre = 0;
  {
    int stride = 1;
    for (int k = 0; k < d; ++k) {
      centre += h->dir[k].p * stride;
      stride *= bwk[k];
    }
  }
  for (int f = 0; f < 3; ++f) h->sdiag[f].assign((size_t)ns, 0.0);
  for (int64_t i = 0; i < ns; ++i) {
    h->sdiag[0][(size_t)i] = Ms[(size_t)centre * ns + (size_t)i];
    h->sdiag[1][(size_t)i] = Js[(size_t)centre * ns + (size_t)i];
    h->sdiag[2][(size_t)i] = Ls[(size_t)centre * ns + (size_t)i];
  }
  h->hsten[0].swap(Ms);
  h->hsten[1].swap(Js);
  h->hsten[2].swap(Ls);
  // --- FD factors
  const Dir& Dt = h->dir[d];
  if (prec == 1) {
    // coefficients at the element barycentres, elements colex with time slowest
    std::vector<int> shape;
    std::vector<std::vector<double>> mids(d);
    for (int k = 0; k < d; ++k) {
      for (int s : Q[k].span) mids[k].push_back(0.5 * (h->dir[k].knots[s] + h->dir[k].knots[s + 1]));
      shape.push_back((int)mids[k].size());
    }
    int net = 0;
    for (int s = Dt.p; s < Dt.m; ++s)
      if (Dt.knots[s + 1] > Dt.knots[s]) ++net;
    shape.push_back(net);
    size_t nsp = 1;
    for (int k = 0; k < d; ++k) nsp *= (size_t)shape[k];
    std::vector<std::vector<double>> C(d + 1, std::vector<double>(nsp * (size_t)net));
    for (size_t e = 0; e < nsp; ++e) {
      double eta[3];
      size_t rem = e;
      for (int k = 0; k < d; ++k) {
        eta[k] = mids[k][rem % shape[k]];
        rem /= shape[k];
      }
      Metric m;
      metric_at(geometry, d, eta, m);
      for (int t = 0; t < net; ++t) {
        for (int k = 0; k < d; ++k) C[k][e + nsp * t] = m.g[k][k] * m.g[k][k] * m.det;  // T = 1
        C[d][e + nsp * t] = m.det;
      }
    }
    std::vector<std::vector<double>> mu, om;
    separate(C, shape, 2, mu, om);
    for (int k = 0; k <= d; ++k) {
      Dir& D = h->dir[k];
      const bool tm = k == d;
      std::vector<double> Mw = weighted_band(D, mu[k], 0);
      std::vector<double> Kw = weighted_band(D, om[k], tm ? 1 : 2);  // time: K^G_t, space: J^G_k
      std::vector<double> Kd, Md;
      band_to_dense(Kw, D.n, D.p, Kd);
      band_to_dense(Mw, D.n, D.p, Md);
      sym_generalized_eig(D.n, Kd, Md, D.U, D.lam);
      const int bw = 2 * D.p + 1;
      h->wdiag[k][0].assign(D.n, 0.0);
      h->wdiag[k][1].assign(D.n, 0.0);
      for (int i = 0; i < D.n; ++i) {
        // space: [M, J]; time: [K, M]
        h->wdiag[k][0][i] = tm ? Kw[(size_t)i * bw + D.p] : Mw[(size_t)i * bw + D.p];
        h->wdiag[k][1][i] = tm ? Mw[(size_t)i * bw + D.p] : Kw[(size_t)i * bw + D.p];
      }
    }
  }
  return STLS_OK;
}

// sigma_i = (Pbar^G_ii / A_ii)^(1/2) from the diagonals, uploaded (P^G only).
int mapped_update_sigma(stls_ctx* h) {
  if (h->geo_prec != 1) return STLS_OK;
  const int d = h->d;
  const Dir& Dt = h->dir[d];
  const int nt = Dt.n, bwt = 2 * Dt.p + 1;
  const double k2 = h->kappa * h->kappa;
  std::vector<double> pbar_s((size_t)h->ns * 2);  // prod m, sum_k j_k prod_{l!=k} m_l
  for (int64_t i = 0; i < h->ns; ++i) {
    int64_t rem = i;
    double pm = 1.0, sj = 0.0;
    for (int k = 0; k < d; ++k) {
      const int ik = (int)(rem % h->dir[k].n);
      rem /= h->dir[k].n;
      const double m = h->wdiag[k][0][ik], j = h->wdiag[k][1][ik];
      sj = sj * m + pm * j;
      pm *= m;
    }
    pbar_s[2 * (size_t)i] = pm;
    pbar_s[2 * (size_t)i + 1] = sj;
  }
  std::vector<double> sig((size_t)h->ndof);
  for (int t = 0; t < nt; ++t) {
    const double kt = h->wdiag[d][0][t], mt = h->wdiag[d][1][t];
    const double Kt = Dt.K[(size_t)t * bwt + Dt.p], Mt = Dt.M[(size_t)t * bwt + Dt.p];
    const double Wt = t == nt - 1 ? Dt.wend : 0.0;
    for (int64_t i = 0; i < h->ns; ++i) {
      const double P = kt * pbar_s[2 * (size_t)i] + k2 * mt * pbar_s[2 * (size_t)i + 1];
      const double A = Kt * h->sdiag[0][(size_t)i] + k2 * Mt * h->sdiag[1][(size_t)i] +
                       h->kappa * Wt * h->sdiag[2][(size_t)i];
      sig[(size_t)t * h->ns + (size_t)i] = std::sqrt(P / A);
    }
  }
  hipError_t e;
  if (!h->sigma) {
    e = hipMalloc((void**)&h->sigma, sizeof(double) * sig.size());
    if (e != hipSuccess) { set_error("hipMalloc (P^G scaling)"); return STLS_ENOMEM; }
  }
  e = hipMemcpyAsync(h->sigma, sig.data(), sizeof(double) * sig.size(), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return e == hipSuccess ? STLS_OK : hip_fail(e, "upload of the P^G scaling");
}

// Device copies of the stencils (the host copies are released).
int mapped_upload(stls_ctx* h) {
  for (int f = 0; f < 3; ++f) {
    const size_t bytes = sizeof(double) * h->hsten[f].size();
    hipError_t e = hipMalloc((void**)&h->sten[f], std::max<size_t>(bytes, 8));
    if (e != hipSuccess) { set_error("hipMalloc (mapped-domain stencils)"); return STLS_ENOMEM; }
    e = hipMemcpyAsync(h->sten[f], h->hsten[f].data(), bytes, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "upload of the mapped-domain stencils");
    std::vector<double>().swap(h->hsten[f]);
  }
  return mapped_update_sigma(h);
}

}  // namespace stls
