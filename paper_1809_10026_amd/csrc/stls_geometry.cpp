// Mapped spatial domains of the stls library (host side).
//
// Paper: Montardini, Negri, Sangalli, Tani, arXiv:1809.10026.  The discrete
// space on Omega = G((0,1)^d) is the restricted tensor B-spline space
// composed with G^{-1} (§2.2).  The least-squares matrix keeps the time
// Kronecker structure of §4.1,
//   A = K_t (x) M_s + kappa^2 M_t (x) J_s + kappa W_t (x) L_s,
// with sparse spatial factors M_s = int B_i B_j, L_s = int grad B_i . grad B_j
// and J_s = int Lap B_i Lap B_j over Omega.  They are assembled on the
// device (stls_mapped.hip, metric terms in stls_geomap.h) by tensor Gauss
// quadrature in the parametric domain (p + 3 points per non-empty span: the
// integrands carry the geometry and are not polynomial) and stored as
// stencils: row i of the restricted tensor basis holds its
// prod_k (2 p_k + 1) entries at the column offsets o in [-p_k, p_k]^d,
// colexicographic in o (zero where the column leaves the box).  This file
// prepares the quadrature data of the space directions.
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
#include <vector>

#include "stls_geomap.h"
#include "stls_internal.h"

namespace stls {

namespace {

// Quadrature points of one direction: per non-empty span, q Gauss points
// with the values and first two derivatives of the span's p + 1 functions.
struct Quad1 {
  int p = 0, q = 0;
  std::vector<int> span;         // knot span index of each non-empty span
  std::vector<double> x, w;      // points and weights (span-major)
  std::vector<double> v;         // [point][3][p+1]
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
  // --- quadrature of the spatial factors; the stencils are assembled on the device
  Quad1 Q[kMaxDim];
  MappedQuad mq;
  mq.d = d;
  mq.geom = geometry;
  for (int k = 0; k < d; ++k) {
    build_quad(h->dir[k], h->dir[k].p + 3, Q[k]);
    mq.nel[k] = (int)Q[k].span.size();
    mq.q[k] = Q[k].q;
    mq.p[k] = Q[k].p;
    mq.n[k] = h->dir[k].n;
    mq.x[k] = Q[k].x;
    mq.w[k] = Q[k].w;
    mq.v[k] = Q[k].v;
    for (int s : Q[k].span) mq.first[k].push_back(s - Q[k].p - 1);
  }
  const int st = mapped_assemble(h, mq);
  if (st) return st;
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

// Last step of the mapped setup, after the workspaces: the P^G scaling.
int mapped_upload(stls_ctx* h) { return mapped_update_sigma(h); }

}  // namespace stls
