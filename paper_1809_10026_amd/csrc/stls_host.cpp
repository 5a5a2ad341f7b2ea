// Host side of the stls library: input validation, B-spline quadrature of the
// univariate banded matrices, generalized symmetric eigendecompositions, device
// upload and the non-compute C ABI entry points.
//
// Paper: Montardini, Negri, Sangalli, Tani, arXiv:1809.10026.  B-splines and
// knot vectors: §2.1; restricted spaces: §2.2 eq. basis_par; univariate
// matrices: §4.1 (eq. A_kron) and §4.2 (eq. preconditioner); generalized
// eigendecompositions: §4.3 eq. eig_dec (Algorithm 1, step 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "stls_internal.h"

namespace stls {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return STLS_EHIP;
}

// ---------------------------------------------------------------------------
// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_q, using
// the three-term Legendre recurrence (q <= 16 is all the library needs).
static void legendre_eval(int q, double z, double& pq, double& dpq) {
  double pk = z, pkm1 = 1.0;  // P_1, P_0
  for (int k = 2; k <= q; ++k) {
    const double pn = ((2.0 * k - 1.0) * z * pk - (k - 1.0) * pkm1) / k;
    pkm1 = pk;
    pk = pn;
  }
  pq = pk;
  dpq = q * (z * pk - pkm1) / (z * z - 1.0);  // P_q'(z) from P_q and P_{q-1}
}

void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < (q + 1) / 2; ++i) {
    double z = std::cos(pi * (i + 0.75) / (q + 0.5));  // descending initial guesses
    double pq = 0.0, dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      legendre_eval(q, z, pq, dp);
      const double dz = pq / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    legendre_eval(q, z, pq, dp);
    x[i] = -z;
    x[q - 1 - i] = z;
    w[i] = w[q - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  if (q % 2 == 1) x[q / 2] = 0.0;
}

// ---------------------------------------------------------------------------
// Nonzero B-splines of degree p on knot span s (xi[s] <= u <= xi[s+1], a
// non-empty span) and their first two derivatives.  The degree-q functions
// nonzero on the span are N_{s-q+a,q}, a = 0..q; each degree is formed from
// the previous one by the Cox-de Boor recursion of §2.1 (0/0 = 0), and the
// derivatives by differentiating that recursion.  v[k][a] = d^k/du^k
// N_{s-p+a,p}(u), k = 0..2.
static inline double ratio(double num, double den) { return den == 0.0 ? 0.0 : num / den; }

void span_basis(const std::vector<double>& xi, int p, int s, double u, double v[3][16]) {
  // tab[q][a] = N_{s-q+a, q}(u)
  double tab[16][16];
  tab[0][0] = 1.0;
  for (int q = 1; q <= p; ++q) {
    for (int a = 0; a <= q; ++a) {
      const int i = s - q + a;
      double val = 0.0;
      if (a >= 1) val += ratio(u - xi[i], xi[i + q] - xi[i]) * tab[q - 1][a - 1];
      if (a <= q - 1) val += ratio(xi[i + q + 1] - u, xi[i + q + 1] - xi[i + 1]) * tab[q - 1][a];
      tab[q][a] = val;
    }
  }
  // first derivatives of degree q from values of degree q-1
  auto deriv = [&](int q, const double* lower, double* outv) {
    for (int a = 0; a <= q; ++a) {
      const int i = s - q + a;
      double val = 0.0;
      if (a >= 1) val += q * ratio(lower[a - 1], xi[i + q] - xi[i]);
      if (a <= q - 1) val -= q * ratio(lower[a], xi[i + q + 1] - xi[i + 1]);
      outv[a] = val;
    }
  };
  for (int a = 0; a <= p; ++a) v[0][a] = tab[p][a];
  if (p >= 1) deriv(p, tab[p - 1], v[1]); else for (int a = 0; a <= p; ++a) v[1][a] = 0.0;
  if (p >= 2) {
    double d1[16];
    deriv(p - 1, tab[p - 2], d1);  // first derivatives of degree p-1
    deriv(p, d1, v[2]);
  } else {
    for (int a = 0; a <= p; ++a) v[2][a] = 0.0;
  }
}

// ---------------------------------------------------------------------------
int validate_and_build_dir(const double* knots, int nknots, int p, bool is_time, Dir& out,
                           std::string& err) {
  const char* what = is_time ? "time" : "space";
  if (!knots) { err = std::string(what) + " knot pointer is NULL"; return STLS_EINVAL; }
  if (p < (is_time ? 1 : 2) || p > 12) {
    err = std::string(what) + " degree out of range (space 2..12, time 1..12)";
    return STLS_EINVAL;
  }
  const int m = nknots - p - 1;
  const int n = is_time ? m - 1 : m - 2;
  if (m < p + 1 || n < 1) { err = std::string(what) + " knot vector too short"; return STLS_EINVAL; }
  if (n > kMaxDirN) { err = std::string(what) + " direction larger than supported (n <= 256)"; return STLS_EINVAL; }
  for (int i = 0; i < nknots; ++i) {
    if (!std::isfinite(knots[i])) { err = "non-finite knot"; return STLS_EINVAL; }
    if (i > 0 && knots[i] < knots[i - 1]) { err = "knots must be non-decreasing"; return STLS_EINVAL; }
  }
  for (int i = 0; i <= p; ++i) {
    if (knots[i] != 0.0 || knots[nknots - 1 - i] != 1.0) {
      err = std::string(what) + " knot vector must be open on [0,1] (p+1 zeros and ones)";
      return STLS_EINVAL;
    }
  }
  if (!(knots[p + 1] > 0.0) || !(knots[nknots - p - 2] < 1.0)) {
    err = std::string(what) + " end knots must have multiplicity exactly p+1";
    return STLS_EINVAL;
  }
  // interior multiplicity: space <= p-1 (C^1), time <= p (C^0) (Assumption 2)
  const int maxmult = is_time ? p : p - 1;
  int run = 1;
  for (int i = p + 2; i < nknots - p - 1; ++i) {
    run = (knots[i] == knots[i - 1]) ? run + 1 : 1;
    if (run > maxmult) {
      err = std::string(what) + (is_time ? " interior knot multiplicity > p (not C^0)"
                                         : " interior knot multiplicity > p-1 (not C^1)");
      return STLS_EINVAL;
    }
  }
  out = Dir();
  out.p = p;
  out.m = m;
  out.n = n;
  out.is_time = is_time;
  out.knots.assign(knots, knots + nknots);

  // --- assembly of the full banded matrices by Gauss quadrature (p+1 points,
  // exact for the piecewise polynomial integrands of degree <= 2p)
  const int bw = 2 * p + 1;
  std::vector<double> Mf((size_t)m * bw, 0.0), Kf((size_t)m * bw, 0.0), Jf((size_t)m * bw, 0.0);
  std::vector<double> D1f((size_t)m * bw, 0.0), G2f((size_t)m * bw, 0.0);  // int b'_i b_j, int b''_i b_j
  std::vector<double> D0f((size_t)m * bw, 0.0), H2f((size_t)m * bw, 0.0);  // int b_i b'_j, int b_i b''_j
  std::vector<double> gx, gw;
  gauss_legendre(p + 1, gx, gw);
  for (int s = p; s < m; ++s) {
    const double a = knots[s], b = knots[s + 1];
    if (!(b > a)) continue;
    for (int g = 0; g < p + 1; ++g) {
      const double u = 0.5 * (b - a) * gx[g] + 0.5 * (a + b);
      const double wq = 0.5 * (b - a) * gw[g];
      double v[3][16];
      span_basis(out.knots, p, s, u, v);
      for (int r = 0; r <= p; ++r) {
        const int i = s - p + r;
        for (int c = 0; c <= p; ++c) {
          const int j = s - p + c;
          const size_t e = (size_t)i * bw + (j - i + p);
          Mf[e] += wq * v[0][r] * v[0][c];
          Kf[e] += wq * v[1][r] * v[1][c];
          Jf[e] += wq * v[2][r] * v[2][c];
          D1f[e] += wq * v[1][r] * v[0][c];
          G2f[e] += wq * v[2][r] * v[0][c];
          D0f[e] += wq * v[0][r] * v[1][c];
          H2f[e] += wq * v[0][r] * v[2][c];
        }
      }
    }
  }
  // --- restriction: space drops functions 0 and m-1, time drops function 0
  const int off = 1;
  out.M.assign((size_t)n * bw, 0.0);
  out.K.assign((size_t)n * bw, 0.0);
  out.J.assign((size_t)n * bw, 0.0);
  for (int ri = 0; ri < n; ++ri) {
    for (int o = 0; o < bw; ++o) {
      const int rj = ri + o - p;
      if (rj < 0 || rj >= n) continue;
      const size_t src = (size_t)(ri + off) * bw + o;
      out.M[(size_t)ri * bw + o] = Mf[src];
      out.K[(size_t)ri * bw + o] = Kf[src];
      if (!is_time) out.J[(size_t)ri * bw + o] = Jf[src];
    }
  }
  // rectangular restricted x full bands: restricted row ri is full row ri + 1
  out.Mbar.assign((size_t)n * bw, 0.0);
  out.Cbar.assign((size_t)n * bw, 0.0);
  out.Gbar.assign((size_t)n * bw, 0.0);
  out.Kbar.assign((size_t)n * bw, 0.0);
  out.Jbar.assign((size_t)n * bw, 0.0);
  out.Hbar.assign((size_t)n * bw, 0.0);
  out.Dbar.assign((size_t)n * bw, 0.0);
  for (int ri = 0; ri < n; ++ri)
    for (int o = 0; o < bw; ++o) {
      const int j = ri + 1 + o - p;
      if (j < 0 || j >= m) continue;
      const size_t src = (size_t)(ri + 1) * bw + o;
      out.Mbar[(size_t)ri * bw + o] = Mf[src];
      out.Cbar[(size_t)ri * bw + o] = D1f[src];
      out.Gbar[(size_t)ri * bw + o] = G2f[src];
      out.Kbar[(size_t)ri * bw + o] = Kf[src];
      out.Jbar[(size_t)ri * bw + o] = Jf[src];
      out.Hbar[(size_t)ri * bw + o] = H2f[src];
      out.Dbar[(size_t)ri * bw + o] = D0f[src];
    }
  if (is_time) {
    out.J.clear();
    // W_t = b(1) b(1)^T: evaluate the last non-empty span at its right end
    int s = m - 1;
    while (s > p && !(knots[s + 1] > knots[s])) --s;
    double v[3][16];
    span_basis(out.knots, p, s, 1.0, v);
    // only the last function is nonzero at the closed right end of an open
    // knot vector; it is the last restricted function
    out.wend = v[0][p] * v[0][p];
  }
  // --- generalized eigendecomposition (Algorithm 1, step 1)
  std::vector<double> Kd((size_t)n * n, 0.0), Md((size_t)n * n, 0.0);
  const std::vector<double>& Kb = is_time ? out.K : out.J;
  for (int i = 0; i < n; ++i)
    for (int o = 0; o < bw; ++o) {
      const int j = i + o - p;
      if (j < 0 || j >= n) continue;
      Kd[(size_t)j * n + i] = Kb[(size_t)i * bw + o];
      Md[(size_t)j * n + i] = out.M[(size_t)i * bw + o];
    }
  sym_generalized_eig(n, Kd, Md, out.U, out.lam);
  return STLS_OK;
}

// ---------------------------------------------------------------------------
// Generalized symmetric-definite eigenproblem K U = M U diag(lam), U^T M U = I.
// Cholesky M = L L^T, C = L^{-1} K L^{-T}, cyclic Jacobi C = V diag(lam) V^T
// (rotations chosen by the classical two-sided formula, a rotation is applied
// when |c_pq| exceeds eps * sqrt(|c_pp c_qq|), which keeps small eigenvalues
// relatively accurate on graded matrices), U = L^{-T} V.  Column-major n x n.
void sym_generalized_eig(int n, const std::vector<double>& Kd, const std::vector<double>& Md,
                         std::vector<double>& U, std::vector<double>& lam) {
  auto at = [n](std::vector<double>& A, int i, int j) -> double& { return A[(size_t)j * n + i]; };
  std::vector<double> L(Md);
  // Cholesky (lower), column-major
  for (int j = 0; j < n; ++j) {
    double s = at(L, j, j);
    for (int k = 0; k < j; ++k) s -= at(L, j, k) * at(L, j, k);
    const double ljj = std::sqrt(s);
    at(L, j, j) = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = at(L, i, j);
      for (int k = 0; k < j; ++k) t -= at(L, i, k) * at(L, j, k);
      at(L, i, j) = t / ljj;
    }
    for (int i = 0; i < j; ++i) at(L, i, j) = 0.0;
  }
  // C = L^{-1} K L^{-T}: first Y = L^{-1} K (forward solves on columns)
  std::vector<double> Y(Kd);
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double t = at(Y, i, c);
      for (int k = 0; k < i; ++k) t -= at(L, i, k) * at(Y, k, c);
      at(Y, i, c) = t / at(L, i, i);
    }
  // C = Y L^{-T}  <=>  C^T = L^{-1} Y^T; C symmetric, solve on rows of Y
  std::vector<double> C((size_t)n * n);
  for (int r = 0; r < n; ++r)
    for (int i = 0; i < n; ++i) {
      double t = at(Y, r, i);
      for (int k = 0; k < i; ++k) t -= at(L, i, k) * at(C, r, k);
      at(C, r, i) = t / at(L, i, i);
    }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double s = 0.5 * (at(C, i, j) + at(C, j, i));
      at(C, i, j) = at(C, j, i) = s;
    }
  std::vector<double> V((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) at(V, i, i) = 1.0;
  const double eps = 2.220446049250313e-16;
  for (int sweep = 0; sweep < 60; ++sweep) {
    int rotations = 0;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = at(C, p, q);
        const double app = at(C, p, p), aqq = at(C, q, q);
        if (std::fabs(apq) <= eps * std::sqrt(std::fabs(app * aqq)) || apq == 0.0) continue;
        ++rotations;
        const double tau = (aqq - app) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double ckp = at(C, k, p), ckq = at(C, k, q);
          at(C, k, p) = c * ckp - s * ckq;
          at(C, k, q) = s * ckp + c * ckq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double cpk = at(C, p, k), cqk = at(C, q, k);
          at(C, p, k) = c * cpk - s * cqk;
          at(C, q, k) = s * cpk + c * cqk;
        }
        at(C, p, q) = at(C, q, p) = 0.0;
        for (int k = 0; k < n; ++k) {
          const double vkp = at(V, k, p), vkq = at(V, k, q);
          at(V, k, p) = c * vkp - s * vkq;
          at(V, k, q) = s * vkp + c * vkq;
        }
      }
    if (rotations == 0) break;
  }
  // sort ascending
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return at(C, a, a) < at(C, b, b); });
  lam.resize(n);
  std::vector<double> Vs((size_t)n * n);
  for (int jj = 0; jj < n; ++jj) {
    lam[jj] = at(C, order[jj], order[jj]);
    for (int i = 0; i < n; ++i) Vs[(size_t)jj * n + i] = at(V, i, order[jj]);
  }
  // U = L^{-T} V: back substitution with L^T on each column
  U.assign((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c)
    for (int i = n - 1; i >= 0; --i) {
      double t = Vs[(size_t)c * n + i];
      for (int k = i + 1; k < n; ++k) t -= at(L, k, i) * U[(size_t)c * n + k];
      U[(size_t)c * n + i] = t / at(L, i, i);
    }
}

// ---------------------------------------------------------------------------
// bf16 round-to-nearest-even of a float (bit manipulation, finite inputs).
static inline uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}
static inline float from_bf16(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

template <typename T>
static int dev_upload(T** dst, const T* src, size_t count, hipStream_t st) {
  hipError_t e = hipMalloc((void**)dst, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) {
    set_error(std::string("hipMalloc failed: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? STLS_ENOMEM : STLS_EHIP;
  }
  if (count) {
    e = hipMemcpyAsync(*dst, src, count * sizeof(T), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  }
  return STLS_OK;
}

// FD operands of direction k.  The mode product Y[i] = sum_j W(i,j) X[j] uses
// W = U^T (forward, step 2) or W = U (backward, step 4).  MFMA f64/f32 read
// W through [j*npad + i] (column-major W, padded with zeros); the bf16 path
// reads W row-major [i*kpad + k] split into hi and lo halves.
int upload_fd_operands(stls_ctx* h, int k) {
  const Dir& D = h->dir[k];
  DevDir& dd = h->dd[k];
  const int n = D.n, np = (n + 15) / 16 * 16, kp = (n + 31) / 32 * 32;
  dd.npad = np;
  dd.kpad = kp;
  std::vector<double> af((size_t)np * np, 0.0), ab((size_t)np * np, 0.0);
  auto U = [&](int i, int j) { return D.U[(size_t)j * n + i]; };
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      af[(size_t)j * np + i] = U(j, i);  // W = U^T: W(i,j) = U(j,i)
      ab[(size_t)j * np + i] = U(i, j);  // W = U
    }
  std::vector<float> af32(af.begin(), af.end()), ab32(ab.begin(), ab.end());
  std::vector<uint16_t> hf((size_t)np * kp, 0), lf((size_t)np * kp, 0), hb((size_t)np * kp, 0),
      lb((size_t)np * kp, 0);
  std::vector<float> rf32((size_t)np * kp, 0.f), rb32((size_t)np * kp, 0.f);
  std::vector<double> rf64((size_t)np * kp, 0.0), rb64((size_t)np * kp, 0.0);
  for (int i = 0; i < n; ++i)
    for (int kk = 0; kk < n; ++kk) {
      const float wf = (float)U(kk, i), wb = (float)U(i, kk);
      const uint16_t h1 = to_bf16(wf), h2 = to_bf16(wb);
      hf[(size_t)i * kp + kk] = h1;
      lf[(size_t)i * kp + kk] = to_bf16(wf - from_bf16(h1));
      hb[(size_t)i * kp + kk] = h2;
      lb[(size_t)i * kp + kk] = to_bf16(wb - from_bf16(h2));
      rf32[(size_t)i * kp + kk] = wf;
      rb32[(size_t)i * kp + kk] = wb;
      rf64[(size_t)i * kp + kk] = U(kk, i);
      rb64[(size_t)i * kp + kk] = U(i, kk);
    }
  int st;
  if ((st = dev_upload(&dd.Afwd64, af.data(), af.size(), h->stream))) return st;
  if ((st = dev_upload(&dd.Abwd64, ab.data(), ab.size(), h->stream))) return st;
  if ((st = dev_upload(&dd.Afwd32, af32.data(), af32.size(), h->stream))) return st;
  if ((st = dev_upload(&dd.Abwd32, ab32.data(), ab32.size(), h->stream))) return st;
  if ((st = dev_upload(&dd.Hfwd, hf.data(), hf.size(), h->stream))) return st;
  if ((st = dev_upload(&dd.Lfwd, lf.data(), lf.size(), h->stream))) return st;
  if ((st = dev_upload(&dd.Hbwd, hb.data(), hb.size(), h->stream))) return st;
  if ((st = dev_upload(&dd.Lbwd, lb.data(), lb.size(), h->stream))) return st;
  if ((st = dev_upload(&dd.Rfwd32, rf32.data(), rf32.size(), h->stream))) return st;
  if ((st = dev_upload(&dd.Rbwd32, rb32.data(), rb32.size(), h->stream))) return st;
  if ((st = dev_upload(&dd.Rfwd64, rf64.data(), rf64.size(), h->stream))) return st;
  if ((st = dev_upload(&dd.Rbwd64, rb64.data(), rb64.size(), h->stream))) return st;
  return STLS_OK;
}

static int upload_lambda_s(stls_ctx* h) {
  std::vector<double> raw((size_t)h->ns), scaled((size_t)h->ns);
  for (int64_t l = 0; l < h->ns; ++l) {
    int64_t rem = l;
    double s = 0.0;
    for (int k = 0; k < h->d; ++k) {
      const int ik = (int)(rem % h->dir[k].n);
      rem /= h->dir[k].n;
      s += h->dir[k].lam[ik];
    }
    raw[(size_t)l] = s;
    scaled[(size_t)l] = h->kappa * h->kappa * s;
  }
  hipError_t e;
  if (!h->lam_s_raw) {
    int st = dev_upload(&h->lam_s_raw, raw.data(), raw.size(), h->stream);
    if (st) return st;
    st = dev_upload(&h->lam_s, scaled.data(), scaled.size(), h->stream);
    return st;
  }
  e = hipMemcpyAsync(h->lam_s, scaled.data(), scaled.size() * sizeof(double), hipMemcpyHostToDevice,
                     h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return STLS_OK;
}

// Packed univariate diagonals for the diagonal scaling of the FD
// preconditioner (DiagScale layout): [m_k | k_k | j_k] per space direction,
// then [k_t | m_t]; the band's diagonal is its column p.
static int upload_diagonals(stls_ctx* h) {
  std::vector<double> g;
  for (int k = 0; k <= h->d; ++k) {
    const Dir& D = h->dir[k];
    const size_t bw = 2 * (size_t)D.p + 1;
    const std::vector<double>* bands[3] = {&D.M, &D.K, &D.J};
    if (D.is_time) { bands[0] = &D.K; bands[1] = &D.M; }
    for (int b = 0; b < (D.is_time ? 2 : 3); ++b)
      for (int i = 0; i < D.n; ++i) g.push_back((*bands[b])[(size_t)i * bw + (size_t)D.p]);
  }
  std::vector<float> g32(g.begin(), g.end());
  int st = dev_upload(&h->diag64, g.data(), g.size(), h->stream);
  if (!st) st = dev_upload(&h->diag32, g32.data(), g32.size(), h->stream);
  if (st) return st;
  const hipError_t e = hipStreamSynchronize(h->stream);  // the host vectors go out of scope
  return e == hipSuccess ? STLS_OK : hip_fail(e, "hipStreamSynchronize");
}

DiagScale diag_scale_args(const stls_ctx* h) {
  DiagScale S;
  S.g = h->diag64;
  S.g32 = h->diag32;
  S.d = h->d;
  int off = 0;
  for (int k = 0; k < h->d; ++k) {
    S.n[k] = h->dir[k].n;
    S.off[k] = off;
    off += 3 * S.n[k];
  }
  S.n[h->d] = h->dir[h->d].n;
  S.off[h->d] = off;
  S.k2 = h->kappa * h->kappa;
  S.kw = h->kappa * h->dir[h->d].wend;
  return S;
}

// Rectangular (restricted x full) bands of the differentiation and lifting
// operators: small (n x (2p+1) per band), uploaded once at setup so that the
// allocation-free entry points find them on the device.
int upload_diff_bands(stls_ctx* h) {
  if (h->bands_ready) return STLS_OK;
  int st = STLS_OK;
  h->nfull = 1;
  for (int k = 0; k <= h->d && !st; ++k) {
    Dir& D = h->dir[k];
    DevDir& dd = h->dd[k];
    dd.m = D.m;
    h->nfull *= D.m;
    st = dev_upload(&dd.Mbar, D.Mbar.data(), D.Mbar.size(), h->stream);
    if (!st) st = dev_upload(&dd.Cbar, D.Cbar.data(), D.Cbar.size(), h->stream);
    if (!st) st = dev_upload(&dd.Gbar, D.Gbar.data(), D.Gbar.size(), h->stream);
    if (!st) st = dev_upload(&dd.Kbar, D.Kbar.data(), D.Kbar.size(), h->stream);
    if (!st) st = dev_upload(&dd.Jbar, D.Jbar.data(), D.Jbar.size(), h->stream);
    if (!st) st = dev_upload(&dd.Hbar, D.Hbar.data(), D.Hbar.size(), h->stream);
    if (!st) st = dev_upload(&dd.Dbar, D.Dbar.data(), D.Dbar.size(), h->stream);
  }
  if (!st) h->bands_ready = true;
  return st;
}

// Full-space temporaries of the differentiation operators (first use).
int ensure_diff_operands(stls_ctx* h) {
  if (h->diff_ready) return STLS_OK;
  int st = upload_diff_bands(h);
  if (!st && h->nfull > 2147483647LL) { set_error("forcing space too large"); st = STLS_EINVAL; }
  for (int i = 0; i < 2 && !st; ++i) {
    hipError_t e = hipMalloc((void**)&h->ftmp[i], sizeof(double) * (size_t)h->nfull);
    if (e != hipSuccess) { set_error("hipMalloc forcing workspace"); st = STLS_ENOMEM; }
  }
  if (!st) h->diff_ready = true;
  return st;
}

static void free_ctx(stls_ctx* h) {
  if (!h) return;
  for (int k = 0; k <= kMaxDim; ++k) {
    DevDir& dd = h->dd[k];
    void* ptrs[] = {dd.M,      dd.K,      dd.J,      dd.Afwd64, dd.Abwd64, dd.Afwd32, dd.Abwd32,
                    dd.Hfwd,   dd.Lfwd,   dd.Hbwd,   dd.Lbwd,   dd.Rfwd32, dd.Rbwd32, dd.Rfwd64,
                    dd.Rbwd64, dd.lam,    dd.Mbar,   dd.Cbar,   dd.Gbar,   dd.Kbar,   dd.Jbar,
                    dd.Hbar,   dd.Dbar};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
  }
  void* ptrs[] = {h->diag64, h->diag32, h->lam_s, h->lam_s_raw, h->work[0], h->work[1], h->work[2], h->work[3], h->work[4],
                  h->work[5], h->fdbuf[0], h->fdbuf[1], h->r, h->z, h->pvec, h->q, h->partials, h->scal,
                  h->dres, h->ftmp[0], h->ftmp[1], h->lgrp[0], h->lgrp[1], h->lgrp[2], h->lgrp[3], h->lcls[0], h->lcls[1], h->lcls[2], h->lcls[3],
                  h->sten[0], h->sten[1], h->sten[2], h->sigma, h->mapped_lx, h->norm_ws};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (h->scal_host) (void)hipHostFree(h->scal_host);
  for (hipEvent_t e : h->check_ev)
    if (e) (void)hipEventDestroy(e);
  prof_flush(h);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  delete h;
}

static hipEvent_t prof_event(stls_ctx* h) {
  if (!h->ev_pool.empty()) {
    hipEvent_t e = h->ev_pool.back();
    h->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

void prof_begin(stls_ctx* h) {
  if (!h->prof) return;
  h->ev_open = prof_event(h);
  (void)hipEventRecord(h->ev_open, h->stream);
}

void prof_end(stls_ctx* h, int id) {
  if (!h->prof || !h->ev_open) return;
  hipEvent_t e1 = prof_event(h);
  (void)hipEventRecord(e1, h->stream);
  h->ev_pending.push_back({h->ev_open, e1, id});
  h->ev_open = nullptr;
}

void prof_flush(stls_ctx* h) {
  if (h->ev_pending.empty()) return;
  (void)hipEventSynchronize(h->ev_pending.back().b);
  for (auto& pe : h->ev_pending) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, pe.a, pe.b);
    h->prof_launch[pe.id] += 1;
    h->prof_ms[pe.id] += ms;
    h->ev_pool.push_back(pe.a);
    h->ev_pool.push_back(pe.b);
  }
  h->ev_pending.clear();
}

}  // namespace stls

using namespace stls;

extern "C" {

static int setup_common(int d, const int* nknots, const double* const* knots, const int* degree, double kappa,
                        void* stream, int geometry, int prec, stls_handle* out) {
  if (!out) { set_error("out is NULL"); return STLS_EINVAL; }
  *out = nullptr;
  if (d < 1 || d > kMaxDim) { set_error("d must be 1, 2 or 3"); return STLS_EINVAL; }
  if (!nknots || !knots || !degree) { set_error("NULL argument"); return STLS_EINVAL; }
  if (!(kappa > 0.0) || !std::isfinite(kappa)) { set_error("kappa must be finite and > 0"); return STLS_EINVAL; }
  stls_ctx* h = new stls_ctx();
  h->d = d;
  h->kappa = kappa;
  h->stream = (hipStream_t)stream;
  for (int k = 0; k <= d; ++k) {
    std::string err;
    int st = validate_and_build_dir(knots[k], nknots[k], degree[k], k == d, h->dir[k], err);
    if (st) {
      set_error(err);
      delete h;
      return st;
    }
  }
  h->ns = 1;
  for (int k = 0; k < d; ++k) h->ns *= h->dir[k].n;
  h->ndof = h->ns * h->dir[d].n;
  if (h->ndof > 2147483647LL) {
    set_error("ndof must stay below 2^31 (32-bit index arithmetic in the kernels)");
    delete h;
    return STLS_EINVAL;
  }
  int st = STLS_OK;
  // mapped domain: spatial stencils, and for P^G the weighted FD factors
  // (they replace dir[k].U and lam before the upload below)
  if (geometry != STLS_GEOM_UNIT_BOX) st = mapped_host_setup(h, geometry, prec);
  for (int k = 0; k <= d && !st; ++k) {
    Dir& D = h->dir[k];
    DevDir& dd = h->dd[k];
    dd.p = D.p;
    dd.n = D.n;
    st = dev_upload(&dd.M, D.M.data(), D.M.size(), h->stream);
    if (!st) st = dev_upload(&dd.K, D.K.data(), D.K.size(), h->stream);
    if (!st && !D.is_time) st = dev_upload(&dd.J, D.J.data(), D.J.size(), h->stream);
    if (!st) st = dev_upload(&dd.lam, D.lam.data(), D.lam.size(), h->stream);
    if (!st) st = upload_fd_operands(h, k);
  }
  if (!st) st = upload_lambda_s(h);
  if (!st) st = upload_diagonals(h);
  if (!st) st = upload_diff_bands(h);
  if (!st) st = resolve_noalloc_scratch(h);
  const size_t nb = (size_t)h->ndof * sizeof(double);
  auto alloc = [&](double** p, size_t bytes) {
    if (st) return;
    hipError_t e = hipMalloc((void**)p, bytes);
    if (e != hipSuccess) {
      set_error(std::string("hipMalloc workspace: ") + hipGetErrorString(e));
      st = e == hipErrorOutOfMemory ? STLS_ENOMEM : STLS_EHIP;
    }
  };
  const int nwork = d == 1 ? 1 : 3;  // matvec intermediates (d >= 2); the scaled FD's input copy
  for (int i = 0; i < nwork; ++i) alloc(&h->work[i], nb);
  alloc(&h->fdbuf[0], nb);
  alloc(&h->fdbuf[1], nb);
  alloc(&h->r, nb);
  alloc(&h->z, nb);
  alloc(&h->pvec, nb);
  alloc(&h->q, nb);
  alloc(&h->partials, 2 * kPartialsCap * sizeof(double));  // two sets: dot products and r.r
  alloc(&h->dres, 8 * sizeof(double));
  if (!st && hipMalloc((void**)&h->scal, sizeof(PcgScalars)) != hipSuccess) { set_error("hipMalloc"); st = STLS_ENOMEM; }
  for (int i = 0; i < 2 && !st; ++i)
    if (hipEventCreateWithFlags(&h->check_ev[i], hipEventDisableTiming) != hipSuccess) {
      set_error("hipEventCreate");
      st = STLS_EHIP;
    }
  if (!st && hipHostMalloc((void**)&h->scal_host, 2 * sizeof(PcgScalars), hipHostMallocDefault) != hipSuccess) {
    set_error("hipHostMalloc");
    st = STLS_ENOMEM;
  }
  if (!st && geometry != STLS_GEOM_UNIT_BOX) st = mapped_upload(h);
  if (st) {
    free_ctx(h);
    return st;
  }
  *out = h;
  return STLS_OK;
}

int stls_setup(int d, const int* nknots, const double* const* knots, const int* degree, double kappa,
               void* stream, stls_handle* out) {
  return setup_common(d, nknots, knots, degree, kappa, stream, STLS_GEOM_UNIT_BOX, STLS_PREC_PARAMETRIC, out);
}

int stls_setup_mapped(int d, const int* nknots, const double* const* knots, const int* degree, double kappa,
                      int geometry, int prec, void* stream, stls_handle* out) {
  if (geometry != STLS_GEOM_QUARTER_ANNULUS && geometry != STLS_GEOM_ROTATED_QUARTER_ANNULUS) {
    set_error("geometry must be STLS_GEOM_QUARTER_ANNULUS or STLS_GEOM_ROTATED_QUARTER_ANNULUS");
    if (out) *out = nullptr;
    return STLS_EINVAL;
  }
  if (prec != STLS_PREC_PARAMETRIC && prec != STLS_PREC_GEOMETRY) {
    set_error("prec must be STLS_PREC_PARAMETRIC or STLS_PREC_GEOMETRY");
    if (out) *out = nullptr;
    return STLS_EINVAL;
  }
  return setup_common(d, nknots, knots, degree, kappa, stream, geometry, prec, out);
}

int stls_destroy(stls_handle h) {
  if (!h) return STLS_OK;
  (void)hipStreamSynchronize(h->stream);
  free_ctx(h);
  return STLS_OK;
}

int stls_get_shape(stls_handle h, int* n, int64_t* ndof) {
  if (!h) { set_error("NULL handle"); return STLS_EINVAL; }
  if (n)
    for (int k = 0; k <= h->d; ++k) n[k] = h->dir[k].n;
  if (ndof) *ndof = h->ndof;
  return STLS_OK;
}

int stls_get_factor(stls_handle h, int dir, int what, double* out, int64_t* count) {
  if (!h || dir < 0 || dir > h->d) { set_error("bad handle or direction"); return STLS_EINVAL; }
  const Dir& D = h->dir[dir];
  const std::vector<double>* src = nullptr;
  std::vector<double> tmp;
  switch (what) {
    case 0: src = &D.M; break;
    case 1: src = &D.K; break;
    case 2:
      if (D.is_time) { set_error("J is a space factor"); return STLS_EINVAL; }
      src = &D.J;
      break;
    case 3: src = &D.U; break;
    case 4: src = &D.lam; break;
    case 5:
      if (!D.is_time) { set_error("W is a time factor"); return STLS_EINVAL; }
      tmp.assign(1, D.wend);
      src = &tmp;
      break;
    default: set_error("unknown factor id"); return STLS_EINVAL;
  }
  if (count) *count = (int64_t)src->size();
  if (out) std::memcpy(out, src->data(), src->size() * sizeof(double));
  return STLS_OK;
}

int stls_set_kappa(stls_handle h, double kappa) {
  if (!h || !(kappa > 0.0) || !std::isfinite(kappa)) { set_error("bad handle or kappa"); return STLS_EINVAL; }
  h->kappa = kappa;
  const int st = upload_lambda_s(h);
  return st ? st : mapped_update_sigma(h);  // P^G on a mapped domain: D depends on kappa
}

int stls_set_fd_precision(stls_handle h, int mode) {
  if (!h || mode < STLS_FD_FP64 || mode > STLS_FD_ASYM) { set_error("bad handle or precision mode"); return STLS_EINVAL; }
  h->fd_mode = mode;
  return STLS_OK;
}

int stls_set_fd_scaling(stls_handle h, int on) {
  if (!h) { set_error("NULL handle"); return STLS_EINVAL; }
  if (h->geometry && on) {
    set_error("mapped domains take their preconditioner (P or the scaled P^G) at stls_setup_mapped");
    return STLS_EINVAL;
  }
  h->fd_scale = on != 0;
  return STLS_OK;
}

int stls_pcg_history(stls_handle h, double* out, int max, int* count) {
  if (!h) { set_error("NULL handle"); return STLS_EINVAL; }
  const int c = (int)h->history.size();
  if (count) *count = c;
  if (out)
    for (int i = 0; i < c && i < max; ++i) out[i] = h->history[i];
  return STLS_OK;
}

static const char* kProfNames[PROF_COUNT] = {"fd_space", "fd_time", "mv_inner1",   "mv_inner2",   "mv_outer",
                                             "vec_xr",   "reduce",  "diff",        "fd_slab_fwd", "fd_slab_bwd",
                                             "vec_p",    "misc",    "mv_mapped"};

int stls_set_profiling(stls_handle h, int on) {
  if (!h) { set_error("NULL handle"); return STLS_EINVAL; }
  h->prof = on != 0;
  return STLS_OK;
}
int stls_profile_count(void) { return PROF_COUNT; }
int stls_profile_get(stls_handle h, int idx, const char** name, int64_t* launches, double* ms) {
  if (!h || idx < 0 || idx >= PROF_COUNT) { set_error("bad handle or index"); return STLS_EINVAL; }
  prof_flush(h);
  if (name) *name = kProfNames[idx];
  if (launches) *launches = h->prof_launch[idx];
  if (ms) *ms = h->prof_ms[idx];
  return STLS_OK;
}
int stls_profile_reset(stls_handle h) {
  if (!h) { set_error("NULL handle"); return STLS_EINVAL; }
  prof_flush(h);
  for (int i = 0; i < PROF_COUNT; ++i) { h->prof_launch[i] = 0; h->prof_ms[i] = 0.0; }
  return STLS_OK;
}

const char* stls_status_string(int status) {
  switch (status) {
    case STLS_OK: return "ok";
    case STLS_EINVAL: return "invalid argument";
    case STLS_ENOMEM: return "out of memory";
    case STLS_EHIP: return "HIP runtime error";
    case STLS_ENOCONV: return "PCG did not converge within maxit";
    case STLS_ENAN: return "non-finite value in PCG";
    case STLS_EBREAKDOWN: return "PCG breakdown";
    default: return "unknown status";
  }
}

const char* stls_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
