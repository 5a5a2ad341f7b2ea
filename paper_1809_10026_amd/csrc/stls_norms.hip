// Error norms of a discrete space-time solution on the GPU (§3.1 eq. norm_V0,
// §5.1): u_h = sum_i u_i B_i and its derivatives are evaluated on a tensor
// grid of Gauss points (p + 3 per non-empty knot span and direction) by
// evaluation mode products (eq. kron_vec_multi with rectangular
// basis-evaluation factors), and the weighted squared differences to a
// separable exact solution u = sum_s prod_k g_{s,k}(x_k) are summed.
//
// The space directions are evaluated first (one chain per spatial derivative
// pattern, kept as a (grid_s, n_t) tensor), then the time direction in chunks
// of quadrature points, each chunk evaluated inside the reduction that
// compares it with the exact solution; the device temporaries live in a
// per-handle workspace that grows when a call needs more.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "stls_internal.h"

namespace stls {

namespace {

constexpr int kNT = 256;
constexpr int kNormBlocks = 4096;
constexpr int kMaxTerms = 64;
constexpr long long kChunkPoints = 1LL << 26;  // grid points per time chunk (one reduction launch)

// Quadrature grid of one direction and the basis values at its points.
struct Grid1 {
  std::vector<double> x, w;
  std::vector<int> first;  // restricted index of the first of the p+1 functions nonzero at the point
  std::vector<double> E;   // [order][q][a]: d^order/dx^order of that function a (0 if not restricted)
  int nq = 0, np = 0;
};

void build_grid(const Dir& D, Grid1& G) {
  G = Grid1();
  G.np = D.p + 1;
  std::vector<double> gx, gw;
  gauss_legendre(D.p + 3, gx, gw);
  const std::vector<double>& xi = D.knots;
  for (int s = D.p; s < D.m; ++s) {
    const double a = xi[s], b = xi[s + 1];
    if (!(b > a)) continue;
    for (size_t g = 0; g < gx.size(); ++g) {
      G.x.push_back(0.5 * (b - a) * gx[g] + 0.5 * (a + b));
      G.w.push_back(0.5 * (b - a) * gw[g]);
      // full index of function a on span s is s - p + a; restricted index
      // (space drops full 0 and m-1, time drops full 0) is one less
      G.first.push_back(s - D.p - 1);
    }
  }
  G.nq = (int)G.x.size();
  G.E.assign((size_t)3 * G.nq * G.np, 0.0);
  for (int q = 0; q < G.nq; ++q) {
    double v[3][16];
    span_basis(xi, D.p, G.first[q] + D.p + 1, G.x[q], v);
    for (int o = 0; o < 3; ++o)
      for (int a = 0; a < G.np; ++a) {
        const int r = G.first[q] + a;
        G.E[((size_t)o * G.nq + q) * G.np + a] = (r >= 0 && r < D.n) ? v[o][a] : 0.0;
      }
  }
}

// One evaluation mode product over the (L, n_in, R) view:
//   out(l, q, r) (+)= sum_a E[q0 + q][a] in(l, first[q0 + q] + a, r),  0 <= q < nq_out.
__global__ __launch_bounds__(kNT) void eval_mode_kernel(const double* __restrict__ in, double* __restrict__ out,
                                                        long long L, int n_in, int nq_out, long long R,
                                                        const double* __restrict__ E, const int* __restrict__ first,
                                                        int np, int q0, int accumulate) {
  const long long total = L * nq_out * R;
  for (long long e = blockIdx.x * (long long)kNT + threadIdx.x; e < total; e += (long long)gridDim.x * kNT) {
    const long long l = e % L;
    const long long rest = e / L;
    const int q = (int)(rest % nq_out);
    const long long r = rest / nq_out;
    const int f = first[q0 + q];
    const double* row = E + (size_t)(q0 + q) * np;
    const double* src = in + l + r * L * n_in;
    double s = 0.0;
    for (int a = 0; a < np; ++a) {
      const int j = f + a;
      if (j >= 0 && j < n_in) s += row[a] * src[(size_t)j * L];
    }
    out[e] = accumulate ? out[e] + s : s;
  }
}

// Exact-solution factors and weights on the device:
//   g[gbase[k] + (s*3 + order)*nq[k] + q],  w[wbase[k] + q].
// A field is compared with sum over the npat derivative patterns pat[] of
// sum_s prod_k g_{s,k}^(pat[k]).
struct NormArgs {
  const double* g = nullptr;
  const double* w = nullptr;
  int d = 0, nterms = 0, npat = 0;
  int nq[kMaxDim + 1] = {0, 0, 0, 0};
  long long gbase[kMaxDim + 1] = {0, 0, 0, 0};
  int wbase[kMaxDim + 1] = {0, 0, 0, 0};
  int pat[kMaxDim][kMaxDim + 1] = {};
  int q0 = 0;  // first time point of the chunk
};

__device__ inline double block_sum_n(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kNT / 64; ++i) s += red[i];
  return s;
}

// partials[2b], partials[2b+1]: block b's sums of w (F - f)^2 and w f^2 over
// a chunk of time points, with F, the field on the grid, formed on the fly
// from the space-evaluated S (shape (grid_s, n_t), grid_s = Gs):
//   F(l, q) = sum_a Et[q0 + q][a] S(l, first_t[q0 + q] + a),
// so the chunk never goes through memory.  One thread per spatial point l
// and run of kTimeSub time points walks the run: the point's decomposition,
// spatial weight and the spatial factors of the exact solution
// (kSpatialCache products at most; beyond that they are formed per point)
// are computed once per run.
constexpr int kSpatialCache = 8;
constexpr int kTimeSub = 32;

__global__ __launch_bounds__(kNT) void err_reduce_kernel(const double* __restrict__ S, int Gs, int nt, int chunk,
                                                         const double* __restrict__ Et, const int* __restrict__ first_t,
                                                         int np, NormArgs A, double* __restrict__ partials) {
  __shared__ double red[kNT / 64];
  double se = 0.0, sr = 0.0;
  const int d = A.d, nfac = A.npat * A.nterms;
  const int nsub = (chunk + kTimeSub - 1) / kTimeSub;
  const long long items = (long long)Gs * nsub;
  for (long long it = blockIdx.x * (long long)kNT + threadIdx.x; it < items; it += (long long)gridDim.x * kNT) {
    const int l = (int)(it % Gs), qs = (int)(it / Gs) * kTimeSub;
    int idx[kMaxDim] = {0, 0, 0};
    int rest = l;
#pragma unroll
    for (int k = 0; k < kMaxDim; ++k) {
      if (k >= d) break;
      idx[k] = rest % A.nq[k];
      rest /= A.nq[k];
    }
    double ws = 1.0;
    for (int k = 0; k < d; ++k) ws *= A.w[A.wbase[k] + idx[k]];
    // spatial factor of (pattern pt, term s): prod_{k<d} g_{s,k}^(pat[pt][k])(x_k)
    auto spatial = [&](int pt, int s) {
      double prod = 1.0;
      for (int k = 0; k < d; ++k) prod *= A.g[A.gbase[k] + ((long long)s * 3 + A.pat[pt][k]) * A.nq[k] + idx[k]];
      return prod;
    };
    double sp[kSpatialCache];
#pragma unroll
    for (int c = 0; c < kSpatialCache; ++c) sp[c] = c < nfac ? spatial(c / A.nterms, c % A.nterms) : 0.0;
    for (int q = qs; q < min(chunk, qs + kTimeSub); ++q) {
      const int qt = A.q0 + q;
      double Fv = 0.0;
      const int f0 = first_t[qt];
      const double* row = Et + (size_t)qt * np;
      for (int a = 0; a < np; ++a) {
        const int j = f0 + a;
        if (j >= 0 && j < nt) Fv += row[a] * S[(size_t)l + (size_t)j * Gs];
      }
      double f = 0.0;
      for (int c = 0; c < nfac; ++c) {
        const int pt = c / A.nterms, s2 = c % A.nterms;
        double spc = 0.0;
#pragma unroll
        for (int cc = 0; cc < kSpatialCache; ++cc)
          if (cc == c) spc = sp[cc];
        if (c >= kSpatialCache) spc = spatial(pt, s2);
        f += spc * A.g[A.gbase[d] + ((long long)s2 * 3 + A.pat[pt][d]) * A.nq[d] + qt];
      }
      const double wq = ws * A.w[A.wbase[d] + qt];
      const double diff = Fv - f;
      se += wq * diff * diff;
      sr += wq * f * f;
    }
  }
  const double a = block_sum_n(se, red);
  const double b = block_sum_n(sr, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = a;
    partials[2 * blockIdx.x + 1] = b;
  }
}

int blocks_for(long long n) { return (int)std::max<long long>(1, std::min<long long>((n + kNT - 1) / kNT, kNormBlocks)); }

// Carves the call's device buffers out of the handle's norm workspace (kept
// between calls, grown when a call needs more): 256-byte aligned pieces.
struct Arena {
  size_t used = 0;
  char* base = nullptr;
  template <typename T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base ? base + used : nullptr);
    used += (std::max<size_t>(count, 1) * sizeof(T) + 255) / 256 * 256;
    return p;
  }
};

}  // namespace

}  // namespace stls

using namespace stls;

int stls_norm_points(stls_handle h, int dir, double* x, double* w, int* nq) {
  if (!h || dir < 0 || dir > h->d || !nq) { set_error("bad handle, direction or nq"); return STLS_EINVAL; }
  Grid1 G;
  build_grid(h->dir[dir], G);
  *nq = G.nq;
  if (x) std::copy(G.x.begin(), G.x.end(), x);
  if (w) std::copy(G.w.begin(), G.w.end(), w);
  return STLS_OK;
}

int stls_error_norms(stls_handle h, const double* u, int nterms, const double* const* g, double* out) {
  if (h && h->geometry) { set_error("stls_error_norms: unit box only (not available on a mapped domain)"); return STLS_EINVAL; }
  if (!h || !u || !g || !out || nterms < 1 || nterms > kMaxTerms) {
    set_error("bad handle, pointers or number of terms (1..64)");
    return STLS_EINVAL;
  }
  const int d = h->d;
  Grid1 G[kMaxDim + 1];
  for (int k = 0; k <= d; ++k) build_grid(h->dir[k], G[k]);
  for (int s = 0; s < nterms; ++s)
    for (int k = 0; k <= d; ++k)
      if (!g[s * (d + 1) + k]) { set_error("NULL exact-solution factor"); return STLS_EINVAL; }
  hipStream_t st = h->stream;
  int rc = STLS_OK;
  // evaluation tables, weights and exact factors (host side)
  NormArgs A;
  A.d = d;
  A.nterms = nterms;
  std::vector<double> wall, gall;
  for (int k = 0; k <= d; ++k) {
    A.nq[k] = G[k].nq;
    A.wbase[k] = (int)wall.size();
    wall.insert(wall.end(), G[k].w.begin(), G[k].w.end());
  }
  for (int k = 0; k <= d; ++k) {
    A.gbase[k] = (long long)gall.size();
    for (int s = 0; s < nterms; ++s) {
      const double* gs = g[s * (d + 1) + k];
      gall.insert(gall.end(), gs, gs + 3 * (size_t)G[k].nq);
    }
  }
  // tensor sizes
  const int nt = h->dir[d].n;
  long long Gs = 1;
  for (int k = 0; k < d; ++k) Gs *= G[k].nq;
  const long long chunk = std::max<long long>(1, std::min<long long>(G[d].nq, kChunkPoints / Gs));
  if (Gs >= (1LL << 31)) { set_error("error norms: too many spatial grid points"); return STLS_EINVAL; }
  // device buffers, carved from the handle's workspace: sized by a dry run
  double* dE[kMaxDim + 1];
  int* dF[kMaxDim + 1];
  double *dw, *dg, *S, *t0 = nullptr, *t1 = nullptr, *parts;
  auto carve = [&](Arena& ar) {
    for (int k = 0; k <= d; ++k) {
      dE[k] = ar.take<double>(G[k].E.size());
      dF[k] = ar.take<int>(G[k].first.size());
    }
    dw = ar.take<double>(wall.size());
    dg = ar.take<double>(gall.size());
    S = ar.take<double>((size_t)(Gs * nt));
    if (d > 1) t0 = ar.take<double>((size_t)(Gs * nt));
    if (d > 2) t1 = ar.take<double>((size_t)(Gs * nt));
    parts = ar.take<double>(2 * (size_t)kNormBlocks);
  };
  Arena dry;
  carve(dry);
  if (h->norm_ws_bytes < dry.used) {
    if (h->norm_ws) (void)hipFree(h->norm_ws);
    h->norm_ws = nullptr;
    h->norm_ws_bytes = 0;
    if (hipMalloc((void**)&h->norm_ws, dry.used) != hipSuccess) {
      h->norm_ws = nullptr;
      set_error("hipMalloc (error norms workspace)");
      return STLS_ENOMEM;
    }
    h->norm_ws_bytes = dry.used;
  }
  Arena ar;
  ar.base = h->norm_ws;
  carve(ar);
  auto put = [&](void* dst, const void* src, size_t bytes) {
    return bytes == 0 || hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) == hipSuccess;
  };
  bool ok = true;
  for (int k = 0; k <= d; ++k) {
    ok = ok && put(dE[k], G[k].E.data(), G[k].E.size() * sizeof(double));
    ok = ok && put(dF[k], G[k].first.data(), G[k].first.size() * sizeof(int));
  }
  ok = ok && put(dw, wall.data(), wall.size() * sizeof(double)) && put(dg, gall.data(), gall.size() * sizeof(double));
  if (!ok) {
    set_error("hipMemcpyAsync (error norms)");
    return STLS_EHIP;
  }
  A.w = dw;
  A.g = dg;
  std::vector<double> hp(2 * (size_t)kNormBlocks);

  // spatial chain: S (+)= u x_1 E_1^(ord[0]) ... x_d E_d^(ord[d-1])
  auto spatial = [&](const int* ord, bool accumulate) -> int {
    std::vector<long long> cur(d + 1);
    for (int k = 0; k < d; ++k) cur[k] = h->dir[k].n;
    cur[d] = nt;
    const double* in = u;
    for (int k = 0; k < d; ++k) {
      long long L = 1, R = 1;
      for (int m = 0; m < k; ++m) L *= cur[m];
      for (int m = k + 1; m <= d; ++m) R *= cur[m];
      const bool last = k == d - 1;
      double* o = last ? S : (k % 2 == 0 ? t0 : t1);
      const long long total = L * G[k].nq * R;
      hipLaunchKernelGGL(eval_mode_kernel, dim3(blocks_for(total)), dim3(kNT), 0, st, in, o, L, (int)cur[k],
                         G[k].nq, R, dE[k] + (size_t)ord[k] * G[k].nq * G[k].np, dF[k], G[k].np, 0,
                         (last && accumulate) ? 1 : 0);
      if (hipGetLastError() != hipSuccess) { set_error("eval_mode_kernel launch"); return STLS_EHIP; }
      cur[k] = G[k].nq;
      in = o;
    }
    return STLS_OK;
  };
  // time chunks of S x_t E_t^(tord), each compared with the patterns in A
  auto time_reduce = [&](int tord, double& err, double& ref) -> int {
    err = ref = 0.0;
    for (long long q0 = 0; q0 < G[d].nq; q0 += chunk) {
      const int c = (int)std::min<long long>(chunk, G[d].nq - q0);
      A.q0 = (int)q0;
      const int nb = blocks_for(Gs * ((c + kTimeSub - 1) / kTimeSub));
      hipLaunchKernelGGL(err_reduce_kernel, dim3(nb), dim3(kNT), 0, st, S, (int)Gs, nt, c,
                         dE[d] + (size_t)tord * G[d].nq * G[d].np, dF[d], G[d].np, A, parts);
      if (hipGetLastError() != hipSuccess) { set_error("error-norm kernel launch"); return STLS_EHIP; }
      if (hipMemcpyAsync(hp.data(), parts, 2 * (size_t)nb * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) {
        set_error("error-norm partial sums");
        return STLS_EHIP;
      }
      for (int b = 0; b < nb; ++b) {  // fixed order: deterministic
        err += hp[2 * (size_t)b];
        ref += hp[2 * (size_t)b + 1];
      }
    }
    return STLS_OK;
  };
  auto set_pat = [&](int npat, const int (*pats)[kMaxDim + 1]) {
    A.npat = npat;
    for (int pt = 0; pt < npat; ++pt)
      for (int k = 0; k <= d; ++k) A.pat[pt][k] = pats[pt][k];
  };
  int ord[kMaxDim] = {0, 0, 0};
  int pats[kMaxDim][kMaxDim + 1] = {};
  double Eu, Ru, Eut, Rut, Elap, Rlap, Eg = 0.0, Rg = 0.0;
  // u and d_t u (spatial values)
  if ((rc = spatial(ord, false))) return rc;
  pats[0][d] = 0;
  set_pat(1, pats);
  if ((rc = time_reduce(0, Eu, Ru))) return rc;
  pats[0][d] = 1;
  set_pat(1, pats);
  if ((rc = time_reduce(1, Eut, Rut))) return rc;
  // Laplacian: sum over k of the second derivative in direction k
  for (int k = 0; k < d; ++k) {
    int o2[kMaxDim] = {0, 0, 0};
    o2[k] = 2;
    if ((rc = spatial(o2, k > 0))) return rc;
    for (int m = 0; m <= d; ++m) pats[k][m] = (m == k) ? 2 : 0;
  }
  set_pat(d, pats);
  if ((rc = time_reduce(0, Elap, Rlap))) return rc;
  // spatial gradient
  for (int k = 0; k < d; ++k) {
    int o1[kMaxDim] = {0, 0, 0};
    o1[k] = 1;
    if ((rc = spatial(o1, false))) return rc;
    int p1[kMaxDim][kMaxDim + 1] = {};
    p1[0][k] = 1;
    set_pat(1, p1);
    double e, r;
    if ((rc = time_reduce(0, e, r))) return rc;
    Eg += e;
    Rg += r;
  }
  out[0] = std::sqrt((Eut + Elap) / (Rut + Rlap));
  out[1] = std::sqrt(Eu / Ru);
  out[2] = std::sqrt((Eu + Eut + Eg) / (Ru + Rut + Rg));
  return STLS_OK;
}
