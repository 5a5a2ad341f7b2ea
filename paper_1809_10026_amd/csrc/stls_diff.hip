// Differentiation operators of the stls library (gfx950): load operator of a
// forcing in the full spline space and its transpose, space-time mass matrix,
// derivative of the load and of the system matrix with respect to kappa, and
// deterministic dot products.  They serve the adjoint gradient of the misfit
// L = (u - u*)^T M_Q (u - u*), u = A_kappa^{-1} B_kappa f:
//   B_kappa = C_t (x) Mbar_s - kappa Mbar_t (x) Dbar_s   (load F_i = int int f (d_t B_i - kappa Lap B_i), §3.2)
//   dL/df = B_kappa^T lambda,  lambda = A_kappa^{-1} (2 M_Q e)
//   dL/dkappa = lambda^T (-(Mbar_t (x) Dbar_s) f - (2 kappa M_t (x) J_s + W_t (x) L_s) u)
// Every operator is a sum of Kronecker products of banded univariate factors
// (square restricted factors, or restricted x full rectangular ones), applied
// mode by mode (eq. kron_vec_multi).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <mutex>
#include <vector>

#include "stls_internal.h"

// Workspace of the allocation-free entry point (stls_load_apply_noalloc): one
// copy of this array on every device the library runs on, held from module
// load until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol); it uses the
// device address that resolve_noalloc_scratch looks up per device.
constexpr size_t kNoAllocScratchDoubles = size_t(1) << 23;  // 64 MiB
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace stls {

namespace {

constexpr int kT = 256;
constexpr int kMaxBlocks = 8192;

// One banded mode product over the (L, n_in, R) view:
//   not transposed: out(l, i, r) (+)= coef sum_j B(i, j) in(l, j, r)
//   transposed:     out(l, i, r) (+)= coef sum_q B(q, i) in(l, q, r)
// B stored n_rows x (2p+1) with entry (q, j) at q*(2p+1) + (j - q - off + p);
// off = 0 for the square restricted factors, 1 for restricted x full ones.
__global__ __launch_bounds__(kT) void band_rect_kernel(const double* __restrict__ in, double* __restrict__ out, int L,
                                                       int n_in, int n_out, int R, const double* __restrict__ band,
                                                       int p, int off, int trans, double coef, int accumulate) {
  const int bw = 2 * p + 1;
  const long long total = (long long)L * n_out * R;
  for (long long e = (long long)blockIdx.x * kT + threadIdx.x; e < total; e += (long long)gridDim.x * kT) {
    const int l = (int)(e % L);
    const long long rest = e / L;
    const int i = (int)(rest % n_out);
    const int r = (int)(rest / n_out);
    const size_t base = (size_t)l + (size_t)r * L * n_in;
    double s = 0.0;
    if (!trans) {
      const int jlo = max(0, i + off - p), jhi = min(n_in - 1, i + off + p);
      for (int j = jlo; j <= jhi; ++j) s += band[(size_t)i * bw + (j - i - off + p)] * in[base + (size_t)j * L];
    } else {
      const int qlo = max(0, i - off - p), qhi = min(n_in - 1, i - off + p);
      for (int q = qlo; q <= qhi; ++q) s += band[(size_t)q * bw + (i - q - off + p)] * in[base + (size_t)q * L];
    }
    out[e] = accumulate ? out[e] + coef * s : coef * s;
  }
}

// One mode of the general lifting's class recurrence (see stls_lift_apply),
// over the (L, n_in, R) view of the four class arrays M, J, H, G:
//   FIRST (from u_B alone): M' = B0 u, J' = B1 u, H' = B2 u, G' = B3 u
//   MID:   M' = B0 M, J' = B0 J + B1 M + B3 H + B2 G, H' = B0 H + B2 M,
//          G' = B0 G + B3 M                 (B0..B3 = Mbar, Jbar, Hbar, Gbar)
//   TIME:  F += c0 B0 M + c1 B1 J + c2 B2 G + c3 B3 H
//                                           (B0..B3 = Kbar_t, Mbar_t, Dbar_t, Cbar_t)
// Rectangular bands (restricted rows x full columns, offset 1), staged in
// LDS; the four bands' taps are shared by every class that uses them.
constexpr int kCls = 4;
enum { kLiftFirst = 0, kLiftMid = 1, kLiftTime = 2 };
// output rows per thread: 4 where four class arrays are read (their taps
// shared by the run), 1 for the first mode (one input)
template <int MODE>
constexpr int lift_rows() { return MODE == kLiftFirst ? 1 : 4; }

struct LiftPass {
  const double* in[kCls];
  double* out[kCls];
  const double* band[kCls];
  double coef[kCls];
  int L, n_in, n_out, R, p;
};

template <int MODE>
__global__ __launch_bounds__(kT) void lift_class_kernel(LiftPass a) {
  constexpr int kLiftRows = lift_rows<MODE>();
  extern __shared__ double bs[];  // [4][n_out * bw]
  const int p = a.p, bw = 2 * p + 1, nb = a.n_out * bw;
  for (int q = threadIdx.x; q < kCls * nb; q += kT) bs[q] = a.band[q / nb][q % nb];
  __syncthreads();
  // one thread per (l, run of kLiftRows consecutive rows i, r): the runs'
  // overlapping taps are loaded once
  const unsigned L = (unsigned)a.L, n_out = (unsigned)a.n_out;
  const unsigned nrun = (n_out + kLiftRows - 1) / kLiftRows;
  const unsigned total = L * nrun * (unsigned)a.R;
  for (unsigned w = blockIdx.x * kT + threadIdx.x; w < total; w += gridDim.x * kT) {
    const unsigned l = w % L, rest = w / L;
    const int i0 = (int)(rest % nrun) * kLiftRows;
    const unsigned r = rest / nrun;
    const size_t base = (size_t)l + (size_t)r * L * (unsigned)a.n_in;
    const int jlo = max(0, i0 + 1 - p), jhi = min(a.n_in - 1, i0 + kLiftRows + p);
    double oM[kLiftRows], oJ[kLiftRows], oH[kLiftRows], oG[kLiftRows];
#pragma unroll
    for (int u = 0; u < kLiftRows; ++u) oM[u] = oJ[u] = oH[u] = oG[u] = 0.0;
    for (int j = jlo; j <= jhi; ++j) {
      const size_t g = base + (size_t)j * L;
      const double vM = a.in[0][g];
      double vJ = 0.0, vH = 0.0, vG = 0.0;
      if constexpr (MODE != kLiftFirst) {
        vJ = a.in[1][g];
        vH = a.in[2][g];
        vG = a.in[3][g];
      }
#pragma unroll
      for (int u = 0; u < kLiftRows; ++u) {
        const int i = i0 + u, o = j - i - 1 + p;  // tap of row i, B(i, j) at i*bw + o
        if (o < 0 || o > 2 * p || i >= a.n_out) continue;
        const double* b0 = bs + i * bw + o;
        const double c0 = b0[0], c1 = b0[nb], c2 = b0[2 * nb], c3 = b0[3 * nb];
        if constexpr (MODE == kLiftFirst) {
          oM[u] += c0 * vM;
          oJ[u] += c1 * vM;
          oH[u] += c2 * vM;
          oG[u] += c3 * vM;
        } else if constexpr (MODE == kLiftMid) {
          oM[u] += c0 * vM;
          oJ[u] += c0 * vJ + c1 * vM + c3 * vH + c2 * vG;
          oH[u] += c0 * vH + c2 * vM;
          oG[u] += c0 * vG + c3 * vM;
        } else {
          oM[u] += a.coef[0] * c0 * vM + a.coef[1] * c1 * vJ + a.coef[2] * c2 * vG + a.coef[3] * c3 * vH;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kLiftRows; ++u) {
      const int i = i0 + u;
      if (i >= a.n_out) break;
      const size_t e = (size_t)l + (size_t)L * ((size_t)i + (size_t)n_out * r);
      if constexpr (MODE == kLiftTime) {
        a.out[0][e] += oM[u];
      } else {
        a.out[0][e] = oM[u];
        a.out[1][e] = oJ[u];
        a.out[2][e] = oH[u];
        a.out[3][e] = oG[u];
      }
    }
  }
}

__global__ __launch_bounds__(kT) void sub_kernel(const double* __restrict__ a, const double* __restrict__ b,
                                                 double* __restrict__ c, long long n) {
  for (long long e = (long long)blockIdx.x * kT + threadIdx.x; e < n; e += (long long)gridDim.x * kT) c[e] = a[e] - b[e];
}

__device__ inline double block_sum_d(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;
}

__global__ __launch_bounds__(kT) void dot_partial_kernel(const double* __restrict__ a, const double* __restrict__ b,
                                                         long long n, double* __restrict__ partials) {
  __shared__ double red[4];
  double s = 0.0;
  for (long long e = (long long)blockIdx.x * kT + threadIdx.x; e < n; e += (long long)gridDim.x * kT) s += a[e] * b[e];
  s = block_sum_d(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// fixed-order final sum of the partials (deterministic)
__global__ __launch_bounds__(kT) void dot_final_kernel(const double* __restrict__ partials, int nparts,
                                                       double* __restrict__ out) {
  __shared__ double red[4];
  double v = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kT) v += partials[i];
  const double s = block_sum_d(v, red);
  if (threadIdx.x == 0) *out = s;
}

int grid_for(long long n) { return (int)std::max<long long>(1, std::min<long long>((n + kT - 1) / kT, kMaxBlocks)); }

// One factor of a Kronecker chain.
struct Fac {
  const double* band;
  int p, off, trans, n_in, n_out;
};

// dst (+)= coef * (F_{d} (x) ... (x) F_0) src on a tensor whose mode sizes are
// fac[k].n_in; intermediate results ping-pong between t0 and t1.
int apply_chain(stls_ctx* h, const double* src, double* dst, const std::vector<Fac>& fac, double coef, bool accumulate,
                double* t0, double* t1) {
  const int nm = (int)fac.size();
  std::vector<int> cur(nm);
  for (int k = 0; k < nm; ++k) cur[k] = fac[k].n_in;
  const double* in = src;
  for (int k = 0; k < nm; ++k) {
    long long L = 1, R = 1;
    for (int m = 0; m < k; ++m) L *= cur[m];
    for (int m = k + 1; m < nm; ++m) R *= cur[m];
    const bool last = k == nm - 1;
    double* out = last ? dst : (k % 2 == 0 ? t0 : t1);
    const long long total = L * fac[k].n_out * R;
    prof_begin(h);
    hipLaunchKernelGGL(band_rect_kernel, dim3(grid_for(total)), dim3(kT), 0, h->stream, in, out, (int)L, fac[k].n_in,
                       fac[k].n_out, (int)R, fac[k].band, fac[k].p, fac[k].off, fac[k].trans, last ? coef : 1.0,
                       (last && accumulate) ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "band_rect_kernel launch");
    prof_end(h, PROF_DIFF);
    cur[k] = fac[k].n_out;
    in = out;
  }
  return STLS_OK;
}

// One mode product on a tensor of mode sizes cur[0..nm-1]: out (+)= coef F in.
int apply_mode(stls_ctx* h, const double* in, double* out, const std::vector<int>& cur, int k, const Fac& f,
               double coef, bool accumulate) {
  long long L = 1, R = 1;
  for (int m = 0; m < k; ++m) L *= cur[m];
  for (int m = k + 1; m < (int)cur.size(); ++m) R *= cur[m];
  const long long total = L * f.n_out * R;
  prof_begin(h);
  hipLaunchKernelGGL(band_rect_kernel, dim3(grid_for(total)), dim3(kT), 0, h->stream, in, out, (int)L, f.n_in, f.n_out,
                     (int)R, f.band, f.p, f.off, f.trans, coef, accumulate ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "band_rect_kernel launch");
  prof_end(h, PROF_DIFF);
  return STLS_OK;
}

int device_dot(stls_ctx* h, const double* a, const double* b, long long n, double* host_out) {
  const int nb = std::min(grid_for(n), kPartialsCap);
  hipLaunchKernelGGL(dot_partial_kernel, dim3(nb), dim3(kT), 0, h->stream, a, b, n, h->partials);
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(kT), 0, h->stream, h->partials, nb, h->dres);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "dot kernel launch");
  e = hipMemcpyAsync(h->scal_host, h->dres, sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  *host_out = *reinterpret_cast<double*>(h->scal_host);
  return STLS_OK;
}

Fac sq(const DevDir& D, const double* band) { return Fac{band, D.p, 0, 0, D.n, D.n}; }
Fac rect(const DevDir& D, const double* band) { return Fac{band, D.p, 1, 0, D.m, D.n}; }
Fac rectT(const DevDir& D, const double* band) { return Fac{band, D.p, 1, 1, D.n, D.m}; }

// terms of B_kappa: (coef, factors per mode, time last)
std::vector<std::pair<double, std::vector<Fac>>> load_terms(stls_ctx* h, bool transpose) {
  const int d = h->d;
  auto R = [&](int k, const double* b) { return transpose ? rectT(h->dd[k], b) : rect(h->dd[k], b); };
  std::vector<std::pair<double, std::vector<Fac>>> terms;
  std::vector<Fac> f0;
  for (int k = 0; k < d; ++k) f0.push_back(R(k, h->dd[k].Mbar));
  f0.push_back(R(d, h->dd[d].Cbar));
  terms.push_back({1.0, f0});
  for (int k = 0; k < d; ++k) {
    std::vector<Fac> f;
    for (int m = 0; m < d; ++m) f.push_back(R(m, m == k ? h->dd[m].Gbar : h->dd[m].Mbar));
    f.push_back(R(d, h->dd[d].Mbar));
    terms.push_back({-h->kappa, f});
  }
  return terms;
}

// Terms of a(u0_h b_1, B_i) for initial data u0_h (restricted spatial
// coefficients) on the first time function b_1 (lifting, §2; least-squares
// form §3.2).  For a trial function that vanishes on the spatial boundary the
// spatial integrations by parts of the system matrix hold, and the time one
// leaves [b_1 b_j] from 0 to T, which is zero for the restricted b_j; so the
// coupling is the system matrix with each time factor replaced by its
// column of the first function: K_t -> int b_j' b_1', M_t -> int b_j b_1,
// W_t -> b_j(T) b_1(T) = 0.  J_s = sum_k J_k + 2 sum_{k<l} K_k K_l (other
// modes M), as in the matvec.  The time factor maps a mode of size 1 (the
// coefficient of b_1) to the first min(p_t, n_t) restricted time rows, the
// only ones whose support meets b_1's.
std::vector<std::pair<double, std::vector<Fac>>> lift_terms(stls_ctx* h) {
  const int d = h->d;
  const DevDir& T = h->dd[d];
  auto tcol = [&](const double* band) { return Fac{band, T.p, 1, 0, 1, std::min(T.p, T.n)}; };
  auto S = [&](int k, const double* band) { return sq(h->dd[k], band); };
  std::vector<std::pair<double, std::vector<Fac>>> terms;
  std::vector<Fac> f0;
  for (int k = 0; k < d; ++k) f0.push_back(S(k, h->dd[k].M));
  f0.push_back(tcol(T.Kbar));
  terms.push_back({-1.0, f0});
  const double k2 = h->kappa * h->kappa;
  for (int k = 0; k < d; ++k) {
    std::vector<Fac> f;
    for (int m = 0; m < d; ++m) f.push_back(S(m, m == k ? h->dd[m].J : h->dd[m].M));
    f.push_back(tcol(T.Mbar));
    terms.push_back({-k2, f});
  }
  for (int k = 0; k < d; ++k)
    for (int l = k + 1; l < d; ++l) {
      std::vector<Fac> f;
      for (int m = 0; m < d; ++m) f.push_back(S(m, (m == k || m == l) ? h->dd[m].K : h->dd[m].M));
      f.push_back(tcol(T.Mbar));
      terms.push_back({-2.0 * k2, f});
    }
  return terms;
}

// u[full index of r] += w[r] for every restricted multi-index r: space
// index i is full index i + 1 (the first function is dropped), time too.
struct EmbedShape {
  int nm;
  int n[kMaxDim + 1], m[kMaxDim + 1];
};
__global__ __launch_bounds__(kT) void embed_add_kernel(const double* __restrict__ w, double* __restrict__ u,
                                                       EmbedShape sh, long long total) {
  for (long long e = (long long)blockIdx.x * kT + threadIdx.x; e < total; e += (long long)gridDim.x * kT) {
    long long rest = e, f = 0, stride = 1;
    for (int k = 0; k < sh.nm; ++k) {
      const int i = (int)(rest % sh.n[k]);
      rest /= sh.n[k];
      f += (long long)(i + 1) * stride;
      stride *= sh.m[k];
    }
    u[f] += w[e];
  }
}

}  // namespace

namespace {
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;  // per device index; nullptr until looked up
}  // namespace

int resolve_noalloc_scratch(stls_ctx* h) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  h->noalloc_scratch = g_scratch_ptr[dev];
  return STLS_OK;
}

}  // namespace stls

using namespace stls;

extern "C" {

int stls_get_forcing_shape(stls_handle h, int* m, int64_t* nfull) {
  if (!h) { set_error("NULL handle"); return STLS_EINVAL; }
  int64_t t = 1;
  for (int k = 0; k <= h->d; ++k) {
    if (m) m[k] = h->dir[k].m;
    t *= h->dir[k].m;
  }
  if (nfull) *nfull = t;
  return STLS_OK;
}

int stls_load_apply(stls_handle h, const double* f, double* F) {
  if (h && h->geometry) { set_error("stls_load_apply: unit box only (not available on a mapped domain)"); return STLS_EINVAL; }
  if (!h || !f || !F) { set_error("bad handle or pointers"); return STLS_EINVAL; }
  int st = ensure_diff_operands(h);
  if (st) return st;
  bool first = true;
  for (auto& t : load_terms(h, false)) {
    if ((st = apply_chain(h, f, F, t.second, t.first, !first, h->ftmp[0], h->ftmp[1]))) return st;
    first = false;
  }
  return STLS_OK;
}

// F = B_kappa f with the chain temporaries in the device's static workspace:
// the same terms, kernels and launch order as stls_load_apply, without any
// allocation (host or device).  Each mode product overwrites its whole
// output, so nothing in the workspace has to start at zero.
int stls_load_apply_noalloc(stls_handle h, const double* f, double* F) {
  if (h && h->geometry) { set_error("stls_load_apply_noalloc: unit box only (not available on a mapped domain)"); return STLS_EINVAL; }
  if (!h || !f || !F) { set_error("bad handle or pointers"); return STLS_EINVAL; }
  if (!h->bands_ready || !h->noalloc_scratch) {
    set_error("handle has no device bands or workspace address (stls_setup did not complete)");
    return STLS_EINVAL;
  }
  const int d = h->d, nm = d + 1;
  // terms of B_kappa: C_t (x) Mbar_s, then -kappa Mbar_t (x) (Gbar_k, Mbar elsewhere)
  Fac fac[kMaxDim + 1][kMaxDim + 1];
  double coef[kMaxDim + 1];
  const int nterm = d + 1;
  for (int t = 0; t < nterm; ++t) {
    for (int k = 0; k < d; ++k) fac[t][k] = rect(h->dd[k], (t == k + 1) ? h->dd[k].Gbar : h->dd[k].Mbar);
    fac[t][d] = rect(h->dd[d], t == 0 ? h->dd[d].Cbar : h->dd[d].Mbar);
    coef[t] = t == 0 ? 1.0 : -h->kappa;
  }
  // sizes of the intermediates: mode k's result goes to t0 (k even) or t1 (k odd)
  long long need[2] = {0, 0};
  long long cur[kMaxDim + 1];
  for (int k = 0; k < nm; ++k) cur[k] = fac[0][k].n_in;
  for (int k = 0; k + 1 < nm; ++k) {
    cur[k] = fac[0][k].n_out;
    long long sz = 1;
    for (int m = 0; m < nm; ++m) sz *= cur[m];
    need[k % 2] = std::max(need[k % 2], sz);
  }
  const long long off1 = (need[0] + 31) / 32 * 32;  // 256-byte aligned second region
  if (off1 + need[1] > (long long)kNoAllocScratchDoubles) {
    set_error("stls_load_apply_noalloc: the chain temporaries need " + std::to_string(off1 + need[1]) +
              " doubles, more than the static workspace of " + std::to_string(kNoAllocScratchDoubles) +
              " doubles (64 MiB); use stls_load_apply");
    return STLS_EINVAL;
  }
  double* t0 = h->noalloc_scratch;
  double* t1 = h->noalloc_scratch + off1;
  for (int t = 0; t < nterm; ++t) {
    for (int k = 0; k < nm; ++k) cur[k] = fac[t][k].n_in;
    const double* in = f;
    for (int k = 0; k < nm; ++k) {
      long long L = 1, R = 1;
      for (int m = 0; m < k; ++m) L *= cur[m];
      for (int m = k + 1; m < nm; ++m) R *= cur[m];
      const bool last = k == nm - 1;
      double* out = last ? F : (k % 2 == 0 ? t0 : t1);
      const long long total = L * fac[t][k].n_out * R;
      hipLaunchKernelGGL(band_rect_kernel, dim3(grid_for(total)), dim3(kT), 0, h->stream, in, out, (int)L,
                         fac[t][k].n_in, fac[t][k].n_out, (int)R, fac[t][k].band, fac[t][k].p, fac[t][k].off,
                         fac[t][k].trans, last ? coef[t] : 1.0, (last && t > 0) ? 1 : 0);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "band_rect_kernel launch");
      cur[k] = fac[t][k].n_out;
      in = out;
    }
  }
  return STLS_OK;
}

int stls_lift_initial(stls_handle h, const double* u0, double* F) {
  if (h && h->geometry) { set_error("stls_lift_initial: unit box only (not available on a mapped domain)"); return STLS_EINVAL; }
  if (!h || !u0 || !F) { set_error("bad handle or pointers"); return STLS_EINVAL; }
  int st = ensure_diff_operands(h);
  if (st) return st;
  for (auto& t : lift_terms(h))
    if ((st = apply_chain(h, u0, F, t.second, t.first, true, h->ftmp[0], h->ftmp[1]))) return st;
  return STLS_OK;
}

int stls_lift_combine(stls_handle h, const double* u0, const double* x, double* u) {
  if (h && h->geometry) { set_error("stls_lift_combine: unit box only (not available on a mapped domain)"); return STLS_EINVAL; }
  if (!h || !u0 || !x || !u) { set_error("bad handle or pointers"); return STLS_EINVAL; }
  hipError_t e = hipMemcpyAsync(u, u0, sizeof(double) * (size_t)h->ns, hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(u + h->ns, x, sizeof(double) * (size_t)h->ndof, hipMemcpyDeviceToDevice, h->stream);
  return e == hipSuccess ? STLS_OK : hip_fail(e, "hipMemcpyAsync");
}

// General lifting, F -= a(u_B, B_i), for a lifting u_B anywhere in the full
// space (boundary and/or initial coefficients): least-squares form of §3.2
// assembled term by term, since for such a trial function the integrations
// by parts that give the system matrix leave boundary terms.  Factors are
// restricted (test) rows x full (trial) columns:
//   int int d_t u d_t v          : Kbar_t (x) Mbar_s
//   kappa^2 int int Lap u Lap v  : Mbar_t (x) (Jbar_k, or Hbar_k Gbar_l for k != l)
//   -kappa int int d_t u Lap v   : Dbar_t (x) Gbar_k
//   -kappa int int Lap u d_t v   : Cbar_t (x) Hbar_k
// (other modes Mbar; G: test function differentiated twice, H: trial;
// 16 terms at d = 3), evaluated one mode at a time.  After the
// space modes 0 .. m every partial product lies in one of four classes by
// which special factors it has taken: none (M), the whole second-derivative
// part, J_k or H_k with G_l (J), H only (H), G only (G).  A space mode maps
// the classes as
//   M' = Mbar M,  J' = Mbar J + Jbar M + Gbar H + Hbar G,
//   H' = Mbar H + Hbar M,  G' = Mbar G + Gbar M,
// starting from u_B in class M alone, and the time mode closes them:
//   F -= Kbar_t M + kappa^2 Mbar_t J - kappa Dbar_t G - kappa Cbar_t H.
// (At d = 3: 4 passes of lift_class_kernel in place of 16 chains of 4
// products.)
int stls_lift_apply(stls_handle h, const double* ub, double* F) {
  if (h && h->geometry) { set_error("stls_lift_apply: unit box only (not available on a mapped domain)"); return STLS_EINVAL; }
  if (!h || !ub || !F) { set_error("bad handle or pointers"); return STLS_EINVAL; }
  int st = ensure_diff_operands(h);
  if (st) return st;
  const int d = h->d;
  for (int g = 0; g < 4 && !st; ++g)
    if ((!h->lgrp[g] && hipMalloc((void**)&h->lgrp[g], sizeof(double) * (size_t)h->nfull) != hipSuccess) ||
        (!h->lcls[g] && hipMalloc((void**)&h->lcls[g], sizeof(double) * (size_t)h->nfull) != hipSuccess)) {
      set_error("hipMalloc lifting workspace");
      st = STLS_ENOMEM;
    }
  if (st) return st;
  std::vector<long long> cur(d + 1);
  for (int k = 0; k <= d; ++k) cur[k] = h->dd[k].m;
  long long full = 1;
  for (int k = 0; k <= d; ++k) full *= cur[k];
  if (full >= 0xffffffffLL - (long long)kMaxBlocks * kT) { set_error("lifting: too many entries"); return STLS_EINVAL; }
  double* const* sets[2] = {h->lgrp, h->lcls};
  const double* cls[kCls] = {ub, nullptr, nullptr, nullptr};
  for (int m = 0; m <= d; ++m) {
    const DevDir& D = h->dd[m];
    LiftPass a = {};
    long long L = 1, R = 1;
    for (int q = 0; q < m; ++q) L *= cur[q];
    for (int q = m + 1; q <= d; ++q) R *= cur[q];
    a.L = (int)L;
    a.R = (int)R;
    a.n_in = D.m;
    a.n_out = D.n;
    a.p = D.p;
    for (int k = 0; k < kCls; ++k) a.in[k] = cls[k];
    const int mode = m == d ? kLiftTime : m == 0 ? kLiftFirst : kLiftMid;
    if (mode == kLiftTime) {
      const double k2 = h->kappa * h->kappa, kap = h->kappa;
      const double* bands[kCls] = {D.Kbar, D.Mbar, D.Dbar, D.Cbar};
      const double coef[kCls] = {-1.0, -k2, kap, kap};
      for (int k = 0; k < kCls; ++k) {
        a.band[k] = bands[k];
        a.coef[k] = coef[k];
      }
      a.out[0] = F;
    } else {
      const double* bands[kCls] = {D.Mbar, D.Jbar, D.Hbar, D.Gbar};
      for (int k = 0; k < kCls; ++k) {
        a.band[k] = bands[k];
        a.out[k] = sets[m % 2][k];
      }
    }
    const size_t shmem = sizeof(double) * kCls * D.n * (2 * D.p + 1);
    if (shmem > 160 * 1024) { set_error("lifting: bands too large for the pass's LDS"); return STLS_EINVAL; }
    const int rows = mode == kLiftFirst ? lift_rows<kLiftFirst>() : lift_rows<kLiftMid>();
    const long long total = L * ((a.n_out + rows - 1) / rows) * R;
    auto kern = mode == kLiftFirst ? lift_class_kernel<kLiftFirst>
                : mode == kLiftMid ? lift_class_kernel<kLiftMid> : lift_class_kernel<kLiftTime>;
    if (shmem > 65536) {
      const hipError_t ea = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
      if (ea != hipSuccess) return hip_fail(ea, "hipFuncSetAttribute(LDS)");
    }
    prof_begin(h);
    hipLaunchKernelGGL(kern, dim3(grid_for(total)), dim3(kT), shmem, h->stream, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "lift_class_kernel launch");
    prof_end(h, PROF_DIFF);
    cur[m] = D.n;
    for (int g = 0; g < kCls; ++g) cls[g] = sets[m % 2][g];
  }
  return STLS_OK;
}

int stls_lift_embed(stls_handle h, const double* ub, const double* w, double* u) {
  if (h && h->geometry) { set_error("stls_lift_embed: unit box only (not available on a mapped domain)"); return STLS_EINVAL; }
  if (!h || !ub || !w || !u) { set_error("bad handle or pointers"); return STLS_EINVAL; }
  int st = ensure_diff_operands(h);
  if (st) return st;
  EmbedShape sh{};
  sh.nm = h->d + 1;
  for (int k = 0; k <= h->d; ++k) {
    sh.n[k] = h->dd[k].n;
    sh.m[k] = h->dd[k].m;
  }
  hipError_t e = hipMemcpyAsync(u, ub, sizeof(double) * (size_t)h->nfull, hipMemcpyDeviceToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  hipLaunchKernelGGL(embed_add_kernel, dim3(grid_for(h->ndof)), dim3(kT), 0, h->stream, w, u, sh,
                     (long long)h->ndof);
  e = hipGetLastError();
  return e == hipSuccess ? STLS_OK : hip_fail(e, "embed_add_kernel launch");
}

int stls_load_apply_T(stls_handle h, const double* lam, double* gf) {
  if (h && h->geometry) { set_error("stls_load_apply_T: unit box only (not available on a mapped domain)"); return STLS_EINVAL; }
  if (!h || !lam || !gf) { set_error("bad handle or pointers"); return STLS_EINVAL; }
  int st = ensure_diff_operands(h);
  if (st) return st;
  bool first = true;
  for (auto& t : load_terms(h, true)) {
    if ((st = apply_chain(h, lam, gf, t.second, t.first, !first, h->ftmp[0], h->ftmp[1]))) return st;
    first = false;
  }
  return STLS_OK;
}

int stls_mass_apply(stls_handle h, const double* x, double* y) {
  if (h && h->geometry) { set_error("stls_mass_apply: unit box only (not available on a mapped domain)"); return STLS_EINVAL; }
  if (!h || !x || !y || x == y) { set_error("bad handle or pointers (x and y must differ)"); return STLS_EINVAL; }
  int st = ensure_diff_operands(h);
  if (st) return st;
  std::vector<Fac> f;
  for (int k = 0; k <= h->d; ++k) f.push_back(sq(h->dd[k], h->dd[k].M));
  return apply_chain(h, x, y, f, 1.0, false, h->ftmp[0], h->ftmp[1]);
}

int stls_dot(stls_handle h, const double* a, const double* b, int64_t n, double* out) {
  if (!h || !a || !b || !out || n < 0) { set_error("bad handle or pointers"); return STLS_EINVAL; }
  return device_dot(h, a, b, n, out);
}

int stls_dkappa(stls_handle h, const double* f, const double* u, const double* lam, double* dk) {
  if (h && h->geometry) { set_error("stls_dkappa: unit box only (not available on a mapped domain)"); return STLS_EINVAL; }
  if (!h || !f || !u || !lam || !dk) { set_error("bad handle or pointers"); return STLS_EINVAL; }
  int st = ensure_diff_operands(h);
  if (st) return st;
  const int d = h->d;
  double* V = h->fdbuf[0];
  bool first = true;
  // -(Mbar_t x Dbar_s) f
  for (int k = 0; k < d; ++k) {
    std::vector<Fac> fac;
    for (int m = 0; m < d; ++m) fac.push_back(rect(h->dd[m], m == k ? h->dd[m].Gbar : h->dd[m].Mbar));
    fac.push_back(rect(h->dd[d], h->dd[d].Mbar));
    if ((st = apply_chain(h, f, V, fac, -1.0, !first, h->ftmp[0], h->ftmp[1]))) return st;
    first = false;
  }
  // -2 kappa (M_t x J_s) u with J_s = sum_k (J_k) + 2 sum_{k<l} (K_k K_l)
  const double c2 = -2.0 * h->kappa;
  for (int k = 0; k < d; ++k) {
    std::vector<Fac> fac;
    for (int m = 0; m < d; ++m) fac.push_back(sq(h->dd[m], m == k ? h->dd[m].J : h->dd[m].M));
    fac.push_back(sq(h->dd[d], h->dd[d].M));
    if ((st = apply_chain(h, u, V, fac, c2, true, h->ftmp[0], h->ftmp[1]))) return st;
    for (int l = k + 1; l < d; ++l) {
      std::vector<Fac> g;
      for (int m = 0; m < d; ++m) g.push_back(sq(h->dd[m], (m == k || m == l) ? h->dd[m].K : h->dd[m].M));
      g.push_back(sq(h->dd[d], h->dd[d].M));
      if ((st = apply_chain(h, u, V, g, 2.0 * c2, true, h->ftmp[0], h->ftmp[1]))) return st;
    }
  }
  // -(W_t x L_s) u: only the final time slice, W_t = w e_T e_T^T
  const size_t last = (size_t)(h->dir[d].n - 1) * h->ns;
  const double w = h->dir[d].wend;
  for (int k = 0; k < d; ++k) {
    std::vector<Fac> fac;
    for (int m = 0; m < d; ++m) fac.push_back(sq(h->dd[m], m == k ? h->dd[m].K : h->dd[m].M));
    if ((st = apply_chain(h, u + last, V + last, fac, -w, true, h->ftmp[0], h->ftmp[1]))) return st;
  }
  return device_dot(h, lam, V, h->ndof, dk);
}

int stls_dkappa_terms(stls_handle h, const double* f, const double* u, const double* lam, double* dk) {
  return stls_dkappa(h, f, u, lam, dk);
}

int stls_misfit(stls_handle h, const double* u, const double* ustar, double* q, double* loss) {
  if (h && h->geometry) { set_error("stls_misfit: unit box only (not available on a mapped domain)"); return STLS_EINVAL; }
  if (!h || !u || !ustar || !q || !loss) { set_error("bad handle or pointers"); return STLS_EINVAL; }
  int st = ensure_diff_operands(h);
  if (st) return st;
  double* e = h->fdbuf[1];
  hipLaunchKernelGGL(sub_kernel, dim3(grid_for(h->ndof)), dim3(kT), 0, h->stream, u, ustar, e, (long long)h->ndof);
  hipError_t er = hipGetLastError();
  if (er != hipSuccess) return hip_fail(er, "sub_kernel launch");
  // q = 2 M_Q e: the factor 2 in the last mode product is an exact scaling,
  // so e . q / 2 is the loss e^T M_Q e bit for bit
  std::vector<Fac> f;
  for (int k = 0; k <= h->d; ++k) f.push_back(sq(h->dd[k], h->dd[k].M));
  if ((st = apply_chain(h, e, q, f, 2.0, false, h->ftmp[0], h->ftmp[1]))) return st;
  double two_loss = 0.0;
  if ((st = device_dot(h, e, q, h->ndof, &two_loss))) return st;
  *loss = 0.5 * two_loss;
  return STLS_OK;
}

}  // extern "C"
