// Kernels of the stls library for mapped spatial domains (gfx950):
//   y = (K_t (x) M_s + kappa^2 M_t (x) J_s + kappa W_t (x) L_s) x
// with the pulled-back spatial factors stored as stencils [S][ns] (row i's
// entry for column offset o at o*ns + i; §4.1 with the geometry of §2.2),
// and the diagonal scaling of P^G = D^1/2 Pbar^G D^1/2 (§4.4).
//
// The matvec runs in two passes.  The time band first:
//   XK = (K_t (x) I) x,  XM = (M_t (x) I) x   (read x, write XK, XM: 24 B/DOF),
// then the spatial stencils applied to all time slices of a row:
//   y(:, t) = M_s XK(:, t) + kappa^2 J_s XM(:, t)  [+ kappa w L_s x(:, T)]
// one thread per (row, chunk of time slices): the row's stencil entries are
// read once per chunk and reused for every slice; the neighbours' values
// are read coalesced across the rows of a wave.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "stls_internal.h"

namespace stls {

namespace {

constexpr int kMT = 256;
constexpr int kMapTT = 8;  // time slices per thread in the spatial pass
constexpr int kMapBlocks = 8192;

struct MapShape {
  int d, ns, nt;
  int n[3], p[3];
};

__device__ inline bool finished(const PcgScalars* gate) { return gate && (gate->done | gate->flag); }

__global__ __launch_bounds__(kMT) void mapped_time_kernel(const double* __restrict__ x, double* __restrict__ XK,
                                                          double* __restrict__ XM, int ns, int nt, int pt,
                                                          const double* __restrict__ Kt,
                                                          const double* __restrict__ Mt,
                                                          const PcgScalars* __restrict__ gate) {
  if (finished(gate)) return;
  const int bw = 2 * pt + 1;
  const long long total = (long long)ns * nt;
  for (long long e = (long long)blockIdx.x * kMT + threadIdx.x; e < total; e += (long long)gridDim.x * kMT) {
    const int is = (int)(e % ns), t = (int)(e / ns);
    double a = 0.0, b = 0.0;
    for (int o = 0; o < bw; ++o) {
      const int tau = t + o - pt;
      if (tau < 0 || tau >= nt) continue;
      const double v = x[(size_t)tau * ns + is];
      a += Kt[t * bw + o] * v;
      b += Mt[t * bw + o] * v;
    }
    XK[e] = a;
    XM[e] = b;
  }
}

template <bool DOT>
__global__ __launch_bounds__(kMT) void mapped_space_kernel(
    const double* __restrict__ XK, const double* __restrict__ XM, const double* __restrict__ x,
    double* __restrict__ y, MapShape sh, const double* __restrict__ Ms, const double* __restrict__ Js,
    const double* __restrict__ Ls, double k2, double kw, const double* __restrict__ dotv,
    double* __restrict__ partials, const PcgScalars* __restrict__ gate) {
  if (finished(gate)) return;
  __shared__ double red[kMT / 64];
  const int ns = sh.ns, nt = sh.nt;
  const int nchunk = (nt + kMapTT - 1) / kMapTT;
  const long long total = (long long)ns * nchunk;
  const int bw0 = 2 * sh.p[0] + 1, bw1 = sh.d > 1 ? 2 * sh.p[1] + 1 : 1, bw2 = sh.d > 2 ? 2 * sh.p[2] + 1 : 1;
  const int n0 = sh.n[0], n1 = sh.d > 1 ? sh.n[1] : 1, n2 = sh.d > 2 ? sh.n[2] : 1;
  const int p0 = sh.p[0], p1 = sh.d > 1 ? sh.p[1] : 0, p2 = sh.d > 2 ? sh.p[2] : 0;
  double dsum = 0.0;
  for (long long e = (long long)blockIdx.x * kMT + threadIdx.x; e < total; e += (long long)gridDim.x * kMT) {
    const int is = (int)(e % ns), tc = (int)(e / ns);
    const int t0 = tc * kMapTT;
    const int i0 = is % n0, i1 = (is / n0) % n1, i2 = is / (n0 * n1);
    const bool has_last = t0 + kMapTT >= nt;  // the final time slice is in this chunk
    double acc[kMapTT];
#pragma unroll
    for (int u = 0; u < kMapTT; ++u) acc[u] = 0.0;
    double accL = 0.0;
    for (int o2 = 0; o2 < bw2; ++o2) {
      const int j2 = i2 + o2 - p2;
      if (j2 < 0 || j2 >= n2) continue;
      for (int o1 = 0; o1 < bw1; ++o1) {
        const int j1 = i1 + o1 - p1;
        if (j1 < 0 || j1 >= n1) continue;
        for (int o0 = 0; o0 < bw0; ++o0) {
          const int j0 = i0 + o0 - p0;
          if (j0 < 0 || j0 >= n0) continue;
          const int o = o0 + bw0 * (o1 + bw1 * o2);
          const int js = j0 + n0 * (j1 + n1 * j2);
          const double cm = Ms[(size_t)o * ns + is], cj = k2 * Js[(size_t)o * ns + is];
#pragma unroll
          for (int u = 0; u < kMapTT; ++u) {
            const int t = min(t0 + u, nt - 1);  // slices past nt are computed and dropped
            acc[u] += cm * XK[(size_t)t * ns + js] + cj * XM[(size_t)t * ns + js];
          }
          if (has_last) accL += Ls[(size_t)o * ns + is] * x[(size_t)(nt - 1) * ns + js];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kMapTT; ++u) {
      const int t = t0 + u;
      if (t >= nt) break;
      const double v = acc[u] + (t == nt - 1 ? kw * accL : 0.0);
      y[(size_t)t * ns + is] = v;
      if constexpr (DOT) dsum += v * dotv[(size_t)t * ns + is];
    }
  }
  if constexpr (DOT) {
    for (int off = 32; off > 0; off >>= 1) dsum += __shfl_xor(dsum, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = dsum;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int w = 0; w < kMT / 64; ++w) s += red[w];
      partials[blockIdx.x] = s;
    }
  }
}

// y = sigma o x (x and y may alias), optional partial sums of y . dotv
template <bool DOT>
__global__ __launch_bounds__(kMT) void mapped_scale_kernel(const double* x, double* y, const double* __restrict__ sigma,
                                                           long long n, const double* __restrict__ dotv,
                                                           double* __restrict__ partials,
                                                           const PcgScalars* __restrict__ gate) {
  if (finished(gate)) return;
  __shared__ double red[kMT / 64];
  double dsum = 0.0;
  for (long long i = (long long)blockIdx.x * kMT + threadIdx.x; i < n; i += (long long)gridDim.x * kMT) {
    const double v = sigma[i] * x[i];
    y[i] = v;
    if constexpr (DOT) dsum += v * dotv[i];
  }
  if constexpr (DOT) {
    for (int off = 32; off > 0; off >>= 1) dsum += __shfl_xor(dsum, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = dsum;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int w = 0; w < kMT / 64; ++w) s += red[w];
      partials[blockIdx.x] = s;
    }
  }
}

int blocks_for(long long n) {
  return (int)std::max<long long>(1, std::min<long long>((n + kMT - 1) / kMT, kMapBlocks));
}

}  // namespace

int launch_mapped_matvec(stls_ctx* h, const double* x, double* y, const double* dot_with, double* partials,
                         int* nparts) {
  const int d = h->d;
  const DevDir& Dt = h->dd[d];
  MapShape sh;
  sh.d = d;
  sh.ns = (int)h->ns;
  sh.nt = Dt.n;
  for (int k = 0; k < 3; ++k) {
    sh.n[k] = k < d ? h->dd[k].n : 1;
    sh.p[k] = k < d ? h->dd[k].p : 0;
  }
  double* XK = h->work[1];
  double* XM = h->work[2];
  prof_begin(h);
  hipLaunchKernelGGL(mapped_time_kernel, dim3(blocks_for(h->ndof)), dim3(kMT), 0, h->stream, x, XK, XM, sh.ns, sh.nt,
                     Dt.p, Dt.K, Dt.M, h->gate);
  const long long total = (long long)sh.ns * ((sh.nt + kMapTT - 1) / kMapTT);
  const int blocks = blocks_for(total);
  if (dot_with && blocks > kPartialsCap) { set_error("too many partial sums"); return STLS_EINVAL; }
  const double k2 = h->kappa * h->kappa, kw = h->kappa * h->dir[d].wend;
  if (dot_with)
    hipLaunchKernelGGL(mapped_space_kernel<true>, dim3(blocks), dim3(kMT), 0, h->stream, XK, XM, x, y, sh, h->sten[0],
                       h->sten[1], h->sten[2], k2, kw, dot_with, partials, h->gate);
  else
    hipLaunchKernelGGL(mapped_space_kernel<false>, dim3(blocks), dim3(kMT), 0, h->stream, XK, XM, x, y, sh,
                       h->sten[0], h->sten[1], h->sten[2], k2, kw, nullptr, nullptr, h->gate);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "mapped matvec launch");
  prof_end(h, PROF_MV_MAPPED);
  if (nparts) *nparts = blocks;
  return STLS_OK;
}

int launch_mapped_scale(stls_ctx* h, const double* x, double* y, const double* dot_with, double* partials,
                        int* nparts) {
  const int blocks = blocks_for(h->ndof);
  prof_begin(h);
  if (dot_with)
    hipLaunchKernelGGL(mapped_scale_kernel<true>, dim3(blocks), dim3(kMT), 0, h->stream, x, y, h->sigma,
                       (long long)h->ndof, dot_with, partials, h->gate);
  else
    hipLaunchKernelGGL(mapped_scale_kernel<false>, dim3(blocks), dim3(kMT), 0, h->stream, x, y, h->sigma,
                       (long long)h->ndof, nullptr, nullptr, h->gate);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "mapped scaling launch");
  prof_end(h, PROF_MISC);
  if (nparts) *nparts = blocks;
  return STLS_OK;
}

}  // namespace stls
