// HIP kernels (gfx950) and launchers of the stls library.
//
//  * Fast-diagonalization preconditioner (§4.3, Algorithm 1 steps 2-4):
//    dense n-mode products on MFMA, one LDS-staged panel of columns per
//    workgroup; the time mode fuses forward product, eigenvalue division
//    and backward product in one pass.
//  * Matrix-free system matvec (§4.1 eq. A_kron, §4.5): banded mode products
//    of the univariate factors, grouped so that every pass reads each input
//    once.
//  * PCG vector updates and deterministic two-stage dot products (wavefront
//    shuffles, fixed-order final sum).
//
// Tensor layout everywhere: colexicographic (first space index fastest, time
// slowest).  A mode-k view of the tensor is (L, n, R) with L the product of
// the faster extents; "column" c = l + L*r holds the n entries of mode k at
// offsets base(c) + j*L, base(c) = l + L*n*r.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "stls_internal.h"

namespace stls {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kCols = 64;          // FD panel width (columns per workgroup)
constexpr int kLdx = kCols + 1;    // LDS row stride of a panel (elements)
constexpr int kMaxBlocksEW = 8192; // grid cap of grid-stride elementwise kernels

// ---------------------------------------------------------------------------
// Block-wide sum of one double per thread; result valid in thread 0.
__device__ inline double block_sum(double v, double* red) {
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

// ---------------------------------------------------------------------------
// MFMA wrappers.  Lane l supplies A(i = l%16, k) and B(k, j = l%16) with
// k = l/16; the 16x16 result lands in 4 registers per lane:
//   f64 16x16x4: register r holds row l/16 + 4r, column l%16
//   f32 16x16x4: register r holds row 4*(l/16) + r, column l%16
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4_t acc_t;
  __device__ static inline acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mfma<float> {
  typedef f4_t acc_t;
  __device__ static inline acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// ---------------------------------------------------------------------------
// FD mode product on one panel of kCols columns:
//   Y(i, c) = sum_j W(i, j) X(j, c),   W given as A[j*npad + i] (zero padded)
// TC: compute type (double -> MFMA f64, float -> MFMA f32); TI/TO: storage
// types of input/output.  With fused_time the panel is the time mode (L =
// number of spatial dofs, one column per spatial index) and the kernel applies
// Y -> (Y / (lambda_t[i] + lambda_s[c])) -> W2 Y before storing (Algorithm 1
// steps 2 (time part), 3 and 4 (time part)); the division is FP64.
// With dotv != nullptr each block also writes sum(Y .* dotv) to partials.
template <typename TC, typename TI, typename TO, int NM>
__global__ __launch_bounds__(kThreads) void fd_mode_kernel(
    const TI* __restrict__ X, TO* __restrict__ Y, int L, int n, int ncols, const TC* __restrict__ A,
    int npad, int fused_time, const TC* __restrict__ A2, const double* __restrict__ lam_t,
    const double* __restrict__ lam_s, const double* __restrict__ dotv, double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TC* Xs = reinterpret_cast<TC*>(smem_raw);                        // npad x kLdx
  int* colbase = reinterpret_cast<int*>(smem_raw + sizeof(TC) * npad * kLdx);  // kCols
  double* red = reinterpret_cast<double*>(colbase + kCols);        // 4 (8-byte aligned: kCols ints)
  typedef typename Mfma<TC>::acc_t acc_t;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c0 = blockIdx.x * kCols;
  if (tid < kCols) {
    const int cc = c0 + tid;
    colbase[tid] = (cc < ncols) ? (cc % L) + (cc / L) * L * n : -1;
  }
  __syncthreads();
  const int total = kCols * npad;
  for (int e = tid; e < total; e += kThreads) {
    int j, c;
    if (L == 1) { c = e / npad; j = e - c * npad; }   // columns are contiguous in memory
    else { j = e / kCols; c = e - j * kCols; }        // rows of kCols contiguous entries
    const int b = colbase[c];
    TC v = TC(0);
    if (j < n && b >= 0) v = (TC)X[(size_t)b + (size_t)j * L];
    Xs[j * kLdx + c] = v;
  }
  __syncthreads();

  acc_t acc[NM];
  const int ccol = wave * 16 + (lane & 15);
  const int krow = lane >> 4;
  auto gemm = [&](const TC* __restrict__ W) {
#pragma unroll
    for (int mt = 0; mt < NM; ++mt) acc[mt] = acc_t{0, 0, 0, 0};
    for (int k0 = 0; k0 < n; k0 += 4) {
      const TC b = Xs[(k0 + krow) * kLdx + ccol];
      const TC* __restrict__ Ap = W + (size_t)(k0 + krow) * npad + (lane & 15);
#pragma unroll
      for (int mt = 0; mt < NM; ++mt) acc[mt] = Mfma<TC>::step(Ap[mt * 16], b, acc[mt]);
    }
  };
  gemm(A);
  if (fused_time) {
    __syncthreads();  // every wave is done reading the panel
    const int cc = c0 + ccol;
    const double ls = (cc < ncols) ? lam_s[cc] : 1.0;
#pragma unroll
    for (int mt = 0; mt < NM; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = mt * 16 + Mfma<TC>::row(lane, r);
        double v = 0.0;
        if (i < n && cc < ncols) v = (double)acc[mt][r] / (lam_t[i] + ls);
        Xs[i * kLdx + ccol] = (TC)v;
      }
    __syncthreads();
    gemm(A2);
  }
  __syncthreads();
#pragma unroll
  for (int mt = 0; mt < NM; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) Xs[(mt * 16 + Mfma<TC>::row(lane, r)) * kLdx + ccol] = acc[mt][r];
  __syncthreads();
  double dsum = 0.0;
  for (int e = tid; e < total; e += kThreads) {
    int j, c;
    if (L == 1) { c = e / npad; j = e - c * npad; }
    else { j = e / kCols; c = e - j * kCols; }
    const int b = colbase[c];
    if (j < n && b >= 0) {
      const size_t off = (size_t)b + (size_t)j * L;
      const TO v = (TO)Xs[j * kLdx + c];
      Y[off] = v;
      if (dotv) dsum += (double)v * dotv[off];
    }
  }
  if (dotv) {
    const double s = block_sum(dsum, red);
    if (tid == 0) partials[blockIdx.x] = s;
  }
}

template <typename TC, typename TI, typename TO>
static int launch_fd_mode(stls_ctx* h, const TI* X, TO* Y, int L, int n, int ncols, const TC* A, int npad,
                          int fused, const TC* A2, const double* lam_t, const double* dotv,
                          double* partials, int* nparts) {
  const int nm = npad / 16;
  const int blocks = (ncols + kCols - 1) / kCols;
  const size_t shmem = sizeof(TC) * (size_t)npad * kLdx + sizeof(int) * kCols + 4 * sizeof(double);
  if (dotv && blocks > kPartialsCap) { set_error("too many partial sums"); return STLS_EINVAL; }
  if (nparts) *nparts = blocks;
  prof_begin(h);
#define STLS_FD_CASE(NMV)                                                                          \
  case NMV:                                                                                        \
    kern = fd_mode_kernel<TC, TI, TO, NMV>;                                                        \
    break;
  void (*kern)(const TI*, TO*, int, int, int, const TC*, int, int, const TC*, const double*, const double*,
               const double*, double*) = nullptr;
  switch (nm) {
    STLS_FD_CASE(1) STLS_FD_CASE(2) STLS_FD_CASE(3) STLS_FD_CASE(4) STLS_FD_CASE(5) STLS_FD_CASE(6)
    STLS_FD_CASE(7) STLS_FD_CASE(8) STLS_FD_CASE(9) STLS_FD_CASE(10) STLS_FD_CASE(11) STLS_FD_CASE(12)
    STLS_FD_CASE(13) STLS_FD_CASE(14) STLS_FD_CASE(15) STLS_FD_CASE(16)
    default: set_error("direction too large for the FD kernel"); return STLS_EINVAL;
  }
  if (shmem > 65536) {
    hipError_t ea = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (ea != hipSuccess) return hip_fail(ea, "hipFuncSetAttribute(LDS)");
  }
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(kThreads), shmem, h->stream, X, Y, L, n, ncols, A, npad, fused, A2,
                     lam_t, h->lam_s, dotv, partials);
#undef STLS_FD_CASE
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "fd_mode_kernel launch");
  prof_end(h, fused ? PROF_FD_TIME : PROF_FD_SPACE);
  return STLS_OK;
}

// Forward chain over space modes, fused time kernel, backward chain; the
// last backward product writes s (FP64) and optionally the partial sums of
// s . dot_with.
template <typename TC>
static int prec_apply_t(stls_ctx* h, const double* r, double* s, const double* dot_with, double* partials,
                        int* nparts) {
  const int d = h->d;
  const int nt = h->dir[d].n;
  const int ns = (int)h->ns;
  TC* buf[2] = {reinterpret_cast<TC*>(h->fdbuf[0]), reinterpret_cast<TC*>(h->fdbuf[1])};
  auto fwdA = [&](int k) -> const TC* {
    if constexpr (sizeof(TC) == 8) return (const TC*)h->dd[k].Afwd64; else return (const TC*)h->dd[k].Afwd32;
  };
  auto bwdA = [&](int k) -> const TC* {
    if constexpr (sizeof(TC) == 8) return (const TC*)h->dd[k].Abwd64; else return (const TC*)h->dd[k].Abwd32;
  };
  int st;
  int cur = 0;
  // forward chain over space modes 1..d: r -> buf
  int L = 1;
  for (int k = 0; k < d; ++k) {
    const int n = h->dir[k].n;
    const int ncols = (int)(h->ndof / n);
    if (k == 0) st = launch_fd_mode<TC, double, TC>(h, r, buf[cur], L, n, ncols, fwdA(k), h->dd[k].npad, 0,
                                                    nullptr, nullptr, nullptr, nullptr, nullptr);
    else {
      st = launch_fd_mode<TC, TC, TC>(h, buf[cur], buf[cur ^ 1], L, n, ncols, fwdA(k), h->dd[k].npad, 0,
                                      nullptr, nullptr, nullptr, nullptr, nullptr);
      cur ^= 1;
    }
    if (st) return st;
    L *= n;
  }
  // time: forward product, division, backward product
  st = launch_fd_mode<TC, TC, TC>(h, buf[cur], buf[cur ^ 1], ns, nt, ns, fwdA(d), h->dd[d].npad, 1,
                                  bwdA(d), h->dd[d].lam, nullptr, nullptr, nullptr);
  if (st) return st;
  cur ^= 1;
  // backward chain over space modes d..1
  for (int k = d - 1; k >= 0; --k) {
    const int n = h->dir[k].n;
    L /= n;
    const int ncols = (int)(h->ndof / n);
    if (k == 0)
      st = launch_fd_mode<TC, TC, double>(h, buf[cur], s, L, n, ncols, bwdA(k), h->dd[k].npad, 0, nullptr,
                                          nullptr, dot_with, partials, nparts);
    else {
      st = launch_fd_mode<TC, TC, TC>(h, buf[cur], buf[cur ^ 1], L, n, ncols, bwdA(k), h->dd[k].npad, 0,
                                      nullptr, nullptr, nullptr, nullptr, nullptr);
      cur ^= 1;
    }
    if (st) return st;
  }
  return STLS_OK;
}

int launch_prec_apply(stls_ctx* h, const double* r, double* s, const double* dot_with, double* partials,
                      int* nparts) {
  switch (h->fd_mode) {
    case STLS_FD_FP64: return prec_apply_t<double>(h, r, s, dot_with, partials, nparts);
    case STLS_FD_FP32: return prec_apply_t<float>(h, r, s, dot_with, partials, nparts);
    default: set_error("FD precision mode not available"); return STLS_EINVAL;
  }
}

// ---------------------------------------------------------------------------
// Banded mode products of the matvec.  Each output is a short sum of terms
// coef * B_t (in_s) along one mode, B_t a banded univariate matrix stored
// n x (2p+1) row-major.  One thread per output entry; the band neighbours of
// an entry are L apart, so consecutive threads read consecutive addresses.
struct BandTerm {
  int in;      // input slot
  int band;    // band matrix slot
  double coef;
};
struct BandProg {
  const double* in[3];
  double* out[3];
  const double* band[3];
  int nin, nout;
  int nterm[3];
  BandTerm term[3][4];
  const double* last_add;  // optional: out[0](l, n-1) += last_add[l] (R must be 1)
  const double* dotv;      // optional: partial sums of out[0] .* dotv
  double* partials;
};

__global__ __launch_bounds__(kThreads) void band_mode_kernel(BandProg P, int L, int n, int total, int p) {
  __shared__ double red[4];
  const int bw = 2 * p + 1;
  double dsum = 0.0;
  for (int e = blockIdx.x * kThreads + threadIdx.x; e < total; e += gridDim.x * kThreads) {
    const int l = e % L;
    const int rest = e / L;
    const int i = rest % n;
    const int r = rest / n;
    const size_t base = (size_t)l + (size_t)r * L * n;
    double acc[3] = {0.0, 0.0, 0.0};
    const int jlo = max(0, i - p), jhi = min(n - 1, i + p);
    for (int j = jlo; j <= jhi; ++j) {
      double v[3];
      for (int s = 0; s < P.nin; ++s) v[s] = P.in[s][base + (size_t)j * L];
      const int o = j - i + p;
      for (int q = 0; q < P.nout; ++q)
        for (int t = 0; t < P.nterm[q]; ++t) {
          const BandTerm& T = P.term[q][t];
          acc[q] += T.coef * P.band[T.band][i * bw + o] * v[T.in];
        }
    }
    if (P.last_add && i == n - 1) acc[0] += P.last_add[l];
    for (int q = 0; q < P.nout; ++q) P.out[q][e] = acc[q];
    if (P.dotv) dsum += acc[0] * P.dotv[e];
  }
  if (P.dotv) {
    const double s = block_sum(dsum, red);
    if (threadIdx.x == 0) P.partials[blockIdx.x] = s;
  }
}

static int launch_band(stls_ctx* h, const BandProg& P, int L, int n, int total, int p, int prof_id,
                       int* nparts) {
  int blocks = (total + kThreads - 1) / kThreads;
  blocks = std::min(blocks, kMaxBlocksEW);
  if (nparts) *nparts = blocks;
  prof_begin(h);
  hipLaunchKernelGGL(band_mode_kernel, dim3(blocks), dim3(kThreads), 0, h->stream, P, L, n, total, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "band_mode_kernel launch");
  prof_end(h, prof_id);
  return STLS_OK;
}

// y = (K_t x M_s + kappa^2 M_t x J_s + kappa W_t x L_s) x on the unit box.
// On the Dirichlet-restricted space int b_i'' b_j = -int b_i' b_j', so the
// mixed second-derivative terms of J_s are K_k x K_l and
//   J_s = sum_k (J_k, M elsewhere) + 2 sum_{k<l} (K_k, K_l, M elsewhere),
//   L_s = sum_k (K_k, M elsewhere).
// Grouping by the operator of the last space direction d:
//   A = (M..M) x,  B = [J_s inner part] x,  C = [L_s inner part] x  over modes < d,
//   S1 = M_d A,  S2 = kappa^2 (J_d A + M_d B + 2 K_d C),  S3 = kappa w (K_d A + M_d C) at t = T,
//   y = K_t S1 + M_t S2 + e_T (x) S3.
int launch_matvec(stls_ctx* h, const double* x, double* y, const double* dot_with, double* partials,
                  int* nparts) {
  const int d = h->d;
  const int N = (int)h->ndof;
  const double k2 = h->kappa * h->kappa;
  double** w = h->work;
  const double* A = x;
  const double* B = nullptr;
  const double* C = nullptr;
  int st;
  int L = 1;
  if (d >= 2) {
    // mode 1: XM = M1 x, XJ = J1 x, XK = K1 x
    const DevDir& D1 = h->dd[0];
    BandProg P{};
    P.in[0] = x;
    P.nin = 1;
    P.band[0] = D1.M; P.band[1] = D1.J; P.band[2] = D1.K;
    P.nout = 3;
    P.out[0] = w[0]; P.out[1] = w[1]; P.out[2] = w[2];
    for (int q = 0; q < 3; ++q) { P.nterm[q] = 1; P.term[q][0] = {0, q, 1.0}; }
    if ((st = launch_band(h, P, 1, D1.n, N, D1.p, PROF_MV_INNER1, nullptr))) return st;
    L = D1.n;
    if (d == 2) {
      A = w[0]; B = w[1]; C = w[2];
    } else {
      // mode 2: A = M2 XM, B = J2 XM + M2 XJ + 2 K2 XK, C = K2 XM + M2 XK
      const DevDir& D2 = h->dd[1];
      BandProg Q{};
      Q.in[0] = w[0]; Q.in[1] = w[1]; Q.in[2] = w[2];
      Q.nin = 3;
      Q.band[0] = D2.M; Q.band[1] = D2.J; Q.band[2] = D2.K;
      Q.nout = 3;
      Q.out[0] = w[3]; Q.out[1] = w[4]; Q.out[2] = w[5];
      Q.nterm[0] = 1; Q.term[0][0] = {0, 0, 1.0};
      Q.nterm[1] = 3; Q.term[1][0] = {0, 1, 1.0}; Q.term[1][1] = {1, 0, 1.0}; Q.term[1][2] = {2, 2, 2.0};
      Q.nterm[2] = 2; Q.term[2][0] = {0, 2, 1.0}; Q.term[2][1] = {2, 0, 1.0};
      if ((st = launch_band(h, Q, L, D2.n, N, D2.p, PROF_MV_INNER2, nullptr))) return st;
      L *= D2.n;
      A = w[3]; B = w[4]; C = w[5];
    }
  }
  // last space mode d: S1, S2 over all time slices, S3 on the final slice
  const DevDir& Dd = h->dd[d - 1];
  const DevDir& Dt = h->dd[d];
  const int nt = Dt.n;
  double* S1 = (d == 3) ? w[0] : (d == 2 ? w[3] : w[0]);
  double* S2 = (d == 3) ? w[1] : (d == 2 ? w[4] : w[1]);
  double* S3 = h->fdbuf[0];  // ns entries are enough
  {
    BandProg P{};
    P.in[0] = A; P.in[1] = B; P.in[2] = C;
    P.nin = B ? 3 : 1;
    P.band[0] = Dd.M; P.band[1] = Dd.J; P.band[2] = Dd.K;
    P.nout = 2;
    P.out[0] = S1; P.out[1] = S2;
    P.nterm[0] = 1; P.term[0][0] = {0, 0, 1.0};
    if (B) {
      P.nterm[1] = 3; P.term[1][0] = {0, 1, k2}; P.term[1][1] = {1, 0, k2}; P.term[1][2] = {2, 2, 2.0 * k2};
    } else {
      P.nterm[1] = 1; P.term[1][0] = {0, 1, k2};
    }
    if ((st = launch_band(h, P, L, Dd.n, N, Dd.p, PROF_MV_SPACE, nullptr))) return st;
    // final-time slice: S3 = kappa w (K_d A + M_d C)
    const size_t last = (size_t)(nt - 1) * h->ns;
    BandProg Q{};
    Q.in[0] = A + last;
    Q.in[1] = C ? C + last : nullptr;
    Q.nin = C ? 2 : 1;
    Q.band[0] = Dd.K; Q.band[1] = Dd.M;
    Q.nout = 1;
    Q.out[0] = S3;
    const double kw = h->kappa * h->dir[d].wend;
    Q.nterm[0] = C ? 2 : 1;
    Q.term[0][0] = {0, 0, kw};
    if (C) Q.term[0][1] = {1, 1, kw};
    if ((st = launch_band(h, Q, L, Dd.n, (int)h->ns, Dd.p, PROF_MV_LAST, nullptr))) return st;
  }
  // time mode: y = K_t S1 + M_t S2 (+ S3 on the last slice)
  {
    BandProg P{};
    P.in[0] = S1; P.in[1] = S2;
    P.nin = 2;
    P.band[0] = Dt.K; P.band[1] = Dt.M;
    P.nout = 1;
    P.out[0] = y;
    P.nterm[0] = 2; P.term[0][0] = {0, 0, 1.0}; P.term[0][1] = {1, 1, 1.0};
    P.last_add = S3;
    P.dotv = dot_with;
    P.partials = partials;
    if ((st = launch_band(h, P, (int)h->ns, nt, N, Dt.p, PROF_MV_TIME, nparts))) return st;
  }
  return STLS_OK;
}

// ---------------------------------------------------------------------------
// PCG vector kernels.  Scalars live in device memory (PcgScalars); every
// kernel after convergence or breakdown returns immediately.
__global__ __launch_bounds__(kThreads) void dot_kernel(const double* __restrict__ a, const double* __restrict__ b,
                                                       int n, double* __restrict__ partials) {
  __shared__ double red[4];
  double s = 0.0;
  for (int e = blockIdx.x * kThreads + threadIdx.x; e < n; e += gridDim.x * kThreads) s += a[e] * b[e];
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

enum FinKind { FIN_BNORM = 0, FIN_RHO0, FIN_ALPHA, FIN_RR, FIN_BETA };

// One workgroup sums the partials in a fixed order and updates the scalars.
__global__ __launch_bounds__(kThreads) void finalize_kernel(const double* __restrict__ partials, int nparts,
                                                            PcgScalars* __restrict__ S, int kind,
                                                            double* __restrict__ hist, int it) {
  __shared__ double red[4];
  if (S->done || S->flag) return;
  double v = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kThreads) v += partials[i];
  const double s = block_sum(v, red);
  if (threadIdx.x != 0) return;
  switch (kind) {
    case FIN_BNORM:
      S->bnorm2 = s;
      S->relres = 1.0;
      S->iters = 0;
      if (!isfinite(s)) S->flag = 2;
      else if (s == 0.0) { S->done = 1; S->relres = 0.0; }
      break;
    case FIN_RHO0:
      S->rho = s;
      if (!isfinite(s)) S->flag = 2;
      else if (!(s > 0.0)) S->flag = 1;
      break;
    case FIN_ALPHA:
      if (!isfinite(s)) S->flag = 2;
      else if (!(s > 0.0)) S->flag = 1;
      else S->alpha = S->rho / s;
      break;
    case FIN_RR: {
      const double rel = sqrt(s / S->bnorm2);
      S->relres = rel;
      S->iters = it;
      if (hist) hist[it] = rel;
      if (!isfinite(rel)) S->flag = 2;
      else if (rel <= S->rtol) S->done = 1;
      break;
    }
    case FIN_BETA:
      if (!isfinite(s)) S->flag = 2;
      else if (!(s > 0.0)) S->flag = 1;
      else { S->beta = s / S->rho; S->rho = s; }
      break;
  }
}

// x += alpha p; r -= alpha q; partial sums of r.r
__global__ __launch_bounds__(kThreads) void update_xr_kernel(double* __restrict__ x, double* __restrict__ r,
                                                             const double* __restrict__ p,
                                                             const double* __restrict__ q, int n,
                                                             const PcgScalars* __restrict__ S,
                                                             double* __restrict__ partials) {
  __shared__ double red[4];
  if (S->done || S->flag) return;
  const double alpha = S->alpha;
  double s = 0.0;
  for (int e = blockIdx.x * kThreads + threadIdx.x; e < n; e += gridDim.x * kThreads) {
    x[e] += alpha * p[e];
    const double rn = r[e] - alpha * q[e];
    r[e] = rn;
    s += rn * rn;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// p = z + beta p
__global__ __launch_bounds__(kThreads) void update_p_kernel(double* __restrict__ p, const double* __restrict__ z,
                                                            int n, const PcgScalars* __restrict__ S) {
  if (S->done || S->flag) return;
  const double beta = S->beta;
  for (int e = blockIdx.x * kThreads + threadIdx.x; e < n; e += gridDim.x * kThreads) p[e] = z[e] + beta * p[e];
}

__global__ void init_scalars_kernel(PcgScalars* S, double rtol) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    S->rho = S->alpha = S->beta = S->bnorm2 = 0.0;
    S->relres = 1.0;
    S->rtol = rtol;
    S->done = S->flag = S->iters = S->pad = 0;
  }
}

static int ew_blocks(int n) { return std::max(1, std::min((n + kThreads - 1) / kThreads, kMaxBlocksEW)); }

static int fin(stls_ctx* h, int nparts, int kind, double* hist, int it) {
  prof_begin(h);
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kThreads), 0, h->stream, h->partials, nparts, h->scal, kind,
                     hist, it);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "finalize_kernel launch");
  prof_end(h, PROF_REDUCE);
  return STLS_OK;
}

static int read_scalars(stls_ctx* h) {
  hipError_t e = hipMemcpyAsync(h->scal_host, h->scal, sizeof(PcgScalars), hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync scalars");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return STLS_OK;
}

int pcg_run(stls_ctx* h, const double* b, double* x, double rtol, int maxit, int* iters, double* relres) {
  const int N = (int)h->ndof;
  const int nb = ew_blocks(N);
  int st, np = 0;
  hipError_t e;
  h->history.clear();
  e = hipMemsetAsync(x, 0, sizeof(double) * N, h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
  e = hipMemcpyAsync(h->r, b, sizeof(double) * N, hipMemcpyDeviceToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  hipLaunchKernelGGL(init_scalars_kernel, dim3(1), dim3(64), 0, h->stream, h->scal, rtol);
  prof_begin(h);
  hipLaunchKernelGGL(dot_kernel, dim3(nb), dim3(kThreads), 0, h->stream, b, b, N, h->partials);
  prof_end(h, PROF_VEC);
  if ((st = fin(h, nb, FIN_BNORM, nullptr, 0))) return st;
  if ((st = read_scalars(h))) return st;
  PcgScalars* S = h->scal_host;
  if (S->flag) { set_error("non-finite right-hand side"); return STLS_ENAN; }
  h->history.push_back(S->relres);
  if (S->done) {
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    h->last_iters = 0;
    return STLS_OK;
  }
  // z = P^{-1} r, rho = r.z, p = z
  if ((st = launch_prec_apply(h, h->r, h->z, h->r, h->partials, &np))) return st;
  if ((st = fin(h, np, FIN_RHO0, nullptr, 0))) return st;
  e = hipMemcpyAsync(h->pvec, h->z, sizeof(double) * N, hipMemcpyDeviceToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  int k = 0;
  int status = STLS_ENOCONV;
  for (k = 1; k <= maxit; ++k) {
    if ((st = launch_matvec(h, h->pvec, h->q, h->pvec, h->partials, &np))) return st;
    if ((st = fin(h, np, FIN_ALPHA, nullptr, k))) return st;
    prof_begin(h);
    hipLaunchKernelGGL(update_xr_kernel, dim3(nb), dim3(kThreads), 0, h->stream, x, h->r, h->pvec, h->q, N, h->scal,
                       h->partials);
    prof_end(h, PROF_VEC);
    if ((st = fin(h, nb, FIN_RR, nullptr, k))) return st;
    if ((st = read_scalars(h))) return st;
    if (S->flag == 2) { set_error("non-finite value in PCG"); status = STLS_ENAN; break; }
    if (S->flag == 1) { set_error("PCG breakdown (non-positive curvature)"); status = STLS_EBREAKDOWN; break; }
    h->history.push_back(S->relres);
    if (S->done) { status = STLS_OK; break; }
    if (k == maxit) break;
    if ((st = launch_prec_apply(h, h->r, h->z, h->r, h->partials, &np))) return st;
    if ((st = fin(h, np, FIN_BETA, nullptr, k))) return st;
    prof_begin(h);
    hipLaunchKernelGGL(update_p_kernel, dim3(nb), dim3(kThreads), 0, h->stream, h->pvec, h->z, N, h->scal);
    prof_end(h, PROF_VEC);
  }
  const int done_iters = (int)h->history.size() - 1;
  if (iters) *iters = done_iters;
  if (relres) *relres = S->relres;
  h->last_iters = done_iters;
  prof_flush(h);
  if (status == STLS_ENOCONV) set_error("PCG did not reach rtol within maxit");
  return status;
}

}  // namespace stls

using namespace stls;

extern "C" {

int stls_prec_apply(stls_handle h, const double* r, double* s) {
  if (!h || !r || !s || r == s) { set_error("bad handle or pointers (r and s must differ)"); return STLS_EINVAL; }
  return launch_prec_apply(h, r, s, nullptr, nullptr, nullptr);
}

int stls_matvec(stls_handle h, const double* x, double* y) {
  if (!h || !x || !y || x == y) { set_error("bad handle or pointers (x and y must differ)"); return STLS_EINVAL; }
  return launch_matvec(h, x, y, nullptr, nullptr, nullptr);
}

int stls_pcg_solve(stls_handle h, const double* b, double* x, double rtol, int maxit, int* iters,
                   double* relres) {
  if (!h || !b || !x || b == x) { set_error("bad handle or pointers"); return STLS_EINVAL; }
  if (!(rtol > 0.0) || maxit < 1) { set_error("rtol must be > 0 and maxit >= 1"); return STLS_EINVAL; }
  return pcg_run(h, b, x, rtol, maxit, iters, relres);
}

}  // extern "C"
