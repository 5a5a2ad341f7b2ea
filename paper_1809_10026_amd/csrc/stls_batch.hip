// Batched FD-preconditioned PCG for many independent heat problems of uneven
// sizes and degrees (gfx950).  Each problem is a regular stls handle (its
// factors stay where stls_setup put them); the batch concatenates the PCG
// vectors of all problems and runs every PCG step as ONE launch over a work
// list of (problem, tile) items, with per-problem scalars alpha, beta, rho,
// convergence flags and fixed-order segmented reductions in device memory.
// Problems that have converged skip their items.
//
// Operators per problem are those of the single-problem path (FD of §4.3
// Algorithm 1 in FP64 on MFMA, Kronecker-sum matvec of §4.1 eq. A_kron);
// supported: d = 1 or 2, the same degree (<= 6) in every direction, n <= 112
// per direction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "stls_buf.h"
#include "stls_internal.h"

namespace stls {

namespace {

constexpr int kT = 256;
constexpr int kBCols = 64;            // FD panel width
constexpr int kBLdx = kBCols + 1;     // panel LDS row stride (static LDS stays below 64 KB)
constexpr int kBNM = 7;               // max 16-row tiles per direction (n <= 112)
constexpr int kOLb = 16, kOMaxTd = 16, kOSlots = 2;

typedef double d4b_t __attribute__((ext_vector_type(4)));

// Device descriptor of one problem.
struct BProb {
  long long off;   // offset of the problem's vectors in the concatenated buffers
  int N, ns, d, vchunk;  // vchunk: elements per vector work item
  int n[3], p[3], npad[3];
  const double* Af[3];
  const double* Ab[3];
  const double* M[3];
  const double* K[3];
  const double* J[3];
  const double* lam_t;
  const double* lam_s;
  double k2, kw;
  int Td, nlb, ntd, nchunk, Tc, insteps;  // insteps: column steps per inner-stage work item
};

struct Item {
  int prob, idx;
};

__device__ inline double bsum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  __syncthreads();
  return s;
}

__device__ inline bool skip(const PcgScalars* S, int prob) { return S[prob].done || S[prob].flag; }

// ---------------------------------------------------------------------------
// FD mode product over one panel of kBCols columns of one problem; W (n x n,
// zero padded to npad) read from global memory as W[j*npad + i].  mode: space
// direction (0..d-1) or d = fused time (forward product, FP64 division by
// lambda_t[i] + lambda_s[c], backward product).  TRANS: contiguous mode 0.
// NMT: 16-row tiles of the operator (the items of one launch are those of
// the problems whose direction has that padded size); the panel is staged in
// NMT * 16 rows of dynamic LDS.  item0: index of items[0] in the pass's
// list (partial sums are indexed by list position).
template <bool TRANS, bool FUSED, bool DOT, int NMT>
__global__ __launch_bounds__(kT) void bfd_kernel(const double* __restrict__ X, double* __restrict__ Y,
                                                 const BProb* __restrict__ P, const Item* __restrict__ items,
                                                 int nitems, int item0, int mode, int bwd,
                                                 const PcgScalars* __restrict__ S, const double* __restrict__ dotv,
                                                 double* __restrict__ partials) {
  extern __shared__ __align__(16) double Xs[];  // NMT * 16 x kBLdx
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // 2 x 2 wave split of the output panel: wave (wr, wq) owns row tiles
  // [wr * kH, wr * kH + kH) (the last one may be past NMT: computed on a
  // clamped operand column, not stored) and columns [32 wq, 32 wq + 32)
  constexpr int kH = (NMT + 1) / 2;
  const int wr = wave >> 1, wq = wave & 1;
  const int col0 = wq * 32 + (lane & 15), krow = lane >> 4;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item I = items[it];
    const BProb& B = P[I.prob];
    if (skip(S, I.prob)) continue;
    constexpr int npad = NMT * 16;  // == B.npad[mode] for every item of this launch
    const int n = B.n[mode];
    int L = 1;
    for (int m = 0; m < mode; ++m) L *= B.n[m];
    const int ncols = B.N / n;
    const double* W = FUSED ? B.Af[mode] : (bwd ? B.Ab[mode] : B.Af[mode]);
    const double* Xp = X + B.off;
    double* Yp = Y + B.off;
    const int c0 = I.idx * kBCols;
    auto base = [&](int cc) -> int { return TRANS ? cc * n : (cc % L) + (cc / L) * L * n; };
    // panel load: all 4 * NMT loads of a thread in flight before the LDS writes
    constexpr int kLd = kBCols * npad / kT;
    double v[kLd];
#pragma unroll
    for (int q = 0; q < kLd; ++q) {
      const int e = tid + q * kT;
      int j, c;
      if (TRANS) { c = e / npad; j = e - c * npad; }
      else { j = e / kBCols; c = e - j * kBCols; }
      const int cc = c0 + c;
      const bool ok = cc < ncols && j < n;
      v[q] = Xp[ok ? (size_t)base(cc) + (size_t)j * L : 0];
      v[q] = ok ? v[q] : 0.0;
    }
    __syncthreads();  // previous item's LDS reads are done
#pragma unroll
    for (int q = 0; q < kLd; ++q) {
      const int e = tid + q * kT;
      int j, c;
      if (TRANS) { c = e / npad; j = e - c * npad; }
      else { j = e / kBCols; c = e - j * kBCols; }
      Xs[j * kBLdx + c] = v[q];
    }
    __syncthreads();
    d4b_t acc[kH][2];
    auto tile = [&](int t) { return min(wr * kH + t, NMT - 1); };
    // k in 16-row blocks; the W fragments of block kb + 1 are loaded while
    // block kb's MFMAs run (W is zero padded to npad rows); each fragment
    // feeds the wave's two column tiles
    auto gemm = [&](const double* Wm) {
#pragma unroll
      for (int t = 0; t < kH; ++t) acc[t][0] = acc[t][1] = d4b_t{0, 0, 0, 0};
      double wc[4][kH], wn[4][kH];
      auto wload = [&](double (&w)[4][kH], int kb) {
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
          for (int t = 0; t < kH; ++t)
            w[s4][t] = Wm[(size_t)(kb * 16 + s4 * 4 + krow) * npad + tile(t) * 16 + (lane & 15)];
      };
      wload(wc, 0);
#pragma unroll
      for (int kb = 0; kb < NMT; ++kb) {
        if (kb + 1 < NMT) wload(wn, kb + 1);
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const double* xr = Xs + (kb * 16 + s4 * 4 + krow) * kBLdx + col0;
          const double x0 = xr[0], x1 = xr[16];
#pragma unroll
          for (int t = 0; t < kH; ++t) {
            if (TRANS) {
              acc[t][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, wc[s4][t], acc[t][0], 0, 0, 0);
              acc[t][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, wc[s4][t], acc[t][1], 0, 0, 0);
            } else {
              acc[t][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(wc[s4][t], x0, acc[t][0], 0, 0, 0);
              acc[t][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(wc[s4][t], x1, acc[t][1], 0, 0, 0);
            }
          }
        }
        if (kb + 1 < NMT) {
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
            for (int t = 0; t < kH; ++t) wc[s4][t] = wn[s4][t];
        }
      }
    };
    gemm(W);
    if (FUSED) {
      double ls[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) ls[q] = B.lam_s[min(c0 + col0 + 16 * q, ncols - 1)];
      __syncthreads();
#pragma unroll
      for (int t = 0; t < kH; ++t) {
        if (wr * kH + t >= NMT) continue;
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = (wr * kH + t) * 16 + (lane >> 4) + 4 * r;
            const double v2 = acc[t][q][r] / (B.lam_t[min(i, n - 1)] + ls[q]);
            Xs[i * kBLdx + col0 + 16 * q] = i < n ? v2 : 0.0;
          }
      }
      __syncthreads();
      gemm(B.Ab[mode]);
    }
    // outputs through range-checked buffer accesses (padding rows, columns
    // past the problem and the clamped tile are out of range): a row tile's
    // dot operand loads are all issued before the first is used
    const size_t bytes = sizeof(double) * (size_t)B.N;
    const __amdgpu_buffer_rsrc_t rY = buf_rsrc(Yp, bytes);
    const __amdgpu_buffer_rsrc_t rD = buf_rsrc(DOT ? dotv + B.off : Yp, bytes);
    double ds = 0.0;
#pragma unroll
    for (int t = 0; t < kH; ++t) {  // one row tile at a time: 8 dot operands live
      int off[2][4];
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int i, cc;
          if (TRANS) { cc = c0 + wq * 32 + 16 * q + (lane >> 4) + 4 * r; i = (wr * kH + t) * 16 + (lane & 15); }
          else { cc = c0 + col0 + 16 * q; i = (wr * kH + t) * 16 + (lane >> 4) + 4 * r; }
          const bool ok = wr * kH + t < NMT && cc < ncols && i < n;
          off[q][r] = ok ? (int)sizeof(double) * (base(cc) + i * L) : kOutOfRange;
        }
      double dv[2][4];
      if (DOT) {
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) dv[q][r] = buf_load_f64(rD, off[q][r]);
      }
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          buf_store(acc[t][q][r], rY, off[q][r]);
          if (DOT) ds += acc[t][q][r] * dv[q][r];  // 0 where out of range
        }
    }
    if (DOT) {
      const double s = bsum(ds, red);
      if (tid == 0) partials[item0 + it] = s;
    }
  }
}

// Inner stage of the matvec for d = 2: A = M1 x, B = J1 x, C = K1 x along the
// contiguous columns of n1 entries, for the problems of degree PP.  Thread t
// of a workgroup owns row i = t mod n1 of the three banded operators (its
// 3 (2PP+1) band entries stay in registers for the whole item) and column
// lane t / n1 of G = kT / n1; an item is B.insteps column steps of G columns.
// The 2PP+1 taps are unrolled with clamped columns (band entries outside the
// matrix are stored as zeros, so the clamped reads add nothing).
template <int PP>
__global__ __launch_bounds__(kT) void binner1_kernel(const double* __restrict__ x, double* __restrict__ A,
                                                     double* __restrict__ Bo, double* __restrict__ C,
                                                     const BProb* __restrict__ P, const Item* __restrict__ items,
                                                     int nitems, const PcgScalars* __restrict__ S) {
  constexpr int BW = 2 * PP + 1;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item I = items[it];
    if (skip(S, I.prob)) continue;
    const BProb& B = P[I.prob];
    const int n1 = B.n[0], G = kT / n1, ncols = B.N / n1;
    const int t = threadIdx.x, cg = t / n1;
    const int i = min(t - cg * n1, n1 - 1);
    const bool act = cg < G;
    double cm[BW], cj[BW], ck[BW];
#pragma unroll
    for (int o = 0; o < BW; ++o) {
      cm[o] = B.M[0][i * BW + o];
      cj[o] = B.J[0][i * BW + o];
      ck[o] = B.K[0][i * BW + o];
    }
    int tap[BW];  // clamped row offsets of the window
#pragma unroll
    for (int o = 0; o < BW; ++o) tap[o] = (int)sizeof(double) * min(max(i + o - PP, 0), n1 - 1);
    const size_t bytes = sizeof(double) * (size_t)B.N;
    const __amdgpu_buffer_rsrc_t rX = buf_rsrc(x + B.off, bytes);
    const __amdgpu_buffer_rsrc_t rA = buf_rsrc(A + B.off, bytes);
    const __amdgpu_buffer_rsrc_t rB = buf_rsrc(Bo + B.off, bytes);
    const __amdgpu_buffer_rsrc_t rC = buf_rsrc(C + B.off, bytes);
    const int cb = I.idx * G * B.insteps + cg;
#pragma unroll 2
    for (int s = 0; s < B.insteps; ++s) {
      const int c = cb + s * G;
      const bool ok = act && c < ncols;
      const int colb = (int)sizeof(double) * min(c, ncols - 1) * n1;
      double v[BW];
#pragma unroll
      for (int o = 0; o < BW; ++o) v[o] = buf_load_f64(rX, ok ? colb + tap[o] : kOutOfRange);
      double a = 0.0, b = 0.0, cc = 0.0;
#pragma unroll
      for (int o = 0; o < BW; ++o) {
        a += cm[o] * v[o];
        b += cj[o] * v[o];
        cc += ck[o] * v[o];
      }
      const int so = ok ? colb + (int)sizeof(double) * i : kOutOfRange;
      buf_store(a, rA, so);
      buf_store(b, rB, so);
      buf_store(cc, rC, so);
    }
  }
}

// Outer stage (last space direction and time), same streaming scheme as the
// single-problem kernel: per item 16 inner indices x Td rows of i_d x a chunk
// of output time slices, register window of 2P+1 slices, fused final-time
// term and fused partial dot product y . dotv (DOT).  P: degree in space and
// time; THREE: d = 2 (the inner stage's A, B, C), else d = 1 (x alone).
// Slices t + 1 and t + 2 are in flight in registers while slice t is applied
// from LDS (double buffered, one barrier per step); the dot operand of the
// output slice travels with them.  All reads and the y store are
// range-checked buffer accesses of the problem's own vectors, so no load is
// consumed in the step that issues it.
typedef __attribute__((address_space(4))) double kconst_f64;

template <int PP, bool THREE, bool DOT>
__global__ __launch_bounds__(kT) void bouter_kernel(const double* __restrict__ A, const double* __restrict__ Bi,
                                                    const double* __restrict__ C, double* __restrict__ y,
                                                    const BProb* __restrict__ P, const Item* __restrict__ items,
                                                    int nitems, const PcgScalars* __restrict__ S,
                                                    const double* __restrict__ dotv, double* __restrict__ partials) {
  constexpr int W = 2 * PP + 1;
  constexpr int ROWS = kOMaxTd * kOSlots;  // >= Td + 2P: every thread's slots have a row
  static_assert(kOMaxTd + 2 * PP <= ROWS, "halo rows exceed the slots");
  constexpr int NA = THREE ? 3 : 1;
  __shared__ double sbuf[2][NA][ROWS * kOLb];
  __shared__ double red[4];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item I = items[it];
    if (skip(S, I.prob)) {
      if (DOT && threadIdx.x == 0) partials[it] = 0.0;
      continue;
    }
    const BProb& B = P[I.prob];
    const int d = THREE ? 2 : 1;
    const int L = THREE ? B.n[0] : 1;
    const int nd = B.n[d - 1], nt = B.n[d];
    const int Td = B.Td, rows = Td + 2 * PP;
    const int td = I.idx % B.ntd, lb = (I.idx / B.ntd) % B.nlb, ch = I.idx / (B.ntd * B.nlb);
    const int l0 = lb * kOLb, d0 = td * Td, c0 = ch * B.Tc, c1 = min(nt, c0 + B.Tc);
    const int li = threadIdx.x % kOLb, di = threadIdx.x / kOLb;
    const int l = l0 + li, id = d0 + di;
    const bool mine = di < Td && l < L && id < nd;
    const int dic = min(di, Td - 1), idc = min(id, nd - 1);
    const int plane = L * nd;
    const size_t bytes = sizeof(double) * (size_t)B.N;
    const __amdgpu_buffer_rsrc_t rA = buf_rsrc(A + B.off, bytes);
    const __amdgpu_buffer_rsrc_t rB = buf_rsrc(THREE ? Bi + B.off : A + B.off, bytes);
    const __amdgpu_buffer_rsrc_t rC = buf_rsrc(THREE ? C + B.off : A + B.off, bytes);
    const __amdgpu_buffer_rsrc_t rY = buf_rsrc(y + B.off, bytes);
    const __amdgpu_buffer_rsrc_t rD = buf_rsrc(DOT ? dotv + B.off : A + B.off, bytes);
    const double* Md = B.M[d - 1];
    const double* Jd = B.J[d - 1];
    const double* Kd = B.K[d - 1];
    // time band rows at a uniform index: read through the constant address
    // space (the bands are not written by any kernel), i.e. scalar loads that
    // do not share the vector memory counter with the prefetched slices
    const kconst_f64* Kt = (const kconst_f64*)B.K[d];
    const kconst_f64* Mt = (const kconst_f64*)B.M[d];
    double cm[W], cj[W], ck[W];
#pragma unroll
    for (int o = 0; o < W; ++o) { cm[o] = Md[idc * W + o]; cj[o] = Jd[idc * W + o]; ck[o] = Kd[idc * W + o]; }
    double S1w[W], S2w[W];
#pragma unroll
    for (int k = 0; k < W; ++k) { S1w[k] = 0.0; S2w[k] = 0.0; }
    double S3 = 0.0, ds = 0.0;
    const int tb = max(0, c0 - PP), te = c1 - 1 + PP;
    struct Slice {
      double v[kOSlots][NA];
      double dv;
    };
    // Slices past nt are read clamped and zeroed in step(); only per-lane
    // selects here, so the loads are not split by uniform branches.
    auto fetch = [&](int t, Slice& R) {
      const int tc = min(t, nt - 1);
#pragma unroll
      for (int s = 0; s < kOSlots; ++s) {
        const int rr = di + kOMaxTd * s;
        const int row = d0 - PP + rr;
        const bool ok = rr < rows && row >= 0 && row < nd && l < L;
        const int off = ok ? (int)sizeof(double) * (tc * plane + row * L + l) : kOutOfRange;
        R.v[s][0] = buf_load_f64(rA, off);
        if (THREE) {
          R.v[s][1] = buf_load_f64(rB, off);
          R.v[s][2] = buf_load_f64(rC, off);
        }
      }
      if (DOT) {
        const int tp = min(max(t - PP, 0), nt - 1);
        R.dv = buf_load_f64(rD, mine ? (int)sizeof(double) * (tp * plane + id * L + l) : kOutOfRange);
      }
    };
    auto put = [&](int buf, const Slice& R) {
#pragma unroll
      for (int s = 0; s < kOSlots; ++s) {
        const int rr = di + kOMaxTd * s;
#pragma unroll
        for (int q = 0; q < NA; ++q) sbuf[buf][q][rr * kOLb + li] = R.v[s][q];
      }
    };
    double dvc = 0.0;  // dot operand at slice t - PP
    auto step = [&](int cur, Slice& R, int t) {
      double s1 = 0.0, jA = 0.0, mB = 0.0, kC = 0.0, kA = 0.0, mC = 0.0;
#pragma unroll
      for (int o = 0; o < W; ++o) {
        const int rr = dic + o;
        const double a = sbuf[cur][0][rr * kOLb + li];
        s1 += cm[o] * a;
        jA += cj[o] * a;
        kA += ck[o] * a;
        if (THREE) {
          const double bv = sbuf[cur][1][rr * kOLb + li], cv = sbuf[cur][2][rr * kOLb + li];
          mB += cm[o] * bv;
          kC += ck[o] * cv;
          mC += cm[o] * cv;
        }
      }
      if (t == nt - 1) S3 = B.kw * (kA + mC);
      const bool live = t < nt;
#pragma unroll
      for (int k = 0; k < W - 1; ++k) { S1w[k] = S1w[k + 1]; S2w[k] = S2w[k + 1]; }
      S1w[W - 1] = live ? s1 : 0.0;
      S2w[W - 1] = live ? B.k2 * (jA + mB + 2.0 * kC) : 0.0;
      const int tp = t - PP, tpc = min(max(tp, 0), nt - 1);
      const bool out = tp >= c0 && tp < c1;
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < W; ++k) v += Kt[tpc * W + k] * S1w[k] + Mt[tpc * W + k] * S2w[k];
      if (tp == nt - 1) v += S3;
      buf_store(v, rY, out && mine ? (int)sizeof(double) * (tpc * plane + id * L + l) : kOutOfRange);
      if (DOT) ds += out && mine ? v * dvc : 0.0;
      put(cur ^ 1, R);  // slice t + 1
      if (DOT) dvc = R.dv;
      fetch(t + 3, R);
      __syncthreads();
    };
    Slice R0, R1;
    __syncthreads();  // previous item's LDS reads are done
    fetch(tb, R0);
    put(0, R0);
    if (DOT) dvc = R0.dv;
    fetch(tb + 1, R0);
    fetch(tb + 2, R1);
    __syncthreads();
    for (int t = tb; t <= te; t += 2) {
      step(0, R0, t);
      if (t + 1 <= te) step(1, R1, t + 1);
    }
    if (DOT) {
      const double s = bsum(ds, red);
      if (threadIdx.x == 0) partials[it] = s;
    }
  }
}

// vector kernels over (problem, chunk) items
enum BVec { BV_DOT_BB = 0, BV_XR = 1, BV_P = 2, BV_INIT = 3 };
__global__ __launch_bounds__(kT) void bvec_kernel(int kind, double* __restrict__ x, double* __restrict__ r,
                                                  double* __restrict__ p, const double* __restrict__ q,
                                                  const double* __restrict__ b, const BProb* __restrict__ P,
                                                  const Item* __restrict__ items, int nitems,
                                                  const PcgScalars* __restrict__ S, double* __restrict__ partials) {
  __shared__ double red[4];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item I = items[it];
    const BProb& B = P[I.prob];
    const size_t e0 = B.off + (size_t)I.idx * B.vchunk;
    const size_t e1 = B.off + std::min<size_t>((size_t)(I.idx + 1) * B.vchunk, (size_t)B.N);
    double s = 0.0;
    if (kind == BV_INIT) {  // x = 0, r = b; partial sums of b.b
      for (size_t e = e0 + threadIdx.x; e < e1; e += kT) {
        const double bv = b[e];
        x[e] = 0.0;
        r[e] = bv;
        s += bv * bv;
      }
    } else if (!skip(S, I.prob)) {
      if (kind == BV_XR) {
        const double alpha = S[I.prob].alpha;
        for (size_t e = e0 + threadIdx.x; e < e1; e += kT) {
          x[e] += alpha * p[e];
          const double rn = r[e] - alpha * q[e];
          r[e] = rn;
          s += rn * rn;
        }
      } else if (kind == BV_P) {  // p = z + beta p   (z passed in q)
        const double beta = S[I.prob].beta;
        for (size_t e = e0 + threadIdx.x; e < e1; e += kT) p[e] = q[e] + beta * p[e];
      }
    }
    if (kind != BV_P) {
      s = bsum(s, red);
      if (threadIdx.x == 0) partials[it] = s;
    }
  }
}

__global__ void bcopy_kernel(double* __restrict__ dst, const double* __restrict__ src, const BProb* __restrict__ P,
                             const Item* __restrict__ items, int nitems, const PcgScalars* __restrict__ S) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item I = items[it];
    if (skip(S, I.prob)) continue;
    const BProb& B = P[I.prob];
    const size_t e0 = B.off + (size_t)I.idx * B.vchunk;
    const size_t e1 = B.off + std::min<size_t>((size_t)(I.idx + 1) * B.vchunk, (size_t)B.N);
    for (size_t e = e0 + threadIdx.x; e < e1; e += kT) dst[e] = src[e];
  }
}

enum BFin { BF_BNORM = 0, BF_RHO0, BF_ALPHA, BF_RR, BF_BETA };
// One workgroup per problem: fixed-order sum of the problem's partials
// [beg[prob], end[prob]) and update of its scalars.
__global__ __launch_bounds__(kT) void bfinalize_kernel(const double* __restrict__ partials, const int* __restrict__ beg,
                                                       const int* __restrict__ end, PcgScalars* __restrict__ S,
                                                       int kind, double rtol) {
  __shared__ double red[4];
  const int prob = blockIdx.x;
  PcgScalars& s = S[prob];
  if (kind == BF_BNORM && threadIdx.x == 0) {
    s.rho = s.alpha = s.beta = 0.0;
    s.relres = 1.0;
    s.rtol = rtol;
    s.done = s.flag = s.iters = 0;
  }
  __syncthreads();
  if (s.done || s.flag) return;
  double v = 0.0;
  for (int i = beg[prob] + threadIdx.x; i < end[prob]; i += kT) v += partials[i];
  const double t = bsum(v, red);
  if (threadIdx.x != 0) return;
  switch (kind) {
    case BF_BNORM:
      s.bnorm2 = t;
      if (!isfinite(t)) s.flag = 2;
      else if (t == 0.0) { s.done = 1; s.relres = 0.0; }
      break;
    case BF_RHO0:
      s.rho = t;
      if (!isfinite(t)) s.flag = 2; else if (!(t > 0.0)) s.flag = 1;
      break;
    case BF_ALPHA:
      if (!isfinite(t)) s.flag = 2; else if (!(t > 0.0)) s.flag = 1; else s.alpha = s.rho / t;
      break;
    case BF_RR: {
      const double rel = sqrt(t / s.bnorm2);
      s.relres = rel;
      s.iters += 1;  // active problems finalise r.r once per iteration (replayable as a graph)
      if (!isfinite(rel)) s.flag = 2; else if (rel <= s.rtol) s.done = 1;
      break;
    }
    case BF_BETA:
      if (!isfinite(t)) s.flag = 2; else if (!(t > 0.0)) s.flag = 1; else { s.beta = t / s.rho; s.rho = t; }
      break;
  }
}

template <typename T>
int upload_vec(T** dst, const std::vector<T>& v, hipStream_t st) {
  if (hipMalloc((void**)dst, std::max<size_t>(1, v.size()) * sizeof(T)) != hipSuccess) {
    set_error("hipMalloc (batch)");
    return STLS_ENOMEM;
  }
  // synchronised: the host vector is a temporary of the caller
  if (!v.empty() && (hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st) != hipSuccess ||
                     hipStreamSynchronize(st) != hipSuccess)) {
    set_error("hipMemcpyAsync (batch)");
    return STLS_EHIP;
  }
  return STLS_OK;
}

struct ItemList {
  Item* dev = nullptr;
  int count = 0;
  int* beg = nullptr;  // per problem, into this list
  int* end = nullptr;
};

// Work-item shapes and launch geometry of the batched kernels (chosen by
// stls_batch_autotune; the defaults are the shapes measured best on the
// 256-problem uneven batch by hand).  Field order = enum stls_batch_tune_field.
struct BatchTuning {
  int vec_chunk = 4096;   // elements per vector work item
  int inner_steps = 8;    // column steps per inner-stage work item
  int outer_chunk = 32;   // time slices per outer-stage work item (at most)
  int grid_fd = 2048;     // workgroup caps per launch
  int grid_inner = 2048;
  int grid_outer = 2048;
  int grid_vec = 2048;
  int graph_depth = 1;    // PCG iterations per captured graph launch
};
constexpr int kTuneFields = 8;
static_assert(sizeof(BatchTuning) == kTuneFields * sizeof(int), "tuning fields");

}  // namespace

}  // namespace stls

using namespace stls;

struct stls_batch_ctx {
  int nprob = 0, d = 0;
  hipStream_t stream = nullptr;
  std::vector<stls_handle> probs;
  std::vector<BProb> hdesc;
  BProb* desc = nullptr;
  std::vector<int64_t> off;  // nprob + 1
  int64_t total = 0;
  ItemList fd[4];       // FD passes per direction (index d = fused time), items ordered by padded size
  std::vector<std::array<int, 3>> fd_grp[4];  // per pass: {16-row tiles, first item, item count}
  ItemList vec;
  std::vector<ItemList> inner;   // d = 2 inner-stage items per degree group
  std::vector<int> inner_p;      // degree of each group
  std::vector<ItemList> outer;   // per degree group
  std::vector<int> outer_p;      // degree of each group
  ItemList outer_all;            // concatenation (for the dot ranges)
  std::vector<int> outer_base;   // item offset of each group within outer_all
  double* buf[10] = {nullptr};   // r z p q fd0 fd1 A B C spare
  double* partials = nullptr;
  int partials_cap = 0;
  PcgScalars* S = nullptr;
  PcgScalars* Sh = nullptr;
  std::vector<int> last_iters;
  bool use_graph = true;  // PCG iterations replayed from a captured hipGraph
  // the solve runs on a stream of its own (capturable whatever the caller's
  // stream is), ordered after and before the caller's stream by events
  hipStream_t solve_stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  int graph_used = 0;  // 1 if the last solve replayed a captured graph
  BatchTuning tune;
};

namespace {

// make a list of items (prob, idx) for idx < count[prob]
int make_list(stls_batch_ctx* B, ItemList& L, const std::vector<int>& count, const std::vector<int>* probs = nullptr) {
  std::vector<Item> items;
  std::vector<int> beg(B->nprob, 0), end(B->nprob, 0);
  auto add = [&](int p) {
    beg[p] = (int)items.size();
    for (int i = 0; i < count[p]; ++i) items.push_back({p, i});
    end[p] = (int)items.size();
  };
  if (probs) for (int p : *probs) add(p);
  else for (int p = 0; p < B->nprob; ++p) add(p);
  L.count = (int)items.size();
  int st = upload_vec(&L.dev, items, B->stream);
  if (!st) st = upload_vec(&L.beg, beg, B->stream);
  if (!st) st = upload_vec(&L.end, end, B->stream);
  return st;
}

void free_list(ItemList& L) {
  if (L.dev) (void)hipFree(L.dev);
  if (L.beg) (void)hipFree(L.beg);
  if (L.end) (void)hipFree(L.end);
  L = ItemList();
}

void free_batch(stls_batch_ctx* B) {
  if (!B) return;
  for (auto& L : B->fd) free_list(L);
  free_list(B->vec);
  for (auto& L : B->inner) free_list(L);
  for (auto& L : B->outer) free_list(L);
  free_list(B->outer_all);
  for (double* p : B->buf)
    if (p) (void)hipFree(p);
  if (B->partials) (void)hipFree(B->partials);
  if (B->S) (void)hipFree(B->S);
  if (B->Sh) (void)hipHostFree(B->Sh);
  if (B->desc) (void)hipFree(B->desc);
  if (B->ev_in) (void)hipEventDestroy(B->ev_in);
  if (B->ev_out) (void)hipEventDestroy(B->ev_out);
  if (B->solve_stream) (void)hipStreamDestroy(B->solve_stream);
  for (auto h : B->probs)
    if (h) stls_destroy(h);
  delete B;
}

// (Re)build the work lists whose item shapes the tuning sets: vector chunks,
// inner-stage column steps and outer-stage time chunks; upload the problem
// descriptors carrying those shapes; size the partial-sum buffer.  The
// stream must be idle (no enqueued kernel reads the old lists).
int build_tuned_lists(stls_batch_ctx* B) {
  const BatchTuning& T = B->tune;
  const int nprob = B->nprob, d = B->d;
  free_list(B->vec);
  for (auto& L : B->inner) free_list(L);
  for (auto& L : B->outer) free_list(L);
  free_list(B->outer_all);
  B->inner.clear();
  B->inner_p.clear();
  B->outer.clear();
  B->outer_p.clear();
  B->outer_base.clear();
  std::vector<int> cnt_vec(nprob), cnt_in(nprob), cnt_outer(nprob);
  for (int i = 0; i < nprob; ++i) {
    BProb& P = B->hdesc[i];
    const int nt = P.n[d];
    P.vchunk = T.vec_chunk;
    P.insteps = T.inner_steps;
    P.nchunk = (nt + T.outer_chunk - 1) / T.outer_chunk;  // time chunks (each re-reads 2p halo slices)
    P.Tc = (nt + P.nchunk - 1) / P.nchunk;
    cnt_outer[i] = P.nlb * P.ntd * P.nchunk;
    cnt_vec[i] = (P.N + P.vchunk - 1) / P.vchunk;
    const int G = kT / P.n[0], ncols = P.N / P.n[0];  // n[0] <= 112: G >= 2
    cnt_in[i] = (ncols + G * P.insteps - 1) / (G * P.insteps);
  }
  if (hipMemcpyAsync(B->desc, B->hdesc.data(), sizeof(BProb) * nprob, hipMemcpyHostToDevice, B->stream) !=
      hipSuccess) {
    set_error("hipMemcpyAsync (batch descriptors)");
    return STLS_EHIP;
  }
  int st = make_list(B, B->vec, cnt_vec);
  std::vector<int> uniq;
  for (int i = 0; i < nprob; ++i) uniq.push_back(B->hdesc[i].p[0]);
  std::sort(uniq.begin(), uniq.end());
  uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
  if (!st && d == 2) {  // inner items grouped by degree
    for (int p : uniq) {
      std::vector<int> members;
      for (int i = 0; i < nprob; ++i)
        if (B->hdesc[i].p[0] == p) members.push_back(i);
      ItemList L;
      if ((st = make_list(B, L, cnt_in, &members))) break;
      B->inner.push_back(L);
      B->inner_p.push_back(p);
    }
  }
  // outer items grouped by degree; the concatenated list fixes the partial ranges
  if (!st) {
    std::vector<int> order;
    int base = 0;
    for (int p : uniq) {
      std::vector<int> members;
      for (int i = 0; i < nprob; ++i)
        if (B->hdesc[i].p[0] == p) members.push_back(i);
      ItemList L;
      if ((st = make_list(B, L, cnt_outer, &members))) break;
      B->outer.push_back(L);
      B->outer_p.push_back(p);
      B->outer_base.push_back(base);
      base += L.count;
      for (int m : members) order.push_back(m);
    }
    if (!st) st = make_list(B, B->outer_all, cnt_outer, &order);
  }
  int cap = 0;
  for (int k = 0; k <= d; ++k) cap = std::max(cap, B->fd[k].count);
  cap = std::max({cap, B->vec.count, B->outer_all.count, 1});
  if (!st && cap > B->partials_cap) {
    if (B->partials) (void)hipFree(B->partials);
    B->partials = nullptr;
    B->partials_cap = 0;
    if (hipMalloc((void**)&B->partials, sizeof(double) * cap) != hipSuccess) {
      set_error("hipMalloc (batch partial sums)");
      st = STLS_ENOMEM;
    } else {
      B->partials_cap = cap;
    }
  }
  if (!st && hipStreamSynchronize(B->stream) != hipSuccess) {
    set_error("hipStreamSynchronize (batch lists)");
    st = STLS_EHIP;
  }
  return st;
}

int grid_items(int n, int cap) { return std::max(1, std::min(n, cap)); }

int bfin(stls_batch_ctx* B, const ItemList& L, int kind, double rtol) {
  hipLaunchKernelGGL(bfinalize_kernel, dim3(B->nprob), dim3(kT), 0, B->stream, B->partials, L.beg, L.end, B->S, kind,
                     rtol);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STLS_OK : hip_fail(e, "bfinalize_kernel launch");
}

// One FD pass over all problems: a launch per padded-size group.
template <bool TRANS, bool FUSED, bool DOT>
int bfd_pass(stls_batch_ctx* B, int k, const double* in, double* out, int bwd, const double* dotv) {
  for (const auto& g : B->fd_grp[k]) {
    const int nm = g[0], first = g[1], count = g[2];
    if (count == 0) continue;
    void (*kern)(const double*, double*, const BProb*, const Item*, int, int, int, int, const PcgScalars*,
                 const double*, double*) = nullptr;
    switch (nm) {
      case 1: kern = bfd_kernel<TRANS, FUSED, DOT, 1>; break;
      case 2: kern = bfd_kernel<TRANS, FUSED, DOT, 2>; break;
      case 3: kern = bfd_kernel<TRANS, FUSED, DOT, 3>; break;
      case 4: kern = bfd_kernel<TRANS, FUSED, DOT, 4>; break;
      case 5: kern = bfd_kernel<TRANS, FUSED, DOT, 5>; break;
      case 6: kern = bfd_kernel<TRANS, FUSED, DOT, 6>; break;
      case 7: kern = bfd_kernel<TRANS, FUSED, DOT, 7>; break;
      default: set_error("batch: direction too large for the FD kernel"); return STLS_EINVAL;
    }
    const size_t shmem = sizeof(double) * (size_t)nm * 16 * kBLdx;
    hipLaunchKernelGGL(kern, dim3(grid_items(count, B->tune.grid_fd)), dim3(kT), shmem, B->stream, in, out, B->desc,
                       B->fd[k].dev + first, count, first, k, bwd, B->S, dotv, B->partials);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? STLS_OK : hip_fail(e, "batched FD launch");
}

int bprec(stls_batch_ctx* B, const double* r, double* s, const double* dotv) {
  const int d = B->d;
  double* outs[2] = {B->buf[4], B->buf[5]};
  const double* in = r;
  int cur = 0, st;
  // forward space modes
  for (int k = 0; k < d; ++k) {
    double* out = outs[cur];
    st = k == 0 ? bfd_pass<true, false, false>(B, k, in, out, 0, nullptr)
                : bfd_pass<false, false, false>(B, k, in, out, 0, nullptr);
    if (st) return st;
    in = out;
    cur ^= 1;
  }
  if ((st = bfd_pass<false, true, false>(B, d, in, outs[cur], 0, nullptr))) return st;
  in = outs[cur];
  cur ^= 1;
  for (int k = d - 1; k >= 0; --k) {
    double* out = (k == 0) ? s : outs[cur];
    if (k == 0)
      st = dotv ? bfd_pass<true, false, true>(B, k, in, out, 1, dotv) : bfd_pass<true, false, false>(B, k, in, out, 1, nullptr);
    else
      st = bfd_pass<false, false, false>(B, k, in, out, 1, nullptr);
    if (st) return st;
    in = out;
    cur ^= 1;
  }
  return STLS_OK;
}

template <int PP>
auto outer_instance(bool three, bool dot) {
  return three ? (dot ? bouter_kernel<PP, true, true> : bouter_kernel<PP, true, false>)
               : (dot ? bouter_kernel<PP, false, true> : bouter_kernel<PP, false, false>);
}

int bmatvec(stls_batch_ctx* B, const double* x, double* y, const double* dotv) {
  hipStream_t st = B->stream;
  const double* A = x;
  const double* Bv = nullptr;
  const double* C = nullptr;
  if (B->d == 2) {
    for (size_t g = 0; g < B->inner.size(); ++g) {
      const ItemList& L = B->inner[g];
      if (L.count == 0) continue;
      void (*kern)(const double*, double*, double*, double*, const BProb*, const Item*, int, const PcgScalars*) =
          nullptr;
      switch (B->inner_p[g]) {
        case 1: kern = binner1_kernel<1>; break;
        case 2: kern = binner1_kernel<2>; break;
        case 3: kern = binner1_kernel<3>; break;
        case 4: kern = binner1_kernel<4>; break;
        case 5: kern = binner1_kernel<5>; break;
        case 6: kern = binner1_kernel<6>; break;
        default: set_error("batch degree not supported"); return STLS_EINVAL;
      }
      hipLaunchKernelGGL(kern, dim3(grid_items(L.count, B->tune.grid_inner)), dim3(kT), 0, st, x, B->buf[6], B->buf[7],
                         B->buf[8],
                         B->desc, L.dev, L.count, B->S);
    }
    A = B->buf[6];
    Bv = B->buf[7];
    C = B->buf[8];
  }
  for (size_t g = 0; g < B->outer.size(); ++g) {
    const ItemList& L = B->outer[g];
    if (L.count == 0) continue;
    double* parts = B->partials + B->outer_base[g];
    void (*kern)(const double*, const double*, const double*, double*, const BProb*, const Item*, int,
                 const PcgScalars*, const double*, double*) = nullptr;
    switch (B->outer_p[g]) {
      case 1: kern = outer_instance<1>(B->d == 2, dotv != nullptr); break;
      case 2: kern = outer_instance<2>(B->d == 2, dotv != nullptr); break;
      case 3: kern = outer_instance<3>(B->d == 2, dotv != nullptr); break;
      case 4: kern = outer_instance<4>(B->d == 2, dotv != nullptr); break;
      case 5: kern = outer_instance<5>(B->d == 2, dotv != nullptr); break;
      case 6: kern = outer_instance<6>(B->d == 2, dotv != nullptr); break;
      default: set_error("batch degree not supported"); return STLS_EINVAL;
    }
    hipLaunchKernelGGL(kern, dim3(grid_items(L.count, B->tune.grid_outer)), dim3(kT), 0, st, A, Bv, C, y, B->desc, L.dev,
                       L.count, B->S,
                       dotv, parts);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STLS_OK : hip_fail(e, "batched matvec launch");
}

int read_scalars(stls_batch_ctx* B) {
  hipError_t e = hipMemcpyAsync(B->Sh, B->S, sizeof(PcgScalars) * B->nprob, hipMemcpyDeviceToHost, B->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  e = hipStreamSynchronize(B->stream);
  return e == hipSuccess ? STLS_OK : hip_fail(e, "hipStreamSynchronize");
}

}  // namespace

extern "C" {

int stls_batch_setup(int nprob, int d, const int* nknots, const double* const* knots, const int* degree,
                     const double* kappa, void* stream, stls_batch_handle* out) {
  if (!out) { set_error("out is NULL"); return STLS_EINVAL; }
  *out = nullptr;
  if (nprob < 1 || (d != 1 && d != 2) || !nknots || !knots || !degree || !kappa) {
    set_error("batch: nprob >= 1, d in {1, 2} and non-NULL arrays required");
    return STLS_EINVAL;
  }
  for (int i = 0; i < nprob; ++i)
    for (int k = 1; k <= d; ++k)
      if (degree[i * (d + 1) + k] != degree[i * (d + 1)] || degree[i * (d + 1)] > 6) {
        set_error("batch: every problem needs the same degree (<= 6) in all directions");
        return STLS_EINVAL;
      }
  stls_batch_ctx* B = new stls_batch_ctx();
  B->nprob = nprob;
  B->d = d;
  B->stream = (hipStream_t)stream;
  B->probs.assign(nprob, nullptr);
  // per-problem setup (host quadrature and eigensolves) in parallel threads
  std::vector<int> status(nprob, STLS_OK);
  std::vector<std::string> errs(nprob);
  const int nthreads = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (int t = 0; t < nthreads; ++t)
    pool.emplace_back([&, t]() {
      for (int i = t; i < nprob; i += nthreads) {
        status[i] = stls_setup(d, nknots + i * (d + 1), knots + i * (d + 1), degree + i * (d + 1), kappa[i], stream,
                               &B->probs[i]);
        if (status[i]) errs[i] = stls_last_error();
      }
    });
  for (auto& th : pool) th.join();
  for (int i = 0; i < nprob; ++i)
    if (status[i]) {
      set_error("batch problem " + std::to_string(i) + ": " + errs[i]);
      const int st = status[i];
      free_batch(B);
      return st;
    }
  // descriptors, offsets and the FD work lists (independent of the tuning)
  B->off.assign(nprob + 1, 0);
  B->hdesc.resize(nprob);
  std::vector<int> cnt_fd[4];
  for (int k = 0; k <= d; ++k) cnt_fd[k].assign(nprob, 0);
  for (int i = 0; i < nprob; ++i) {
    stls_ctx* h = B->probs[i];
    BProb& P = B->hdesc[i];
    std::memset(&P, 0, sizeof(P));
    P.off = B->off[i];
    P.N = (int)h->ndof;
    P.ns = (int)h->ns;
    P.d = d;
    for (int k = 0; k <= d; ++k) {
      const DevDir& D = h->dd[k];
      if (D.n > kBNM * 16) {
        set_error("batch: directions are limited to n <= 112");
        free_batch(B);
        return STLS_EINVAL;
      }
      P.n[k] = D.n;
      P.p[k] = D.p;
      P.npad[k] = D.npad;
      P.Af[k] = D.Afwd64;
      P.Ab[k] = D.Abwd64;
      P.M[k] = D.M;
      P.K[k] = D.K;
      P.J[k] = D.J;
      cnt_fd[k][i] = (P.N / D.n + kBCols - 1) / kBCols;
    }
    cnt_fd[d][i] = (P.ns + kBCols - 1) / kBCols;  // fused time: one column per spatial index
    P.lam_t = h->dd[d].lam;
    P.lam_s = h->lam_s;
    P.k2 = h->kappa * h->kappa;
    P.kw = h->kappa * h->dir[d].wend;
    const int L = d == 2 ? P.n[0] : 1, nd = P.n[d - 1];
    P.ntd = (nd + kOMaxTd - 1) / kOMaxTd;
    P.Td = (nd + P.ntd - 1) / P.ntd;
    P.nlb = (L + kOLb - 1) / kOLb;
    B->off[i + 1] = B->off[i] + P.N;
  }
  B->total = B->off[nprob];
  int st = STLS_OK;
  if (hipMalloc((void**)&B->desc, sizeof(BProb) * nprob) != hipSuccess) { set_error("hipMalloc"); st = STLS_ENOMEM; }
  // FD items of each pass ordered by the direction's padded size, one group
  // (kernel instance with that many tiles) per size
  for (int k = 0; k <= d && !st; ++k) {
    std::vector<int> order(nprob);
    for (int i = 0; i < nprob; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return B->hdesc[a].npad[k] < B->hdesc[b].npad[k]; });
    st = make_list(B, B->fd[k], cnt_fd[k], &order);
    int first = 0;
    for (size_t j = 0; j < order.size();) {
      const int nm = B->hdesc[order[j]].npad[k] / 16;
      int count = 0;
      for (; j < order.size() && B->hdesc[order[j]].npad[k] / 16 == nm; ++j) count += cnt_fd[k][order[j]];
      B->fd_grp[k].push_back({nm, first, count});
      first += count;
    }
  }
  // vector, inner and outer work lists (shaped by the tuning) and partials
  if (!st) st = build_tuned_lists(B);
  for (int i = 0; i < 9 && !st; ++i)
    if (hipMalloc((void**)&B->buf[i], sizeof(double) * std::max<int64_t>(1, B->total)) != hipSuccess) {
      set_error("hipMalloc batch vectors");
      st = STLS_ENOMEM;
    }
  if (!st && hipMalloc((void**)&B->S, sizeof(PcgScalars) * nprob) != hipSuccess) { set_error("hipMalloc"); st = STLS_ENOMEM; }
  if (!st && hipHostMalloc((void**)&B->Sh, sizeof(PcgScalars) * nprob, hipHostMallocDefault) != hipSuccess) {
    set_error("hipHostMalloc");
    st = STLS_ENOMEM;
  }
  if (!st && hipMemsetAsync(B->S, 0, sizeof(PcgScalars) * nprob, B->stream) != hipSuccess) st = STLS_EHIP;
  if (!st && hipStreamSynchronize(B->stream) != hipSuccess) st = STLS_EHIP;
  if (!st && (hipStreamCreateWithFlags(&B->solve_stream, hipStreamNonBlocking) != hipSuccess ||
              hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming) != hipSuccess ||
              hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming) != hipSuccess)) {
    set_error("batch solve stream");
    st = STLS_EHIP;
  }
  if (st) {
    free_batch(B);
    return st;
  }
  B->last_iters.assign(nprob, 0);
  *out = B;
  return STLS_OK;
}

int stls_batch_destroy(stls_batch_handle B) {
  if (!B) return STLS_OK;
  (void)hipStreamSynchronize(B->stream);
  free_batch(B);
  return STLS_OK;
}

int stls_batch_offsets(stls_batch_handle B, int64_t* off) {
  if (!B || !off) { set_error("bad batch handle or pointer"); return STLS_EINVAL; }
  for (int i = 0; i <= B->nprob; ++i) off[i] = B->off[i];
  return STLS_OK;
}

int stls_batch_problem(stls_batch_handle B, int i, stls_handle* h) {
  if (!B || !h || i < 0 || i >= B->nprob) { set_error("bad batch handle or index"); return STLS_EINVAL; }
  *h = B->probs[i];
  return STLS_OK;
}

int stls_batch_matvec(stls_batch_handle B, const double* x, double* y) {
  if (!B || !x || !y || x == y) { set_error("bad batch handle or pointers"); return STLS_EINVAL; }
  const hipError_t e = hipMemsetAsync(B->S, 0, sizeof(PcgScalars) * B->nprob, B->stream);  // no problem is masked
  if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
  return bmatvec(B, x, y, nullptr);
}

int stls_batch_prec_apply(stls_batch_handle B, const double* r, double* s) {
  if (!B || !r || !s || r == s) { set_error("bad batch handle or pointers"); return STLS_EINVAL; }
  const hipError_t e = hipMemsetAsync(B->S, 0, sizeof(PcgScalars) * B->nprob, B->stream);  // no problem is masked
  if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
  return bprec(B, r, s, nullptr);
}

int stls_batch_graph_used(stls_batch_handle B) {
  if (!B) { set_error("NULL batch handle"); return STLS_EINVAL; }
  return B->graph_used;
}

int stls_batch_set_graph(stls_batch_handle B, int on) {
  if (!B) { set_error("NULL batch handle"); return STLS_EINVAL; }
  B->use_graph = on != 0;
  return STLS_OK;
}

static int batch_pcg(stls_batch_handle B, const double* b, double* x, double rtol, int maxit, int* iters,
                     double* relres) {
  hipStream_t st = B->stream;
  double* r = B->buf[0];
  double* z = B->buf[1];
  double* p = B->buf[2];
  double* q = B->buf[3];
  int s = STLS_OK;
  const int gv = grid_items(B->vec.count, B->tune.grid_vec);
  hipLaunchKernelGGL(bvec_kernel, dim3(gv), dim3(kT), 0, st, (int)BV_INIT, x, r, p, q, b, B->desc, B->vec.dev,
                     B->vec.count, B->S, B->partials);
  if ((s = bfin(B, B->vec, BF_BNORM, rtol))) return s;
  if ((s = bprec(B, r, z, r))) return s;
  if ((s = bfin(B, B->fd[0], BF_RHO0, rtol))) return s;
  hipLaunchKernelGGL(bcopy_kernel, dim3(gv), dim3(kT), 0, st, p, z, B->desc, B->vec.dev, B->vec.count, B->S);
  // One PCG iteration of every problem; converged or broken-down problems
  // are masked by every kernel (their scalars say so), so the body is the
  // same in every iteration and can be replayed from a graph.
  auto body = [&]() -> int {
    int t;
    if ((t = bmatvec(B, p, q, p))) return t;
    if ((t = bfin(B, B->outer_all, BF_ALPHA, rtol))) return t;
    hipLaunchKernelGGL(bvec_kernel, dim3(gv), dim3(kT), 0, st, (int)BV_XR, x, r, p, q, b, B->desc, B->vec.dev,
                       B->vec.count, B->S, B->partials);
    if ((t = bfin(B, B->vec, BF_RR, rtol))) return t;
    if ((t = bprec(B, r, z, r))) return t;
    if ((t = bfin(B, B->fd[0], BF_BETA, rtol))) return t;
    hipLaunchKernelGGL(bvec_kernel, dim3(gv), dim3(kT), 0, st, (int)BV_P, x, r, p, z, b, B->desc, B->vec.dev,
                       B->vec.count, B->S, B->partials);
    const hipError_t le = hipGetLastError();
    return le == hipSuccess ? STLS_OK : hip_fail(le, "batched PCG launch");
  };
  // graphs of one iteration and (graph_depth > 1) of graph_depth iterations:
  // the host reads the scalars once per graph launch, and the one-iteration
  // graph takes the last iterations before maxit, so no problem runs more
  // than maxit iterations
  const int depth = std::max(1, B->tune.graph_depth);
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  if (B->use_graph) {  // capture failure falls back to direct launches
    for (int g = 0; g < (depth > 1 ? 2 : 1); ++g) {
      const int reps = g == 0 ? 1 : depth;
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) break;
      int cs = STLS_OK;
      for (int r = 0; r < reps && cs == STLS_OK; ++r) cs = body();
      if (hipStreamEndCapture(st, &graph[g]) != hipSuccess || cs != STLS_OK ||
          hipGraphInstantiate(&exec[g], graph[g], nullptr, nullptr, 0) != hipSuccess) {
        if (graph[g]) (void)hipGraphDestroy(graph[g]);
        graph[g] = nullptr;
        exec[g] = nullptr;
        (void)hipGetLastError();
        break;
      }
    }
  }
  B->graph_used = exec[0] != nullptr;
  int status = STLS_ENOCONV;
  for (int k = 0; k < maxit;) {
    const bool deep = exec[1] != nullptr && maxit - k >= depth;
    if (deep || exec[0]) {
      const hipError_t ge = hipGraphLaunch(deep ? exec[1] : exec[0], st);
      if (ge != hipSuccess) { s = hip_fail(ge, "hipGraphLaunch"); break; }
    } else if ((s = body())) {
      break;
    }
    k += deep ? depth : 1;
    if ((s = read_scalars(B))) break;
    bool all = true, bad = false;
    for (int i = 0; i < B->nprob; ++i) {
      if (B->Sh[i].flag) bad = true;
      else if (!B->Sh[i].done) all = false;
    }
    if (all) { status = bad ? STLS_EBREAKDOWN : STLS_OK; break; }
  }
  for (int g = 0; g < 2; ++g) {
    if (exec[g]) (void)hipGraphExecDestroy(exec[g]);
    if (graph[g]) (void)hipGraphDestroy(graph[g]);
  }
  if (s) return s;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "batched PCG launch");
  if ((s = read_scalars(B))) return s;
  bool nan = false;
  for (int i = 0; i < B->nprob; ++i) {
    if (iters) iters[i] = B->Sh[i].iters;
    if (relres) relres[i] = B->Sh[i].relres;
    B->last_iters[i] = B->Sh[i].iters;
    if (B->Sh[i].flag == 2) nan = true;
  }
  if (nan) { set_error("non-finite value in a batched problem"); return STLS_ENAN; }
  if (status == STLS_ENOCONV) set_error("some batched problems did not reach rtol within maxit");
  return status;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Autotuner of the batched kernels' work-item shapes and launch geometry.

#ifndef STLS_BATCH_SOURCE_HASH
#define STLS_BATCH_SOURCE_HASH "unhashed"
#endif

namespace {

const char* const kTuneNames[kTuneFields] = {"vec_chunk",  "inner_steps", "outer_chunk", "grid_fd",
                                             "grid_inner", "grid_outer",  "grid_vec",    "graph_depth"};

int* tune_field(BatchTuning& T, int f) { return reinterpret_cast<int*>(&T) + f; }

bool tune_valid(const BatchTuning& T) {
  auto in = [](int v, int lo, int hi) { return v >= lo && v <= hi; };
  return in(T.vec_chunk, 256, 1 << 20) && T.vec_chunk % 256 == 0 && in(T.inner_steps, 1, 64) &&
         in(T.outer_chunk, 1, 1 << 16) && in(T.grid_fd, 1, 1 << 16) && in(T.grid_inner, 1, 1 << 16) &&
         in(T.grid_outer, 1, 1 << 16) && in(T.grid_vec, 1, 1 << 16) && in(T.graph_depth, 1, 64);
}

// Cache key: the batch kernels' source hash, the device's architecture and a
// 64-bit FNV-1a hash of the batch's shape (d and every problem's sizes and
// degree): a cached choice is reused only for the same kernels on the same
// kind of device and the same problem set.
std::string tune_key(const stls_batch_ctx* B) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int v) {
    for (int b = 0; b < 4; ++b) {
      h ^= (uint64_t)((v >> (8 * b)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  mix(B->d);
  mix(B->nprob);
  for (const BProb& P : B->hdesc) {
    for (int k = 0; k <= B->d; ++k) mix(P.n[k]);
    mix(P.p[0]);
  }
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  for (char& c : arch)
    if (c == ':' || c == '"' || c == ' ') c = '_';
  char buf[32];
  std::snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)h);
  return std::string(STLS_BATCH_SOURCE_HASH).substr(0, 16) + "/" + arch + "/" + buf;
}

// The cache file is a JSON object of objects of integers,
//   {"<key>": {"vec_chunk": 4096, ...}, ...};
// the reader accepts exactly that shape (what the writer produces).
using TuneCache = std::map<std::string, std::map<std::string, long long>>;

bool read_cache(const char* path, TuneCache& out) {
  std::ifstream f(path);
  if (!f) return true;  // no file yet: empty cache
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  size_t i = 0;
  auto ws = [&]() { while (i < t.size() && std::isspace((unsigned char)t[i])) ++i; };
  auto str = [&](std::string& v) -> bool {
    ws();
    if (i >= t.size() || t[i] != '"') return false;
    const size_t j = t.find('"', i + 1);
    if (j == std::string::npos) return false;
    v = t.substr(i + 1, j - i - 1);
    i = j + 1;
    return true;
  };
  auto ch = [&](char c) -> bool { ws(); if (i < t.size() && t[i] == c) { ++i; return true; } return false; };
  if (!ch('{')) return false;
  if (ch('}')) return true;
  do {
    std::string key;
    if (!str(key) || !ch(':') || !ch('{')) return false;
    auto& ent = out[key];
    if (!ch('}')) {
      do {
        std::string name;
        if (!str(name) || !ch(':')) return false;
        ws();
        size_t used = 0;
        long long v = 0;
        try { v = std::stoll(t.substr(i, 24), &used); } catch (...) { return false; }
        i += used;
        ent[name] = v;
      } while (ch(','));
      if (!ch('}')) return false;
    }
  } while (ch(','));
  return ch('}');
}

bool write_cache(const char* path, const TuneCache& c) {
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return false;
    f << "{";
    bool first = true;
    for (const auto& e : c) {
      f << (first ? "\n" : ",\n") << " \"" << e.first << "\": {";
      first = false;
      bool f2 = true;
      for (const auto& kv : e.second) {
        f << (f2 ? "" : ", ") << "\"" << kv.first << "\": " << kv.second;
        f2 = false;
      }
      f << "}";
    }
    f << "\n}\n";
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path) == 0;
}

// Mean time of `reps` back-to-back runs of `launch` on the batch's stream
// (after one untimed run), in milliseconds.
template <class F>
int time_ms(stls_batch_ctx* B, F&& launch, int reps, float* ms) {
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return hip_fail(hipGetLastError(), "hipEventCreate");
  int st = launch();
  if (!st && hipEventRecord(a, B->stream) != hipSuccess) st = STLS_EHIP;
  for (int r = 0; r < reps && !st; ++r) st = launch();
  if (!st && hipEventRecord(b, B->stream) != hipSuccess) st = STLS_EHIP;
  if (!st && hipEventSynchronize(b) != hipSuccess) st = STLS_EHIP;
  float t = 0.f;
  if (!st && hipEventElapsedTime(&t, a, b) != hipSuccess) st = STLS_EHIP;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st) return st == STLS_EHIP ? hip_fail(hipGetLastError(), "autotune timing") : st;
  *ms = t / reps;
  return STLS_OK;
}

// Best of three timings (the minimum rejects interference).
template <class F>
int best_of(stls_batch_ctx* B, F&& launch, int reps, float* ms) {
  float best = 1e30f;
  for (int k = 0; k < 3; ++k) {
    float t;
    const int st = time_ms(B, launch, reps, &t);
    if (st) return st;
    best = std::min(best, t);
  }
  *ms = best;
  return STLS_OK;
}

}  // namespace

extern "C" {

int stls_batch_get_tuning(stls_batch_handle B, int* vals) {
  if (!B || !vals) { set_error("NULL batch or values"); return STLS_EINVAL; }
  for (int f = 0; f < kTuneFields; ++f) vals[f] = *tune_field(B->tune, f);
  return STLS_OK;
}

int stls_batch_set_tuning(stls_batch_handle B, const int* vals) {
  if (!B || !vals) { set_error("NULL batch or values"); return STLS_EINVAL; }
  BatchTuning T;
  for (int f = 0; f < kTuneFields; ++f) *tune_field(T, f) = vals[f];
  if (!tune_valid(T)) { set_error("batch tuning value out of range"); return STLS_EINVAL; }
  if (hipStreamSynchronize(B->stream) != hipSuccess || hipStreamSynchronize(B->solve_stream) != hipSuccess)
    return hip_fail(hipGetLastError(), "hipStreamSynchronize");
  B->tune = T;
  return build_tuned_lists(B);
}

int stls_batch_autotune(stls_batch_handle B, const char* cache_path, int* measured) {
  if (!B) { set_error("NULL batch"); return STLS_EINVAL; }
  if (measured) *measured = 0;
  const std::string key = tune_key(B);
  TuneCache cache;
  if (cache_path && !read_cache(cache_path, cache)) {
    set_error(std::string("autotune cache is not in the expected format: ") + cache_path);
    return STLS_EINVAL;
  }
  if (cache_path && cache.count(key)) {  // reuse the stored choice
    BatchTuning T = B->tune;
    for (int f = 0; f < kTuneFields; ++f) {
      auto it = cache[key].find(kTuneNames[f]);
      if (it != cache[key].end()) *tune_field(T, f) = (int)it->second;
    }
    if (tune_valid(T)) {
      int v[kTuneFields];
      for (int f = 0; f < kTuneFields; ++f) v[f] = *tune_field(T, f);
      return stls_batch_set_tuning(B, v);
    }
  }
  if (hipStreamSynchronize(B->stream) != hipSuccess) return hip_fail(hipGetLastError(), "hipStreamSynchronize");
  // the measurements run on the batch's own (capturable) stream; the caller's
  // stream is idle meanwhile and is restored on every return path
  hipStream_t caller = B->stream;
  B->stream = B->solve_stream;
  struct Restore {
    stls_batch_ctx* B;
    hipStream_t s;
    ~Restore() {
      (void)hipStreamSynchronize(B->solve_stream);
      B->stream = s;
    }
  } restore{B, caller};
  // every problem active (done = flag = 0) so that no kernel skips its items;
  // operands are the batch's work vectors (their values do not change the
  // kernels' work)
  hipStream_t st = B->stream;
  if (hipMemsetAsync(B->S, 0, sizeof(PcgScalars) * B->nprob, st) != hipSuccess)
    return hip_fail(hipGetLastError(), "hipMemsetAsync");
  for (int i = 0; i < 4; ++i)
    if (hipMemsetAsync(B->buf[i], 0, sizeof(double) * B->total, st) != hipSuccess)
      return hip_fail(hipGetLastError(), "hipMemsetAsync");
  int rc = STLS_OK;
  auto apply = [&](const BatchTuning& T) -> int {
    int v[kTuneFields];
    for (int f = 0; f < kTuneFields; ++f) v[f] = *tune_field(const_cast<BatchTuning&>(T), f);
    return stls_batch_set_tuning(B, v);
  };
  // one knob group at a time, the others held at their current values
  struct Group {
    std::vector<int> fields;
    std::vector<std::vector<int>> cands;
    std::function<int()> stage;
  };
  auto vec_stage = [&]() -> int {
    hipLaunchKernelGGL(bvec_kernel, dim3(grid_items(B->vec.count, B->tune.grid_vec)), dim3(kT), 0, st, (int)BV_XR,
                       B->buf[4], B->buf[5], B->buf[2], B->buf[3], B->buf[0], B->desc, B->vec.dev, B->vec.count, B->S,
                       B->partials);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? STLS_OK : hip_fail(e, "bvec_kernel launch");
  };
  auto mv_stage = [&]() -> int { return bmatvec(B, B->buf[2], B->buf[3], B->buf[2]); };
  auto fd_stage = [&]() -> int { return bprec(B, B->buf[0], B->buf[1], B->buf[0]); };
  std::vector<Group> groups;
  {
    Group g{{0, 6}, {}, vec_stage};
    for (int c : {1024, 2048, 4096, 8192, 16384})
      for (int gr : {1024, 2048, 4096}) g.cands.push_back({c, gr});
    groups.push_back(g);
  }
  if (B->d == 2) {
    Group g{{1, 4}, {}, mv_stage};
    for (int c : {2, 4, 8, 16})
      for (int gr : {1024, 2048, 4096}) g.cands.push_back({c, gr});
    groups.push_back(g);
  }
  {
    Group g{{2, 5}, {}, mv_stage};
    for (int c : {8, 16, 32, 64, 128})
      for (int gr : {1024, 2048, 4096}) g.cands.push_back({c, gr});
    groups.push_back(g);
  }
  {
    Group g{{3}, {}, fd_stage};
    for (int gr : {512, 1024, 2048, 4096, 8192}) g.cands.push_back({gr});
    groups.push_back(g);
  }
  for (Group& g : groups) {
    BatchTuning best = B->tune;
    float best_ms = 1e30f;
    for (const auto& cand : g.cands) {
      BatchTuning T = B->tune;
      for (size_t j = 0; j < g.fields.size(); ++j) *tune_field(T, g.fields[j]) = cand[j];
      if ((rc = apply(T))) return rc;
      float ms = 0.f;
      if ((rc = best_of(B, g.stage, 3, &ms))) return rc;
      if (ms < best_ms) { best_ms = ms; best = T; }
    }
    if ((rc = apply(best))) return rc;
  }
  // PCG iterations per graph launch: whole solves of a right-hand side of
  // ones on scratch vectors
  double *tb = nullptr, *tx = nullptr;
  if (hipMalloc((void**)&tb, sizeof(double) * B->total) != hipSuccess ||
      hipMalloc((void**)&tx, sizeof(double) * B->total) != hipSuccess) {
    if (tb) (void)hipFree(tb);
    set_error("hipMalloc (autotune vectors)");
    return STLS_ENOMEM;
  }
  {
    std::vector<double> ones((size_t)B->total, 1.0);
    if (hipMemcpy(tb, ones.data(), sizeof(double) * B->total, hipMemcpyHostToDevice) != hipSuccess)
      rc = hip_fail(hipGetLastError(), "hipMemcpy");
  }
  if (!rc) {
    BatchTuning best = B->tune;
    float best_ms = 1e30f;
    const bool graph_on = B->use_graph;
    B->use_graph = true;
    for (int depth : {1, 2, 4, 8}) {
      BatchTuning T = B->tune;
      T.graph_depth = depth;
      if ((rc = apply(T))) break;
      float ms = 0.f;
      auto solve = [&]() -> int {
        const int r = batch_pcg(B, tb, tx, 1e-8, 500, nullptr, nullptr);
        return (r == STLS_OK || r == STLS_ENOCONV) ? STLS_OK : r;
      };
      if ((rc = best_of(B, solve, 1, &ms))) break;
      if (ms < best_ms) { best_ms = ms; best = T; }
    }
    B->use_graph = graph_on;
    if (!rc) rc = apply(best);
  }
  (void)hipFree(tb);
  (void)hipFree(tx);
  if (rc) return rc;
  if (measured) *measured = 1;
  if (cache_path) {
    auto& ent = cache[key];
    ent.clear();
    for (int f = 0; f < kTuneFields; ++f) ent[kTuneNames[f]] = *tune_field(B->tune, f);
    if (!write_cache(cache_path, cache)) {
      set_error(std::string("cannot write the autotune cache ") + cache_path);
      return STLS_EINVAL;
    }
  }
  return STLS_OK;
}

int stls_batch_pcg_solve(stls_batch_handle B, const double* b, double* x, double rtol, int maxit, int* iters,
                         double* relres) {
  if (!B || !b || !x || b == x || !(rtol > 0.0) || maxit < 1) { set_error("bad batch arguments"); return STLS_EINVAL; }
  // run on the batch's own stream, after the caller's stream's earlier work
  // and before its later work
  hipStream_t caller = B->stream;
  if (hipEventRecord(B->ev_in, caller) != hipSuccess || hipStreamWaitEvent(B->solve_stream, B->ev_in, 0) != hipSuccess) {
    set_error("batch solve stream ordering");
    return STLS_EHIP;
  }
  B->stream = B->solve_stream;
  const int st = batch_pcg(B, b, x, rtol, maxit, iters, relres);
  B->stream = caller;
  if (hipEventRecord(B->ev_out, B->solve_stream) != hipSuccess || hipStreamWaitEvent(caller, B->ev_out, 0) != hipSuccess) {
    set_error("batch solve stream ordering");
    return STLS_EHIP;
  }
  return st;
}

}  // extern "C"
