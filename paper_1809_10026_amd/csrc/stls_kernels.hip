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
#include <type_traits>
#include <vector>

#include "stls_diag.h"
#include "stls_internal.h"

namespace stls {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kCols = 64;          // FD panel width (columns per workgroup)
constexpr int kLdx = kCols + 16;   // LDS row stride of a panel: rows fill distinct banks
constexpr int kStageBatch = 4;     // operator pieces per thread in flight while staging
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
// Hand the logical tile index of a block so that consecutive logical tiles
// run on the same XCD (blocks are dealt round-robin to the 8 XCDs, each with
// its own L2): neighbouring tiles then share halo and operand lines in L2.
__device__ inline int xcd_tile(int bid, int nblocks) {
  constexpr int kXcd = 8;
  const int full = nblocks - nblocks % kXcd;
  if (bid >= full) return bid;
  return (bid % kXcd) * (full / kXcd) + bid / kXcd;
}

// ---------------------------------------------------------------------------
// FD mode product, one panel of kCols columns at a time:
//   Y(i, c) = sum_j W(i, j) X(j, c),   W read as Aop[j*npad + i] (zero padded)
// The operand W is staged in LDS once per workgroup; the workgroup then loops
// over panels (grid-stride).  A panel is staged through LDS with coalesced
// loads; results go straight from the MFMA registers to HBM in 16-wide
// contiguous runs.  TRANS selects the orientation: for the contiguous mode
// (L == 1) the MFMA rows are panel columns (output rows of 16 contiguous i),
// otherwise MFMA rows are i and the 16 lanes of a row are contiguous columns.
// TC: compute type (double -> MFMA f64, float -> MFMA f32); TI/TO storage
// types.  fused_time: time mode, Y -> (Y / (lambda_t[i] + lambda_s[c])) -> W2 Y
// (Algorithm 1, time part of step 2, step 3, time part of step 4), division
// in FP64.  dotv: each block adds sum(Y .* dotv) of its panels to partials.
template <typename TC, typename TI, typename TO, int NM, bool TRANS, bool WLDS, bool FUSED, bool DOT>
__global__ __launch_bounds__(kThreads) void fd_mode_kernel(
    const TI* __restrict__ X, TO* __restrict__ Y, int L, int n, int ncols, const TC* __restrict__ Aop,
    const TC* __restrict__ Aop2, int w2lds, const double* __restrict__ lam_t, const double* __restrict__ lam_s,
    const double* __restrict__ dotv, double* __restrict__ partials, const PcgScalars* __restrict__ gate) {
  if (gate && (gate->done | gate->flag)) return;  // PCG already finished: nothing to do
  constexpr int NPAD = NM * 16;
  constexpr int PER = NPAD * kCols / kThreads;  // panel entries per thread
  constexpr bool PREF = NM <= 4;                // register prefetch of the next panel
  constexpr int LDW = NPAD + 16;                // rows of 16-lane fragments land on distinct banks
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TC* Ws = reinterpret_cast<TC*>(smem_raw);            // NPAD x LDW (if WLDS)
  TC* Ws2 = Ws + (WLDS ? NPAD * LDW : 0);              // second operand (if w2lds)
  TC* Xs = Ws2 + (w2lds ? NPAD * LDW : 0);             // NPAD x kLdx: panel
  double* red = reinterpret_cast<double*>(Xs + NPAD * kLdx);
  typedef typename Mfma<TC>::acc_t acc_t;
  const TC* __restrict__ Wsrc = WLDS ? Ws : Aop;
  const int ldw1 = WLDS ? LDW : NPAD;
  const TC* __restrict__ W2src = w2lds ? Ws2 : Aop2;
  const int ldw2 = w2lds ? LDW : NPAD;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int npanels = (ncols + kCols - 1) / kCols;
  const int ccol = wave * 16 + (lane & 15);
  const int krow = lane >> 4;
  double dsum = 0.0;

  // operators into LDS in pairs of entries, kStageBatch pairs per thread
  // with their loads in flight before the stores
  auto stage_w = [&](const TC* __restrict__ src, TC* dst) {
    typedef TC pair_t __attribute__((ext_vector_type(2)));
    constexpr int P2 = NPAD / 2, TOT = NPAD * P2;
    for (int e0 = tid; e0 < TOT; e0 += kThreads * kStageBatch) {
      pair_t v[kStageBatch];
#pragma unroll
      for (int b = 0; b < kStageBatch; ++b)
        v[b] = *reinterpret_cast<const pair_t*>(src + (size_t)min(e0 + b * kThreads, TOT - 1) * 2);
#pragma unroll
      for (int b = 0; b < kStageBatch; ++b) {
        const int e = e0 + b * kThreads;
        if (e < TOT) {
          const int j = e / P2, i2 = e - j * P2;
          *reinterpret_cast<pair_t*>(dst + j * LDW + 2 * i2) = v[b];
        }
      }
    }
  };
  if (WLDS) stage_w(Aop, Ws);
  if (FUSED && w2lds) stage_w(Aop2, Ws2);
  // eigenvalues of this thread's output rows (rows are fixed per lane)
  double lt[FUSED ? NM * 4 : 1];
  if constexpr (FUSED) {
#pragma unroll
    for (int t = 0; t < NM; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = t * 16 + Mfma<TC>::row(lane, r);
        lt[t * 4 + r] = lam_t[min(i, n - 1)];
      }
  }

  // Column c of the (L, n, R) view starts at base(c) = c % L + (c / L) * L * n.
  auto column_base = [&](int cc) -> int {
    if constexpr (TRANS) return cc * n;
    return (cc % L) + (cc / L) * L * n;
  };
  // Panel entry s of this thread: strided layout (64 contiguous columns per
  // row): c = tid % 64, j = tid / 64 + 4 s; contiguous columns (TRANS):
  // e = tid + 256 s, c = e / NPAD, j = e % NPAD.  Loads are unconditional
  // (clamped address) so that no branch separates them from their use.
  TI pre[PREF ? PER : 1];
  auto fetch_panel = [&](int c0p, TI* dst) {
    if constexpr (TRANS) {
#pragma unroll
      for (int s = 0; s < PER; ++s) {
        const int e = tid + kThreads * s;
        const int c = e / NPAD, j = e - c * NPAD;
        const int cc = c0p + c;
        const bool ok = cc < ncols && j < n;
        const TI v = X[ok ? (size_t)cc * n + j : 0];
        dst[s] = ok ? v : TI(0);
      }
    } else {
      const int cc = c0p + (tid & (kCols - 1));
      const bool okc = cc < ncols;
      const size_t b = okc ? (size_t)column_base(cc) : 0;
#pragma unroll
      for (int s = 0; s < PER; ++s) {
        const int j = (tid >> 6) + (kThreads / kCols) * s;
        const bool ok = okc && j < n;
        const TI v = X[ok ? b + (size_t)j * L : 0];
        dst[s] = ok ? v : TI(0);
      }
    }
  };
  auto park_entry = [&](int s, TC v) {
    int j, c;
    if constexpr (TRANS) { const int e = tid + kThreads * s; c = e / NPAD; j = e - c * NPAD; }
    else { c = tid & (kCols - 1); j = (tid >> 6) + (kThreads / kCols) * s; }
    Xs[j * kLdx + c] = v;
  };

  acc_t acc[NM];
  // W(i, j) sits at W[j*ldw + i] (LDS copy or the global operand).  FP64
  // from global memory: the fragments of the next k step are loaded while
  // the current step's products run (two register sets in turn; measured
  // 1.8x on the FP64 passes at n = 130, slower in FP32); the products and
  // their order are the same either way.
  auto gemm = [&](const TC* __restrict__ W, int ldw) {
#pragma unroll
    for (int t = 0; t < NM; ++t) acc[t] = acc_t{0, 0, 0, 0};
    auto step_k = [&](int k0, const TC* wv) {
      const TC xv = Xs[(k0 + krow) * kLdx + ccol];
#pragma unroll
      for (int t = 0; t < NM; ++t) {
        if constexpr (TRANS) acc[t] = Mfma<TC>::step(xv, wv[t], acc[t]);
        else acc[t] = Mfma<TC>::step(wv[t], xv, acc[t]);
      }
    };
    if constexpr (!WLDS && std::is_same_v<TC, double>) {
      TC wa[NM], wb[NM];
      auto load_w = [&](TC* w, int k0) {
        const int kk = min(k0, NPAD - 4) + krow;  // past the end: in range, unused
#pragma unroll
        for (int t = 0; t < NM; ++t) w[t] = W[kk * ldw + t * 16 + (lane & 15)];
      };
      load_w(wa, 0);
      for (int k0 = 0; k0 < n; k0 += 8) {
        load_w(wb, k0 + 4);
        step_k(k0, wa);
        if (k0 + 4 < n) {
          load_w(wa, k0 + 8);
          step_k(k0 + 4, wb);
        }
      }
    } else {
      for (int k0 = 0; k0 < n; k0 += 4) {
        TC wv[NM];
#pragma unroll
        for (int t = 0; t < NM; ++t) wv[t] = W[(k0 + krow) * ldw + t * 16 + (lane & 15)];
        step_k(k0, wv);
      }
    }
  };
  // output position of accumulator (t, r): offset base + i * L
  auto out_pos = [&](int c0p, int t, int r, int& i, int& cc) {
    if constexpr (TRANS) { cc = c0p + wave * 16 + Mfma<TC>::row(lane, r); i = t * 16 + (lane & 15); }
    else { cc = c0p + ccol; i = t * 16 + Mfma<TC>::row(lane, r); }
  };

  if constexpr (PREF) {
    if (blockIdx.x < npanels) fetch_panel(blockIdx.x * kCols, pre);
  }
  for (int pn = blockIdx.x; pn < npanels; pn += gridDim.x) {
    const int c0 = pn * kCols;
    __syncthreads();  // W staged; previous panel's readers of Xs are done
    if constexpr (PREF) {
#pragma unroll
      for (int s = 0; s < PER; ++s) park_entry(s, (TC)pre[s]);
    } else {
      TI tmp[PER];
      fetch_panel(c0, tmp);
#pragma unroll
      for (int s = 0; s < PER; ++s) park_entry(s, (TC)tmp[s]);
    }
    // per-panel operands needed after the GEMM, loaded before the prefetch
    // of the next panel is issued (loads complete in order)
    double ls = 1.0;
    if constexpr (FUSED) ls = lam_s[min(c0 + ccol, ncols - 1)];
    double dv[DOT ? NM * 4 : 1];
    if constexpr (DOT) {
#pragma unroll
      for (int t = 0; t < NM; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int i, cc;
          out_pos(c0, t, r, i, cc);
          const bool ok = cc < ncols && i < n;
          const double v = dotv[ok ? (size_t)column_base(cc) + (size_t)i * L : 0];
          dv[t * 4 + r] = ok ? v : 0.0;
        }
    }
    __syncthreads();
    if constexpr (PREF) {
      const int nx = pn + gridDim.x;
      if (nx < npanels) fetch_panel(nx * kCols, pre);
    }
    gemm(Wsrc, ldw1);
    if constexpr (FUSED) {
      // Q = (U_t^T X) / Lambda, then U_t Q with the backward operand.
      __syncthreads();  // all waves are done reading Xs
#pragma unroll
      for (int t = 0; t < NM; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = t * 16 + Mfma<TC>::row(lane, r);
          const double v = (double)acc[t][r] / (lt[t * 4 + r] + ls);
          Xs[i * kLdx + ccol] = (i < n) ? (TC)v : TC(0);
        }
      __syncthreads();
      gemm(W2src, ldw2);
    }
    // direct stores from the accumulators
#pragma unroll
    for (int t = 0; t < NM; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int i, cc;
        out_pos(c0, t, r, i, cc);
        const TO v = (TO)acc[t][r];
        if constexpr (DOT) dsum += (double)v * dv[t * 4 + r];
        if (cc < ncols && i < n) Y[(size_t)column_base(cc) + (size_t)i * L] = v;
      }
  }
  if constexpr (DOT) {
    const double s = block_sum(dsum, red);
    if (tid == 0) partials[blockIdx.x] = s;
  }
}

template <typename TC, typename TI, typename TO, bool TRANS, bool FUSED, bool DOT>
using FdKernelPtr = void (*)(const TI*, TO*, int, int, int, const TC*, const TC*, int, const double*, const double*,
                             const double*, double*, const PcgScalars*);

template <typename TC, typename TI, typename TO, bool TRANS, bool FUSED, bool DOT, int NM>
static FdKernelPtr<TC, TI, TO, TRANS, FUSED, DOT> fd_pick(bool wlds) {
  if constexpr (NM <= 8) {
    if (wlds) return fd_mode_kernel<TC, TI, TO, NM, TRANS, true, FUSED, DOT>;
  }
  return fd_mode_kernel<TC, TI, TO, NM, TRANS, false, FUSED, DOT>;
}

// One mode product (or the fused time kernel) over the (L, n, R) view.
// TRANS: contiguous mode (L == 1); FUSED: time kernel with A2 = backward
// operand; DOT: also write partial sums of Y . dotv.
template <typename TC, typename TI, typename TO, bool TRANS, bool FUSED, bool DOT>
static int launch_fd_mode(stls_ctx* h, const TI* X, TO* Y, int L, int n, int ncols, const TC* A, const TC* A2,
                          int npad, const double* lam_t, const double* dotv, double* partials, int* nparts) {
  const int nm = npad / 16;
  const int npanels = (ncols + kCols - 1) / kCols;
  const size_t tail = sizeof(TC) * (size_t)npad * kLdx + 4 * sizeof(double);
  const size_t wbytes = sizeof(TC) * (size_t)npad * (npad + 16);
  // W in LDS while two or more workgroups still fit on a CU; FP32 also up to
  // the whole LDS (one workgroup per CU) where each workgroup then has many
  // panels to amortise the staging over (measured: d = 3, n = 98, FP32
  // 2.96 -> 2.40 ms per FD apply; slower with few panels, and in FP64)
  const bool wlds = (nm <= 8 && wbytes + tail <= 64 * 1024) ||
                    (std::is_same_v<TC, float> && wbytes + tail <= 160 * 1024 && npanels >= 16 * 256);
  const bool w2lds = FUSED && wlds && 2 * wbytes + tail <= 80 * 1024;
  const size_t shmem = (wlds ? wbytes : 0) + (w2lds ? wbytes : 0) + tail;
  if (shmem > 160 * 1024) { set_error("direction too large for the FD kernel's LDS budget"); return STLS_EINVAL; }
  const int per_cu = std::max(1, std::min(4, (int)((160 * 1024) / shmem)));
  const int blocks = std::min(npanels, 256 * per_cu);
  if (DOT && blocks > kPartialsCap) { set_error("too many partial sums"); return STLS_EINVAL; }
  if (nparts) *nparts = blocks;
  FdKernelPtr<TC, TI, TO, TRANS, FUSED, DOT> kern = nullptr;
#define STLS_FD_PICK(NMV) \
  case NMV: kern = fd_pick<TC, TI, TO, TRANS, FUSED, DOT, NMV>(wlds); break;
  switch (nm) {
    STLS_FD_PICK(1) STLS_FD_PICK(2) STLS_FD_PICK(3) STLS_FD_PICK(4) STLS_FD_PICK(5) STLS_FD_PICK(6)
    STLS_FD_PICK(7) STLS_FD_PICK(8) STLS_FD_PICK(9) STLS_FD_PICK(10) STLS_FD_PICK(11) STLS_FD_PICK(12)
    STLS_FD_PICK(13) STLS_FD_PICK(14) STLS_FD_PICK(15) STLS_FD_PICK(16)
    default: set_error("direction too large for the FD kernel"); return STLS_EINVAL;
  }
#undef STLS_FD_PICK
  if (shmem > 65536) {
    hipError_t ea = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (ea != hipSuccess) return hip_fail(ea, "hipFuncSetAttribute(LDS)");
  }
  prof_begin(h);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(kThreads), shmem, h->stream, X, Y, L, n, ncols, A, A2, (int)w2lds, lam_t,
                     h->lam_s, dotv, partials, h->gate);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "fd_mode_kernel launch");
  prof_end(h, FUSED ? PROF_FD_TIME : PROF_FD_SPACE);
  return STLS_OK;
}

// ---------------------------------------------------------------------------
// BF16x3 mode product.  Operands are FP32; each is split into bf16 hi + lo
// (hi = bf16(x), lo = bf16(x - hi)) and the product is formed as
// W_hi X_hi + W_hi X_lo + W_lo X_hi on MFMA bf16 16x16x32 with FP32
// accumulation (the lo*lo term, relative size 2^-18, is dropped).
// Fragment layout (16x16x32): lane l supplies A(i = l%16, k = 8(l/16)+e) and
// B(k = 8(l/16)+e, j = l%16), e = 0..7; results as for f32 16x16x4.
// The panel is staged as hi/lo halves in [column][k] order (8 consecutive k
// per 16-byte read); W halves are row-major [i][k].  Same orientation, fused
// time and dot conventions as fd_mode_kernel.
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef unsigned short us8_t __attribute__((ext_vector_type(8)));

__device__ inline unsigned short bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float bf16_to_float(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

template <typename TI, typename TO, int NM, bool TRANS, bool FUSED, bool DOT, bool DIV>
__global__ __launch_bounds__(kThreads) void fd_mode_bf16x3_kernel(
    const TI* __restrict__ X, TO* __restrict__ Y, int L, int n, int ncols, const unsigned short* __restrict__ Wh,
    const unsigned short* __restrict__ Wl, const unsigned short* __restrict__ W2h,
    const unsigned short* __restrict__ W2l, const double* __restrict__ lam_t, const double* __restrict__ lam_s,
    const double* __restrict__ dotv, double* __restrict__ partials, const PcgScalars* __restrict__ gate) {
  if (gate && (gate->done | gate->flag)) return;  // PCG already finished: nothing to do
  constexpr int NPAD = NM * 16;
  constexpr int NK = (NM + 1) / 2;  // 32-wide k steps
  constexpr int KPAD = NK * 32;
  constexpr int LDK = KPAD + 8;     // bf16 row stride: 16-byte fragment reads hit distinct banks
  constexpr int PER = NPAD * kCols / kThreads;
  constexpr int NW = FUSED ? 2 : 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned short* Ws = reinterpret_cast<unsigned short*>(smem_raw);  // NW x {hi, lo} x NPAD x LDK
  unsigned short* Xh = Ws + NW * 2 * NPAD * LDK;                     // kCols x LDK
  unsigned short* Xl = Xh + kCols * LDK;
  double* red = reinterpret_cast<double*>(Xl + kCols * LDK);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int npanels = (ncols + kCols - 1) / kCols;
  const int ccol = wave * 16 + (lane & 15);
  double dsum = 0.0;

  // operator rows into LDS in 16-byte pieces (8 bf16), kStageBatch pieces
  // per thread with their loads in flight before the stores
  auto stage_w = [&](const unsigned short* __restrict__ h, const unsigned short* __restrict__ l, int slot) {
    unsigned short* dh = Ws + slot * 2 * NPAD * LDK;
    unsigned short* dl = dh + NPAD * LDK;
    constexpr int P8 = KPAD / 8, TOT = NPAD * P8;
    for (int e0 = tid; e0 < TOT; e0 += kThreads * kStageBatch) {
      us8_t vh[kStageBatch], vl[kStageBatch];
#pragma unroll
      for (int b = 0; b < kStageBatch; ++b) {
        const int e = min(e0 + b * kThreads, TOT - 1);
        vh[b] = *reinterpret_cast<const us8_t*>(h + (size_t)e * 8);
        vl[b] = *reinterpret_cast<const us8_t*>(l + (size_t)e * 8);
      }
#pragma unroll
      for (int b = 0; b < kStageBatch; ++b) {
        const int e = e0 + b * kThreads;
        if (e < TOT) {
          const int i = e / P8, k8 = e - i * P8;
          *reinterpret_cast<us8_t*>(dh + i * LDK + k8 * 8) = vh[b];
          *reinterpret_cast<us8_t*>(dl + i * LDK + k8 * 8) = vl[b];
        }
      }
    }
  };
  stage_w(Wh, Wl, 0);
  if constexpr (FUSED) stage_w(W2h, W2l, 1);
  constexpr bool TIME = FUSED || DIV;  // the eigenvalue division of the time pass
  double lt[TIME ? NM * 4 : 1];
  if constexpr (TIME) {
#pragma unroll
    for (int t = 0; t < NM; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) lt[t * 4 + r] = lam_t[min(t * 16 + 4 * (lane >> 4) + r, n - 1)];
  }
  auto column_base = [&](int cc) -> int {
    if constexpr (TRANS) return cc * n;
    return (cc % L) + (cc / L) * L * n;
  };
  auto put = [&](int j, int c, float v) {
    const unsigned short hi = bf16_rne(v);
    Xh[c * LDK + j] = hi;
    Xl[c * LDK + j] = bf16_rne(v - bf16_to_float(hi));
  };
  typedef float f4v __attribute__((ext_vector_type(4)));
  f4v acc[NM];
  auto gemm = [&](int slot) {
    const unsigned short* wh = Ws + slot * 2 * NPAD * LDK;
    const unsigned short* wl = wh + NPAD * LDK;
#pragma unroll
    for (int t = 0; t < NM; ++t) acc[t] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < NK; ++kb) {
      const int koff = kb * 32 + 8 * (lane >> 4);
      const bf8_t xh = __builtin_bit_cast(bf8_t, *reinterpret_cast<const us8_t*>(Xh + ccol * LDK + koff));
      const bf8_t xl = __builtin_bit_cast(bf8_t, *reinterpret_cast<const us8_t*>(Xl + ccol * LDK + koff));
#pragma unroll
      for (int t = 0; t < NM; ++t) {
        const int row = (t * 16 + (lane & 15)) * LDK + koff;
        const bf8_t ah = __builtin_bit_cast(bf8_t, *reinterpret_cast<const us8_t*>(wh + row));
        const bf8_t al = __builtin_bit_cast(bf8_t, *reinterpret_cast<const us8_t*>(wl + row));
        if constexpr (TRANS) {
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, ah, acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, ah, acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, al, acc[t], 0, 0, 0);
        } else {
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, xh, acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, xl, acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, xh, acc[t], 0, 0, 0);
        }
      }
    }
  };
  auto out_pos = [&](int c0p, int t, int r, int& i, int& cc) {
    if constexpr (TRANS) { cc = c0p + wave * 16 + 4 * (lane >> 4) + r; i = t * 16 + (lane & 15); }
    else { cc = c0p + ccol; i = t * 16 + 4 * (lane >> 4) + r; }
  };

  for (int pn = blockIdx.x; pn < npanels; pn += gridDim.x) {
    const int c0 = pn * kCols;
    __syncthreads();  // W staged; previous panel's readers are done
    // stage the panel (entries with j >= n, including the k padding, are zero)
    if constexpr (TRANS) {
#pragma unroll
      for (int s = 0; s < PER; ++s) {
        const int e = tid + kThreads * s;
        const int c = e / NPAD, j = e - c * NPAD;
        const int cc = c0 + c;
        const bool ok = cc < ncols && j < n;
        const TI v = X[ok ? (size_t)cc * n + j : 0];
        put(j, c, ok ? (float)v : 0.f);
      }
    } else {
      const int c = tid & (kCols - 1);
      const int cc = c0 + c;
      const bool okc = cc < ncols;
      const size_t b = okc ? (size_t)column_base(cc) : 0;
#pragma unroll
      for (int s = 0; s < PER; ++s) {
        const int j = (tid >> 6) + (kThreads / kCols) * s;
        const bool ok = okc && j < n;
        const TI v = X[ok ? b + (size_t)j * L : 0];
        put(j, c, ok ? (float)v : 0.f);
      }
    }
    if constexpr (KPAD > NPAD) {  // k padding beyond NPAD rows
      for (int e = tid; e < kCols * (KPAD - NPAD); e += kThreads) {
        const int c = e / (KPAD - NPAD), j = NPAD + e % (KPAD - NPAD);
        Xh[c * LDK + j] = 0;
        Xl[c * LDK + j] = 0;
      }
    }
    double ls = 1.0;
    if constexpr (TIME) ls = lam_s[min(c0 + ccol, ncols - 1)];
    double dv[DOT ? NM * 4 : 1];
    if constexpr (DOT) {
#pragma unroll
      for (int t = 0; t < NM; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int i, cc;
          out_pos(c0, t, r, i, cc);
          const bool ok = cc < ncols && i < n;
          const double v = dotv[ok ? (size_t)column_base(cc) + (size_t)i * L : 0];
          dv[t * 4 + r] = ok ? v : 0.0;
        }
    }
    __syncthreads();
    gemm(0);
    if constexpr (FUSED) {
      __syncthreads();  // all waves are done reading the panel
#pragma unroll
      for (int t = 0; t < NM; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = t * 16 + 4 * (lane >> 4) + r;
          const double v = (double)acc[t][r] / (lt[t * 4 + r] + ls);
          put(i, ccol, i < n ? (float)v : 0.f);
        }
      __syncthreads();
      gemm(1);
    }
#pragma unroll
    for (int t = 0; t < NM; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int i, cc;
        out_pos(c0, t, r, i, cc);
        TO v;
        if constexpr (DIV && !FUSED) v = (TO)((double)acc[t][r] / (lt[t * 4 + r] + ls));  // FP64, as the fused pass
        else v = (TO)acc[t][r];
        if constexpr (DOT) dsum += (double)v * dv[t * 4 + r];
        if (cc < ncols && i < n) Y[(size_t)column_base(cc) + (size_t)i * L] = v;
      }
  }
  if constexpr (DOT) {
    const double s = block_sum(dsum, red);
    if (tid == 0) partials[blockIdx.x] = s;
  }
}

// LDS bytes of the bf16 mode kernel: the operator (two for the fused time
// pass) in bf16 hi + lo with padded rows, and the panel.
static size_t bf16_shmem(const DevDir& D, bool fused) {
  const int nm = D.npad / 16;
  const int ldk = (nm + 1) / 2 * 32 + 8;
  return sizeof(unsigned short) * ((fused ? 2 : 1) * 2 * (size_t)D.npad * ldk + 2 * (size_t)kCols * ldk) +
         4 * sizeof(double) + 16;
}

template <typename TI, typename TO, bool TRANS, bool FUSED, bool DOT, bool DIV = false>
static int launch_fd_bf16(stls_ctx* h, const TI* X, TO* Y, int L, int n, int ncols, int k, bool fwd, int k2,
                          const double* lam_t, const double* dotv, double* partials, int* nparts) {
  const DevDir& D = h->dd[k];
  const int nm = D.npad / 16;
  const int nk = (nm + 1) / 2, kpad = nk * 32, ldk = kpad + 8;
  if (kpad != D.kpad) { set_error("bf16 operand padding mismatch"); return STLS_EINVAL; }
  const int npanels = (ncols + kCols - 1) / kCols;
  const size_t shmem = bf16_shmem(D, FUSED);
  if (shmem > 160 * 1024) { set_error("direction too large for the bf16 FD kernel"); return STLS_EINVAL; }
  const int per_cu = std::max(1, std::min(4, (int)((160 * 1024) / shmem)));
  const int blocks = std::min(npanels, 256 * per_cu);
  if (DOT && blocks > kPartialsCap) { set_error("too many partial sums"); return STLS_EINVAL; }
  if (nparts) *nparts = blocks;
  const unsigned short* Wh = fwd ? D.Hfwd : D.Hbwd;
  const unsigned short* Wl = fwd ? D.Lfwd : D.Lbwd;
  const unsigned short* W2h = FUSED ? h->dd[k2].Hbwd : nullptr;
  const unsigned short* W2l = FUSED ? h->dd[k2].Lbwd : nullptr;
  void (*kern)(const TI*, TO*, int, int, int, const unsigned short*, const unsigned short*, const unsigned short*,
               const unsigned short*, const double*, const double*, const double*, double*,
               const PcgScalars*) = nullptr;
#define STLS_BF_PICK(NMV) \
  case NMV: kern = fd_mode_bf16x3_kernel<TI, TO, NMV, TRANS, FUSED, DOT, DIV>; break;
  switch (nm) {
    STLS_BF_PICK(1) STLS_BF_PICK(2) STLS_BF_PICK(3) STLS_BF_PICK(4) STLS_BF_PICK(5) STLS_BF_PICK(6)
    STLS_BF_PICK(7) STLS_BF_PICK(8) STLS_BF_PICK(9) STLS_BF_PICK(10) STLS_BF_PICK(11) STLS_BF_PICK(12)
    STLS_BF_PICK(13) STLS_BF_PICK(14) STLS_BF_PICK(15) STLS_BF_PICK(16)
    default: set_error("direction too large for the bf16 FD kernel"); return STLS_EINVAL;
  }
#undef STLS_BF_PICK
  if (shmem > 65536) {
    hipError_t ea = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (ea != hipSuccess) return hip_fail(ea, "hipFuncSetAttribute(LDS)");
  }
  prof_begin(h);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(kThreads), shmem, h->stream, X, Y, L, n, ncols, Wh, Wl, W2h, W2l, lam_t,
                     h->lam_s, dotv, partials, h->gate);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "fd_mode_bf16x3_kernel launch");
  prof_end(h, (FUSED || k == h->d) ? PROF_FD_TIME : PROF_FD_SPACE);
  return STLS_OK;
}

// BF16x3 chain: FP32 intermediates, bf16 split products.
static int prec_apply_bf16x3(stls_ctx* h, const double* r, double* s, const double* dot_with, double* partials,
                             int* nparts) {
  const int d = h->d;
  const int nt = h->dir[d].n;
  const int ns = (int)h->ns;
  float* buf[2] = {reinterpret_cast<float*>(h->fdbuf[0]), reinterpret_cast<float*>(h->fdbuf[1])};
  int st, cur = 0, L = 1;
  for (int k = 0; k < d; ++k) {
    const int n = h->dir[k].n;
    const int ncols = (int)(h->ndof / n);
    if (k == 0) st = launch_fd_bf16<double, float, true, false, false>(h, r, buf[cur], L, n, ncols, k, true, 0, nullptr,
                                                                      nullptr, nullptr, nullptr);
    else {
      st = launch_fd_bf16<float, float, false, false, false>(h, buf[cur], buf[cur ^ 1], L, n, ncols, k, true, 0,
                                                             nullptr, nullptr, nullptr, nullptr);
      cur ^= 1;
    }
    if (st) return st;
    L *= n;
  }
  if (bf16_shmem(h->dd[d], true) <= 160 * 1024) {
    st = launch_fd_bf16<float, float, false, true, false>(h, buf[cur], buf[cur ^ 1], ns, nt, ns, d, true, d,
                                                          h->dd[d].lam, nullptr, nullptr, nullptr);
    if (st) return st;
    cur ^= 1;
  } else {
    // the two time operators do not fit in LDS together (n_t > 128): the
    // forward product with the division, then the backward product
    st = launch_fd_bf16<float, float, false, false, false, true>(h, buf[cur], buf[cur ^ 1], ns, nt, ns, d, true, 0,
                                                                 h->dd[d].lam, nullptr, nullptr, nullptr);
    if (st) return st;
    cur ^= 1;
    st = launch_fd_bf16<float, float, false, false, false>(h, buf[cur], buf[cur ^ 1], ns, nt, ns, d, false, 0,
                                                           nullptr, nullptr, nullptr, nullptr);
    if (st) return st;
    cur ^= 1;
  }
  for (int k = d - 1; k >= 0; --k) {
    const int n = h->dir[k].n;
    L /= n;
    const int ncols = (int)(h->ndof / n);
    if (k == 0)
      st = dot_with ? launch_fd_bf16<float, double, true, false, true>(h, buf[cur], s, L, n, ncols, k, false, 0,
                                                                       nullptr, dot_with, partials, nparts)
                    : launch_fd_bf16<float, double, true, false, false>(h, buf[cur], s, L, n, ncols, k, false, 0,
                                                                        nullptr, nullptr, nullptr, nparts);
    else {
      st = launch_fd_bf16<float, float, false, false, false>(h, buf[cur], buf[cur ^ 1], L, n, ncols, k, false, 0,
                                                             nullptr, nullptr, nullptr, nullptr);
      cur ^= 1;
    }
    if (st) return st;
  }
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
  int L = 1;
  for (int k = 0; k < d; ++k) {
    const int n = h->dir[k].n;
    const int ncols = (int)(h->ndof / n);
    if (k == 0)
      st = launch_fd_mode<TC, double, TC, true, false, false>(h, r, buf[cur], L, n, ncols, fwdA(k), nullptr,
                                                              h->dd[k].npad, nullptr, nullptr, nullptr, nullptr);
    else {
      st = launch_fd_mode<TC, TC, TC, false, false, false>(h, buf[cur], buf[cur ^ 1], L, n, ncols, fwdA(k), nullptr,
                                                           h->dd[k].npad, nullptr, nullptr, nullptr, nullptr);
      cur ^= 1;
    }
    if (st) return st;
    L *= n;
  }
  st = launch_fd_mode<TC, TC, TC, false, true, false>(h, buf[cur], buf[cur ^ 1], ns, nt, ns, fwdA(d), bwdA(d),
                                                      h->dd[d].npad, h->dd[d].lam, nullptr, nullptr, nullptr);
  if (st) return st;
  cur ^= 1;
  for (int k = d - 1; k >= 0; --k) {
    const int n = h->dir[k].n;
    L /= n;
    const int ncols = (int)(h->ndof / n);
    if (k == 0)
      st = dot_with ? launch_fd_mode<TC, TC, double, true, false, true>(h, buf[cur], s, L, n, ncols, bwdA(k), nullptr,
                                                                        h->dd[k].npad, nullptr, dot_with, partials,
                                                                        nparts)
                    : launch_fd_mode<TC, TC, double, true, false, false>(h, buf[cur], s, L, n, ncols, bwdA(k),
                                                                         nullptr, h->dd[k].npad, nullptr, nullptr,
                                                                         nullptr, nparts);
    else {
      st = launch_fd_mode<TC, TC, TC, false, false, false>(h, buf[cur], buf[cur ^ 1], L, n, ncols, bwdA(k), nullptr,
                                                           h->dd[k].npad, nullptr, nullptr, nullptr, nullptr);
      cur ^= 1;
    }
    if (st) return st;
  }
  return STLS_OK;
}

// Asymmetric chain: the forward space products in FP32 (MFMA f32, FP32
// intermediates); the fused time pass (both time products and the
// eigenvalue division) and the backward space products in FP64.  Rounding in
// the backward half is what costs PCG iterations; the forward half tolerates
// FP32 with little effect on the count.
static int prec_apply_asym(stls_ctx* h, const double* r, double* s, const double* dot_with, double* partials,
                           int* nparts) {
  const int d = h->d;
  const int nt = h->dir[d].n;
  const int ns = (int)h->ns;
  float* fb[2] = {reinterpret_cast<float*>(h->fdbuf[0]), reinterpret_cast<float*>(h->fdbuf[1])};
  double* db[2] = {h->fdbuf[0], h->fdbuf[1]};
  int st, cur = 0, L = 1;
  for (int k = 0; k < d; ++k) {
    const int n = h->dir[k].n;
    const int ncols = (int)(h->ndof / n);
    if (k == 0)
      st = launch_fd_mode<float, double, float, true, false, false>(h, r, fb[cur], L, n, ncols, h->dd[k].Afwd32,
                                                                    nullptr, h->dd[k].npad, nullptr, nullptr, nullptr,
                                                                    nullptr);
    else {
      st = launch_fd_mode<float, float, float, false, false, false>(h, fb[cur], fb[cur ^ 1], L, n, ncols,
                                                                    h->dd[k].Afwd32, nullptr, h->dd[k].npad, nullptr,
                                                                    nullptr, nullptr, nullptr);
      cur ^= 1;
    }
    if (st) return st;
    L *= n;
  }
  st = launch_fd_mode<double, float, double, false, true, false>(h, fb[cur], db[cur ^ 1], ns, nt, ns, h->dd[d].Afwd64,
                                                                 h->dd[d].Abwd64, h->dd[d].npad, h->dd[d].lam, nullptr,
                                                                 nullptr, nullptr);
  if (st) return st;
  cur ^= 1;
  for (int k = d - 1; k >= 0; --k) {
    const int n = h->dir[k].n;
    L /= n;
    const int ncols = (int)(h->ndof / n);
    if (k == 0)
      st = dot_with ? launch_fd_mode<double, double, double, true, false, true>(h, db[cur], s, L, n, ncols,
                                                                                h->dd[k].Abwd64, nullptr, h->dd[k].npad,
                                                                                nullptr, dot_with, partials, nparts)
                    : launch_fd_mode<double, double, double, true, false, false>(h, db[cur], s, L, n, ncols,
                                                                                 h->dd[k].Abwd64, nullptr,
                                                                                 h->dd[k].npad, nullptr, nullptr,
                                                                                 nullptr, nparts);
    else {
      st = launch_fd_mode<double, double, double, false, false, false>(h, db[cur], db[cur ^ 1], L, n, ncols,
                                                                       h->dd[k].Abwd64, nullptr, h->dd[k].npad,
                                                                       nullptr, nullptr, nullptr, nullptr);
      cur ^= 1;
    }
    if (st) return st;
  }
  return STLS_OK;
}

// Diagonal scaling around the FD chains (§4.4, closing definition):
// y_i = sigma_i x_i with sigma_i = (P_ii / A_ii)^1/2 in FP64, the multi-index
// decoded from the colex position; optional partial sums of y . dotv (one
// per block).  x and y may alias.
constexpr int kScaleBlocks = 2048;
template <bool DOT>
__global__ __launch_bounds__(kThreads) void diag_scale_kernel(const double* x, double* y, int64_t n, DiagScale S,
                                                              const double* __restrict__ dotv,
                                                              double* __restrict__ partials,
                                                              const PcgScalars* __restrict__ gate) {
  if (gate && (gate->done | gate->flag)) return;  // PCG already finished: nothing to do
  __shared__ double red[kThreads / 64];
  double dsum = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    int idx[kMaxDim + 1];
    int64_t rest = i;
#pragma unroll
    for (int k = 0; k <= kMaxDim; ++k) {
      if (k > S.d) break;
      idx[k] = (int)(rest % S.n[k]);
      rest /= S.n[k];
    }
    double Pm, Pj, Ek, Em;
    diag_row_coeffs<double>(S, S.g, idx, Pm, Pj, Ek, Em);
    const double* g1 = S.g + S.off[0];
    const int i1 = idx[0];
    const double v = diag_sigma(g1[i1], g1[S.n[0] + i1], g1[2 * S.n[0] + i1], Pm, Pj, Ek, Em) * x[i];
    y[i] = v;
    if constexpr (DOT) dsum += v * dotv[i];
  }
  if constexpr (DOT) {
    const double t = block_sum(dsum, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
  }
}

static int launch_diag_scale(stls_ctx* h, const double* x, double* y, const double* dot_with, double* partials,
                             int* nparts) {
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((h->ndof + kThreads - 1) / kThreads, kScaleBlocks));
  const DiagScale S = diag_scale_args(h);
  prof_begin(h);
  if (dot_with)
    hipLaunchKernelGGL(diag_scale_kernel<true>, dim3(blocks), dim3(kThreads), 0, h->stream, x, y, h->ndof, S,
                       dot_with, partials, h->gate);
  else
    hipLaunchKernelGGL(diag_scale_kernel<false>, dim3(blocks), dim3(kThreads), 0, h->stream, x, y, h->ndof, S,
                       nullptr, nullptr, h->gate);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "diag_scale_kernel launch");
  prof_end(h, PROF_MISC);
  if (nparts) *nparts = blocks;
  return STLS_OK;
}

static int prec_apply_plain(stls_ctx* h, const double* r, double* s, const double* dot_with, double* partials,
                            int* nparts) {
  switch (h->fd_mode) {
    case STLS_FD_FP64: return prec_apply_t<double>(h, r, s, dot_with, partials, nparts);
    case STLS_FD_FP32: return prec_apply_t<float>(h, r, s, dot_with, partials, nparts);
    case STLS_FD_BF16X3: return prec_apply_bf16x3(h, r, s, dot_with, partials, nparts);
    case STLS_FD_ASYM: return prec_apply_asym(h, r, s, dot_with, partials, nparts);
    default: set_error("FD precision mode not available"); return STLS_EINVAL;
  }
}

int launch_prec_apply(stls_ctx* h, const double* r, double* s, const double* dot_with, double* partials,
                      int* nparts) {
  if (h->geometry && h->sigma) {
    // P^G on a mapped domain: sigma o r, the chain with the weighted
    // factors, sigma o s in place with the dot product
    double* tmp = h->work[0];
    int st = launch_mapped_scale(h, r, tmp, nullptr, nullptr, nullptr);
    if (!st)
      st = fd_five_pass_covers(h) ? prec_apply_five_pass(h, tmp, s, nullptr, nullptr, nullptr, false)
                                  : prec_apply_plain(h, tmp, s, nullptr, nullptr, nullptr);
    if (!st) st = launch_mapped_scale(h, s, s, dot_with, partials, nparts);
    return st;
  }
  if (fd_five_pass_covers(h))
    return prec_apply_five_pass(h, r, s, dot_with, partials, nparts, h->fd_scale);  // scaling fused
  if (!h->fd_scale) return prec_apply_plain(h, r, s, dot_with, partials, nparts);
  // scaled: sigma o r into a matvec intermediate (free while the FD runs),
  // the chain, then sigma o s in place with the dot product
  double* tmp = h->work[0];
  int st = launch_diag_scale(h, r, tmp, nullptr, nullptr, nullptr);
  if (!st) st = prec_apply_plain(h, tmp, s, nullptr, nullptr, nullptr);
  if (!st) st = launch_diag_scale(h, s, s, dot_with, partials, nparts);
  return st;
}

// ---------------------------------------------------------------------------
// Matrix-free matvec y = (K_t x M_s + kappa^2 M_t x J_s + kappa W_t x L_s) x
// on the unit box (§4.1 eq. A_kron with the diffusivity).  On the
// Dirichlet-restricted space int b_i'' b_j = -int b_i' b_j', so the mixed
// second-derivative terms of J_s are K_k x K_l:
//   J_s = sum_k (J_k, M elsewhere) + 2 sum_{k<l} (K_k, K_l, M elsewhere),
//   L_s = sum_k (K_k, M elsewhere).
// Grouped by the operator of the last space direction d and time:
//   inner (directions < d):  A = (M..M) x,  B = (J_s part of dirs < d) x,
//                            C = (L_s part of dirs < d) x
//   outer ((i_d, t) plane):  S1 = M_d A,  S2 = kappa^2 (J_d A + M_d B + 2 K_d C),
//                            y  = K_t S1 + M_t S2 + e_T (x) kappa w (K_d A + M_d C)
// d = 1 has no inner stage (A = x, B = C = 0).  Banded factors are stored
// n x (2p+1) row-major, zero outside the matrix.

// Inner stage, d = 2: banded products along contiguous columns of n1.
constexpr int kInnerChunk = 1024;
__global__ __launch_bounds__(kThreads) void mv_inner1_kernel(const double* __restrict__ x, double* __restrict__ A,
                                                             double* __restrict__ B, double* __restrict__ C, int n1,
                                                             int N, int p, const double* __restrict__ Mb,
                                                             const double* __restrict__ Jb,
                                                             const double* __restrict__ Kb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int bw = 2 * p + 1;
  double* xs = reinterpret_cast<double*>(smem_raw);
  double* bM = xs + kInnerChunk + 2 * p;
  double* bJ = bM + n1 * bw;
  double* bK = bJ + n1 * bw;
  for (int t = threadIdx.x; t < n1 * bw; t += kThreads) { bM[t] = Mb[t]; bJ[t] = Jb[t]; bK[t] = Kb[t]; }
  const int nchunks = (N + kInnerChunk - 1) / kInnerChunk;
  for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const int e0 = ch * kInnerChunk;
    __syncthreads();
    for (int t = threadIdx.x; t < kInnerChunk + 2 * p; t += kThreads) {
      const int g = e0 - p + t;
      xs[t] = (g >= 0 && g < N) ? x[g] : 0.0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kInnerChunk; t += kThreads) {
      const int e = e0 + t;
      if (e >= N) break;
      const int i = e % n1;
      double a = 0.0, b = 0.0, c = 0.0;
      for (int o = 0; o < bw; ++o) {
        const int j = i + o - p;
        if (j < 0 || j >= n1) continue;
        const double v = xs[t + o];
        a += bM[i * bw + o] * v;
        b += bJ[i * bw + o] * v;
        c += bK[i * bw + o] * v;
      }
      A[e] = a;
      B[e] = b;
      C[e] = c;
    }
  }
}

// Inner stage, d = 3: one workgroup per (i3, t) slab and chunk of T2 rows in
// i2; direction-1 products for the rows of the chunk plus a halo of p2 rows,
// then direction-2 products:
//   A = M2 (M1 x),  B = J2 (M1 x) + M2 (J1 x) + 2 K2 (K1 x),  C = K2 (M1 x) + M2 (K1 x)
// Lanes run along i1 (contiguous), the four waves along rows.  P > 0: both
// degrees equal P, direction-1 band rows live in registers; P = 0: runtime
// degrees.  Row indices are wave-uniform, so direction-2 coefficients come
// through scalar loads.
constexpr int kInnerPf = 8;

template <int P>
__global__ __launch_bounds__(kThreads) void mv_inner12_kernel(
    const double* __restrict__ x, double* __restrict__ A, double* __restrict__ B, double* __restrict__ C, int n1,
    int n2, int T2, int ntile2, int nwork, int p1r, int p2r, const double* __restrict__ M1,
    const double* __restrict__ J1, const double* __restrict__ K1, const double* __restrict__ M2,
    const double* __restrict__ J2, const double* __restrict__ K2) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int p1 = P > 0 ? P : p1r, p2 = P > 0 ? P : p2r;
  const int bw1 = 2 * p1 + 1, bw2 = 2 * p2 + 1;
  const int hmax = min(n2, T2 + 2 * p2);
  double* xs = reinterpret_cast<double*>(smem_raw);  // hmax x n1
  double* XM = xs + hmax * n1;
  double* XJ = XM + hmax * n1;
  double* XK = XJ + hmax * n1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int BW = P > 0 ? 2 * P + 1 : 1;
  double cM[BW], cJ[BW], cK[BW];
  // The chunk of x of the next work item is fetched into registers while the
  // current one is processed (hmax * n1 <= kInnerPf * kThreads by the LDS budget).
  double pf[kInnerPf];
  auto fetch = [&](int wi_) {
    const int w_ = xcd_tile(wi_, nwork);
    const int slab_ = w_ / ntile2, tile_ = w_ - slab_ * ntile2;
    const int r0_ = tile_ * T2, r1_ = min(n2, r0_ + T2);
    const int h0_ = max(0, r0_ - p2), nh_ = min(n2, r1_ + p2) - h0_;
    const size_t off = (size_t)slab_ * n1 * n2 + (size_t)h0_ * n1;
#pragma unroll
    for (int s = 0; s < kInnerPf; ++s) {
      const int t = threadIdx.x + kThreads * s;
      const bool ok = t < nh_ * n1;
      const double v = x[off + (ok ? t : 0)];
      pf[s] = ok ? v : 0.0;
    }
  };
  if (blockIdx.x < nwork) fetch(blockIdx.x);
  for (int wi = blockIdx.x; wi < nwork; wi += gridDim.x) {
    const int w = xcd_tile(wi, nwork);
    const int slab = w / ntile2, tile = w - slab * ntile2;
    const int r0 = tile * T2, r1 = min(n2, r0 + T2);
    const int h0 = max(0, r0 - p2), h1 = min(n2, r1 + p2), nh = h1 - h0;
    const size_t base = (size_t)slab * n1 * n2;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kInnerPf; ++s) {
      const int t = threadIdx.x + kThreads * s;
      if (t < nh * n1) xs[t] = pf[s];
    }
    __syncthreads();
    if (wi + (int)gridDim.x < nwork) fetch(wi + gridDim.x);
    for (int i1 = lane; i1 < n1; i1 += 64) {
      if constexpr (P > 0) {
#pragma unroll
        for (int o = 0; o < BW; ++o) {
          cM[o] = M1[i1 * BW + o]; cJ[o] = J1[i1 * BW + o]; cK[o] = K1[i1 * BW + o];
        }
      }
      for (int row = wave; row < nh; row += kThreads / 64) {
        double m = 0.0, jj = 0.0, kk = 0.0;
        if constexpr (P > 0) {
#pragma unroll
          for (int o = 0; o < BW; ++o) {
            // band entries outside the matrix are stored as zeros: clamp the
            // column so that every LDS read stays inside the slab
            const int j = min(max(i1 + o - P, 0), n1 - 1);
            const double v = xs[row * n1 + j];
            m += cM[o] * v; jj += cJ[o] * v; kk += cK[o] * v;
          }
        } else {
          for (int o = 0; o < bw1; ++o) {
            const int j = i1 + o - p1;
            if (j < 0 || j >= n1) continue;
            const double v = xs[row * n1 + j];
            m += M1[i1 * bw1 + o] * v; jj += J1[i1 * bw1 + o] * v; kk += K1[i1 * bw1 + o] * v;
          }
        }
        XM[row * n1 + i1] = m;
        XJ[row * n1 + i1] = jj;
        XK[row * n1 + i1] = kk;
      }
    }
    __syncthreads();
    for (int rr = wave; rr < r1 - r0; rr += kThreads / 64) {
      const int i2 = __builtin_amdgcn_readfirstlane(r0 + rr);  // wave-uniform row
      for (int i1 = lane; i1 < n1; i1 += 64) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int o = 0; o < bw2; ++o) {
          const int j2 = i2 + o - p2;
          if (j2 < 0 || j2 >= n2) continue;
          const int hr = (j2 - h0) * n1 + i1;
          const double m = XM[hr], jv = XJ[hr], kv = XK[hr];
          const double cm = M2[i2 * bw2 + o], cj = J2[i2 * bw2 + o], ck = K2[i2 * bw2 + o];
          a += cm * m;
          b += cj * m + cm * jv + 2.0 * ck * kv;
          c += ck * m + cm * kv;
        }
        const size_t g = base + (size_t)i2 * n1 + i1;
        A[g] = a;
        B[g] = b;
        C[g] = c;
      }
    }
  }
}

// Outer stage.  A workgroup owns 16 consecutive inner indices l (one 128-byte
// run per row) x Td rows of i_d x a chunk [c0, c1) of output time slices.  It
// streams the input slices t in [c0 - PT, c1 + PT): slice t + 2 is being
// loaded into registers while slice t + 1 waits in LDS and slice t is
// processed (3-slot LDS ring).  Every thread keeps for its (l, i_d) pencil a
// window of S1, S2 over 2 PT + 1 slices and emits
//   y(t') = sum_k K_t(t', t'-PT+k) S1w[k] + M_t(t', t'-PT+k) S2w[k]
// once slice t' + PT is in.  The final-time term and the partial dot product
// y . dotv are fused.  PD > 0: space degree PD known at compile time (band
// rows of the thread's i_d in registers); PD = 0: runtime space degree.
constexpr int kOuterLb = 16;             // inner indices per workgroup
constexpr int kOuterLds = kOuterLb;      // LDS row: 16 doubles, two rows per half wave fill the banks
constexpr int kOuterMaxTd = 16;
constexpr int kOuterSlots = 2;           // staged rows per thread and input: rows <= 32

template <int PT, int PD, bool THREE, bool DOT>
__global__ __launch_bounds__(kThreads) void mv_outer_kernel(
    const double* __restrict__ A, const double* __restrict__ B, const double* __restrict__ C, double* __restrict__ y,
    int L, int nd, int nt, int pdr, int Td, int nlb, int ntd, int nchunk, int Tc, const double* __restrict__ Md,
    const double* __restrict__ Jd, const double* __restrict__ Kd, const double* __restrict__ Kt,
    const double* __restrict__ Mt, double k2, double kw, const double* __restrict__ dotv,
    double* __restrict__ partials) {
  constexpr int W = 2 * PT + 1;
  constexpr int BWD = PD > 0 ? 2 * PD + 1 : 1;
  constexpr int NQ = THREE ? 3 : 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[4];
  const int pd = PD > 0 ? PD : pdr;
  const int bwd = 2 * pd + 1;
  const int rows = Td + 2 * pd;
  double* bands = reinterpret_cast<double*>(smem_raw);  // Md | Jd | Kd, nd x bwd each (PD == 0)
  double* sbuf = bands + (PD > 0 ? 0 : 3 * nd * bwd);    // 3 slots x (NQ x rows x kOuterLds)
  const int buf_stride = NQ * rows * kOuterLds;
  if (PD == 0)
    for (int t = threadIdx.x; t < nd * bwd; t += kThreads) {
      bands[t] = Md[t]; bands[nd * bwd + t] = Jd[t]; bands[2 * nd * bwd + t] = Kd[t];
    }
  const int ntile = nlb * ntd * nchunk;
  const int tile = xcd_tile(blockIdx.x, ntile);
  const int td = tile % ntd;
  const int lb = (tile / ntd) % nlb;
  const int ch = tile / (ntd * nlb);
  const int l0 = lb * kOuterLb, d0 = td * Td;
  const int c0 = ch * Tc, c1 = min(nt, c0 + Tc);
  const int li = threadIdx.x % kOuterLb, di = threadIdx.x / kOuterLb;
  const int l = l0 + li, id = d0 + di;
  const bool mine = (di < Td) && (l < L) && (id < nd);
  // clamped coordinates: threads outside the tile compute on valid data and
  // their results are discarded, so the loop has no divergent branches
  const int dic = min(di, Td - 1), idc = min(id, nd - 1), lc = min(l, L - 1);
  const size_t plane = (size_t)L * nd;  // one time slice

  // staging coordinates of this thread: lane li, staged rows di + 16 s
  int soff[kOuterSlots];
  bool sok[kOuterSlots];
#pragma unroll
  for (int s = 0; s < kOuterSlots; ++s) {
    const int rr = di + kOuterMaxTd * s;
    const int row = d0 - pd + rr;
    sok[s] = rr < rows && row >= 0 && row < nd && l < L;
    soff[s] = sok[s] ? row * L + l : 0;
  }
  double cm[BWD], cj[BWD], ck[BWD];
  if constexpr (PD > 0) {
#pragma unroll
    for (int o = 0; o < BWD; ++o) {
      cm[o] = Md[idc * BWD + o];
      cj[o] = Jd[idc * BWD + o];
      ck[o] = Kd[idc * BWD + o];
    }
  }
  auto load_slice = [&](int t, double (&regs)[NQ][kOuterSlots]) {
    const size_t tb0 = (size_t)t * plane;
#pragma unroll
    for (int s = 0; s < kOuterSlots; ++s) {
      const size_t g = tb0 + soff[s];
      const double a = A[g];
      regs[0][s] = sok[s] ? a : 0.0;
      if constexpr (THREE) {
        const double bv = B[g], cv = C[g];
        regs[1][s] = sok[s] ? bv : 0.0;
        regs[2][s] = sok[s] ? cv : 0.0;
      }
    }
  };
  auto park_slice = [&](const double (&regs)[NQ][kOuterSlots], double* buf) {
#pragma unroll
    for (int s = 0; s < kOuterSlots; ++s) {
      const int rr = di + kOuterMaxTd * s;
      if (rr < rows) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) buf[q * rows * kOuterLds + rr * kOuterLds + li] = regs[q][s];
      }
    }
  };

  double S1w[W], S2w[W];
#pragma unroll
  for (int k = 0; k < W; ++k) { S1w[k] = 0.0; S2w[k] = 0.0; }
  double S3 = 0.0, dsum = 0.0;
  const int tb = max(0, c0 - PT);   // first input slice (tb < nt)
  const int te = c1 - 1 + PT;       // last window position (inputs beyond nt are zero)
  const int tl = min(te, nt - 1);   // last input slice
  double ra[NQ][kOuterSlots], rb[NQ][kOuterSlots];
  load_slice(tb, ra);
  __syncthreads();  // bands in LDS
  park_slice(ra, sbuf);
  load_slice(min(tb + 1, tl), ra);
  __syncthreads();
  // One input slice: prefetch slice t + 2 into `nxt`, process slice t from
  // LDS, park slice t + 1 (held in `cur`).  The loop is unrolled by two with
  // the register sets swapped so that no copy forces an early wait.
  auto step = [&](int t, double (&nxt)[NQ][kOuterSlots], double (&cur)[NQ][kOuterSlots]) {
    const int tp = t - PT;  // output slice completed by this input
    // operand of the fused dot product, requested before the slice prefetch
    double dvv = 0.0;
    const size_t gout = (size_t)max(tp, 0) * plane + (size_t)idc * L + lc;
    if constexpr (DOT) dvv = dotv[gout];
    load_slice(min(t + 2, tl), nxt);  // unconditional: a repeated load at the end is harmless
    const double* buf = sbuf + ((t - tb) % 3) * buf_stride;
    double s1 = 0.0, jA = 0.0, mB = 0.0, kC = 0.0;
    auto tap = [&](int o, double m_, double j_, double k_) {
      const int rr = dic + o;  // staged row of i_d + o - pd
      const double a = buf[rr * kOuterLds + li];
      s1 += m_ * a;
      jA += j_ * a;
      if constexpr (THREE) {
        mB += m_ * buf[rows * kOuterLds + rr * kOuterLds + li];
        kC += k_ * buf[2 * rows * kOuterLds + rr * kOuterLds + li];
      }
    };
    if constexpr (PD > 0) {
#pragma unroll
      for (int o = 0; o < BWD; ++o) tap(o, cm[o], cj[o], ck[o]);
    } else {
      for (int o = 0; o < bwd; ++o)
        tap(o, bands[idc * bwd + o], bands[nd * bwd + idc * bwd + o], bands[2 * nd * bwd + idc * bwd + o]);
    }
    const bool have = t < nt;
    double s2 = k2 * (jA + mB + 2.0 * kC);
    s1 = have ? s1 : 0.0;
    s2 = have ? s2 : 0.0;
    if (t == nt - 1) {  // final-time term kappa w (K_d A + M_d C) (uniform branch, LDS only)
      double kA = 0.0, mC = 0.0;
      if constexpr (PD > 0) {
#pragma unroll
        for (int o = 0; o < BWD; ++o) {
          kA += ck[o] * buf[(dic + o) * kOuterLds + li];
          if constexpr (THREE) mC += cm[o] * buf[2 * rows * kOuterLds + (dic + o) * kOuterLds + li];
        }
      } else {
        for (int o = 0; o < bwd; ++o) {
          kA += bands[2 * nd * bwd + idc * bwd + o] * buf[(dic + o) * kOuterLds + li];
          if constexpr (THREE) mC += bands[idc * bwd + o] * buf[2 * rows * kOuterLds + (dic + o) * kOuterLds + li];
        }
      }
      S3 = kw * (kA + mC);
    }
#pragma unroll
    for (int k = 0; k < W - 1; ++k) { S1w[k] = S1w[k + 1]; S2w[k] = S2w[k + 1]; }
    S1w[W - 1] = s1;
    S2w[W - 1] = s2;
    if (tp >= c0 && tp < c1) {  // uniform
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < W; ++k) v += Kt[tp * W + k] * S1w[k] + Mt[tp * W + k] * S2w[k];
      if (tp == nt - 1) v += S3;
      if constexpr (DOT) dsum += mine ? v * dvv : 0.0;
      if (mine) y[gout] = v;
    }
    park_slice(cur, sbuf + ((t + 1 - tb) % 3) * buf_stride);
    __syncthreads();
  };
  for (int t = tb; t <= te; t += 2) {
    step(t, rb, ra);
    if (t + 1 <= te) step(t + 1, ra, rb);
  }
  if constexpr (DOT) {
    const double s = block_sum(dsum, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

// Inner stage, d = 3, one whole (i3, t) slab per work item (n1, n2 <= 64).
// The slab of x is kept transposed in LDS (xT[i1][i2]) so that the
// direction-1 products run with lanes along i2 and a wave-uniform run of R1
// columns i1: the band coefficients of those columns are uniform and come
// through scalar loads, and the R1 + 2P input columns are read once for R1
// outputs.  The direction-2 products run with lanes along i1 (coalesced
// stores) and a wave-uniform run of R2 rows, again with scalar coefficients.
// Both band operators are applied with clamped, branch-free taps: entries
// outside the matrix are stored as zeros.  The next slab of x is fetched into
// registers while the current one is processed.
constexpr int kSlabWaves = 8;
constexpr int kSlabR1 = 7;
constexpr int kSlabR2 = 2;

template <int P>
__global__ __launch_bounds__(kSlabWaves * 64) void mv_inner_slab_kernel(
    const double* __restrict__ x, double* __restrict__ A, double* __restrict__ B, double* __restrict__ C, int n1,
    int n2, int nslab, int ld, const double* __restrict__ M1, const double* __restrict__ J1,
    const double* __restrict__ K1, const double* __restrict__ M2, const double* __restrict__ J2,
    const double* __restrict__ K2) {
  constexpr int BW = 2 * P + 1;
  constexpr int NW = kSlabWaves, R1 = kSlabR1, R2 = kSlabR2;
  constexpr int PF = 64 / NW;  // rows of the slab fetched per wave (n2 <= 64)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* xT = reinterpret_cast<double*>(smem_raw);  // n1 x n2
  double* XM = xT + n1 * n2;                         // n2 x ld each
  double* XJ = XM + n2 * ld;
  double* XK = XJ + n2 * ld;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ns = n1 * n2;
  const int i1l = min(lane, n1 - 1);
  double pf[PF];
  auto fetch = [&](int s) {
    const double* xs = x + (size_t)s * ns;
#pragma unroll
    for (int k = 0; k < PF; ++k) pf[k] = xs[min(wave + NW * k, n2 - 1) * n1 + i1l];
  };
  int s = blockIdx.x;
  if (s < nslab) fetch(s);
  const int nb1 = (n1 + R1 - 1) / R1;
  const int nb2 = (n2 + R2 - 1) / R2;
  const int i2 = lane, i2c = min(lane, n2 - 1);
  for (; s < nslab; s += gridDim.x) {
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int row = wave + NW * k;
      if (row < n2 && lane < n1) xT[lane * n2 + row] = pf[k];
    }
    __syncthreads();
    if (s + (int)gridDim.x < nslab) fetch(s + gridDim.x);
    // direction 1: XM = M1 x, XJ = J1 x, XK = K1 x along i1
    for (int it = wave; it < nb1; it += NW) {
      const int c0 = it * R1;
      double v[R1 + 2 * P];
#pragma unroll
      for (int j = 0; j < R1 + 2 * P; ++j) v[j] = xT[min(max(c0 - P + j, 0), n1 - 1) * n2 + i2c];
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        const int c = min(c0 + r, n1 - 1);
        const double* cm = M1 + c * BW;
        const double* cj = J1 + c * BW;
        const double* ck = K1 + c * BW;
        double m = 0.0, jj = 0.0, kk = 0.0;
#pragma unroll
        for (int o = 0; o < BW; ++o) {
          m += cm[o] * v[r + o];
          jj += cj[o] * v[r + o];
          kk += ck[o] * v[r + o];
        }
        if (i2 < n2 && c0 + r < n1) {
          XM[i2 * ld + c] = m;
          XJ[i2 * ld + c] = jj;
          XK[i2 * ld + c] = kk;
        }
      }
    }
    __syncthreads();
    // direction 2: A = M2 XM, B = J2 XM + M2 XJ + 2 K2 XK, C = K2 XM + M2 XK along i2
    const size_t base = (size_t)s * ns;
    for (int it = wave; it < nb2; it += NW) {
      const int r0 = it * R2;
      double m[R2 + 2 * P], jv[R2 + 2 * P], kv[R2 + 2 * P];
#pragma unroll
      for (int j = 0; j < R2 + 2 * P; ++j) {
        const int row = min(max(r0 - P + j, 0), n2 - 1);
        m[j] = XM[row * ld + i1l];
        jv[j] = XJ[row * ld + i1l];
        kv[j] = XK[row * ld + i1l];
      }
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        const int rr = min(r0 + r, n2 - 1);
        const double* cm = M2 + rr * BW;
        const double* cj = J2 + rr * BW;
        const double* ck = K2 + rr * BW;
        // independent partial sums (short dependent FMA chains)
        double a = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0, c1 = 0.0, c2 = 0.0;
#pragma unroll
        for (int o = 0; o < BW; ++o) {
          a += cm[o] * m[r + o];
          b1 += cj[o] * m[r + o];
          b2 += cm[o] * jv[r + o];
          b3 += ck[o] * kv[r + o];
          c1 += ck[o] * m[r + o];
          c2 += cm[o] * kv[r + o];
        }
        const double b = (b1 + b2) + 2.0 * b3, c = c1 + c2;
        if (lane < n1 && r0 + r < n2) {
          const size_t g = base + (size_t)(r0 + r) * n1 + lane;
          A[g] = a;
          B[g] = b;
          C[g] = c;
        }
      }
    }
  }
}

// Outer stage with a direct-to-LDS load pipeline.  Workgroup = 4 waves, one
// (l, i_d) pencil per thread (16 consecutive l x up to 16 rows i_d); it walks
// the time slices of its chunk.  Each time slice of A, B, C (rows
// d0-P .. d0+Td+P-1) and the slice t-PT of the dot operand are copied
// global -> LDS by global_load_lds (16 B per lane, 8 rows of 16 l per wave
// instruction) into a ring of kDmaSlots slots, kDmaSlots-1 slices ahead of
// use.  Every wave issues exactly K copies per slice (surplus copies land in
// a trash block), so that "slice t has arrived" is s_waitcnt vmcnt((D-2) K):
// loads return in issue order, and only the copies of later slices may still
// be outstanding.  Lanes past the staged rows read the first row of their
// copy (a cache line that is fetched anyway).  Requires L even (16 B source
// alignment of l pairs).
//   space (i_d): s1 = M_d A, s2 = kappa^2 (J_d A + M_d B + 2 K_d C)
//   time:        y(t') = sum_t K_t(t', t) s1(t) + M_t(t', t) s2(t), scattered
//                into 2 PT + 1 accumulators as slice t arrives
//   final time:  y(T) += kappa w (K_d A + M_d C)(T)
typedef __attribute__((address_space(3))) void lds_void_t;
constexpr int kDmaSlots = 4;
constexpr int kDmaLb = 16;

template <int N>
__device__ inline void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  // gfx9 s_waitcnt: vmcnt in bits 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at their maxima
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

template <int PT, int P, int K, bool DOT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void mv_outer_dma_kernel(
    const double* __restrict__ A, const double* __restrict__ B, const double* __restrict__ C, double* __restrict__ y,
    int L, int nd, int nt, int Td, int nlb, int ntd, int nchunk, int Tc, const double* __restrict__ Md,
    const double* __restrict__ Jd, const double* __restrict__ Kd, const double* __restrict__ Kt,
    const double* __restrict__ Mt, double k2, double kw, const double* __restrict__ dotv,
    double* __restrict__ partials) {
  constexpr int W = 2 * PT + 1;
  constexpr int BW = 2 * P + 1;
  constexpr int LB = kDmaLb;
  constexpr int D = kDmaSlots;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sm = reinterpret_cast<double*>(smem_raw);
  __shared__ double red[4];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // row tiles fastest: the tiles sharing halo rows run together on one XCD
  const int ntile = nlb * ntd * nchunk;
  const int tile = xcd_tile(blockIdx.x, ntile);
  const int td = tile % ntd;
  const int lb = (tile / ntd) % nlb;
  const int ch = tile / (nlb * ntd);
  const int li = lane & 15, dr = 4 * wave + (lane >> 4);
  const int l0 = lb * LB;
  const int l = l0 + li, lc = min(l, L - 1);
  const int d0 = td * Td, d1 = min(nd, d0 + Td);
  const int row = d0 + dr, rowc = min(row, nd - 1), drc = min(dr, Td - 1);
  double cm[BW], cj[BW], ck[BW];
#pragma unroll
  for (int o = 0; o < BW; ++o) {
    cm[o] = Md[rowc * BW + o];
    cj[o] = Jd[rowc * BW + o];
    ck[o] = Kd[rowc * BW + o];
  }
  const int rows = Td + 2 * P;
  const int rb8 = (rows + 7) >> 3;          // 8-row blocks per input array
  const int rbd = DOT ? (Td + 7) >> 3 : 0;  // 8-row blocks of the dot operand
  const int arr = rb8 * 8 * LB;             // doubles per input array in a slot
  const int slot = 3 * arr + rbd * 8 * LB + 8 * LB;  // + trash block
  const int njob = 3 * rb8 + rbd;
  const bool mine = l < L && dr < Td && row < d1;
  const int c0 = ch * Tc, c1 = min(nt, c0 + Tc);
  const size_t plane = (size_t)L * nd;
  const double* jsrc[K];
  int jdst[K], jsh[K];
  {
    const int lp = lane & 7, lr = lane >> 3;
    const int ls = min(l0 + 2 * lp, L - 2);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int jr = wave + 4 * k;
      const bool dup = jr >= njob;
      const int j = min(jr, njob - 1);
      const int q = j < 3 * rb8 ? j / rb8 : 3;
      const int rb = j - q * rb8;
      const int nr = q < 3 ? rows : Td;
      const bool pad = dup || rb * 8 + lr >= nr;
      const int rr = pad ? rb * 8 : rb * 8 + lr;
      const int lsx = pad ? min(l0, L - 2) : ls;
      const int gr = q < 3 ? min(max(d0 - P + rr, 0), nd - 1) : min(d0 + rr, nd - 1);
      const double* base = q == 0 ? A : (q == 1 ? B : (q == 2 ? C : dotv));
      jsrc[k] = base + (size_t)gr * L + lsx;
      jdst[k] = dup ? 3 * arr + rbd * 8 * LB : q * arr + rb * 8 * LB;
      jsh[k] = q == 3 ? PT : 0;
    }
  }
  auto issue = [&](int t, int sl) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const size_t toff = (size_t)min(max(t - jsh[k], 0), nt - 1) * plane;
      __builtin_amdgcn_global_load_lds((const void*)(jsrc[k] + toff), (lds_void_t*)(sm + sl * slot + jdst[k]), 16,
                                       0, 0);
    }
  };
  double acc[W];
#pragma unroll
  for (int k = 0; k < W; ++k) acc[k] = 0.0;
  double s3 = 0.0, dsum = 0.0;
  const int tb = max(0, c0 - PT);
  const int te = c1 - 1 + PT;
  const int tl = min(te, nt - 1);
#pragma unroll
  for (int sidx = 0; sidx < D - 1; ++sidx) issue(tb + sidx, (tb + sidx) % D);
  for (int t = tb; t <= te; ++t) {
    wait_vmcnt<(D - 2) * K>();
    __syncthreads();
    issue(t + D - 1, (t + D - 1) % D);  // always K copies (clamped slices past the end)
    const double* buf = sm + (t % D) * slot;
    if (t <= tl) {  // uniform
      // four independent partial sums: no long dependent FMA chain per step
      double x1 = 0.0, xa = 0.0, xb = 0.0, xc = 0.0;
#pragma unroll
      for (int o = 0; o < BW; ++o) {
        const int rr = drc + o;
        const double a = buf[rr * LB + li];
        const double b = buf[arr + rr * LB + li];
        const double c = buf[2 * arr + rr * LB + li];
        x1 += cm[o] * a;
        xa += cj[o] * a;
        xb += cm[o] * b;
        xc += ck[o] * c;
      }
      const double s1 = x1, s2 = k2 * ((xa + xb) + 2.0 * xc);
      if (t == nt - 1) {  // final-time term, last slice only (uniform)
        double x3 = 0.0;
#pragma unroll
        for (int o = 0; o < BW; ++o) x3 += ck[o] * buf[(drc + o) * LB + li] + cm[o] * buf[2 * arr + (drc + o) * LB + li];
        s3 = kw * x3;
      }
      const double* kt = Kt + t * W;
      const double* mt = Mt + t * W;
#pragma unroll
      for (int k = 0; k < W; ++k) acc[k] += kt[k] * s1 + mt[k] * s2;
    }
    const int to = t - PT;
    if (to >= c0) {  // uniform
      double v = acc[0];
      if (to == nt - 1) v += s3;
      if (DOT) dsum += mine ? v * buf[3 * arr + drc * LB + li] : 0.0;
      if (mine) y[(size_t)to * plane + (size_t)rowc * L + lc] = v;
    }
#pragma unroll
    for (int k = 0; k < W - 1; ++k) acc[k] = acc[k + 1];
    acc[W - 1] = 0.0;
  }
  if constexpr (DOT) {
    const double sblk = block_sum(dsum, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = sblk;
  }
}

// Launch the slab inner stage when the slab fits (n1, n2 <= 64, equal
// degrees in directions 1 and 2).  Returns 1 when the shape is not covered
// (nothing launched); otherwise 0, with the launch status in *err.
static int launch_inner_slab(stls_ctx* h, const double* x, hipError_t* err) {
  const DevDir& D1 = h->dd[0];
  const DevDir& D2 = h->dd[1];
  const int n1 = D1.n, n2 = D2.n;
  if (n1 > 64 || n2 > 64 || D1.p != D2.p) return 1;
  const int ld = n1 | 1;
  const size_t shmem = sizeof(double) * ((size_t)n1 * n2 + 3 * (size_t)n2 * ld);
  if (shmem > 160 * 1024) return 1;
  void (*kern)(const double*, double*, double*, double*, int, int, int, int, const double*, const double*,
               const double*, const double*, const double*, const double*) = nullptr;
  switch (D1.p) {
    case 1: kern = mv_inner_slab_kernel<1>; break;
    case 2: kern = mv_inner_slab_kernel<2>; break;
    case 3: kern = mv_inner_slab_kernel<3>; break;
    case 4: kern = mv_inner_slab_kernel<4>; break;
    case 5: kern = mv_inner_slab_kernel<5>; break;
    case 6: kern = mv_inner_slab_kernel<6>; break;
    default: return 1;
  }
  *err = hipSuccess;
  if (shmem > 65536) {
    *err = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (*err != hipSuccess) return 0;
  }
  const int nslab = (int)(h->ndof / ((int64_t)n1 * n2));
  double** w = h->work;
  prof_begin(h);
  // persistent grid (two workgroups per CU by LDS): each workgroup prefetches
  // its next slab into registers while it processes the current one
  const int blocks = std::min(nslab, 2 * 256);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(kSlabWaves * 64), shmem, h->stream, x, w[0], w[1], w[2], n1, n2, nslab,
                     ld, D1.M, D1.J, D1.K, D2.M, D2.J, D2.K);
  *err = hipGetLastError();
  prof_end(h, PROF_MV_INNER2);
  return 0;
}

// Launch the DMA-pipelined outer stage when it covers the shape (L even and
// >= 16, equal space and time degrees <= 6).  Returns 1 when not covered,
// 0 when launched, < 0 on error.
static int launch_outer_dma(stls_ctx* h, const double* A, const double* B, const double* C, double* y, int L,
                            const double* dot_with, double* partials, int* nparts) {
  const int d = h->d;
  const DevDir& Dd = h->dd[d - 1];
  const DevDir& Dt = h->dd[d];
  const int nd = Dd.n, nt = Dt.n, P = Dd.p;
  if (L % 2 != 0 || L < kDmaLb || P != Dt.p || P < 1 || P > 6) return 1;
  const int ntd = (nd + 15) / 16;
  const int Td = (nd + ntd - 1) / ntd;
  const int rows = Td + 2 * P;
  const int rb8 = (rows + 7) / 8;
  const int rbd = dot_with ? (Td + 7) / 8 : 0;
  const int K = std::max(2, (3 * rb8 + rbd + 3) / 4);
  if (K > 4) return 1;
  const int nlb = (L + kDmaLb - 1) / kDmaLb;
  int nchunk = 1;
  while (nlb * ntd * nchunk < 512 && (nt + nchunk) / (nchunk + 1) >= std::max(4 * P, 8)) ++nchunk;
  const int Tc = (nt + nchunk - 1) / nchunk;
  nchunk = (nt + Tc - 1) / Tc;
  const int blocks = nlb * ntd * nchunk;
  if (dot_with && blocks > kPartialsCap) return 1;
  if (nparts) *nparts = blocks;
  const size_t shmem = sizeof(double) * kDmaSlots * ((size_t)(3 * rb8 + rbd) * 8 * kDmaLb + 8 * kDmaLb);
  void (*kern)(const double*, const double*, const double*, double*, int, int, int, int, int, int, int, int,
               const double*, const double*, const double*, const double*, const double*, double, double,
               const double*, double*) = nullptr;
  const bool dot = dot_with != nullptr;
#define STLS_DMA_K(PV, KV)                                                                              \
  if (K == KV) kern = dot ? mv_outer_dma_kernel<PV, PV, KV, true> : mv_outer_dma_kernel<PV, PV, KV, false>;
#define STLS_DMA_P(PV) \
  case PV: STLS_DMA_K(PV, 2) STLS_DMA_K(PV, 3) STLS_DMA_K(PV, 4) break;
  switch (P) {
    STLS_DMA_P(1) STLS_DMA_P(2) STLS_DMA_P(3) STLS_DMA_P(4) STLS_DMA_P(5) STLS_DMA_P(6)
    default: return 1;
  }
#undef STLS_DMA_K
#undef STLS_DMA_P
  if (!kern) return 1;
  hipError_t e;
  if (shmem > 65536) {
    e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(LDS)");
  }
  const double k2 = h->kappa * h->kappa, kw = h->kappa * h->dir[d].wend;
  prof_begin(h);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), shmem, h->stream, A, B, C, y, L, nd, nt, Td, nlb, ntd, nchunk,
                     Tc, Dd.M, Dd.J, Dd.K, Dt.K, Dt.M, k2, kw, dot_with, partials);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "mv_outer_dma_kernel launch");
  prof_end(h, PROF_MV_OUTER);
  return 0;
}

int launch_matvec(stls_ctx* h, const double* x, double* y, const double* dot_with, double* partials,
                  int* nparts) {
  if (h->geometry) return launch_mapped_matvec(h, x, y, dot_with, partials, nparts);
  const int d = h->d;
  const int N = (int)h->ndof;
  double** w = h->work;
  const double* A = x;
  const double* B = nullptr;
  const double* C = nullptr;
  hipError_t e;
  int L = 1;
  if (d == 2) {
    const DevDir& D1 = h->dd[0];
    const int bw = 2 * D1.p + 1;
    const size_t shmem = sizeof(double) * (kInnerChunk + 2 * D1.p + 3 * (size_t)D1.n * bw);
    const int chunks = (N + kInnerChunk - 1) / kInnerChunk;
    const int blocks = std::min(chunks, 256 * 8);
    prof_begin(h);
    hipLaunchKernelGGL(mv_inner1_kernel, dim3(blocks), dim3(kThreads), shmem, h->stream, x, w[0], w[1], w[2], D1.n,
                       N, D1.p, D1.M, D1.J, D1.K);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "mv_inner1_kernel launch");
    prof_end(h, PROF_MV_INNER1);
    A = w[0]; B = w[1]; C = w[2];
    L = D1.n;
  } else if (d == 3 && launch_inner_slab(h, x, &e) == 0) {
    if (e != hipSuccess) return hip_fail(e, "mv_inner_slab_kernel launch");
    A = w[0]; B = w[1]; C = w[2];
    L = h->dd[0].n * h->dd[1].n;
  } else if (d == 3) {
    const DevDir& D1 = h->dd[0];
    const DevDir& D2 = h->dd[1];
    const int n1 = D1.n, n2 = D2.n;
    const size_t budget = 64 * 1024;
    int T2 = n2;
    auto lds_for = [&](int t2) { return sizeof(double) * 4 * (size_t)std::min(n2, t2 + 2 * D2.p) * n1; };
    auto fits = [&](int t2) {
      return lds_for(t2) <= budget && (size_t)std::min(n2, t2 + 2 * D2.p) * n1 <= (size_t)kInnerPf * kThreads;
    };
    while (T2 > 1 && !fits(T2)) --T2;
    if (!fits(T2)) { set_error("space direction too large for the matvec kernel"); return STLS_EINVAL; }
    const int ntile = (n2 + T2 - 1) / T2;
    T2 = (n2 + ntile - 1) / ntile;
    const size_t shmem = lds_for(T2);
    const int nwork = ntile * (N / (n1 * n2));
    const int blocks = std::min(nwork, 256 * 8);
    const int P = (D1.p == D2.p) ? D1.p : 0;
    void (*kern)(const double*, double*, double*, double*, int, int, int, int, int, int, int, const double*,
                 const double*, const double*, const double*, const double*, const double*) = nullptr;
    switch (P) {
      case 2: kern = mv_inner12_kernel<2>; break;
      case 3: kern = mv_inner12_kernel<3>; break;
      case 4: kern = mv_inner12_kernel<4>; break;
      case 5: kern = mv_inner12_kernel<5>; break;
      case 6: kern = mv_inner12_kernel<6>; break;
      default: kern = mv_inner12_kernel<0>; break;
    }
    if (shmem > 65536) {
      e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
      if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(LDS)");
    }
    prof_begin(h);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kThreads), shmem, h->stream, x, w[0], w[1], w[2], n1, n2, T2, ntile,
                       nwork, D1.p, D2.p, D1.M, D1.J, D1.K, D2.M, D2.J, D2.K);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "mv_inner12_kernel launch");
    prof_end(h, PROF_MV_INNER2);
    A = w[0]; B = w[1]; C = w[2];
    L = n1 * n2;
  }
  if (B != nullptr) {
    const int st = launch_outer_dma(h, A, B, C, y, L, dot_with, partials, nparts);
    if (st <= 0) return st;  // launched (0) or failed (< 0); > 0: shape not covered
  }
  const DevDir& Dd = h->dd[d - 1];
  const DevDir& Dt = h->dd[d];
  const int nd = Dd.n, nt = Dt.n, pd = Dd.p;
  const int ntd = (nd + kOuterMaxTd - 1) / kOuterMaxTd;
  const int Td = (nd + ntd - 1) / ntd;
  const int nlb = (L + kOuterLb - 1) / kOuterLb;
  const int rows = Td + 2 * pd;
  if (rows > kOuterMaxTd * kOuterSlots) { set_error("space degree too large for the matvec"); return STLS_EINVAL; }
  // time chunks: enough workgroups to cover the chip, each chunk >= 4 PT slices
  int nchunk = 1;
  while (nlb * ntd * nchunk < 1024 && (nt + nchunk) / (nchunk + 1) >= std::max(4 * Dt.p, 8)) ++nchunk;
  const int Tc = (nt + nchunk - 1) / nchunk;
  nchunk = (nt + Tc - 1) / Tc;
  const int blocks = nlb * ntd * nchunk;
  if (dot_with && blocks > kPartialsCap) { set_error("too many partial sums"); return STLS_EINVAL; }
  if (nparts) *nparts = blocks;
  const bool pd_static = (pd == Dt.p);
  const size_t shmem = sizeof(double) * ((pd_static ? 0 : 3 * (size_t)nd * (2 * pd + 1)) +
                                         3 * (B ? 3 : 1) * (size_t)rows * kOuterLds);
  const double k2 = h->kappa * h->kappa, kw = h->kappa * h->dir[d].wend;
  void (*kern)(const double*, const double*, const double*, double*, int, int, int, int, int, int, int, int, int,
               const double*, const double*, const double*, const double*, const double*, double, double,
               const double*, double*) = nullptr;
  const bool three = B != nullptr, dot = dot_with != nullptr;
#define STLS_OUTER_VAR(PV, PDV)                                                                  \
  kern = three ? (dot ? mv_outer_kernel<PV, PDV, true, true> : mv_outer_kernel<PV, PDV, true, false>) \
               : (dot ? mv_outer_kernel<PV, PDV, false, true> : mv_outer_kernel<PV, PDV, false, false>);
#define STLS_OUTER_PICK(PV)                                   \
  case PV:                                                    \
    if (pd_static) { STLS_OUTER_VAR(PV, PV) } else { STLS_OUTER_VAR(PV, 0) } \
    break;
  switch (Dt.p) {
    STLS_OUTER_PICK(1) STLS_OUTER_PICK(2) STLS_OUTER_PICK(3) STLS_OUTER_PICK(4) STLS_OUTER_PICK(5) STLS_OUTER_PICK(6)
    default: set_error("time degree > 6 not supported by the matvec kernel"); return STLS_EINVAL;
  }
#undef STLS_OUTER_VAR
#undef STLS_OUTER_PICK
  prof_begin(h);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(kThreads), shmem, h->stream, A, B, C, y, L, nd, nt, pd, Td, nlb, ntd,
                     nchunk, Tc, Dd.M, Dd.J, Dd.K, Dt.K, Dt.M, k2, kw, dot_with, partials);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "mv_outer_kernel launch");
  prof_end(h, PROF_MV_OUTER);
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

// This thread's share of a fixed-order sum of partials: entries tid,
// tid + stride, tid + 2 stride, ... added in that order, with the loads of
// eight entries issued before their additions.
__device__ inline double strided_sum(const double* __restrict__ partials, int nparts, int tid, int stride) {
  double v = 0.0;
  int i = tid;
  for (; i + 7 * stride < nparts; i += 8 * stride) {
    double b[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) b[k] = partials[i + k * stride];
#pragma unroll
    for (int k = 0; k < 8; ++k) v += b[k];
  }
  for (; i < nparts; i += stride) v += partials[i];
  return v;
}

enum FinKind { FIN_BNORM = 0, FIN_RHO0, FIN_ALPHA, FIN_RR, FIN_BETA };

// One workgroup sums the partials in a fixed order and updates the scalars.
__global__ __launch_bounds__(kThreads) void finalize_kernel(const double* __restrict__ partials, int nparts,
                                                            PcgScalars* __restrict__ S, int kind,
                                                            double* __restrict__ hist, int it) {
  __shared__ double red[4];
  if (S->done || S->flag) return;
  const double s = block_sum(strided_sum(partials, nparts, threadIdx.x, kThreads), red);
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
      S->rho_ring[0] = s;
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

// Sum of nparts partial sums in a fixed order (identical in every block).
__device__ inline double sum_partials(const double* __restrict__ partials, int nparts, double* red) {
  double v = strided_sum(partials, nparts, threadIdx.x, blockDim.x);
  v = block_sum(v, red);
  __syncthreads();
  if (threadIdx.x == 0) red[0] = v;
  __syncthreads();
  return red[0];
}

// Iteration k (parity par = k & 1): alpha = rho_{k-1} / (p.q) from the
// matvec's partial sums (every block forms the same sum; block 0 records
// alpha and any breakdown), then x += alpha p; r -= alpha q; partial sums of
// r.r into rr_parts.
__global__ __launch_bounds__(kThreads) void update_xr_kernel(double* __restrict__ x, double* __restrict__ r,
                                                             const double* __restrict__ p,
                                                             const double* __restrict__ q, int n,
                                                             PcgScalars* __restrict__ S,
                                                             const double* __restrict__ pq_parts, int npq, int par,
                                                             double* __restrict__ rr_parts) {
  __shared__ double red[4];
  // block 0 of this kernel may set S->flag while other blocks start: decide
  // once per block (thread 0) so that every wave of a block takes the same path
  __shared__ int skip;
  if (threadIdx.x == 0) skip = S->done | S->flag;
  __syncthreads();
  if (skip) return;
  const double pq = sum_partials(pq_parts, npq, red);
  const bool bad = !isfinite(pq) || !(pq > 0.0);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (!isfinite(pq)) S->flag = 2;
    else if (!(pq > 0.0)) S->flag = 1;
    else S->alpha = S->rho_ring[par ^ 1] / pq;
  }
  if (bad) return;
  const double alpha = S->rho_ring[par ^ 1] / pq;
  double s = 0.0;
  // 16-byte accesses (pairs; the internal vectors are 256-byte aligned).  x is
  // the caller's buffer: pairs when it is 16-byte aligned, else two scalars;
  // the r.r summation order is the same either way.
  const int n2 = n >> 1;
  const bool xal = (reinterpret_cast<uintptr_t>(x) & 15) == 0;
  double2* r2 = reinterpret_cast<double2*>(r);
  const double2* p2 = reinterpret_cast<const double2*>(p);
  const double2* q2 = reinterpret_cast<const double2*>(q);
  for (int e = blockIdx.x * kThreads + threadIdx.x; e < n2; e += gridDim.x * kThreads) {
    const double2 pv = p2[e], rv = r2[e], qv = q2[e];
    if (xal) {
      double2* x2 = reinterpret_cast<double2*>(x);
      const double2 xv = x2[e];
      x2[e] = make_double2(xv.x + alpha * pv.x, xv.y + alpha * pv.y);
    } else {
      x[2 * e] += alpha * pv.x;
      x[2 * e + 1] += alpha * pv.y;
    }
    const double2 rn = make_double2(rv.x - alpha * qv.x, rv.y - alpha * qv.y);
    r2[e] = rn;
    s += rn.x * rn.x + rn.y * rn.y;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {  // odd tail
    x[n - 1] += alpha * p[n - 1];
    const double rn = r[n - 1] - alpha * q[n - 1];
    r[n - 1] = rn;
    s += rn * rn;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) rr_parts[blockIdx.x] = s;
}

// Iteration k (parity par): rho_k = r.z from the FD's partial sums, beta =
// rho_k / rho_{k-1}; block 0 stores rho_k in the ring slot par (the other
// blocks read slot par ^ 1 only); p = z + beta p.
__global__ __launch_bounds__(kThreads) void update_p_kernel(double* __restrict__ p, const double* __restrict__ z,
                                                            int n, PcgScalars* __restrict__ S,
                                                            const double* __restrict__ rz_parts, int nrz, int par) {
  __shared__ double red[4];
  __shared__ int skip;  // block-uniform decision (see update_xr_kernel)
  if (threadIdx.x == 0) skip = S->done | S->flag;
  __syncthreads();
  if (skip) return;
  const double rz = sum_partials(rz_parts, nrz, red);
  const bool bad = !isfinite(rz) || !(rz > 0.0);
  const double beta = rz / S->rho_ring[par ^ 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (!isfinite(rz)) S->flag = 2;
    else if (!(rz > 0.0)) S->flag = 1;
    else {
      S->beta = beta;
      S->rho = rz;
      S->rho_ring[par] = rz;
    }
  }
  if (bad) return;
  const int n2 = n >> 1;
  double2* p2 = reinterpret_cast<double2*>(p);
  const double2* z2 = reinterpret_cast<const double2*>(z);
  for (int e = blockIdx.x * kThreads + threadIdx.x; e < n2; e += gridDim.x * kThreads) {
    const double2 pv = p2[e], zv = z2[e];
    p2[e] = make_double2(zv.x + beta * pv.x, zv.y + beta * pv.y);
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) p[n - 1] = z[n - 1] + beta * p[n - 1];  // odd tail
}

__global__ void init_scalars_kernel(PcgScalars* S, double rtol) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    S->rho = S->alpha = S->beta = S->bnorm2 = 0.0;
    S->rho_ring[0] = S->rho_ring[1] = 0.0;
    S->relres = 1.0;
    S->rtol = rtol;
    S->done = S->flag = S->iters = S->pad = 0;
  }
}

static int ew_blocks(int n) { return std::max(1, std::min((n + kThreads - 1) / kThreads, kMaxBlocksEW)); }
// grid of the PCG vector kernels: few enough partial sums for a quick
// single-workgroup finalisation, enough workgroups to stream at full rate
static int vec_blocks(int n) { return std::max(1, std::min((n + kThreads - 1) / kThreads, 2048)); }

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
  const int nb = vec_blocks(N);
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
  prof_end(h, PROF_MISC);
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
  // Iteration k enqueues its convergence check (scalars copied to a pinned
  // slot, event) and then, before waiting on it, the preconditioner and the
  // direction update of the same iteration: while the host waits and then
  // enqueues iteration k + 1, the GPU runs the FD chain.  Once the check
  // reports convergence those already-enqueued kernels return at once (they
  // read done through the gate / the scalars).
  double* rr_parts = h->partials + kPartialsCap;
  int k = 0;
  int status = STLS_ENOCONV;
  h->gate = h->scal;
  for (k = 1; k <= maxit; ++k) {
    const int par = k & 1;
    if ((st = launch_matvec(h, h->pvec, h->q, h->pvec, h->partials, &np))) break;
    prof_begin(h);
    hipLaunchKernelGGL(update_xr_kernel, dim3(nb), dim3(kThreads), 0, h->stream, x, h->r, h->pvec, h->q, N, h->scal,
                       h->partials, np, par, rr_parts);
    prof_end(h, PROF_VEC);
    if ((e = hipGetLastError()) != hipSuccess) { st = hip_fail(e, "update_xr_kernel launch"); break; }
    prof_begin(h);
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kThreads), 0, h->stream, rr_parts, nb, h->scal, (int)FIN_RR,
                       nullptr, k);
    prof_end(h, PROF_REDUCE);
    if ((e = hipGetLastError()) != hipSuccess) { st = hip_fail(e, "finalize_kernel launch"); break; }
    e = hipMemcpyAsync(h->scal_host + par, h->scal, sizeof(PcgScalars), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipEventRecord(h->check_ev[par], h->stream);
    if (e != hipSuccess) { st = hip_fail(e, "scalar read-back"); break; }
    if (k < maxit) {
      if ((st = launch_prec_apply(h, h->r, h->z, h->r, h->partials, &np))) break;
      prof_begin(h);
      hipLaunchKernelGGL(update_p_kernel, dim3(nb), dim3(kThreads), 0, h->stream, h->pvec, h->z, N, h->scal,
                         h->partials, np, par);
      prof_end(h, PROF_VEC_P);
      if ((e = hipGetLastError()) != hipSuccess) { st = hip_fail(e, "update_p_kernel launch"); break; }
    }
    if ((e = hipEventSynchronize(h->check_ev[par])) != hipSuccess) { st = hip_fail(e, "hipEventSynchronize"); break; }
    const PcgScalars* Sk = h->scal_host + par;
    if (Sk->flag == 2) { set_error("non-finite value in PCG"); status = STLS_ENAN; break; }
    if (Sk->flag == 1) { set_error("PCG breakdown (non-positive curvature)"); status = STLS_EBREAKDOWN; break; }
    h->history.push_back(Sk->relres);
    if (Sk->done) { status = STLS_OK; break; }
  }
  h->gate = nullptr;
  if (st) return st;
  if ((st = read_scalars(h))) return st;  // drains the stream; final scalars
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
