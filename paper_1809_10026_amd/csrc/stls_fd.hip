// BF16x3 fast-diagonalization chain for three space dimensions (§4.3,
// Algorithm 1 steps 2-4) in five passes:
//   1. slab pass, forward:  modes 1 and 2 of every (i3, t) slab, r (FP64) -> FP32
//   2. strided pass:        mode 3 forward
//   3. strided fused pass:  time mode forward, FP64 division by the FP64
//                           eigenvalue sum (quotient rounded to FP32), time
//                           mode backward
//   4. strided pass:        mode 3 backward
//   5. slab pass, backward: modes 2 and 1, FP32 -> s (FP64), partial sums of s . r
// Every product W X is formed as W_hi X_hi + W_hi X_lo + W_lo X_hi on MFMA
// bf16 16x16x32 with FP32 accumulation; operands are FP32 values split into
// bf16 hi + lo halves by hardware round-to-nearest-even conversions.
// Fragment layout of v_mfma_f32_16x16x32_bf16 (lane l, e = 0..7, r = 0..3):
//   A(i = l%16, k = 8(l/16) + e), B(k = 8(l/16) + e, j = l%16),
//   D(4(l/16) + r, l%16).
// The operator fragments (row-major [i*kpad + k] bf16 halves of W = U^T or
// W = U) stay in registers for the whole kernel; workgroups are persistent.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "stls_buf.h"
#include "stls_diag.h"
#include "stls_internal.h"

namespace stls {
namespace {

typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf4_t __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ inline void split8(const float* v, bf8_t& h, bf8_t& l) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 a = (__bf16)v[e];
    h[e] = a;
    l[e] = (__bf16)(v[e] - (float)a);
  }
}
__device__ inline bf8_t ld8(const void* p) { return *reinterpret_cast<const bf8_t*>(p); }

__device__ inline f4v mfma3(bf8_t ah, bf8_t al, bf8_t bh, bf8_t bl, f4v c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
  return c;
}

// ---------------------------------------------------------------------------
// Slab pass: for each slab X (n2 x n1, i1 fastest) computes
//   Y = X W1^T (mode 1),  Z = W2 Y (mode 2)
// with n1, n2 <= 16 NM (both directions padded to 16 NM rows, n1 even).
// Wave w owns rows i2 in [16w, 16w+16) of the mode-1 product, its A
// fragments read straight from global memory, and rows j2 in [16w, 16w+16)
// of the mode-2 product.  Y crosses waves through a double-buffered LDS tile
// [j1][i2] of bf16 halves (one barrier per slab).  The next slab of X is
// fetched into registers while the current one is processed.
// SCALE: diagonal scaling of the preconditioner, sigma o x on the way in
// (forward pass, TI = double) or sigma o z on the way out (backward pass),
// sigma from the packed univariate diagonals staged in LDS (FP32).
constexpr int kSlabLdy = 72;  // bf16 row stride of the Y tile (64 + 8)
constexpr int kDiagLds = 3 * 3 * 64 + 2 * 64;  // packed diagonals, d = 3, n <= 64

template <int NM, typename TI, typename TO, bool DOT, bool SCALE>
__global__ __launch_bounds__(256) void fd_slab_bf16_kernel(const TI* __restrict__ X, TO* __restrict__ Z, int n1,
                                                           int n2, int nslab, const __bf16* __restrict__ W1h,
                                                           const __bf16* __restrict__ W1l,
                                                           const __bf16* __restrict__ W2h,
                                                           const __bf16* __restrict__ W2l,
                                                           const double* __restrict__ dotv,
                                                           double* __restrict__ partials,
                                                           const PcgScalars* __restrict__ gate, DiagScale S) {
  if (gate && (gate->done | gate->flag)) return;  // PCG already finished: nothing to do
  constexpr int NK = (NM + 1) / 2;
  constexpr int KPAD = NK * 32;
  constexpr int NP = NM * 16;
  constexpr bool FWD = sizeof(TI) == 8;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __bf16* ytile = reinterpret_cast<__bf16*>(smem_raw);  // 2 buffers x {hi, lo} x [64][kSlabLdy]
  __shared__ double red[4];
  __shared__ float dgs[SCALE ? kDiagLds : 1];
  if constexpr (SCALE) {
    for (int i = threadIdx.x; i < S.off[3] + 2 * S.n[3]; i += 256) dgs[i] = S.g32[i];
    __syncthreads();
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, cl = lane & 15;
  bf8_t b1h[NM][NK], b1l[NM][NK], a2h[NK], a2l[NK];
#pragma unroll
  for (int kb = 0; kb < NK; ++kb) {
#pragma unroll
    for (int nt = 0; nt < NM; ++nt) {
      const int off = (16 * nt + cl) * KPAD + 32 * kb + 8 * g;
      b1h[nt][kb] = ld8(W1h + off);
      b1l[nt][kb] = ld8(W1l + off);
    }
    const int off2 = min(16 * wave + cl, NP - 1) * KPAD + 32 * kb + 8 * g;
    a2h[kb] = ld8(W2h + off2);
    a2l[kb] = ld8(W2l + off2);
  }
  const int ns = n1 * n2;
  const int i2 = min(16 * wave + cl, n2 - 1);  // A-fragment row of this lane (rows >= n2 masked below)
  TI px[NK][8];
  auto fetch = [&](int sl) {
    const TI* row = X + (size_t)sl * ns + (size_t)i2 * n1;
#pragma unroll
    for (int kb = 0; kb < NK; ++kb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // raw loads (columns past n1 read the row start and are zeroed at use):
        // no select right after the load, which would force an early wait
        const int c0 = 32 * kb + 8 * g + 2 * q;  // n1 even: pairs never straddle a row
        if constexpr (sizeof(TI) == 8) {
          const double2 w = *reinterpret_cast<const double2*>(row + (c0 < n1 ? c0 : 0));
          px[kb][2 * q] = w.x;
          px[kb][2 * q + 1] = w.y;
        } else {
          const float2 w = *reinterpret_cast<const float2*>(row + (c0 < n1 ? c0 : 0));
          px[kb][2 * q] = w.x;
          px[kb][2 * q + 1] = w.y;
        }
      }
  };
  const int j2o = 16 * wave + 4 * g;  // output rows j2o + r of this lane
  double dsum = 0.0;
  const int s0 = blockIdx.x;
  if (s0 < nslab) fetch(s0);
  int buf = 0;
  for (int sl = s0; sl < nslab; sl += gridDim.x) {
    double dv[DOT ? NM * 4 : 1];
    const size_t base = (size_t)sl * ns;
    if constexpr (DOT) {
#pragma unroll
      for (int nt = 0; nt < NM; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          dv[nt * 4 + r] = dotv[base + (size_t)min(j2o + r, n2 - 1) * n1 + min(16 * nt + cl, n1 - 1)];
    }
    bf8_t xh[NK], xl[NK];
    [[maybe_unused]] float sPm = 0.f, sPj = 0.f, sEk = 0.f, sEm = 0.f;
    if constexpr (SCALE && FWD) {
      const int idx[4] = {0, i2, sl % S.n[2], sl / S.n[2]};
      diag_row_coeffs<float>(S, dgs, idx, sPm, sPj, sEk, sEm);
    }
#pragma unroll
    for (int kb = 0; kb < NK; ++kb) {
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int c = 32 * kb + 8 * g + e;
        float x = (float)px[kb][e];
        if constexpr (SCALE && FWD) {
          const int cc = min(c, n1 - 1);
          x *= diag_sigma(dgs[cc], dgs[n1 + cc], dgs[2 * n1 + cc], sPm, sPj, sEk, sEm);
        }
        v[e] = c < n1 ? x : 0.f;
      }
      split8(v, xh[kb], xl[kb]);
    }
    fetch(min(sl + (int)gridDim.x, nslab - 1));  // always issued: uniform load order
    __bf16* yh = ytile + buf * 2 * 64 * kSlabLdy;
    __bf16* yl = yh + 64 * kSlabLdy;
#pragma unroll
    for (int nt = 0; nt < NM; ++nt) {
      f4v acc = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < NK; ++kb) acc = mfma3(xh[kb], xl[kb], b1h[nt][kb], b1l[nt][kb], acc);
      // the lane holds Y(16w + 4g + r, 16nt + cl); rows past n2 are zeroed
      bf4_t hh, ll;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float yv = (j2o + r < n2) ? acc[r] : 0.f;
        const __bf16 a = (__bf16)yv;
        hh[r] = a;
        ll[r] = (__bf16)(yv - (float)a);
      }
      const int o = (16 * nt + cl) * kSlabLdy + j2o;
      *reinterpret_cast<bf4_t*>(yh + o) = hh;
      *reinterpret_cast<bf4_t*>(yl + o) = ll;
    }
    __syncthreads();
    const __amdgpu_buffer_rsrc_t zr = buf_rsrc(Z + base, (size_t)ns * sizeof(TO));  // this slab of Z
    [[maybe_unused]] float oPm[4], oPj[4], oEk[4], oEm[4];  // SCALE, backward: rows j2o + r
    if constexpr (SCALE && !FWD) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int idx[4] = {0, min(j2o + r, n2 - 1), sl % S.n[2], sl / S.n[2]};
        diag_row_coeffs<float>(S, dgs, idx, oPm[r], oPj[r], oEk[r], oEm[r]);
      }
    }
#pragma unroll
    for (int nt = 0; nt < NM; ++nt) {
      f4v acc = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < NK; ++kb) {
        const int o = (16 * nt + cl) * kSlabLdy + 32 * kb + 8 * g;
        acc = mfma3(a2h[kb], a2l[kb], ld8(yh + o), ld8(yl + o), acc);
      }
      const int j1 = 16 * nt + cl;
      [[maybe_unused]] float m1 = 0.f, k1 = 0.f, jj1 = 0.f;
      if constexpr (SCALE && !FWD) {
        const int cc = min(j1, n1 - 1);
        m1 = dgs[cc];
        k1 = dgs[n1 + cc];
        jj1 = dgs[2 * n1 + cc];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool ok = j1 < n1 && j2o + r < n2;
        float zf = acc[r];
        if constexpr (SCALE && !FWD) zf *= diag_sigma(m1, k1, jj1, oPm[r], oPj[r], oEk[r], oEm[r]);
        const TO zv = (TO)zf;
        if constexpr (DOT) dsum += ok ? (double)zv * dv[nt * 4 + r] : 0.0;
        buf_store(zv, zr, ok ? (int)(((j2o + r) * n1 + j1) * sizeof(TO)) : kOutOfRange);
      }
    }
    buf ^= 1;
  }
  if constexpr (DOT) {
    for (int off = 32; off > 0; off >>= 1) dsum += __shfl_xor(dsum, off, 64);
    if (lane == 0) red[wave] = dsum;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// ---------------------------------------------------------------------------
// Strided pass over the (L, n, R) view (n <= 16 NM): Y(i, c) = sum_k W(i, k) X(k, c).
// One wave handles 16 consecutive columns at a time, its B fragments loaded
// straight from global memory (8 consecutive k of one column per lane), two
// such units prefetched into registers (two register sets, unrolled, so that
// no copy of an in-flight value forces an early wait).  FUSED: time mode,
//   Q(i, c) = (W X)(i, c) / (lambda_t[i] + lambda_s[c])  (FP64 division,
//             quotient rounded to FP32),
//   Y = W2 Q,
// with Q re-fragmented through a per-wave LDS scratch tile.  WL: the
// forward operator's fragments are read from LDS at each product instead of
// being held in registers (fewer registers, more waves per CU).
constexpr int kStridedWaves = 8;
constexpr int kStridedDepth = 2;

template <int NM, bool FUSED, bool WL>
__global__ __launch_bounds__(kStridedWaves * 64, (WL && !FUSED) ? 4 : 2) void fd_strided_bf16_kernel(
    const float* __restrict__ X, float* __restrict__ Y, int L, int n, int ncols, const __bf16* __restrict__ Wh,
    const __bf16* __restrict__ Wl, const __bf16* __restrict__ W2h, const __bf16* __restrict__ W2l,
    const double* __restrict__ lam_t, const double* __restrict__ lam_s, const PcgScalars* __restrict__ gate) {
  if (gate && (gate->done | gate->flag)) return;  // PCG already finished: nothing to do
  constexpr int NK = (NM + 1) / 2;
  constexpr int KPAD = NK * 32;
  constexpr int LDS_S = KPAD + 4;
  constexpr int DEPTH = kStridedDepth;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, cl = lane & 15;
  // LDS: (fused) lambda_t (16 NM doubles, clamped) and the backward
  // operator's bf16 halves [16 NM][KPAD + 8]; (WL) the forward operator's
  // halves, same layout; (fused) the per-wave scratch tiles
  constexpr int LDV = KPAD + 8;
  constexpr int kOpBytes = 2 * 16 * NM * LDV * 2;
  double* lt_lds = reinterpret_cast<double*>(smem_raw);
  __bf16* v2h = reinterpret_cast<__bf16*>(smem_raw + 16 * NM * sizeof(double));
  __bf16* v2l = v2h + 16 * NM * LDV;
  unsigned char* after_fused = smem_raw + (FUSED ? 16 * NM * sizeof(double) + kOpBytes : 0);
  __bf16* w1h = reinterpret_cast<__bf16*>(after_fused);
  __bf16* w1l = w1h + 16 * NM * LDV;
  float* myscr = reinterpret_cast<float*>(after_fused + (WL ? kOpBytes : 0)) + wave * 16 * LDS_S;
  if constexpr (FUSED || WL) {
    if constexpr (FUSED)
      for (int i = threadIdx.x; i < 16 * NM; i += blockDim.x) lt_lds[i] = lam_t[min(i, n - 1)];
    for (int e = threadIdx.x; e < 16 * NM * KPAD; e += blockDim.x) {
      const int i = e / KPAD, k = e - i * KPAD;
      if constexpr (FUSED) {
        v2h[i * LDV + k] = W2h[e];
        v2l[i * LDV + k] = W2l[e];
      }
      if constexpr (WL) {
        w1h[i * LDV + k] = Wh[e];
        w1l[i * LDV + k] = Wl[e];
      }
    }
    __syncthreads();
  }
  const int nunits = (ncols + 15) / 16;
  const int stride = gridDim.x * kStridedWaves;
  const int u0 = blockIdx.x * kStridedWaves + wave;
  if (u0 >= nunits) return;
  bf8_t wh[WL ? 1 : NM][NK], wl[WL ? 1 : NM][NK];
  if constexpr (!WL) {
#pragma unroll
    for (int t = 0; t < NM; ++t)
#pragma unroll
      for (int kb = 0; kb < NK; ++kb) {
        const int off = (16 * t + cl) * KPAD + 32 * kb + 8 * g;
        wh[t][kb] = ld8(Wh + off);
        wl[t][kb] = ld8(Wl + off);
      }
    // the operator fragments arrive before the column prefetch is issued:
    // were they queued behind it, the loop's waits (taken over the entry path
    // as well) would drain the whole prefetch on every unit
    __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (15 << 8));  // vmcnt(0)
    __builtin_amdgcn_sched_barrier(0);
  }
  const int Ln = L * n;
  auto base_of = [&](int c) -> int { return (c % L) + (c / L) * Ln; };
  const __amdgpu_buffer_rsrc_t xr = buf_rsrc(X, (size_t)ncols * n * sizeof(float));
  const __amdgpu_buffer_rsrc_t yr = buf_rsrc(Y, (size_t)ncols * n * sizeof(float));
  float pv[DEPTH][NK][8];
  // fused: lambda_s of the prefetched column, loaded after the unit's last
  // use of the slot (so the slot needs no second register and no copy)
  double pls[DEPTH];
  auto fetch = [&](int u, float (&v)[NK][8]) {  // rows k >= n read as 0 (out of range)
    const int b = base_of(min(u * 16 + cl, ncols - 1));
#pragma unroll
    for (int kb = 0; kb < NK; ++kb)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 32 * kb + 8 * g + e;
        v[kb][e] = buf_load_f32(xr, k < n ? (b + k * L) * (int)sizeof(float) : kOutOfRange);
      }
  };
#pragma unroll
  for (int d = 0; d < DEPTH; ++d) {
    fetch(min(u0 + d * stride, nunits - 1), pv[d]);
    if constexpr (FUSED) pls[d] = lam_s[min(min(u0 + d * stride, nunits - 1) * 16 + cl, ncols - 1)];
    __builtin_amdgcn_sched_barrier(0);  // issue order as in the loop: unit by unit
  }
  for (int ub = u0; ub < nunits; ub += DEPTH * stride) {
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) {
      const int u = ub + d * stride;
      const int c = min(u, nunits - 1) * 16 + cl;
      bf8_t xh[NK], xl[NK];
#pragma unroll
      for (int kb = 0; kb < NK; ++kb) split8(pv[d][kb], xh[kb], xl[kb]);
      __builtin_amdgcn_sched_barrier(0);
      fetch(min(u + DEPTH * stride, nunits - 1), pv[d]);  // always issued: uniform load order
      __builtin_amdgcn_sched_barrier(0);
      f4v acc[NM];
#pragma unroll
      for (int t = 0; t < NM; ++t) {
        acc[t] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < NK; ++kb) {
          if constexpr (WL) {
            const int o = (16 * t + cl) * LDV + 32 * kb + 8 * g;
            acc[t] = mfma3(ld8(w1h + o), ld8(w1l + o), xh[kb], xl[kb], acc[t]);
          } else {
            acc[t] = mfma3(wh[t][kb], wl[t][kb], xh[kb], xl[kb], acc[t]);
          }
        }
      }
      if constexpr (FUSED) {
#pragma unroll
        for (int t = 0; t < NM; ++t) {
          f4v q;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            // eigenvalue sum and division in FP64, the quotient rounded
            // once to FP32 (the precision of the pass's output)
            const int i = 16 * t + 4 * g + r;
            const float qv = (float)((double)acc[t][r] / (lt_lds[i] + pls[d]));
            q[r] = i < n ? qv : 0.f;
          }
          *reinterpret_cast<f4v*>(myscr + cl * LDS_S + 16 * t + 4 * g) = q;
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int kb = 0; kb < NK; ++kb) {
          float v[8];
          const f4v a = *reinterpret_cast<const f4v*>(myscr + cl * LDS_S + 32 * kb + 8 * g);
          const f4v b = *reinterpret_cast<const f4v*>(myscr + cl * LDS_S + 32 * kb + 8 * g + 4);
          // rows past n (including the k padding the tile never holds) are zero
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            v[e] = 32 * kb + 8 * g + e < n ? a[e] : 0.f;
            v[4 + e] = 32 * kb + 8 * g + 4 + e < n ? b[e] : 0.f;
          }
          split8(v, xh[kb], xl[kb]);
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int t = 0; t < NM; ++t) {
          acc[t] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kb = 0; kb < NK; ++kb) {
            const int o = (16 * t + cl) * LDV + 32 * kb + 8 * g;
            acc[t] = mfma3(ld8(v2h + o), ld8(v2l + o), xh[kb], xl[kb], acc[t]);
          }
        }
      }
      {
        const bool colok = u < nunits && c < ncols;
        const int b = base_of(min(c, ncols - 1));
#pragma unroll
        for (int t = 0; t < NM; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 16 * t + 4 * g + r;
            buf_store(acc[t][r], yr, colok && i < n ? (b + i * L) * (int)sizeof(float) : kOutOfRange);
          }
      }
      if constexpr (FUSED) pls[d] = lam_s[min(min(u + DEPTH * stride, nunits - 1) * 16 + cl, ncols - 1)];
    }
  }
}

template <int NM, typename TI, typename TO, bool DOT, bool SCALE>
int launch_slab(stls_ctx* h, const TI* X, TO* Z, bool fwd, const double* dotv, double* partials, int* nparts) {
  const DevDir& D1 = h->dd[0];
  const DevDir& D2 = h->dd[1];
  const int n1 = D1.n, n2 = D2.n;
  const int nslab = (int)(h->ndof / ((int64_t)n1 * n2));
  const int blocks = std::min(nslab, 2 * 256);
  if (nparts) *nparts = blocks;
  const size_t shmem = sizeof(__bf16) * 2 * 2 * 64 * kSlabLdy;
  const __bf16* W1h = (const __bf16*)(fwd ? D1.Hfwd : D1.Hbwd);
  const __bf16* W1l = (const __bf16*)(fwd ? D1.Lfwd : D1.Lbwd);
  const __bf16* W2h = (const __bf16*)(fwd ? D2.Hfwd : D2.Hbwd);
  const __bf16* W2l = (const __bf16*)(fwd ? D2.Lfwd : D2.Lbwd);
  prof_begin(h);
  hipLaunchKernelGGL((fd_slab_bf16_kernel<NM, TI, TO, DOT, SCALE>), dim3(blocks), dim3(256), shmem, h->stream, X, Z,
                     n1, n2, nslab, W1h, W1l, W2h, W2l, dotv, partials, h->gate, diag_scale_args(h));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "fd_slab_bf16_kernel launch");
  prof_end(h, fwd ? PROF_FD_SLAB : PROF_FD_SLAB_BWD);
  return STLS_OK;
}

// forward operator in LDS (WL): measured on the d = 3, p = 4, 48-element
// workload, the fused time pass runs in 23 us with it (128 registers, two
// workgroups per CU) against 26 us without; the mode-3 pass is faster with
// the operator in registers (17.5 us against 18.6 us)
constexpr bool kSpaceOpsInLds = false;
constexpr bool kTimeOpsInLds = true;

template <int NM, bool FUSED>
int launch_strided(stls_ctx* h, const float* X, float* Y, int L, int k, bool fwd, const double* lam_t) {
  constexpr bool WL = FUSED ? kTimeOpsInLds : kSpaceOpsInLds;
  const DevDir& D = h->dd[k];
  const int n = D.n;
  const int ncols = (int)(h->ndof / n);
  const int nunits = (ncols + 15) / 16;
  const int blocks = std::max(1, std::min((nunits + kStridedWaves - 1) / kStridedWaves, WL ? 512 : 256));
  constexpr int NK = (NM + 1) / 2;
  const size_t op_bytes = sizeof(__bf16) * 2 * 16 * NM * (NK * 32 + 8);
  const size_t shmem = (FUSED ? sizeof(double) * 16 * NM + op_bytes + sizeof(float) * kStridedWaves * 16 * (NK * 32 + 4)
                              : 0) +
                       (WL ? op_bytes : 0);
  const __bf16* Wh = (const __bf16*)(fwd ? D.Hfwd : D.Hbwd);
  const __bf16* Wl = (const __bf16*)(fwd ? D.Lfwd : D.Lbwd);
  const __bf16* W2h = FUSED ? (const __bf16*)D.Hbwd : nullptr;
  const __bf16* W2l = FUSED ? (const __bf16*)D.Lbwd : nullptr;
  if (shmem > 65536) {
    const hipError_t ea = hipFuncSetAttribute((const void*)fd_strided_bf16_kernel<NM, FUSED, WL>,
                                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (ea != hipSuccess) return hip_fail(ea, "hipFuncSetAttribute(LDS)");
  }
  prof_begin(h);
  hipLaunchKernelGGL((fd_strided_bf16_kernel<NM, FUSED, WL>), dim3(blocks), dim3(kStridedWaves * 64), shmem, h->stream, X,
                     Y, L, n, ncols, Wh, Wl, W2h, W2l, lam_t, h->lam_s, h->gate);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "fd_strided_bf16_kernel launch");
  prof_end(h, FUSED ? PROF_FD_TIME : PROF_FD_SPACE);
  return STLS_OK;
}

template <bool FUSED>
int strided_nm(stls_ctx* h, const float* X, float* Y, int L, int k, bool fwd, const double* lam_t) {
  switch (h->dd[k].npad / 16) {
    case 1: return launch_strided<1, FUSED>(h, X, Y, L, k, fwd, lam_t);
    case 2: return launch_strided<2, FUSED>(h, X, Y, L, k, fwd, lam_t);
    case 3: return launch_strided<3, FUSED>(h, X, Y, L, k, fwd, lam_t);
    case 4: return launch_strided<4, FUSED>(h, X, Y, L, k, fwd, lam_t);
    default: set_error("direction too large for the strided bf16 pass"); return STLS_EINVAL;
  }
}

template <typename TI, typename TO, bool DOT, bool SCALE>
int slab_nm(stls_ctx* h, const TI* X, TO* Z, bool fwd, const double* dotv, double* partials, int* nparts) {
  switch (h->dd[0].npad / 16) {
    case 1: return launch_slab<1, TI, TO, DOT, SCALE>(h, X, Z, fwd, dotv, partials, nparts);
    case 2: return launch_slab<2, TI, TO, DOT, SCALE>(h, X, Z, fwd, dotv, partials, nparts);
    case 3: return launch_slab<3, TI, TO, DOT, SCALE>(h, X, Z, fwd, dotv, partials, nparts);
    case 4: return launch_slab<4, TI, TO, DOT, SCALE>(h, X, Z, fwd, dotv, partials, nparts);
    default: set_error("direction too large for the slab bf16 pass"); return STLS_EINVAL;
  }
}

}  // namespace

// Shapes covered: d = 3, every restricted size <= 64, n1 even, directions 1
// and 2 padded alike, and the FP32 work vectors addressable by one buffer
// resource (byte offsets below 2^31; out-of-range lanes use 0x7fffffff).
bool fd_bf16_five_pass_covers(const stls_ctx* h) {
  if (h->d != 3) return false;
  for (int k = 0; k <= 3; ++k)
    if (h->dir[k].n > 64) return false;
  if (h->dir[0].n % 2 != 0 || h->dd[0].npad != h->dd[1].npad) return false;
  return h->ndof * (int64_t)sizeof(float) < ((int64_t)1 << 31) - 1;
}

template <bool SCALE>
static int five_pass(stls_ctx* h, const double* r, double* s, const double* dot_with, double* partials,
                     int* nparts) {
  float* b0 = reinterpret_cast<float*>(h->fdbuf[0]);
  float* b1 = reinterpret_cast<float*>(h->fdbuf[1]);
  const int n1 = h->dir[0].n, n2 = h->dir[1].n;
  const int L3 = n1 * n2;
  const int ns = (int)h->ns;
  int st;
  if ((st = slab_nm<double, float, false, SCALE>(h, r, b0, true, nullptr, nullptr, nullptr))) return st;
  if ((st = strided_nm<false>(h, b0, b1, L3, 2, true, nullptr))) return st;
  if ((st = strided_nm<true>(h, b1, b0, ns, 3, true, h->dd[3].lam))) return st;
  if ((st = strided_nm<false>(h, b0, b1, L3, 2, false, nullptr))) return st;
  if (dot_with) return slab_nm<float, double, true, SCALE>(h, b1, s, false, dot_with, partials, nparts);
  return slab_nm<float, double, false, SCALE>(h, b1, s, false, nullptr, nullptr, nparts);
}

int prec_apply_bf16x3_five_pass(stls_ctx* h, const double* r, double* s, const double* dot_with, double* partials,
                                int* nparts, bool scale) {
  return scale ? five_pass<true>(h, r, s, dot_with, partials, nparts)
               : five_pass<false>(h, r, s, dot_with, partials, nparts);
}

}  // namespace stls
