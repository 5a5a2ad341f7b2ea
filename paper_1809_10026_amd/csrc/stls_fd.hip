// Fast-diagonalization chain for three space dimensions (§4.3, Algorithm 1
// steps 2-4) in five passes:
//   1. slab pass, forward:  modes 1 and 2 of every (i3, t) slab, r (FP64) -> T
//   2. strided pass:        mode 3 forward
//   3. strided fused pass:  time mode forward, FP64 division by the FP64
//                           eigenvalue sum (quotient rounded to T), time
//                           mode backward
//   4. strided pass:        mode 3 backward
//   5. slab pass, backward: modes 2 and 1, T -> s (FP64), partial sums of s . r
// The n-mode products run in one of three precisions (T: type of the
// intermediates):
//   bf16x3 (T = float):  W X = W_hi X_hi + W_hi X_lo + W_lo X_hi on MFMA
//                        bf16 16x16x32 with FP32 accumulation, operands split
//                        into bf16 hi + lo halves by round-to-nearest-even;
//   fp32   (T = float):  MFMA f32 16x16x4;
//   fp64   (T = double): MFMA f64 16x16x4.
// One assignment of the summation index serves all three: within a block of
// 32 values of k, lane group g = l/16 of lane l holds the 8 consecutive
// k = 32 kb + 8 g + e (e = 0..7) of its operator row or data column.  The
// bf16 16x16x32 instruction takes the 8 as one operand (A(i = l%16, k),
// B(k, j = l%16)); the x4 instructions take them in 8 steps, step e summing
// k = 32 kb + 8 g + e over the four groups (a fixed permutation of the sum).
// Results: bf16 16x16x32 and f32 16x16x4 leave D(4g + r, l%16) in register
// r, f64 16x16x4 leaves D(g + 4r, l%16).
// Operators are stored row-major [i*kpad + k] (W = U^T forward, W = U
// backward): bf16 hi and lo halves, FP32 or FP64, zero padded.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "stls_buf.h"
#include "stls_diag.h"
#include "stls_internal.h"

namespace stls {
namespace {

typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf4_t __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

enum { kPrecBf16x3 = 0, kPrecF32 = 1, kPrecF64 = 2 };

__device__ inline void split8(const float* v, bf8_t& h, bf8_t& l) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 a = (__bf16)v[e];
    h[e] = a;
    l[e] = (__bf16)(v[e] - (float)a);
  }
}
__device__ inline bf8_t ld8(const __bf16* p) { return *reinterpret_cast<const bf8_t*>(p); }

__device__ inline f4v mfma3(bf8_t ah, bf8_t al, bf8_t bh, bf8_t bl, f4v c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
  return c;
}

// Precision policy: T (intermediates), S (operator and tile storage), the
// fragment of one 32-wide k block, the product of two fragments, the row
// of result register r in lane group g, and the store of 4 results.
template <int PR> struct Prec;

template <> struct Prec<kPrecBf16x3> {
  typedef float T;
  typedef __bf16 S;
  typedef f4v acc_t;
  static constexpr int kHalves = 2;  // hi and lo arrays
  struct Frag { bf8_t h, l; };
  __device__ static inline Frag op(const S* hi, const S* lo, int off) { return Frag{ld8(hi + off), ld8(lo + off)}; }
  __device__ static inline Frag data(const T* v) {
    Frag f;
    split8(v, f.h, f.l);
    return f;
  }
  __device__ static inline acc_t mma(const Frag& a, const Frag& b, acc_t c) { return mfma3(a.h, a.l, b.h, b.l, c); }
  __device__ static inline int row(int g, int r) { return 4 * g + r; }
  // results of rows row(g, 0..3) into a [col][row] tile at col*ld + row(g, 0)
  __device__ static inline void put4(S* hi, S* lo, int off, const T* v) {
    bf4_t hh, ll;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const __bf16 a = (__bf16)v[r];
      hh[r] = a;
      ll[r] = (__bf16)(v[r] - (float)a);
    }
    *reinterpret_cast<bf4_t*>(hi + off) = hh;
    *reinterpret_cast<bf4_t*>(lo + off) = ll;
  }
};

template <> struct Prec<kPrecF32> {
  typedef float T;
  typedef float S;
  typedef f4v acc_t;
  static constexpr int kHalves = 1;
  struct Frag { float v[8]; };
  __device__ static inline Frag op(const S* p, const S*, int off) {
    Frag f;
    const f4v a = *reinterpret_cast<const f4v*>(p + off), b = *reinterpret_cast<const f4v*>(p + off + 4);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      f.v[e] = a[e];
      f.v[4 + e] = b[e];
    }
    return f;
  }
  __device__ static inline Frag data(const T* v) {
    Frag f;
#pragma unroll
    for (int e = 0; e < 8; ++e) f.v[e] = v[e];
    return f;
  }
  __device__ static inline acc_t mma(const Frag& a, const Frag& b, acc_t c) {
#pragma unroll
    for (int e = 0; e < 8; ++e) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[e], b.v[e], c, 0, 0, 0);
    return c;
  }
  __device__ static inline int row(int g, int r) { return 4 * g + r; }
  __device__ static inline void put4(S* p, S*, int off, const T* v) {
    *reinterpret_cast<f4v*>(p + off) = f4v{v[0], v[1], v[2], v[3]};
  }
};

template <> struct Prec<kPrecF64> {
  typedef double T;
  typedef double S;
  typedef d4v acc_t;
  static constexpr int kHalves = 1;
  struct Frag { double v[8]; };
  __device__ static inline Frag op(const S* p, const S*, int off) {
    Frag f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const d2v a = *reinterpret_cast<const d2v*>(p + off + 2 * q);
      f.v[2 * q] = a[0];
      f.v[2 * q + 1] = a[1];
    }
    return f;
  }
  __device__ static inline Frag data(const T* v) {
    Frag f;
#pragma unroll
    for (int e = 0; e < 8; ++e) f.v[e] = v[e];
    return f;
  }
  __device__ static inline acc_t mma(const Frag& a, const Frag& b, acc_t c) {
#pragma unroll
    for (int e = 0; e < 8; ++e) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a.v[e], b.v[e], c, 0, 0, 0);
    return c;
  }
  __device__ static inline int row(int g, int r) { return g + 4 * r; }
  // rows g + 4r are not contiguous: four stores
  __device__ static inline void put4(S* p, S*, int off, const T* v) {
#pragma unroll
    for (int r = 0; r < 4; ++r) p[off + 4 * r] = v[r];
  }
};

// Four results of rows row(g, 0..3) at p[off + row(g, r) - row(g, 0)] in T
// (the per-wave scratch of the fused time pass), and 8 consecutive T.
__device__ inline void put4t(float* p, int off, const float* v) { *reinterpret_cast<f4v*>(p + off) = f4v{v[0], v[1], v[2], v[3]}; }
__device__ inline void put4t(double* p, int off, const double* v) {
#pragma unroll
  for (int r = 0; r < 4; ++r) p[off + 4 * r] = v[r];
}
__device__ inline void get8t(const float* p, float* v) {
  const f4v a = *reinterpret_cast<const f4v*>(p), b = *reinterpret_cast<const f4v*>(p + 4);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    v[e] = a[e];
    v[4 + e] = b[e];
  }
}
__device__ inline void get8t(const double* p, double* v) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const d2v a = *reinterpret_cast<const d2v*>(p + 2 * q);
    v[2 * q] = a[0];
    v[2 * q + 1] = a[1];
  }
}

__device__ inline float buf_load_t(__amdgpu_buffer_rsrc_t r, int off, float) { return buf_load_f32(r, off); }
__device__ inline double buf_load_t(__amdgpu_buffer_rsrc_t r, int off, double) { return buf_load_f64(r, off); }

// ---------------------------------------------------------------------------
// Slab pass: for each slab X (n2 x n1, i1 fastest) computes
//   Y = X W1^T (mode 1),  Z = W2 Y (mode 2)
// with n1, n2 <= 16 NM (both directions padded to 16 NM rows, n1 even).
// Wave w owns rows i2 in [16w, 16w+16) of the mode-1 product, its A
// fragments read straight from global memory, and rows j2 in [16w, 16w+16)
// of the mode-2 product.  Y crosses waves through a double-buffered LDS tile
// [j1][i2] (one barrier per slab).  The next slab of X is fetched into
// registers while the current one is processed.  FWD: r (FP64) in, T out;
// otherwise T in, s (FP64) out with partial sums of s . dotv (DOT).
// SCALE: diagonal scaling of the preconditioner, sigma o x on the way in
// (forward) or sigma o z on the way out (backward), sigma from the packed
// univariate diagonals staged in LDS (in T).  FP64: the mode-1 operator
// (128 registers in registers) is staged in LDS after the Y tile, which then
// has one buffer (a second barrier per slab) so that two workgroups fit on
// a CU.
constexpr int kSlabLdy = 72;  // row stride of the Y tile (64 + 8)
constexpr int kDiagLds = 3 * 3 * 64 + 2 * 64;  // packed diagonals, d = 3, n <= 64

template <int PR>
constexpr bool slab_op1_in_lds() {
  return PR == kPrecF64;
}
template <int PR>
constexpr size_t slab_lds_bytes(int NM) {
  return sizeof(typename Prec<PR>::S) * Prec<PR>::kHalves *
         ((slab_op1_in_lds<PR>() ? 1 : 2) * 64 * kSlabLdy + (slab_op1_in_lds<PR>() ? 16 * NM * (32 * ((NM + 1) / 2) + 8) : 0));
}

// rows x KPAD operator entries (row-major, rows of KPAD) into LDS rows of
// stride LDV: 16-byte pieces, four per thread with their loads in flight
// before the stores (an element per iteration would wait for every load).
template <typename SD, int KPAD, int LDV>
__device__ __forceinline__ void stage_rows(const SD* __restrict__ src, SD* dst, int rows) {
  constexpr int PE = 16 / (int)sizeof(SD), PR = KPAD / PE;
  static_assert(KPAD % PE == 0 && (LDV * (int)sizeof(SD)) % 16 == 0, "16-byte pieces");
  typedef unsigned int u4_t __attribute__((ext_vector_type(4)));
  const int tot = rows * PR;
  for (int e0 = threadIdx.x; e0 < tot; e0 += blockDim.x * 4) {
    u4_t v[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int e = min(e0 + b * (int)blockDim.x, tot - 1);
      v[b] = *reinterpret_cast<const u4_t*>(src + (size_t)(e / PR) * KPAD + (e % PR) * PE);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int e = e0 + b * (int)blockDim.x;
      if (e < tot) *reinterpret_cast<u4_t*>(dst + (e / PR) * LDV + (e % PR) * PE) = v[b];
    }
  }
}

template <int PR, int NM, bool FWD, bool DOT, bool SCALE>
__global__ __launch_bounds__(256) void fd_slab_kernel(
    const typename std::conditional<FWD, double, typename Prec<PR>::T>::type* __restrict__ X,
    typename std::conditional<FWD, typename Prec<PR>::T, double>::type* __restrict__ Z, int n1, int n2, int nslab,
    const typename Prec<PR>::S* __restrict__ W1h, const typename Prec<PR>::S* __restrict__ W1l,
    const typename Prec<PR>::S* __restrict__ W2h, const typename Prec<PR>::S* __restrict__ W2l,
    const double* __restrict__ dotv, double* __restrict__ partials, const PcgScalars* __restrict__ gate, DiagScale S) {
  typedef Prec<PR> P;
  typedef typename P::T T;
  typedef typename P::S SD;
  typedef typename P::Frag Frag;
  typedef typename P::acc_t acc_t;
  typedef typename std::conditional<FWD, double, T>::type TI;
  typedef typename std::conditional<FWD, T, double>::type TO;
  if (gate && (gate->done | gate->flag)) return;  // PCG already finished: nothing to do
  constexpr int NK = (NM + 1) / 2;
  constexpr int KPAD = NK * 32;
  constexpr int NP = NM * 16;
  constexpr int kTile = 64 * kSlabLdy;
  constexpr bool W1L = slab_op1_in_lds<PR>();
  constexpr int NBUF = W1L ? 1 : 2;
  constexpr int LDV = KPAD + 8;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  SD* ytile = reinterpret_cast<SD*>(smem_raw);  // NBUF buffers x kHalves x [64][kSlabLdy]
  SD* w1s = ytile + NBUF * P::kHalves * kTile;  // (W1L) mode-1 operator [16 NM][LDV]
  __shared__ double red[4];
  __shared__ T dgs[SCALE ? kDiagLds : 1];
  if constexpr (SCALE) {
    const int nd = S.off[3] + 2 * S.n[3];
    if constexpr (sizeof(T) == 8) {
      for (int i = threadIdx.x; i < nd; i += 256) dgs[i] = S.g[i];
    } else {
      for (int i = threadIdx.x; i < nd; i += 256) dgs[i] = S.g32[i];
    }
    __syncthreads();
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, cl = lane & 15;
  Frag b1[W1L ? 1 : NM][NK], a2[NK];
  if constexpr (W1L) {
    stage_rows<SD, KPAD, LDV>(W1h, w1s, NP);
    __syncthreads();
  }
#pragma unroll
  for (int kb = 0; kb < NK; ++kb) {
    if constexpr (!W1L) {
#pragma unroll
      for (int nt = 0; nt < NM; ++nt) b1[nt][kb] = P::op(W1h, W1l, (16 * nt + cl) * KPAD + 32 * kb + 8 * g);
    }
    a2[kb] = P::op(W2h, W2l, min(16 * wave + cl, NP - 1) * KPAD + 32 * kb + 8 * g);
  }
  const int ns = n1 * n2;
  const int i2 = min(16 * wave + cl, n2 - 1);  // A-fragment row of this lane (rows >= n2 masked below)
  TI px[NK][8];
  auto fetch = [&](int sl) {
    const TI* rowp = X + (size_t)sl * ns + (size_t)i2 * n1;
#pragma unroll
    for (int kb = 0; kb < NK; ++kb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // raw loads (columns past n1 read the row start and are zeroed at use):
        // no select right after the load, which would force an early wait
        const int c0 = 32 * kb + 8 * g + 2 * q;  // n1 even: pairs never straddle a row
        if constexpr (sizeof(TI) == 8) {
          const double2 w = *reinterpret_cast<const double2*>(rowp + (c0 < n1 ? c0 : 0));
          px[kb][2 * q] = w.x;
          px[kb][2 * q + 1] = w.y;
        } else {
          const float2 w = *reinterpret_cast<const float2*>(rowp + (c0 < n1 ? c0 : 0));
          px[kb][2 * q] = w.x;
          px[kb][2 * q + 1] = w.y;
        }
      }
  };
  const int j2o = 16 * wave;  // output rows j2o + row(g, r) of this lane
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
          dv[nt * 4 + r] = dotv[base + (size_t)min(j2o + P::row(g, r), n2 - 1) * n1 + min(16 * nt + cl, n1 - 1)];
    }
    Frag xf[NK];
    [[maybe_unused]] T sPm = 0, sPj = 0, sEk = 0, sEm = 0;
    if constexpr (SCALE && FWD) {
      const int idx[4] = {0, i2, sl % S.n[2], sl / S.n[2]};
      diag_row_coeffs<T>(S, dgs, idx, sPm, sPj, sEk, sEm);
    }
#pragma unroll
    for (int kb = 0; kb < NK; ++kb) {
      T v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int c = 32 * kb + 8 * g + e;
        T x = (T)px[kb][e];
        if constexpr (SCALE && FWD) {
          const int cc = min(c, n1 - 1);
          x *= diag_sigma(dgs[cc], dgs[n1 + cc], dgs[2 * n1 + cc], sPm, sPj, sEk, sEm);
        }
        v[e] = c < n1 ? x : (T)0;
      }
      xf[kb] = P::data(v);
    }
    fetch(min(sl + (int)gridDim.x, nslab - 1));  // always issued: uniform load order
    SD* yh = ytile + buf * P::kHalves * kTile;
    SD* yl = yh + (P::kHalves - 1) * kTile;
#pragma unroll
    for (int nt = 0; nt < NM; ++nt) {
      acc_t acc = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int kb = 0; kb < NK; ++kb) {
        if constexpr (W1L) acc = P::mma(xf[kb], P::op(w1s, w1s, (16 * nt + cl) * LDV + 32 * kb + 8 * g), acc);
        else acc = P::mma(xf[kb], b1[nt][kb], acc);
      }
      // the lane holds Y(16w + row(g, r), 16nt + cl); rows past n2 are zeroed
      T yv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) yv[r] = (j2o + P::row(g, r) < n2) ? (T)acc[r] : (T)0;
      P::put4(yh, yl, (16 * nt + cl) * kSlabLdy + j2o + P::row(g, 0), yv);
    }
    __syncthreads();
    const __amdgpu_buffer_rsrc_t zr = buf_rsrc(Z + base, (size_t)ns * sizeof(TO));  // this slab of Z
    [[maybe_unused]] T oPm[4], oPj[4], oEk[4], oEm[4];  // SCALE, backward: rows j2o + row(g, r)
    if constexpr (SCALE && !FWD) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int idx[4] = {0, min(j2o + P::row(g, r), n2 - 1), sl % S.n[2], sl / S.n[2]};
        diag_row_coeffs<T>(S, dgs, idx, oPm[r], oPj[r], oEk[r], oEm[r]);
      }
    }
#pragma unroll
    for (int nt = 0; nt < NM; ++nt) {
      acc_t acc = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int kb = 0; kb < NK; ++kb)
        acc = P::mma(a2[kb], P::op(yh, yl, (16 * nt + cl) * kSlabLdy + 32 * kb + 8 * g), acc);
      const int j1 = 16 * nt + cl;
      [[maybe_unused]] T m1 = 0, k1 = 0, jj1 = 0;
      if constexpr (SCALE && !FWD) {
        const int cc = min(j1, n1 - 1);
        m1 = dgs[cc];
        k1 = dgs[n1 + cc];
        jj1 = dgs[2 * n1 + cc];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j2 = j2o + P::row(g, r);
        const bool ok = j1 < n1 && j2 < n2;
        T zf = (T)acc[r];
        if constexpr (SCALE && !FWD) zf *= diag_sigma(m1, k1, jj1, oPm[r], oPj[r], oEk[r], oEm[r]);
        const TO zv = (TO)zf;
        if constexpr (DOT) dsum += ok ? (double)zv * dv[nt * 4 + r] : 0.0;
        buf_store(zv, zr, ok ? (int)((j2 * n1 + j1) * sizeof(TO)) : kOutOfRange);
      }
    }
    if constexpr (NBUF == 1) __syncthreads();  // every wave is done with the tile
    else buf ^= 1;
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
// no copy of an in-flight value forces an early wait); the FP64 mode-3 pass
// prefetches one unit, which fits it in 128 registers and two workgroups per
// CU (37.9 -> 30.6 us at d = 3, p = 4, 48 elements).  FUSED: time mode,
//   Q(i, c) = (W X)(i, c) / (lambda_t[i] + lambda_s[c])  (FP64 division,
//             quotient rounded to T),
//   Y = W2 Q,
// with Q re-fragmented through a per-wave LDS scratch tile.  WL: the
// forward operator's fragments are read from LDS at each product instead of
// being held in registers (fewer registers, more waves per CU).
constexpr int kStridedWaves = 8;
constexpr int kStridedDepth = 2;

// waves per SIMD the registers must allow (the second launch-bounds argument)
template <int PR, bool FUSED, bool WL>
constexpr int strided_min_blocks() {
  return PR == kPrecF64 ? (FUSED ? 1 : 4) : ((WL && !FUSED) ? 4 : 2);
}

template <int PR, int NM, bool FUSED, bool WL>
__global__ __launch_bounds__(kStridedWaves * 64, (strided_min_blocks<PR, FUSED, WL>())) void fd_strided_kernel(
    const typename Prec<PR>::T* __restrict__ X, typename Prec<PR>::T* __restrict__ Y, int L, int n, int ncols,
    const typename Prec<PR>::S* __restrict__ Wh, const typename Prec<PR>::S* __restrict__ Wl,
    const typename Prec<PR>::S* __restrict__ W2h, const typename Prec<PR>::S* __restrict__ W2l,
    const double* __restrict__ lam_t, const double* __restrict__ lam_s, const PcgScalars* __restrict__ gate) {
  typedef Prec<PR> P;
  typedef typename P::T T;
  typedef typename P::S SD;
  typedef typename P::Frag Frag;
  typedef typename P::acc_t acc_t;
  if (gate && (gate->done | gate->flag)) return;  // PCG already finished: nothing to do
  constexpr int NK = (NM + 1) / 2;
  constexpr int KPAD = NK * 32;
  constexpr int LDS_S = KPAD + 4;
  constexpr int DEPTH = (PR == kPrecF64 && !FUSED) ? 1 : kStridedDepth;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, cl = lane & 15;
  // LDS: (fused) lambda_t (16 NM doubles, clamped) and the backward
  // operator [16 NM][KPAD + 8] (kHalves arrays); (WL) the forward operator,
  // same layout; (fused) the per-wave scratch tiles
  constexpr int LDV = KPAD + 8;
  constexpr int kOpBytes = P::kHalves * 16 * NM * LDV * (int)sizeof(SD);
  double* lt_lds = reinterpret_cast<double*>(smem_raw);
  SD* v2h = reinterpret_cast<SD*>(smem_raw + 16 * NM * sizeof(double));
  SD* v2l = v2h + (P::kHalves - 1) * 16 * NM * LDV;
  unsigned char* after_fused = smem_raw + (FUSED ? 16 * NM * sizeof(double) + kOpBytes : 0);
  SD* w1h = reinterpret_cast<SD*>(after_fused);
  SD* w1l = w1h + (P::kHalves - 1) * 16 * NM * LDV;
  T* myscr = reinterpret_cast<T*>(after_fused + (WL ? kOpBytes : 0)) + wave * 16 * LDS_S;
  if constexpr (FUSED || WL) {
    if constexpr (FUSED)
      for (int i = threadIdx.x; i < 16 * NM; i += blockDim.x) lt_lds[i] = lam_t[min(i, n - 1)];
    if constexpr (FUSED) {
      stage_rows<SD, KPAD, LDV>(W2h, v2h, 16 * NM);
      if constexpr (P::kHalves == 2) stage_rows<SD, KPAD, LDV>(W2l, v2l, 16 * NM);
    }
    if constexpr (WL) {
      stage_rows<SD, KPAD, LDV>(Wh, w1h, 16 * NM);
      if constexpr (P::kHalves == 2) stage_rows<SD, KPAD, LDV>(Wl, w1l, 16 * NM);
    }
    __syncthreads();
  }
  const int nunits = (ncols + 15) / 16;
  const int stride = gridDim.x * kStridedWaves;
  const int u0 = blockIdx.x * kStridedWaves + wave;
  if (u0 >= nunits) return;
  Frag wf[WL ? 1 : NM][NK];
  if constexpr (!WL) {
#pragma unroll
    for (int t = 0; t < NM; ++t)
#pragma unroll
      for (int kb = 0; kb < NK; ++kb) wf[t][kb] = P::op(Wh, Wl, (16 * t + cl) * KPAD + 32 * kb + 8 * g);
    // the operator fragments arrive before the column prefetch is issued:
    // were they queued behind it, the loop's waits (taken over the entry path
    // as well) would drain the whole prefetch on every unit
    __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (15 << 8));  // vmcnt(0)
    __builtin_amdgcn_sched_barrier(0);
  }
  const int Ln = L * n;
  auto base_of = [&](int c) -> int { return (c % L) + (c / L) * Ln; };
  const __amdgpu_buffer_rsrc_t xr = buf_rsrc(X, (size_t)ncols * n * sizeof(T));
  const __amdgpu_buffer_rsrc_t yr = buf_rsrc(Y, (size_t)ncols * n * sizeof(T));
  T pv[DEPTH][NK][8];
  // fused: lambda_s of the prefetched column, loaded after the unit's last
  // use of the slot (so the slot needs no second register and no copy)
  double pls[DEPTH];
  auto fetch = [&](int u, T (&v)[NK][8]) {  // rows k >= n read as 0 (out of range)
    const int b = base_of(min(u * 16 + cl, ncols - 1));
#pragma unroll
    for (int kb = 0; kb < NK; ++kb)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 32 * kb + 8 * g + e;
        v[kb][e] = buf_load_t(xr, k < n ? (b + k * L) * (int)sizeof(T) : kOutOfRange, T());
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
      Frag xf[NK];
#pragma unroll
      for (int kb = 0; kb < NK; ++kb) xf[kb] = P::data(pv[d][kb]);
      __builtin_amdgcn_sched_barrier(0);
      fetch(min(u + DEPTH * stride, nunits - 1), pv[d]);  // always issued: uniform load order
      __builtin_amdgcn_sched_barrier(0);
      acc_t acc[NM];
#pragma unroll
      for (int t = 0; t < NM; ++t) {
        acc[t] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int kb = 0; kb < NK; ++kb) {
          if constexpr (WL) {
            acc[t] = P::mma(P::op(w1h, w1l, (16 * t + cl) * LDV + 32 * kb + 8 * g), xf[kb], acc[t]);
          } else {
            acc[t] = P::mma(wf[t][kb], xf[kb], acc[t]);
          }
        }
      }
      if constexpr (FUSED) {
#pragma unroll
        for (int t = 0; t < NM; ++t) {
          T q[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            // eigenvalue sum and division in FP64, the quotient rounded
            // once to T (the precision of the pass's output)
            const int i = 16 * t + P::row(g, r);
            const T qv = (T)((double)acc[t][r] / (lt_lds[i] + pls[d]));
            q[r] = i < n ? qv : (T)0;
          }
          put4t(myscr, cl * LDS_S + 16 * t + P::row(g, 0), q);
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int kb = 0; kb < NK; ++kb) {
          T v[8];
          get8t(myscr + cl * LDS_S + 32 * kb + 8 * g, v);
          // rows past n (including the k padding the tile never holds) are zero
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = 32 * kb + 8 * g + e < n ? v[e] : (T)0;
          xf[kb] = P::data(v);
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int t = 0; t < NM; ++t) {
          acc[t] = acc_t{0, 0, 0, 0};
#pragma unroll
          for (int kb = 0; kb < NK; ++kb)
            acc[t] = P::mma(P::op(v2h, v2l, (16 * t + cl) * LDV + 32 * kb + 8 * g), xf[kb], acc[t]);
        }
      }
      {
        const bool colok = u < nunits && c < ncols;
        const int b = base_of(min(c, ncols - 1));
#pragma unroll
        for (int t = 0; t < NM; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 16 * t + P::row(g, r);
            buf_store((T)acc[t][r], yr, colok && i < n ? (b + i * L) * (int)sizeof(T) : kOutOfRange);
          }
      }
      if constexpr (FUSED) pls[d] = lam_s[min(min(u + DEPTH * stride, nunits - 1) * 16 + cl, ncols - 1)];
    }
  }
}

// Operator storage of direction D for precision PR: (hi, lo) pointers.
template <int PR>
void operators(const DevDir& D, bool fwd, const typename Prec<PR>::S*& hi, const typename Prec<PR>::S*& lo) {
  if constexpr (PR == kPrecBf16x3) {
    hi = (const __bf16*)(fwd ? D.Hfwd : D.Hbwd);
    lo = (const __bf16*)(fwd ? D.Lfwd : D.Lbwd);
  } else if constexpr (PR == kPrecF32) {
    hi = lo = fwd ? D.Rfwd32 : D.Rbwd32;
  } else {
    hi = lo = fwd ? D.Rfwd64 : D.Rbwd64;
  }
}

template <int PR, int NM, bool FWD, bool DOT, bool SCALE>
int launch_slab(stls_ctx* h, const void* X, void* Z, const double* dotv, double* partials, int* nparts) {
  typedef Prec<PR> P;
  typedef typename P::T T;
  typedef typename std::conditional<FWD, double, T>::type TI;
  typedef typename std::conditional<FWD, T, double>::type TO;
  const DevDir& D1 = h->dd[0];
  const DevDir& D2 = h->dd[1];
  const int n1 = D1.n, n2 = D2.n;
  const int nslab = (int)(h->ndof / ((int64_t)n1 * n2));
  const int blocks = std::min(nslab, 2 * 256);
  if (nparts) *nparts = blocks;
  const size_t shmem = slab_lds_bytes<PR>(NM);
  const typename P::S *W1h, *W1l, *W2h, *W2l;
  operators<PR>(D1, FWD, W1h, W1l);
  operators<PR>(D2, FWD, W2h, W2l);
  auto kern = fd_slab_kernel<PR, NM, FWD, DOT, SCALE>;
  if (shmem > 65536) {
    const hipError_t ea = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (ea != hipSuccess) return hip_fail(ea, "hipFuncSetAttribute(LDS)");
  }
  prof_begin(h);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), shmem, h->stream, (const TI*)X, (TO*)Z, n1, n2, nslab, W1h, W1l,
                     W2h, W2l, dotv, partials, h->gate, diag_scale_args(h));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "fd_slab_kernel launch");
  prof_end(h, FWD ? PROF_FD_SLAB : PROF_FD_SLAB_BWD);
  return STLS_OK;
}

// Forward operator in LDS (WL) for the fused time pass: measured on the
// d = 3, p = 4, 48-element workload in bf16x3, 23 us with it (128
// registers, two workgroups per CU) against 26 us without; the bf16x3 and
// FP32 mode-3 passes keep the operator in registers (17.5 us against 18.6
// us in bf16x3); the FP64 operator (128 registers in registers) goes to LDS
// in both passes.
template <int PR, bool FUSED>
constexpr bool ops_in_lds() {
  return FUSED || PR == kPrecF64;
}

template <int PR, int NM, bool FUSED>
int launch_strided(stls_ctx* h, const void* X, void* Y, int L, int k, bool fwd, const double* lam_t) {
  typedef Prec<PR> P;
  typedef typename P::T T;
  constexpr bool WL = ops_in_lds<PR, FUSED>();
  const DevDir& D = h->dd[k];
  const int n = D.n;
  const int ncols = (int)(h->ndof / n);
  const int nunits = (ncols + 15) / 16;
  constexpr int NK = (NM + 1) / 2;
  const size_t op_bytes = sizeof(typename P::S) * P::kHalves * 16 * NM * (NK * 32 + 8);
  const size_t shmem =
      (FUSED ? sizeof(double) * 16 * NM + op_bytes + sizeof(T) * kStridedWaves * 16 * (NK * 32 + 4) : 0) +
      (WL ? op_bytes : 0);
  // operator in registers: one persistent workgroup per CU (256 / 512 /
  // 1024 workgroups gave 17.4 / 20.8 / 29.8 us for the bf16x3 mode-3 pass);
  // operators in LDS: as many per CU as the LDS holds, at most two
  const int per_cu = !WL ? 1 : (int)std::max<size_t>(1, std::min<size_t>(2, (160 * 1024) / shmem));
  const int blocks = std::max(1, std::min((nunits + kStridedWaves - 1) / kStridedWaves, 256 * per_cu));
  const typename P::S *Wh, *Wl, *W2h = nullptr, *W2l = nullptr;
  operators<PR>(D, fwd, Wh, Wl);
  if (FUSED) operators<PR>(D, false, W2h, W2l);
  auto kern = fd_strided_kernel<PR, NM, FUSED, WL>;
  if (shmem > 65536) {
    const hipError_t ea = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (ea != hipSuccess) return hip_fail(ea, "hipFuncSetAttribute(LDS)");
  }
  prof_begin(h);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(kStridedWaves * 64), shmem, h->stream, (const T*)X, (T*)Y, L, n, ncols,
                     Wh, Wl, W2h, W2l, lam_t, h->lam_s, h->gate);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "fd_strided_kernel launch");
  prof_end(h, FUSED ? PROF_FD_TIME : PROF_FD_SPACE);
  return STLS_OK;
}

template <int PR, bool FUSED>
int strided_nm(stls_ctx* h, const void* X, void* Y, int L, int k, bool fwd, const double* lam_t) {
  switch (h->dd[k].npad / 16) {
    case 1: return launch_strided<PR, 1, FUSED>(h, X, Y, L, k, fwd, lam_t);
    case 2: return launch_strided<PR, 2, FUSED>(h, X, Y, L, k, fwd, lam_t);
    case 3: return launch_strided<PR, 3, FUSED>(h, X, Y, L, k, fwd, lam_t);
    case 4: return launch_strided<PR, 4, FUSED>(h, X, Y, L, k, fwd, lam_t);
    default: set_error("direction too large for the strided FD pass"); return STLS_EINVAL;
  }
}

template <int PR, bool FWD, bool DOT, bool SCALE>
int slab_nm(stls_ctx* h, const void* X, void* Z, const double* dotv, double* partials, int* nparts) {
  switch (h->dd[0].npad / 16) {
    case 1: return launch_slab<PR, 1, FWD, DOT, SCALE>(h, X, Z, dotv, partials, nparts);
    case 2: return launch_slab<PR, 2, FWD, DOT, SCALE>(h, X, Z, dotv, partials, nparts);
    case 3: return launch_slab<PR, 3, FWD, DOT, SCALE>(h, X, Z, dotv, partials, nparts);
    case 4: return launch_slab<PR, 4, FWD, DOT, SCALE>(h, X, Z, dotv, partials, nparts);
    default: set_error("direction too large for the slab FD pass"); return STLS_EINVAL;
  }
}

template <int PR, bool SCALE>
int five_pass(stls_ctx* h, const double* r, double* s, const double* dot_with, double* partials, int* nparts) {
  void* b0 = h->fdbuf[0];
  void* b1 = h->fdbuf[1];
  const int n1 = h->dir[0].n, n2 = h->dir[1].n;
  const int L3 = n1 * n2;
  const int ns = (int)h->ns;
  int st;
  if ((st = slab_nm<PR, true, false, SCALE>(h, r, b0, nullptr, nullptr, nullptr))) return st;
  if ((st = strided_nm<PR, false>(h, b0, b1, L3, 2, true, nullptr))) return st;
  if ((st = strided_nm<PR, true>(h, b1, b0, ns, 3, true, h->dd[3].lam))) return st;
  if ((st = strided_nm<PR, false>(h, b0, b1, L3, 2, false, nullptr))) return st;
  if (dot_with) return slab_nm<PR, false, true, SCALE>(h, b1, s, dot_with, partials, nparts);
  return slab_nm<PR, false, false, SCALE>(h, b1, s, nullptr, nullptr, nparts);
}

template <int PR>
int five_pass_scaled(stls_ctx* h, const double* r, double* s, const double* dot_with, double* partials, int* nparts,
                     bool scale) {
  return scale ? five_pass<PR, true>(h, r, s, dot_with, partials, nparts)
               : five_pass<PR, false>(h, r, s, dot_with, partials, nparts);
}

}  // namespace

// Shapes covered: d = 3, every restricted size <= 64, n1 even, directions 1
// and 2 padded alike, and the work vectors of the precision's intermediates
// addressable by one buffer resource (byte offsets below 2^31; out-of-range
// lanes use 0x7fffffff).
bool fd_five_pass_covers(const stls_ctx* h) {
  if (h->d != 3 || h->fd_mode == STLS_FD_ASYM) return false;
  for (int k = 0; k <= 3; ++k)
    if (h->dir[k].n > 64) return false;
  if (h->dir[0].n % 2 != 0 || h->dd[0].npad != h->dd[1].npad) return false;
  const int64_t tsize = h->fd_mode == STLS_FD_FP64 ? 8 : 4;
  return h->ndof * tsize < ((int64_t)1 << 31) - 1;
}

int prec_apply_five_pass(stls_ctx* h, const double* r, double* s, const double* dot_with, double* partials, int* nparts,
                         bool scale) {
  switch (h->fd_mode) {
    case STLS_FD_FP64: return five_pass_scaled<kPrecF64>(h, r, s, dot_with, partials, nparts, scale);
    case STLS_FD_FP32: return five_pass_scaled<kPrecF32>(h, r, s, dot_with, partials, nparts, scale);
    case STLS_FD_BF16X3: return five_pass_scaled<kPrecBf16x3>(h, r, s, dot_with, partials, nparts, scale);
    default: set_error("unknown FD precision"); return STLS_EINVAL;
  }
}

}  // namespace stls
