// Device side of the diagonal scaling of the FD preconditioner (§4.4,
// closing definition): P^G = D^1/2 P D^1/2 with D_ii = A_ii / P_ii, so that
// (P^G)^-1 r = sigma o P^-1 (sigma o r), sigma_i = (P_ii / A_ii)^1/2.
//
// On the unit box both diagonals are sums of products of univariate
// diagonals (the diagonal of a Kronecker product is the product of the
// factors' diagonals).  With m, k, j the diagonals of the restricted M, K, J
// of each space direction, k_t, m_t those of time and w the final-time entry
// of W_t:
//   P_ii = k_t prod m + kappa^2 m_t sum_a j_a prod_{b!=a} m_b
//   A_ii = P_ii + 2 kappa^2 m_t sum_{a<b} k_a k_b prod_{c!=a,b} m_c
//               + kappa w [t = n_t - 1] sum_a k_a prod_{b!=a} m_b
// Grouped by the entries of direction 1 at a fixed (i_2 .. i_d, t):
//   P_ii = m_1 Pm + j_1 Pj,   A_ii - P_ii = k_1 Ek + m_1 Em.
#pragma once

#include "stls_internal.h"

namespace stls {

__device__ inline double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// g: the packed diagonals (S.g, S.g32 or a copy of either with the same
// layout); idx[1 .. d-1]: space indices of directions 2..d, idx[d]: time.
template <typename T>
__device__ inline void diag_row_coeffs(const DiagScale& S, const T* g, const int* idx, T& Pm, T& Pj, T& Ek, T& Em) {
  // running sums over the directions 2..d taken so far:
  //   pm = prod m, sj = sum j prod m, sk = sum k prod m, skk = sum_{a<b} k k prod m
  T pm = 1, sj = 0, sk = 0, skk = 0;
#pragma unroll
  for (int a = 1; a < kMaxDim; ++a) {
    if (a >= S.d) break;
    const T* ga = g + S.off[a];
    const int i = idx[a];
    const T m = ga[i], kk = ga[S.n[a] + i], jj = ga[2 * S.n[a] + i];
    skk = fma_t(skk, m, sk * kk);
    sk = fma_t(sk, m, pm * kk);
    sj = fma_t(sj, m, pm * jj);
    pm = pm * m;
  }
  const int t = idx[S.d];
  const T* gt = g + S.off[S.d];
  const T kt = gt[t], mt = gt[S.n[S.d] + t];
  const T w = t == S.n[S.d] - 1 ? (T)S.kw : (T)0;
  const T k2mt = (T)S.k2 * mt;
  Pm = fma_t(kt, pm, k2mt * sj);
  Pj = k2mt * pm;
  Ek = fma_t((T)2 * k2mt, sk, w * pm);
  Em = fma_t((T)2 * k2mt, skk, w * sk);
}

// sigma = (P_ii / A_ii)^1/2 from the direction-1 entries (m1, k1, j1).
__device__ inline double diag_sigma(double m1, double k1, double j1, double Pm, double Pj, double Ek, double Em) {
  const double p = __builtin_fma(m1, Pm, j1 * Pj);
  const double a = p + __builtin_fma(k1, Ek, m1 * Em);
  return sqrt(p / a);
}
// FP32 (paths whose products are FP32 or bf16x3): hardware reciprocal and
// reciprocal square root, about 1 ulp each.
__device__ inline float diag_sigma(float m1, float k1, float j1, float Pm, float Pj, float Ek, float Em) {
  const float p = __builtin_fmaf(m1, Pm, j1 * Pj);
  const float a = p + __builtin_fmaf(k1, Ek, m1 * Em);
  return __builtin_amdgcn_rsqf(a * __builtin_amdgcn_rcpf(p));
}

}  // namespace stls
