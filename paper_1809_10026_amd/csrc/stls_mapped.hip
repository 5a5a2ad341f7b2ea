// Kernels of the stls library for mapped spatial domains (gfx950):
//   y = (K_t (x) M_s + kappa^2 M_t (x) J_s + kappa W_t (x) L_s) x
// with the pulled-back spatial factors stored as stencils [S][ns] (row i's
// entry for column offset o at o*ns + i; §4.1 with the geometry of §2.2),
// the diagonal scaling of P^G = D^1/2 Pbar^G D^1/2 (§4.4), and the
// element-by-element assembly of the stencils.
//
// The matvec runs in two passes.  The spatial stencils first, on every time
// slice:
//   U(:, t) = M_s x(:, t),  V(:, t) = J_s x(:, t),  Lx = L_s x(:, final slice)
// one workgroup per (block of rows, chunk of slices): the block's x values
// with their halo of p_k rows are staged in LDS slice by slice, and each
// thread reads its row's stencil entries once per chunk and applies them to
// every slice of the chunk (read x, write U and V: 24 B/DOF, plus the
// stencils).  Then the time band:
//   y(:, t) = sum_tau K_t(t, tau) U(:, tau) + kappa^2 M_t(t, tau) V(:, tau)
//             [+ kappa w Lx at the final slice]
// with the p^T q dot fused (read U, V, write y: 24 B/DOF).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "stls_buf.h"
#include "stls_geomap.h"
#include "stls_internal.h"

namespace stls {

namespace {

constexpr int kMT = 256;
constexpr int kMapBlocks = 8192;
constexpr int kMapLds = 80 * 1024;  // LDS budget of a spatial-pass workgroup (two per CU)
constexpr int kSG = 4;              // stencil entries per prefetch group
constexpr int kStageLines = 8;      // staged lines per wave with their loads in flight
// Row blocks of the spatial pass, 256 rows: 32 or 16 along direction 1 (with
// 32, a half-wave reads one run of 32 consecutive rows).
constexpr int kBlk3W[3] = {32, 2, 4}, kBlk3N[3] = {16, 4, 4};
constexpr int kBlk2W[3] = {32, 8, 1}, kBlk2N[3] = {16, 16, 1};

__device__ inline bool finished(const PcgScalars* gate) { return gate && (gate->done | gate->flag); }

// Workgroup index -> work item, so that consecutive work items (the chunks
// of one row block, which read the same stencil rows) land on the same XCD
// (workgroups are dealt to the 8 XCDs round robin).
__device__ inline int xcd_group(int bid, int nblocks) {
  constexpr int kXcd = 8;
  const int full = nblocks - nblocks % kXcd;
  if (bid >= full) return bid;
  return (bid % kXcd) * (full / kXcd) + bid / kXcd;
}

struct MapTile {
  int d, ns, nt, nchunk, nblk, tt;
  int bufsten;  // every stencil below 2 GiB: buffer-addressed loads
  int n[3], p[3], B[3], T[3], nb[3];
  int tsz;  // T[0] T[1] T[2]: staged values per slice
};

// One row of the spatial pass: U, V (and for the final chunk L_s x) over the
// chunk's slices.  xb: the row's place in the staged block; stencil entries
// kSG at a time, the next group in flight while the current one is applied
// (offsets past S re-read the last entry, unused); the offset's row of a
// stencil is a wave-uniform base and the row a 32-bit byte offset.
template <int TT, bool LAST>
__device__ __forceinline__ void space_rows(const double* xb, int T0, int T1, int bw0, int bw1, int S, int ns,
                                           unsigned urow, int tn, const double* __restrict__ Ms,
                                           const double* __restrict__ Js, const double* __restrict__ Ls,
                                           double (&au)[TT], double (&av)[TT], double& al) {
#pragma unroll
  for (int u = 0; u < TT; ++u) au[u] = av[u] = 0.0;
  al = 0.0;
  const unsigned boff = urow * 8u;
  auto at = [&](const double* base, int o) {
    return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base + (size_t)o * ns) + boff);
  };
  double mc[kSG], jc[kSG], lc[kSG], mn[kSG], jn[kSG], ln[kSG];
  auto fetch = [&](int g, double* mm, double* jj, double* ll) {
#pragma unroll
    for (int k = 0; k < kSG; ++k) {
      const int o = min(g + k, S - 1);
      mm[k] = at(Ms, o);
      jj[k] = at(Js, o);
      if constexpr (LAST) ll[k] = at(Ls, o);
    }
  };
  fetch(0, mc, jc, lc);
  int q0 = 0, q1 = 0, lo = 0;  // offset (q0, q1, q2) and its place in the staged block
  for (int g = 0; g < S; g += kSG) {
    fetch(g + kSG, mn, jn, ln);
#pragma unroll
    for (int k = 0; k < kSG; ++k) {
      if (g + k < S) {
        const double* xp = xb + lo * TT;
        double xv[TT];
        if constexpr (TT % 2 == 0) {
#pragma unroll
          for (int u = 0; u < TT; u += 2) {
            const double2 t2 = *reinterpret_cast<const double2*>(xp + u);
            xv[u] = t2.x;
            xv[u + 1] = t2.y;
          }
        } else {
#pragma unroll
          for (int u = 0; u < TT; ++u) xv[u] = xp[u];
        }
#pragma unroll
        for (int u = 0; u < TT; ++u) {  // slices past the chunk's end read unused LDS and are dropped
          au[u] += mc[k] * xv[u];
          av[u] += jc[k] * xv[u];
        }
        if constexpr (LAST) al += lc[k] * xp[tn - 1];
        ++lo;
        if (++q0 == bw0) {
          q0 = 0;
          lo += T0 - bw0;
          if (++q1 == bw1) {
            q1 = 0;
            lo += T0 * (T1 - bw1);
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kSG; ++k) {
      mc[k] = mn[k];
      jc[k] = jn[k];
      if constexpr (LAST) lc[k] = ln[k];
    }
  }
}

// The same for a direction-1 stencil width BW0 known at compile time, with
// stencils below 2 GiB: the loop over the lines (q1, q2) of the offset box
// keeps BW0 offsets unrolled, so the LDS reads of a line take immediate
// offsets; the stencil entries come through buffer loads whose scalar
// offset is the only per-offset scalar work, one line in flight while the
// previous one is applied.
template <int TT, bool LAST, int BW0>
__device__ __forceinline__ void space_rows_u(const double* xb, int T0, int T1, int bw1, int bw2, int nsb,
                                             unsigned boff, int tn, __amdgpu_buffer_rsrc_t rM,
                                             __amdgpu_buffer_rsrc_t rJ, __amdgpu_buffer_rsrc_t rL,
                                             double (&au)[TT], double (&av)[TT], double& al) {
#pragma unroll
  for (int u = 0; u < TT; ++u) au[u] = av[u] = 0.0;
  al = 0.0;
  const int nline = bw1 * bw2;
  auto ld = [&](__amdgpu_buffer_rsrc_t r, int so) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)boff, so, 0));
  };
  // two lines in flight: buffers A and B alternate, each refilled with the
  // line after next as soon as it has been applied
  double ma[BW0], ja[BW0], la[BW0], mb[BW0], jb[BW0], lb[BW0];
  auto fetch = [&](int line, double* mm, double* jj, double* ll) {
    const int so = min(line, nline - 1) * (BW0 * nsb);
#pragma unroll
    for (int q0 = 0; q0 < BW0; ++q0) {
      mm[q0] = ld(rM, so + q0 * nsb);
      jj[q0] = ld(rJ, so + q0 * nsb);
      if constexpr (LAST) ll[q0] = ld(rL, so + q0 * nsb);
    }
  };
  int q1 = 0, lbase = 0;  // line (q1, q2) of the offset box and its first staged value
  auto apply = [&](const double* mm, const double* jj, const double* ll) {
    const double* xp = xb + lbase * TT;
#pragma unroll
    for (int q0 = 0; q0 < BW0; ++q0) {
      double xv[TT];
      if constexpr (TT % 2 == 0) {
#pragma unroll
        for (int u = 0; u < TT; u += 2) {
          const double2 t2 = *reinterpret_cast<const double2*>(xp + q0 * TT + u);
          xv[u] = t2.x;
          xv[u + 1] = t2.y;
        }
      } else {
#pragma unroll
        for (int u = 0; u < TT; ++u) xv[u] = xp[q0 * TT + u];
      }
#pragma unroll
      for (int u = 0; u < TT; ++u) {
        au[u] += mm[q0] * xv[u];
        av[u] += jj[q0] * xv[u];
      }
      if constexpr (LAST) al += ll[q0] * xp[q0 * TT + tn - 1];
    }
    lbase += T0;
    if (++q1 == bw1) {
      q1 = 0;
      lbase += T0 * (T1 - bw1);
    }
  };
  fetch(0, ma, ja, la);
  fetch(1, mb, jb, lb);
  for (int line = 0; line < nline; line += 2) {
    apply(ma, ja, la);
    fetch(line + 2, ma, ja, la);
    if (line + 1 < nline) apply(mb, jb, lb);
    fetch(line + 3, mb, jb, lb);
  }
}

template <int TT, bool LAST>
__device__ __forceinline__ void space_row_any(const double* xb, const MapTile& tl, int bw0, int bw1, int bw2,
                                              unsigned urow, int tn, const double* Ms, const double* Js,
                                              const double* Ls, double (&au)[TT], double (&av)[TT], double& al) {
  const int T0 = tl.T[0], T1 = tl.T[1], S = bw0 * bw1 * bw2, ns = tl.ns;
  if (tl.bufsten && (bw0 == 5 || bw0 == 7 || bw0 == 9)) {
    const int bytes = S * ns * 8;
    const auto rM = buf_rsrc(Ms, bytes), rJ = buf_rsrc(Js, bytes), rL = buf_rsrc(Ls, bytes);
    const unsigned boff = urow * 8u;
    if (bw0 == 5) space_rows_u<TT, LAST, 5>(xb, T0, T1, bw1, bw2, ns * 8, boff, tn, rM, rJ, rL, au, av, al);
    else if (bw0 == 7) space_rows_u<TT, LAST, 7>(xb, T0, T1, bw1, bw2, ns * 8, boff, tn, rM, rJ, rL, au, av, al);
    else space_rows_u<TT, LAST, 9>(xb, T0, T1, bw1, bw2, ns * 8, boff, tn, rM, rJ, rL, au, av, al);
  } else {
    space_rows<TT, LAST>(xb, T0, T1, bw0, bw1, S, ns, urow, tn, Ms, Js, Ls, au, av, al);
  }
}

template <int TT>
__global__ __launch_bounds__(kMT) void mapped_space_kernel(const double* __restrict__ x, double* __restrict__ U,
                                                           double* __restrict__ V, double* __restrict__ Lx,
                                                           MapTile tl, const double* __restrict__ Ms,
                                                           const double* __restrict__ Js,
                                                           const double* __restrict__ Ls,
                                                           const PcgScalars* __restrict__ gate) {
  if (finished(gate)) return;
  extern __shared__ double xs[];  // [tsz][TT]: the chunk's slices of a staged value side by side
  const int w = xcd_group(blockIdx.x, tl.nblk * tl.nchunk);
  const int blk = w / tl.nchunk, ch = w - blk * tl.nchunk;
  const int n0 = tl.n[0], n1 = tl.n[1], n2 = tl.n[2], ns = tl.ns;
  const int T0 = tl.T[0], T1 = tl.T[1], tsz = tl.tsz;
  const int c0 = (blk % tl.nb[0]) * tl.B[0], c1 = ((blk / tl.nb[0]) % tl.nb[1]) * tl.B[1],
            c2 = (blk / (tl.nb[0] * tl.nb[1])) * tl.B[2];
  const int t0 = ch * TT, tn = min(TT, tl.nt - t0);
  // halo'd block of every slice of the chunk, zero outside the box: each
  // wave stages whole lines of T0 (<= 64) values along direction 1, every
  // fourth line (line coordinates wave-uniform and advanced incrementally),
  // kStageLines lines with all their loads in flight before the LDS stores
  {
    const int T2 = tl.T[2], t12 = T1 * T2, nline = tn * t12;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
    const int g0 = c0 + lane - tl.p[0];
    const bool in0 = lane < T0 && g0 >= 0 && g0 < n0;
    int l1 = wv % T1, l2 = (wv / T1) % T2, u = wv / t12;  // coordinates of line lb
    for (int lb = wv; lb < nline; lb += (kMT / 64) * kStageLines) {
      double v[kStageLines];
      int dst[kStageLines];
#pragma unroll
      for (int b = 0; b < kStageLines; ++b) {
        const int ln = lb + (kMT / 64) * b;
        const int g1 = c1 + l1 - tl.p[1], g2 = c2 + l2 - tl.p[2];
        const bool ok = ln < nline && in0 && g1 >= 0 && g1 < n1 && g2 >= 0 && g2 < n2;
        // unconditional load from a clamped index, then a select: no branch
        // around the load, so all of a batch's loads are in flight together
        const double xv = x[ok ? (t0 + u) * ns + n0 * (g1 + n1 * g2) + g0 : 0];
        v[b] = ok ? xv : 0.0;
        dst[b] = ln < nline && lane < T0 ? ((l1 + T1 * l2) * T0 + lane) * TT + u : -1;
        l1 += kMT / 64;  // next line of this wave
        while (l1 >= T1) {
          l1 -= T1;
          if (++l2 == T2) {
            l2 = 0;
            ++u;
          }
        }
      }
#pragma unroll
      for (int b = 0; b < kStageLines; ++b)
        if (dst[b] >= 0) xs[dst[b]] = v[b];
    }
  }
  __syncthreads();
  const int B0 = tl.B[0], B1 = tl.B[1];
  const int r0 = threadIdx.x % B0, r1 = (threadIdx.x / B0) % B1, r2 = threadIdx.x / (B0 * B1);
  const int i0 = c0 + r0, i1 = c1 + r1, i2 = c2 + r2;
  if (r2 >= tl.B[2] || i0 >= n0 || i1 >= n1 || i2 >= n2) return;
  const int row = i0 + n0 * (i1 + n1 * i2);
  const unsigned urow = (unsigned)row;
  const bool last = t0 + tn == tl.nt;  // the chunk holds the final slice
  const int bw0 = 2 * tl.p[0] + 1, bw1 = 2 * tl.p[1] + 1, bw2 = 2 * tl.p[2] + 1;
  const int eb = r0 + T0 * (r1 + T1 * r2);
  double au[TT], av[TT], al = 0.0;
  if (last)
    space_row_any<TT, true>(xs + eb * TT, tl, bw0, bw1, bw2, urow, tn, Ms, Js, Ls, au, av, al);
  else
    space_row_any<TT, false>(xs + eb * TT, tl, bw0, bw1, bw2, urow, tn, Ms, Js, Ls, au, av, al);
#pragma unroll
  for (int u = 0; u < TT; ++u)
    if (u < tn) {
      U[(size_t)(t0 + u) * ns + row] = au[u];
      V[(size_t)(t0 + u) * ns + row] = av[u];
    }
  if (last) Lx[row] = al;
}

// Time band: one thread per (row, chunk of tc slices), the chunk's slices in
// turn, so that the band's overlapping taps of U and V come from the
// thread's own recent loads; consecutive workgroups take consecutive rows of
// one chunk.  tc: 8, or fewer where that leaves under 1024 work items.

template <bool DOT>
__global__ __launch_bounds__(kMT) void mapped_time_kernel(const double* __restrict__ U, const double* __restrict__ V,
                                                          const double* __restrict__ Lx, double* __restrict__ y,
                                                          int ns, int nt, int pt, int tc,
                                                          const double* __restrict__ Kt,
                                                          const double* __restrict__ Mt, double k2, double kw,
                                                          const double* __restrict__ dotv,
                                                          double* __restrict__ partials,
                                                          const PcgScalars* __restrict__ gate) {
  if (finished(gate)) return;
  __shared__ double red[kMT / 64];
  const int bw = 2 * pt + 1;
  const int nrb = (ns + kMT - 1) / kMT, nch = (nt + tc - 1) / tc;
  double dsum = 0.0;
  for (int w = blockIdx.x; w < nrb * nch; w += gridDim.x) {
    const int rb = w % nrb, ch = w / nrb;
    const int is = rb * kMT + threadIdx.x;
    if (is >= ns) continue;
    const int t1 = min(nt, (ch + 1) * tc);
    for (int t = ch * tc; t < t1; ++t) {
      double a = 0.0;
      for (int o = 0; o < bw; ++o) {
        const int tau = t + o - pt;
        if (tau < 0 || tau >= nt) continue;
        const size_t g = (size_t)tau * ns + is;
        a += Kt[t * bw + o] * U[g] + k2 * Mt[t * bw + o] * V[g];
      }
      if (t == nt - 1) a += kw * Lx[is];
      const size_t e = (size_t)t * ns + is;
      y[e] = a;
      if constexpr (DOT) dsum += a * dotv[e];
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

// ---------------------------------------------------------------------------
// Assembly of the stencils of M_s, J_s, L_s, element by element.
//
// One workgroup per element (a product of non-empty spans).  Its
// nf = prod (p_k + 1) functions pair up into nf^2 (test a, trial b) entries;
// each thread owns kAsmPairs of them per pass and sums over the element's
// quadrature points
//   M += W B_a B_b,   J += W Lap_a Lap_b,   L += W grad_a . g grad_b
// (W = weight x |det J|), with the points taken kAsmChunk-wise: the metric
// of a chunk's points and the basis data of every (point, function) are
// formed once into LDS, then read by all pairs.  The element's sums are
// added into row a's stencil at offset b - a.  Elements whose span indices
// agree modulo p_k + 1 in every direction share no function, so each launch
// takes one such colour and adds without atomics; the colours run in a
// fixed order, and every stencil entry is summed in the same order on every
// run.
constexpr int kAsmThreads = 256;
constexpr int kAsmPairs = 4;
constexpr int kAsmMet = 10;  // W, g00 g01 g02 g11 g12 g22, Lap eta_0..2

struct AsmArgs {
  int d, geom, nf, nq, qc, passes;
  int nel[3], q[3], p[3], n[3], bw[3];
  int col[3], ncol[3];
  long long ns;
  const double* x[3];
  const double* w[3];
  const double* v[3];
  const int* first[3];
  double* M;
  double* J;
  double* L;
};

__global__ __launch_bounds__(kAsmThreads) void mapped_assemble_kernel(AsmArgs a) {
  extern __shared__ double lds[];
  double* met = lds;                  // [qc][kAsmMet]
  double* bd = lds + a.qc * kAsmMet;  // [qc][8][nf]: B, grad (3), W g grad (3), Lap
  int e[3] = {0, 0, 0};
  {
    int r = blockIdx.x;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (k < a.d) {
        e[k] = a.col[k] + (r % a.ncol[k]) * (a.p[k] + 1);
        r /= a.ncol[k];
      }
  }
  const int tid = threadIdx.x;
  const int nf = a.nf, npair = nf * nf;
  for (int pass = 0; pass < a.passes; ++pass) {
    double accM[kAsmPairs], accJ[kAsmPairs], accL[kAsmPairs];
    int pa[kAsmPairs], pb[kAsmPairs];
#pragma unroll
    for (int j = 0; j < kAsmPairs; ++j) {
      const int pr = (pass * kAsmPairs + j) * kAsmThreads + tid;
      pa[j] = pr < npair ? pr / nf : -1;
      pb[j] = pr < npair ? pr % nf : 0;
      accM[j] = accJ[j] = accL[j] = 0.0;
    }
    for (int q0 = 0; q0 < a.nq; q0 += a.qc) {
      const int qn = min(a.qc, a.nq - q0);
      if (tid < qn) {
        int qi = q0 + tid;
        double eta[3] = {0.0, 0.0, 0.0}, wt = 1.0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
          if (k < a.d) {
            const int pt = e[k] * a.q[k] + qi % a.q[k];
            qi /= a.q[k];
            eta[k] = a.x[k][pt];
            wt *= a.w[k][pt];
          }
        Metric m = {};
        metric_at(a.geom, a.d, eta, m);
        double* o = met + tid * kAsmMet;
        o[0] = m.det * wt;
        o[1] = m.g[0][0];
        o[2] = m.g[0][1];
        o[3] = m.g[0][2];
        o[4] = m.g[1][1];
        o[5] = m.g[1][2];
        o[6] = m.g[2][2];
        o[7] = m.lap[0];
        o[8] = m.lap[1];
        o[9] = m.lap[2];
      }
      __syncthreads();
      for (int it = tid; it < qn * nf; it += kAsmThreads) {
        const int qc = it / nf, f = it % nf;
        int qi = q0 + qc, fr = f;
        double v0[3] = {1.0, 1.0, 1.0}, v1[3] = {0.0, 0.0, 0.0}, v2[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 3; ++k)
          if (k < a.d) {
            const int pc = a.p[k] + 1;
            const int pt = e[k] * a.q[k] + qi % a.q[k], c = fr % pc;
            qi /= a.q[k];
            fr /= pc;
            const double* vv = a.v[k] + (size_t)pt * 3 * pc;
            v0[k] = vv[c];
            v1[k] = vv[pc + c];
            v2[k] = vv[2 * pc + c];
          }
        const double* m = met + qc * kAsmMet;
        const double B = v0[0] * v0[1] * v0[2];
        const double g0 = v1[0] * v0[1] * v0[2], g1 = v0[0] * v1[1] * v0[2], g2 = v0[0] * v0[1] * v1[2];
        const double h00 = v2[0] * v0[1] * v0[2], h11 = v0[0] * v2[1] * v0[2], h22 = v0[0] * v0[1] * v2[2];
        const double h01 = v1[0] * v1[1] * v0[2], h02 = v1[0] * v0[1] * v1[2], h12 = v0[0] * v1[1] * v1[2];
        const double lap = m[1] * h00 + m[4] * h11 + m[6] * h22 + 2.0 * (m[2] * h01 + m[3] * h02 + m[5] * h12) +
                           m[7] * g0 + m[8] * g1 + m[9] * g2;
        const double W = m[0];
        double* o = bd + (size_t)qc * 8 * nf + f;
        o[0] = B;
        o[nf] = g0;
        o[2 * nf] = g1;
        o[3 * nf] = g2;
        o[4 * nf] = W * (m[1] * g0 + m[2] * g1 + m[3] * g2);
        o[5 * nf] = W * (m[2] * g0 + m[4] * g1 + m[5] * g2);
        o[6 * nf] = W * (m[3] * g0 + m[5] * g1 + m[6] * g2);
        o[7 * nf] = lap;
      }
      __syncthreads();
      for (int qc = 0; qc < qn; ++qc) {
        const double W = met[qc * kAsmMet];
        const double* base = bd + (size_t)qc * 8 * nf;
#pragma unroll
        for (int j = 0; j < kAsmPairs; ++j) {
          if (pa[j] < 0) continue;
          const double* ta = base + pa[j];
          const double* tb = base + pb[j];
          accM[j] += W * ta[0] * tb[0];
          accJ[j] += W * ta[7 * nf] * tb[7 * nf];
          accL[j] += ta[4 * nf] * tb[nf] + ta[5 * nf] * tb[2 * nf] + ta[6 * nf] * tb[3 * nf];
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < kAsmPairs; ++j) {
      if (pa[j] < 0) continue;
      int fa = pa[j], fb = pb[j];
      long long row = 0, rs = 1;
      int o = 0, os = 1;
      bool ok = true;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (k < a.d) {
          const int pc = a.p[k] + 1;
          const int ra = a.first[k][e[k]] + fa % pc, rb = a.first[k][e[k]] + fb % pc;
          fa /= pc;
          fb /= pc;
          ok = ok && ra >= 0 && ra < a.n[k] && rb >= 0 && rb < a.n[k];
          row += (long long)ra * rs;
          rs *= a.n[k];
          o += (rb - ra + a.p[k]) * os;
          os *= a.bw[k];
        }
      if (!ok) continue;
      const size_t at = (size_t)o * (size_t)a.ns + (size_t)row;
      a.M[at] += accM[j];
      a.J[at] += accJ[j];
      a.L[at] += accL[j];
    }
  }
}

int blocks_for(long long n) {
  return (int)std::max<long long>(1, std::min<long long>((n + kMT - 1) / kMT, kMapBlocks));
}

}  // namespace

namespace {

// Spatial-pass geometry of a handle for one row-block shape: staged block
// per slice, and the slices per chunk: the largest of 8, 4, 2, 1 whose
// staged block fits the LDS budget and that still gives at least two
// workgroups per CU, else the smallest that fits (0 where one slice does not
// fit).
MapTile map_tile_for(const stls_ctx* h, const int* B) {
  const int d = h->d;
  MapTile tl = {};
  tl.d = d;
  tl.ns = (int)h->ns;
  tl.nt = h->dir[d].n;
  tl.nblk = 1;
  tl.tsz = 1;
  for (int k = 0; k < 3; ++k) {
    tl.n[k] = k < d ? h->dir[k].n : 1;
    tl.p[k] = k < d ? h->dir[k].p : 0;
    tl.B[k] = B[k];
    tl.T[k] = B[k] + 2 * tl.p[k];
    tl.nb[k] = (tl.n[k] + B[k] - 1) / B[k];
    tl.nblk *= tl.nb[k];
    tl.tsz *= tl.T[k];
  }
  tl.bufsten = (double)h->stencil * (double)h->ns * 8.0 < 2147483648.0;
  tl.tt = 0;
  for (int c : {8, 4, 2, 1}) {
    if (tl.T[0] > 64) break;  // the staging loop covers lines of at most 64 values
    if (sizeof(double) * (size_t)c * tl.tsz > (size_t)kMapLds) continue;
    tl.tt = c;
    if ((long long)tl.nblk * ((tl.nt + c - 1) / c) >= 512) break;
  }
  tl.nchunk = tl.tt ? (tl.nt + tl.tt - 1) / tl.tt : 0;
  return tl;
}

// The row-block shape of a handle: 32 rows along direction 1 where that pads
// direction 1 no more than 16 rows would, and leaves at least 4 slices per
// chunk; else 16 (measured on the rotated quarter annulus: n_1 = 32, p = 2
// favours 32; n_1 = 40, p = 2 and n_1 = 25, p = 3 favour 16).
MapTile map_tile(const stls_ctx* h) {
  const bool d3 = h->d == 3;
  const MapTile w = map_tile_for(h, d3 ? kBlk3W : kBlk2W), n = map_tile_for(h, d3 ? kBlk3N : kBlk2N);
  const int n0 = h->dir[0].n, padw = (n0 + 31) / 32 * 32, padn = (n0 + 15) / 16 * 16;
  if (w.tt && (padw < padn || (padw == padn && w.tt >= 4))) return w;
  return n.tt ? n : w;
}

template <int TT>
int launch_space(const MapTile& tl, hipStream_t st, const double* x, double* U, double* V, double* Lx,
                 const double* Ms, const double* Js, const double* Ls, const PcgScalars* gate) {
  const size_t shmem = sizeof(double) * TT * tl.tsz;
  auto kern = mapped_space_kernel<TT>;
  if (shmem > 65536) {
    const hipError_t ea = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (ea != hipSuccess) return hip_fail(ea, "hipFuncSetAttribute(LDS)");
  }
  hipLaunchKernelGGL(kern, dim3(tl.nblk * tl.nchunk), dim3(kMT), shmem, st, x, U, V, Lx, tl, Ms, Js, Ls, gate);
  return STLS_OK;
}

}  // namespace

int launch_mapped_matvec(stls_ctx* h, const double* x, double* y, const double* dot_with, double* partials,
                         int* nparts) {
  const int d = h->d;
  const DevDir& Dt = h->dd[d];
  const MapTile tl = map_tile(h);
  const int TT = tl.tt;
  if (!TT) {
    set_error("mapped matvec: degree too large for the spatial pass's LDS tile");
    return STLS_EINVAL;
  }
  double* U = h->work[1];
  double* V = h->work[2];
  prof_begin(h);
  const double* const* sten = h->sten;
  double* Lx = h->mapped_lx;
  int st = TT == 8   ? launch_space<8>(tl, h->stream, x, U, V, Lx, sten[0], sten[1], sten[2], h->gate)
           : TT == 4 ? launch_space<4>(tl, h->stream, x, U, V, Lx, sten[0], sten[1], sten[2], h->gate)
           : TT == 2 ? launch_space<2>(tl, h->stream, x, U, V, Lx, sten[0], sten[1], sten[2], h->gate)
                     : launch_space<1>(tl, h->stream, x, U, V, Lx, sten[0], sten[1], sten[2], h->gate);
  if (st) return st;
  const int nrb = (tl.ns + kMT - 1) / kMT;
  int tc = 8;
  while (tc > 1 && (long long)nrb * ((tl.nt + tc - 1) / tc) < 1024) tc /= 2;
  const int blocks = (int)std::min<long long>((long long)nrb * ((tl.nt + tc - 1) / tc), kMapBlocks);
  if (dot_with && blocks > kPartialsCap) { set_error("too many partial sums"); return STLS_EINVAL; }
  const double k2 = h->kappa * h->kappa, kw = h->kappa * h->dir[d].wend;
  if (dot_with)
    hipLaunchKernelGGL(mapped_time_kernel<true>, dim3(blocks), dim3(kMT), 0, h->stream, U, V, h->mapped_lx, y, tl.ns,
                       tl.nt, Dt.p, tc, Dt.K, Dt.M, k2, kw, dot_with, partials, h->gate);
  else
    hipLaunchKernelGGL(mapped_time_kernel<false>, dim3(blocks), dim3(kMT), 0, h->stream, U, V, h->mapped_lx, y,
                       tl.ns, tl.nt, Dt.p, tc, Dt.K, Dt.M, k2, kw, nullptr, nullptr, h->gate);
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

int mapped_assemble(stls_ctx* h, const MappedQuad& mq) {
  const int d = mq.d;
  AsmArgs a = {};
  a.d = d;
  a.geom = mq.geom;
  a.nf = 1;
  a.nq = 1;
  int S = 1;
  for (int k = 0; k < 3; ++k) {
    a.nel[k] = k < d ? mq.nel[k] : 1;
    a.q[k] = k < d ? mq.q[k] : 1;
    a.p[k] = k < d ? mq.p[k] : 0;
    a.n[k] = k < d ? mq.n[k] : 1;
    a.bw[k] = 2 * a.p[k] + 1;
    a.nf *= a.p[k] + 1;
    a.nq *= a.q[k];
    S *= a.bw[k];
  }
  for (int k = 0; k < d; ++k)
    if ((size_t)mq.nel[k] * mq.q[k] != mq.x[k].size() || mq.x[k].size() != mq.w[k].size() ||
        mq.v[k].size() != mq.x[k].size() * 3 * (mq.p[k] + 1) || mq.first[k].size() != (size_t)mq.nel[k] ||
        mq.nel[k] < 1) {
      set_error("mapped assembly: inconsistent quadrature data");
      return STLS_EINVAL;
    }
  if (d < 2 || !map_tile(h).tt) {  // the matvec's spatial pass stages at least one slice of a row block
    set_error("mapped domain: degree too large for the matvec's LDS tile");
    return STLS_EINVAL;
  }
  // points per chunk: the chunk's basis data stays within 64 KB of LDS when nf allows
  a.qc = std::max(1, std::min(32, 1024 / a.nf));
  const size_t lds = sizeof(double) * ((size_t)a.qc * kAsmMet + (size_t)a.qc * 8 * a.nf);
  if (lds > 160 * 1024) {
    set_error("mapped assembly: degree too large for the element kernel's LDS");
    return STLS_EINVAL;
  }
  const long long per_pass = (long long)kAsmThreads * kAsmPairs;
  a.passes = (int)(((long long)a.nf * a.nf + per_pass - 1) / per_pass);
  a.ns = h->ns;
  h->stencil = S;
  const size_t nent = (size_t)S * (size_t)h->ns;
  // device copies of the quadrature data
  std::vector<double> dbuf;
  std::vector<int> ibuf;
  size_t xo[3] = {0, 0, 0}, wo[3] = {0, 0, 0}, vo[3] = {0, 0, 0}, fo[3] = {0, 0, 0};
  for (int k = 0; k < d; ++k) {
    xo[k] = dbuf.size();
    dbuf.insert(dbuf.end(), mq.x[k].begin(), mq.x[k].end());
    wo[k] = dbuf.size();
    dbuf.insert(dbuf.end(), mq.w[k].begin(), mq.w[k].end());
    vo[k] = dbuf.size();
    dbuf.insert(dbuf.end(), mq.v[k].begin(), mq.v[k].end());
    fo[k] = ibuf.size();
    ibuf.insert(ibuf.end(), mq.first[k].begin(), mq.first[k].end());
  }
  double* dq = nullptr;
  int* iq = nullptr;
  auto cleanup = [&]() {
    if (dq) (void)hipFree(dq);
    if (iq) (void)hipFree(iq);
  };
  hipError_t err = hipMalloc((void**)&dq, sizeof(double) * dbuf.size());
  if (err == hipSuccess) err = hipMalloc((void**)&iq, sizeof(int) * ibuf.size());
  for (int f = 0; f < 3 && err == hipSuccess; ++f) err = hipMalloc((void**)&h->sten[f], sizeof(double) * nent);
  if (err == hipSuccess) err = hipMalloc((void**)&h->mapped_lx, sizeof(double) * (size_t)h->ns);
  if (err != hipSuccess) {
    cleanup();
    set_error("hipMalloc (mapped-domain stencils)");
    return STLS_ENOMEM;
  }
  err = hipMemcpyAsync(dq, dbuf.data(), sizeof(double) * dbuf.size(), hipMemcpyHostToDevice, h->stream);
  if (err == hipSuccess)
    err = hipMemcpyAsync(iq, ibuf.data(), sizeof(int) * ibuf.size(), hipMemcpyHostToDevice, h->stream);
  for (int f = 0; f < 3 && err == hipSuccess; ++f)
    err = hipMemsetAsync(h->sten[f], 0, sizeof(double) * nent, h->stream);
  if (err == hipSuccess && lds > 64 * 1024)
    err = hipFuncSetAttribute((const void*)mapped_assemble_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  for (int k = 0; k < 3; ++k) {
    const int kk = k < d ? k : 0;
    a.x[k] = dq + xo[kk];
    a.w[k] = dq + wo[kk];
    a.v[k] = dq + vo[kk];
    a.first[k] = iq + fo[kk];
  }
  a.M = h->sten[0];
  a.J = h->sten[1];
  a.L = h->sten[2];
  // one launch per colour (span index modulo p_k + 1 in every direction)
  const int c1n = d > 1 ? a.p[1] + 1 : 1, c2n = d > 2 ? a.p[2] + 1 : 1;
  for (int c2 = 0; c2 < c2n && err == hipSuccess; ++c2)
    for (int c1 = 0; c1 < c1n && err == hipSuccess; ++c1)
      for (int c0 = 0; c0 <= a.p[0] && err == hipSuccess; ++c0) {
        const int c[3] = {c0, c1, c2};
        long long blocks = 1;
        for (int k = 0; k < 3; ++k) {
          a.col[k] = c[k];
          a.ncol[k] = k < d ? (a.nel[k] - c[k] + a.p[k]) / (a.p[k] + 1) : 1;
          if (a.ncol[k] < 0) a.ncol[k] = 0;
          blocks *= a.ncol[k];
        }
        if (blocks == 0) continue;
        if (blocks > 0x7fffffffLL) {
          cleanup();
          set_error("mapped assembly: too many elements");
          return STLS_EINVAL;
        }
        hipLaunchKernelGGL(mapped_assemble_kernel, dim3((unsigned)blocks), dim3(kAsmThreads), lds, h->stream, a);
        err = hipGetLastError();
      }
  // diagonals (centre entries) back to the host for the P^G scaling
  int centre = 0;
  {
    int stride = 1;
    for (int k = 0; k < d; ++k) {
      centre += a.p[k] * stride;
      stride *= a.bw[k];
    }
  }
  for (int f = 0; f < 3 && err == hipSuccess; ++f) {
    h->sdiag[f].assign((size_t)h->ns, 0.0);
    err = hipMemcpyAsync(h->sdiag[f].data(), h->sten[f] + (size_t)centre * (size_t)h->ns,
                         sizeof(double) * (size_t)h->ns, hipMemcpyDeviceToHost, h->stream);
  }
  if (err == hipSuccess) err = hipStreamSynchronize(h->stream);
  cleanup();
  if (err != hipSuccess) return hip_fail(err, "mapped-domain stencil assembly");
  return STLS_OK;
}

}  // namespace stls
