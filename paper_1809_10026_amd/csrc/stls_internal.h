// Internal declarations of the stls library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/stls.h"

namespace stls {

constexpr int kMaxDim = 3;          // space dimensions supported
constexpr int kMaxDirN = 256;       // largest restricted size per direction
constexpr int kPartialsCap = 1 << 16;

// Host-side description of one parametric direction (space k or time).
struct Dir {
  int p = 0;        // degree
  int m = 0;        // number of B-splines of the knot vector
  int n = 0;        // restricted size (space: m - 2, time: m - 1)
  bool is_time = false;
  std::vector<double> knots;
  // banded restricted matrices, n x (2p+1), entry (i,j) at i*(2p+1)+(j-i+p)
  std::vector<double> M, K, J;
  // restricted x full rectangular bands (forcing in the full space), n x (2p+1):
  // entry (i, j) with j the full index at i*(2p+1) + (j - (i+1) + p)
  std::vector<double> Mbar, Cbar, Gbar;  // int b_i bbar_j, int b'_i bbar_j, int b''_i bbar_j
  std::vector<double> Kbar;              // int b'_i bbar'_j (lifting)
  std::vector<double> Jbar, Hbar, Dbar;  // int b''_i bbar''_j, int b_i bbar''_j, int b_i bbar'_j (lifting)
  std::vector<double> U;    // n x n column-major, U^T M U = I
  std::vector<double> lam;  // generalized eigenvalues
  double wend = 0.0;        // b_{m}(1)^2 (time): the single entry of W_t
};

// Device copies of one direction.
struct DevDir {
  int p = 0, n = 0, npad = 0;  // npad: n rounded up to 16
  double* M = nullptr;         // banded, n x (2p+1)
  double* K = nullptr;
  double* J = nullptr;
  double* Afwd64 = nullptr;    // FD operand for the U^T product: [j*npad + i] = U(j,i)
  double* Abwd64 = nullptr;    // FD operand for the U product:   [j*npad + i] = U(i,j)
  float* Afwd32 = nullptr;
  float* Abwd32 = nullptr;
  uint16_t* Hfwd = nullptr;    // bf16 hi/lo of W, row-major [i*kpad + k], kpad = n rounded to 32
  uint16_t* Lfwd = nullptr;
  uint16_t* Hbwd = nullptr;
  uint16_t* Lbwd = nullptr;
  float* Rfwd32 = nullptr;     // W row-major [i*kpad + k] in FP32 and FP64 (five-pass FD)
  float* Rbwd32 = nullptr;
  double* Rfwd64 = nullptr;
  double* Rbwd64 = nullptr;
  int kpad = 0;
  double* lam = nullptr;
  int m = 0;                   // full space size (forcing coefficients)
  double* Mbar = nullptr;      // rectangular bands (uploaded on first use)
  double* Cbar = nullptr;
  double* Gbar = nullptr;
  double* Kbar = nullptr;
  double* Jbar = nullptr;
  double* Hbar = nullptr;
  double* Dbar = nullptr;
};

// Scalars of the PCG recurrence, resident in device memory.
struct PcgScalars {
  double rho;      // r^T z of the current iterate
  double alpha, beta;
  double bnorm2;   // ||b||^2
  double relres;   // ||r||/||b||
  double rtol;
  double rho_ring[2];  // r^T z by iteration parity (single-problem PCG: the update
                       // kernels read one slot while another block writes the other)
  int done;        // set once relres <= rtol (later kernels become no-ops)
  int flag;        // 0 ok, 1 breakdown, 2 non-finite
  int iters;
  int pad;
};

// Arguments of the diagonal scaling of the FD preconditioner (§4.4, closing
// definition): D_ii = A_ii / P_ii from the univariate diagonals, packed per
// space direction k as [m_k | k_k | j_k] (n_k entries each, diagonals of the
// restricted M, K, J) at off[k], and for time as [k_t | m_t] at off[d].
struct DiagScale {
  const double* g = nullptr;  // packed diagonals, FP64
  const float* g32 = nullptr; // the same, FP32
  int d = 0;
  int n[kMaxDim + 1] = {0, 0, 0, 0};
  int off[kMaxDim + 1] = {0, 0, 0, 0};
  double k2 = 1.0;  // kappa^2
  double kw = 0.0;  // kappa times the single entry of W_t (final time)
};

enum ProfId {
  PROF_FD_SPACE = 0,  // dense n-mode product over one space direction
  PROF_FD_TIME,       // fused time-mode forward product / division / backward product
  PROF_MV_INNER1,     // matvec inner stage, d = 2 (space direction 1)
  PROF_MV_INNER2,     // matvec inner stage, d = 3 (space directions 1 and 2)
  PROF_MV_OUTER,      // matvec outer stage (last space direction and time)
  PROF_VEC,           // PCG update of x and r (with the partial sums of r . r)
  PROF_REDUCE,        // PCG scalar finalisation kernels
  PROF_DIFF,          // differentiation operators (load, transpose, mass, d/dkappa)
  PROF_FD_SLAB,       // FD slab pass, forward: modes 1 and 2 of every (i3, t) slab
  PROF_FD_SLAB_BWD,   // FD slab pass, backward (writes s, partial sums of s . r)
  PROF_VEC_P,         // PCG direction update p = z + beta p
  PROF_MISC,          // other elementwise kernels (initial dot, diagonal scaling)
  PROF_MV_MAPPED,     // matvec on a mapped domain (time band and spatial stencils)
  PROF_COUNT
};

struct stls_ctx_impl;

}  // namespace stls

struct stls_ctx {
  int d = 0;
  double kappa = 1.0;
  hipStream_t stream = nullptr;
  int fd_mode = STLS_FD_FP64;
  bool fd_scale = false;     // diagonal scaling D^-1/2 P^-1 D^-1/2 (stls_set_fd_scaling)
  double* diag64 = nullptr;  // packed univariate diagonals (DiagScale layout)
  float* diag32 = nullptr;
  stls::Dir dir[stls::kMaxDim + 1];
  stls::DevDir dd[stls::kMaxDim + 1];
  int64_t ndof = 0, ns = 0;  // ns = spatial dofs
  double* lam_s = nullptr;   // kappa^2 * sum_k lambda_k[i_k], length ns
  double* lam_s_raw = nullptr;  // sum_k lambda_k[i_k] (kappa-free), length ns
  // workspace
  double* work[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  double* fdbuf[2] = {nullptr, nullptr};   // FD ping-pong (also used as float)
  double* r = nullptr;
  double* z = nullptr;
  double* pvec = nullptr;
  double* q = nullptr;
  double* partials = nullptr;
  double* dres = nullptr;          // device scalar result of stls_dot
  double* ftmp[2] = {nullptr, nullptr};  // full-space temporaries (differentiation ops)
  double* lgrp[4] = {nullptr, nullptr, nullptr, nullptr};  // lifting: the four factor classes (one set)
  double* lcls[4] = {nullptr, nullptr, nullptr, nullptr};  // lifting: the four factor classes (other set)
  int64_t nfull = 0;               // prod of full sizes m_k
  bool bands_ready = false;        // rectangular bands on the device (uploaded at setup)
  bool diff_ready = false;         // and the full-space temporaries allocated
  double* noalloc_scratch = nullptr;  // this device's static workspace (stls_load_apply_noalloc)
  // mapped spatial domain (stls_setup_mapped); geometry == STLS_GEOM_UNIT_BOX
  // for the Kronecker path
  int geometry = 0;
  int geo_prec = 0;               // STLS_PREC_PARAMETRIC (P) or STLS_PREC_GEOMETRY (P^G)
  int stencil = 0;                // entries per stencil row: prod_k (2 p_k + 1)
  double* sten[3] = {nullptr, nullptr, nullptr};  // M_s, J_s, L_s as [stencil][ns] (device)
  double* sigma = nullptr;        // (P^G) sigma_i = (Pbar_ii / A_ii)^(1/2), ndof (device)
  double* mapped_lx = nullptr;    // L_s x(:, final slice) inside the mapped matvec, ns (device)
  char* norm_ws = nullptr;        // stls_error_norms: tables and temporaries (device)
  size_t norm_ws_bytes = 0;
  std::vector<double> sdiag[3];   // diagonals of M_s, J_s, L_s (host, ns)
  std::vector<double> wdiag[stls::kMaxDim + 1][2];  // diagonals of the FD factors: space [M, J], time [K, M]
  stls::PcgScalars* scal = nullptr;
  stls::PcgScalars* scal_host = nullptr;  // pinned, 2 slots (convergence checks of alternate iterations)
  hipEvent_t check_ev[2] = {nullptr, nullptr};
  // set while a PCG solve runs: FD passes that see done or flag here return at once
  const stls::PcgScalars* gate = nullptr;
  std::vector<double> history;
  int last_iters = 0;
  // profiling
  bool prof = false;
  struct PendingEv { hipEvent_t a, b; int id; };
  std::vector<hipEvent_t> ev_pool;
  std::vector<PendingEv> ev_pending;
  hipEvent_t ev_open = nullptr;
  int64_t prof_launch[stls::PROF_COUNT] = {0};
  double prof_ms[stls::PROF_COUNT] = {0};
};

namespace stls {

// error reporting
void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);

// host setup (stls_host.cpp)
int validate_and_build_dir(const double* knots, int nknots, int p, bool is_time, Dir& out,
                           std::string& err);
void sym_generalized_eig(int n, const std::vector<double>& Kdense, const std::vector<double>& Mdense,
                         std::vector<double>& U, std::vector<double>& lam);
// Gauss-Legendre nodes and weights on [-1, 1] (q <= 16)
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w);
// values and first two derivatives of the p+1 B-splines nonzero on the
// non-empty span s at u: v[k][a] = d^k/du^k N_{s-p+a,p}(u)
void span_basis(const std::vector<double>& xi, int p, int s, double u, double v[3][16]);

// kernel launchers (stls_kernels.hip)
int launch_prec_apply(stls_ctx* h, const double* r, double* s, const double* dot_with,
                      double* partials_out, int* nparts);
int launch_matvec(stls_ctx* h, const double* x, double* y, const double* dot_with, double* partials_out,
                  int* nparts);
int pcg_run(stls_ctx* h, const double* b, double* x, double rtol, int maxit, int* iters,
            double* relres);
int upload_fd_operands(stls_ctx* h, int k);
DiagScale diag_scale_args(const stls_ctx* h);
// Five-pass FD chain for d = 3 in the handle's FD precision (stls_fd.hip).
bool fd_five_pass_covers(const stls_ctx* h);
int prec_apply_five_pass(stls_ctx* h, const double* r, double* s, const double* dot_with, double* partials,
                         int* nparts, bool scale);
int upload_diff_bands(stls_ctx* h);
int ensure_diff_operands(stls_ctx* h);
// Mapped domains (stls_geometry.cpp): quadrature data of the pulled-back
// spatial factors, the geometry-weighted FD factors (replacing dir[k].U and
// lam when the preconditioner is P^G) and the scaling vector; the stencils
// are assembled on the device (stls_mapped.hip).
int mapped_host_setup(stls_ctx* h, int geometry, int prec);
// Gauss points of the non-empty spans of the space directions (host arrays,
// span-major): per direction nel spans of q points, the points x, the
// weights w, the values and first two derivatives of the span's p + 1
// functions v[point][3][p+1], and per span the restricted index of its first
// function (span - p - 1, negative where the span's first functions are the
// dropped boundary ones).
struct MappedQuad {
  int d = 0, geom = 0;
  int nel[kMaxDim] = {1, 1, 1}, q[kMaxDim] = {1, 1, 1}, p[kMaxDim] = {0, 0, 0}, n[kMaxDim] = {1, 1, 1};
  std::vector<double> x[kMaxDim], w[kMaxDim], v[kMaxDim];
  std::vector<int> first[kMaxDim];
};
// Allocates h->sten[0..2] (M_s, J_s, L_s as [stencil][ns]), assembles them
// element by element and copies their diagonals into h->sdiag.
int mapped_assemble(stls_ctx* h, const MappedQuad& mq);
int mapped_upload(stls_ctx* h);
int mapped_update_sigma(stls_ctx* h);
int launch_mapped_matvec(stls_ctx* h, const double* x, double* y, const double* dot_with, double* partials,
                         int* nparts);
int launch_mapped_scale(stls_ctx* h, const double* x, double* y, const double* dot_with, double* partials,
                        int* nparts);

// Device address of the static workspace of the allocation-free entry points
// on the current device (looked up once per device; stls_diff.hip).
int resolve_noalloc_scratch(stls_ctx* h);

// profiling helpers
void prof_begin(stls_ctx* h);
void prof_end(stls_ctx* h, int id);
void prof_flush(stls_ctx* h);

}  // namespace stls
