/*
 * stls.h -- C ABI of the MI355X (gfx950) space-time least-squares heat solver.
 *
 * Method: Montardini, Negri, Sangalli, Tani, "Space-time least-squares
 * isogeometric method and efficient solver for parabolic problems"
 * (arXiv:1809.10026).  The heat equation d_t u - kappa Lap u = f on the unit
 * box (0,1)^d x (0,1) with homogeneous Dirichlet data in space and zero
 * initial value (§3.1, eq. heat_eq; kappa = 1 in the paper) is discretised
 * by the least-squares method of §3.2-3.3 with tensor-product B-splines
 * (§2).  The SPD system A u = F (§4.1, eq. A_kron)
 *
 *     A = K_t (x) M_s + kappa^2 M_t (x) J_s + kappa W_t (x) L_s
 *
 * is solved by preconditioned conjugate gradients (PCG) with the
 * preconditioner P = K_t (x) M_s + kappa^2 M_t (x) J~_s (§4.2, eq.
 * preconditioner) applied by fast diagonalization (§4.3, Algorithm 1).
 *
 * Conventions shared by every entry point
 *  - Vectors are FP64, device-resident (HBM), caller-owned, contiguous, in
 *    the colexicographic order of §2.2 / eq. kron_vec_multi: first space
 *    index fastest, ..., d-th space index, time index slowest.  Their
 *    length is ndof = n_1 * ... * n_d * n_t with n_k = m_k - 2 (Dirichlet
 *    functions dropped in space) and n_t = m_t - 1 (initial-time function
 *    dropped), eq. basis_par; m = #knots - degree - 1.
 *  - Work is enqueued on the stream given at setup and is asynchronous with
 *    respect to the host, except where a function says it synchronises.
 *  - No call throws; every call returns a status (stls_status).  A handle
 *    must not be used from two host threads at once; calls on different
 *    handles are independent.
 *  - The handle owns all device memory it allocates (factors, workspace).
 */
#ifndef STLS_H
#define STLS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stls_ctx* stls_handle;

typedef enum stls_status {
  STLS_OK = 0,
  STLS_EINVAL = -1,     /* invalid argument (knots, degrees, sizes, pointers, mode) */
  STLS_ENOMEM = -2,     /* device or host allocation failed */
  STLS_EHIP = -3,       /* a HIP runtime call failed; see stls_last_error */
  STLS_ENOCONV = -4,    /* PCG hit maxit before reaching rtol */
  STLS_ENAN = -5,       /* NaN or Inf met in the right-hand side or the iteration */
  STLS_EBREAKDOWN = -6  /* PCG breakdown: p^T A p <= 0 or r^T z <= 0 */
} stls_status;

typedef enum stls_fd_precision {
  STLS_FD_FP64 = 0,    /* n-mode products in FP64 (MFMA f64) */
  STLS_FD_FP32 = 1,    /* n-mode products and intermediates in FP32 (MFMA f32) */
  STLS_FD_BF16X3 = 2,  /* FP32 operands split into bf16 hi+lo, three bf16 MFMA
                          products (hi*hi + hi*lo + lo*hi), FP32 accumulation */
  STLS_FD_ASYM = 3     /* asymmetric: forward space products (Algorithm 1 step 2)
                          in FP32; the time products, the eigenvalue division
                          (step 3) and the backward space products (step 4) in
                          FP64 */
} stls_fd_precision;

/*
 * stls_setup -- build a solver for one problem (§2.1-2.2, §4.1-4.3 step 1).
 *  d        number of space dimensions, 1..3.
 *  nknots   d + 1 knot-vector lengths (space directions 1..d, then time).
 *  knots    d + 1 host arrays, copied: open knot vectors on [0,1] (§2.1):
 *           non-decreasing, first p+1 entries 0 and last p+1 entries 1.
 *  degree   d + 1 degrees.  Space: p >= 2 and every interior knot of
 *           multiplicity <= p - 1 (C^1 splines, Assumption 2); time:
 *           p >= 1 and multiplicity <= p (C^0).
 *  kappa    diffusivity > 0 (1 = the paper's model problem).
 *  stream   hipStream_t to enqueue on (NULL = default stream).
 *  out      receives the handle.
 * Host work: Gauss quadrature of the banded univariate matrices, generalized
 * eigendecompositions J_k U = M_k U Lambda and K_t U = M_t U Lambda with
 * U^T M U = I (eq. eig_dec), upload.  Synchronises the stream.
 * Errors: STLS_EINVAL for invalid input (nothing allocated), STLS_ENOMEM,
 * STLS_EHIP.
 */
int stls_setup(int d, const int* nknots, const double* const* knots, const int* degree,
               double kappa, void* stream, stls_handle* out);

/* ------------------------------------------------------------------------
 * Mapped spatial domains (§2.2 isoparametric spaces, §4.4, §5.1-5.2).
 * Omega = G((0,1)^d) for one of the paper's domains; trial and test
 * functions are the restricted tensor B-splines composed with G^{-1}.  The
 * system keeps the time Kronecker structure of §4.1 with sparse spatial
 * factors M_s = int B_i B_j, L_s = int grad B_i . grad B_j and
 * J_s = int Lap B_i Lap B_j over Omega, assembled on the device by Gauss
 * quadrature with p + 3 points per non-empty span and applied as stencils.
 * ------------------------------------------------------------------------ */
typedef enum stls_geometry {
  STLS_GEOM_UNIT_BOX = 0,                /* (0,1)^d: stls_setup */
  STLS_GEOM_QUARTER_ANNULUS = 1,         /* d = 2: 1 < r < 2, 0 < theta < pi/2 (§5.1);
                                            x = r cos(theta), y = r sin(theta),
                                            r = 1 + eta_1, theta = (pi/2) eta_2 */
  STLS_GEOM_ROTATED_QUARTER_ANNULUS = 2  /* d = 3: that quarter annulus revolved by pi/2
                                            about the line y = -1, z = 0 (§5.2):
                                            x = x0, y = -1 + (y0 + 1) cos(phi),
                                            z = (y0 + 1) sin(phi), phi = (pi/2) eta_3 */
} stls_geometry;

typedef enum stls_mapped_prec {
  STLS_PREC_PARAMETRIC = 0,  /* P of §4.2 from the parametric factors (G ignored) */
  STLS_PREC_GEOMETRY = 1     /* P^G = D^1/2 Pbar^G D^1/2 (§4.4): factors weighted by the
                                separable approximation (Algorithm 2 of Appendix A.3,
                                maxit = 2) of the geometry coefficients c_k at the element
                                barycentres, D = diag(A) / diag(Pbar^G) */
} stls_mapped_prec;

/*
 * stls_setup on a mapped domain.  Arguments as stls_setup, plus geometry
 * (stls_geometry; d must match) and prec (stls_mapped_prec).  stls_matvec,
 * stls_prec_apply (every FD precision), stls_pcg_solve, stls_set_kappa and
 * the profiling calls work as on the unit box; stls_set_fd_scaling(h, 1)
 * and the differentiation, lifting and error-norm calls return STLS_EINVAL.
 * Setup work: the stencils are assembled on the device element by element
 * (O(elements (p+1)^(2d) (p+3)^d) work, device memory 3 ns prod_k (2p_k+1)
 * doubles); the geometry weights of P^G, their eigendecompositions and the
 * scaling are formed on the host.  Synchronises the stream.  Errors as
 * stls_setup, and STLS_EINVAL where the degree is too large for the
 * matvec's LDS tile (p above 7 in 3-D).
 */
int stls_setup_mapped(int d, const int* nknots, const double* const* knots, const int* degree, double kappa,
                      int geometry, int prec, void* stream, stls_handle* out);

/* Release every device and host resource of the handle (NULL is a no-op). */
int stls_destroy(stls_handle h);

/* Sizes: n[0..d] receives n_1..n_d, n_t; *ndof receives their product. */
int stls_get_shape(stls_handle h, int* n, int64_t* ndof);

/*
 * Copy setup results to host memory (test and inspection use).
 *  dir   0..d-1 space direction, d = time.
 *  what  0 = mass M, 1 = stiffness K, 2 = bilaplacian J (space only): banded
 *        restricted matrix, n x (2p+1) row-major, entry (i,j) at
 *        i*(2p+1) + (j - i + p), zero outside 0 <= j < n;
 *        3 = eigenvectors U, n x n column-major (U^T M U = I);
 *        4 = eigenvalues, n values;
 *        5 = final-time weight b_last(1)^2 (time only), 1 value.
 *  out   host buffer of the documented size; *count receives #doubles.
 * Pass out = NULL to query *count only.
 */
int stls_get_factor(stls_handle h, int dir, int what, double* out, int64_t* count);

/* Change kappa (> 0): rescales the summed eigenvalues; U is independent of kappa. */
int stls_set_kappa(stls_handle h, double kappa);

/* Select the arithmetic of the FD n-mode products (stls_fd_precision).
 * The eigenvalue division, PCG vectors and dot products stay FP64.  The
 * asymmetric mode runs the general (one product per pass) kernels on every
 * shape.  Returns STLS_EINVAL for an unknown mode. */
int stls_set_fd_precision(stls_handle h, int mode);

/*
 * Diagonal scaling of the preconditioner (§4.4, closing definition):
 * P^G = D^{1/2} P D^{1/2} with D_ii = A_ii / P_ii.  On the unit box the
 * geometry-approximated factor of §4.4 is P itself, so with on != 0
 * stls_prec_apply and stls_pcg_solve use s = D^{-1/2} P^{-1} D^{-1/2} r.
 * D is formed on the fly from the univariate diagonals and follows
 * stls_set_kappa; on = 0 (the default) restores s = P^{-1} r.  Batched
 * solves (stls_batch_*) always use the unscaled P.
 */
int stls_set_fd_scaling(stls_handle h, int on);

/*
 * s = P^{-1} r by Algorithm 1 steps 2-4 (§4.3): n-mode products with U^T
 * over every direction, division by lambda_t[i_t] + kappa^2 sum_k
 * lambda_k[i_k], n-mode products with U.  r, s: device, ndof doubles, may
 * not alias.  Asynchronous.
 */
int stls_prec_apply(stls_handle h, const double* r, double* s);

/*
 * y = A x, matrix-free from the banded univariate factors (§4.5; eq. A_kron
 * with kappa).  x, y: device, ndof doubles, may not alias.  Asynchronous.
 */
int stls_matvec(stls_handle h, const double* x, double* y);

/*
 * PCG for A x = b (§4.2; tolerance and zero start as in §5).
 *  b      device, ndof doubles.
 *  x      device, ndof doubles: output (the iteration starts from x = 0;
 *         incoming contents are ignored).
 *  rtol   stop when the recurrence residual satisfies ||r||_2/||b||_2 <= rtol.
 *  maxit  iteration cap (>= 1).
 *  iters, relres  host outputs (may be NULL): iterations done, final
 *         recurrence relative residual.
 * Synchronises the stream.  Returns STLS_OK on convergence, STLS_ENOCONV at
 * maxit, STLS_ENAN for a non-finite b or iterate, STLS_EBREAKDOWN if a
 * curvature or r^T z is not positive.  b = 0 returns x = 0, iters = 0.
 */
int stls_pcg_solve(stls_handle h, const double* b, double* x, double rtol, int maxit,
                   int* iters, double* relres);

/*
 * Quadrature grid of the error norms (§5.1: element-wise Gauss quadrature,
 * p + 3 points per non-empty knot span of the direction).
 *  dir    0..d-1 space directions, d time.
 *  x, w   host buffers of *nq doubles for the points and weights, or both
 *         NULL to query *nq only.
 */
int stls_norm_points(stls_handle h, int dir, double* x, double* w, int* nq);

/*
 * Relative errors of u_h = sum_i u_i B_i against an exact solution given as
 * a sum of separable terms u(x, t) = sum_s prod_k g_{s,k}(x_k) (§3.1
 * eq. norm_V0, §5.1):
 *   out[0] = ||u - u_h||_V0 / ||u||_V0 with ||v||_V0^2 = int int (d_t v)^2 + (Lap v)^2,
 *   out[1] = L^2 relative error,
 *   out[2] = relative error in the space-time H^1 norm (v, d_t v, grad_x v).
 *  u       device, ndof doubles: the coefficients (colex).
 *  nterms  1..64.
 *  g       host array of nterms*(d+1) host pointers; g[s*(d+1)+k] holds
 *          3*nq_k doubles: g_{s,k}, g_{s,k}' and g_{s,k}'' at the points of
 *          stls_norm_points(h, k, ...), in that order.
 *  out     host, 3 doubles.
 * Device temporaries (about 3 * prod_k nq_k(space) * n_t doubles and the
 * tables) live in a workspace of the handle, allocated by the first call
 * that needs it and grown when a later call needs more (freed by
 * stls_destroy); synchronises the stream.  STLS_ENOMEM if they do not fit.
 */
int stls_error_norms(stls_handle h, const double* u, int nterms, const double* const* g, double* out);

/* Residual history of the last stls_pcg_solve: out[k] = ||r_k||/||b||,
 * k = 0..iters (host buffer of at least max entries); *count = iters + 1. */
int stls_pcg_history(stls_handle h, double* out, int max, int* count);

/* ------------------------------------------------------------------------
 * Differentiation operators (adjoint gradients of a space-time misfit).
 * Not in the paper; built on its load functional (§3.2) and Kronecker
 * structure (§4.1).  The forcing f is a spline in the FULL tensor space of
 * the knot vectors (no boundary or initial restriction): coefficient tensor
 * of nfull = m_1 * ... * m_d * m_t entries, colexicographic, FP64, device.
 * kappa is the handle's current diffusivity.  All are stream-ordered and
 * asynchronous unless they return a host scalar (then they synchronise).
 * Full-space workspace (two nfull buffers) is allocated on first use.
 * ------------------------------------------------------------------------ */

/* m[0..d] receives the full sizes m_k (#knots - p - 1), *nfull their product. */
int stls_get_forcing_shape(stls_handle h, int* m, int64_t* nfull);

/* F = B_kappa f with F_i = int int f (d_t B_i - kappa Lap B_i) (the least-
 * squares load of §3.2 for the forcing spline f):
 * B_kappa = C_t (x) Mbar_s - kappa Mbar_t (x) Dbar_s, Mbar = int b_i bbar_j,
 * C = int b'_i bbar_j, Dbar_s = sum_k (int b''_i bbar_j in direction k,
 * Mbar elsewhere).  f: nfull doubles; F: ndof doubles. */
int stls_load_apply(stls_handle h, const double* f, double* F);

/* F = B_kappa f exactly as stls_load_apply (same kernels, same order, same
 * result bit for bit), for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  The call
 * allocates nothing, host or device: its chain temporaries live in a static
 * device array of 64 MiB (2^23 doubles) that every device the library runs
 * on holds until the process ends, looked up once per device at stls_setup.
 * The temporaries need about 2 * nfull * n_1 / m_1 doubles (e.g. 131^3
 * forcing coefficients fit); larger problems get STLS_EINVAL with the sizes
 * in stls_last_error.  Every call on a device shares that device's array:
 * calls that overlap on one device (two streams, or two host threads) race
 * and must be serialised by the caller.  f: nfull doubles; F: ndof doubles;
 * stream-ordered and asynchronous on the handle's stream. */
int stls_load_apply_noalloc(stls_handle h, const double* f, double* F);

/* gf = B_kappa^T l: l ndof doubles, gf nfull doubles. */
int stls_load_apply_T(stls_handle h, const double* l, double* gf);

/* ------------------------------------------------------------------------
 * Non-zero initial data by lifting (§2, the paragraph after the parabolic
 * regularity theorem; least-squares form §3.2).  An initial value u0 in
 * H^1_0 is represented by its coefficients u0_h over the restricted spatial
 * space (ns doubles, colexicographic, FP64, device), carried by the first
 * time B-spline b_1.  The solution is u_h = w_h + u0_h b_1, where w_h in the
 * zero-data space solves A w = F - a(u0_h b_1, B_i).  Stream-ordered and
 * asynchronous.  The full-space workspace of the differentiation operators
 * is allocated on first use.
 * ------------------------------------------------------------------------ */

/* F -= a(u0_h b_1, B_i) for every restricted B_i, i.e. the system matrix with
 * each time factor replaced by its column of b_1 (int b_j' b_1', int b_j b_1;
 * the final-time term vanishes since b_1(T) = 0).  Only the first
 * min(p_t, n_t) time slices of F change.  u0: ns doubles; F: ndof doubles,
 * updated in place.  STLS_EINVAL for NULL arguments. */
int stls_lift_initial(stls_handle h, const double* u0, double* F);

/* u = [u0_h, w_h]: the coefficients of u_h over every time function, time
 * slowest (ns * (n_t + 1) doubles); u0: ns doubles, w: ndof doubles.  The
 * buffers must not overlap.  STLS_EINVAL for NULL arguments. */
int stls_lift_combine(stls_handle h, const double* u0, const double* w, double* u);

/* General data: a lifting u_B anywhere in the full spline space (its
 * boundary coefficients carry the boundary values, its first time
 * coefficients the initial value), nfull doubles laid out as the forcing of
 * the differentiation operators.  For such trial functions the spatial
 * integrations by parts behind the system matrix leave boundary terms, so
 * the least-squares form of §3.2 is assembled term by term:
 * a(u, v) = int int (d_t u - kappa Lap u)(d_t v - kappa Lap v).
 * F -= a(u_B, B_i) for every restricted B_i; F: ndof doubles, in place.
 * On u_B of the zero-data space this equals the system matrix.  Entries of
 * u_B at restricted coefficients are included like any other.  Device
 * temporaries: eight arrays of nfull doubles, allocated by the first call
 * and kept in the handle.  STLS_EINVAL for NULL arguments, on a mapped
 * domain, or where a direction's four bands exceed the 160 KB of LDS of
 * one pass (n_k (2 p_k + 1) > 5120); STLS_ENOMEM if the temporaries do not
 * fit. */
int stls_lift_apply(stls_handle h, const double* ub, double* F);

/* u = u_B + w placed at the restricted coefficients (restricted index i is
 * full index i + 1 in every direction): the coefficients of u_h over the
 * full space, nfull doubles; ub nfull, w ndof.  The buffers must not
 * overlap.  STLS_EINVAL for NULL arguments. */
int stls_lift_embed(stls_handle h, const double* ub, const double* w, double* u);

/* y = (M_t (x) M_s) x, the Gram matrix of L2(space x time) on the discrete
 * space (x, y: ndof doubles, must differ). */
int stls_mass_apply(stls_handle h, const double* x, double* y);

/* *dk (host) = l^T (-(Mbar_t (x) Dbar_s) f - (2 kappa M_t (x) J_s + W_t (x) L_s) u):
 * the derivative of l^T (F_kappa - A_kappa u) with respect to kappa.
 * f: nfull doubles; u, l: ndof doubles.  Synchronises. */
int stls_dkappa(stls_handle h, const double* f, const double* u, const double* l, double* dk);

/* The same derivative under the name of the scope's boundary listing
 * (identical arguments, result and errors). */
int stls_dkappa_terms(stls_handle h, const double* f, const double* u, const double* l, double* dk);

/* *out (host) = a . b over n doubles (device), fixed-order reduction.
 * Synchronises. */
int stls_dot(stls_handle h, const double* a, const double* b, int64_t n, double* out);

/* e = u - ustar, *loss (host) = e^T (M_t (x) M_s) e (squared L2 norm of
 * u_h - u*_h over the space-time cylinder) and q = 2 (M_t (x) M_s) e, its
 * gradient with respect to u (device, ndof).  Synchronises. */
int stls_misfit(stls_handle h, const double* u, const double* ustar, double* q, double* loss);

/* ------------------------------------------------------------------------
 * Batched PCG: many independent problems of uneven sizes and degrees solved
 * together.  Every PCG step of the whole batch is one kernel launch over a
 * work list of (problem, tile) items; alpha, beta, rho and the convergence
 * flag of each problem stay in device memory and converged problems skip
 * their items.  FD products in FP64.  Supported: d = 1 or 2 (the same for
 * the whole batch), the same degree (<= 6) in every direction of a problem,
 * n <= 112 per direction.
 * ------------------------------------------------------------------------ */
typedef struct stls_batch_ctx* stls_batch_handle;

/* nprob problems; problem i has knot vectors knots[i*(d+1) + k] (host, copied)
 * of lengths nknots[i*(d+1) + k], degrees degree[i*(d+1) + k] and diffusivity
 * kappa[i] (validation as in stls_setup).  Per-problem setup runs in host
 * threads.  Synchronises.  Errors: STLS_EINVAL (including the problem index
 * in stls_last_error), STLS_ENOMEM, STLS_EHIP. */
int stls_batch_setup(int nprob, int d, const int* nknots, const double* const* knots, const int* degree,
                     const double* kappa, void* stream, stls_batch_handle* out);

/* Release the batch and its problems (NULL is a no-op). */
int stls_batch_destroy(stls_batch_handle b);

/* Batch vectors are the problems' vectors concatenated: problem i occupies
 * [off[i], off[i+1]) (host array of nprob + 1 entries). */
int stls_batch_offsets(stls_batch_handle b, int64_t* off);

/* Handle of problem i (owned by the batch; valid until stls_batch_destroy),
 * for single-problem calls on the same factors. */
int stls_batch_problem(stls_batch_handle b, int i, stls_handle* h);

/* Batched y = A x and s = P^{-1} r over concatenated vectors (asynchronous). */
int stls_batch_matvec(stls_batch_handle b, const double* x, double* y);
int stls_batch_prec_apply(stls_batch_handle b, const double* r, double* s);

/* Batched PCG from x = 0 to ||r_i||/||b_i|| <= rtol for every problem i.
 * b, x: device, concatenated.  iters, relres: host arrays of nprob (may be
 * NULL).  Synchronises once per iteration (all problems' scalars in one copy).
 * The kernels of one iteration (the same for every iteration: converged
 * problems are masked on the device) are captured once per call into a
 * hipGraph on the handle's stream and replayed; a stream that cannot be
 * captured (the legacy default stream) gets direct launches.
 * Returns STLS_OK when all converged, STLS_ENOCONV if any hit maxit,
 * STLS_ENAN / STLS_EBREAKDOWN if any problem failed. */
int stls_batch_pcg_solve(stls_batch_handle b, const double* bvec, double* x, double rtol, int maxit, int* iters,
                         double* relres);

/* Replay the batched PCG iterations from a captured graph (on != 0, the
 * default) or launch every kernel directly (on = 0); both run the same
 * kernels in the same order and give identical results. */
int stls_batch_set_graph(stls_batch_handle b, int on);
/* 1 if the last stls_batch_pcg_solve replayed a captured graph, 0 if it
 * launched the kernels directly, STLS_EINVAL for a NULL handle. */
int stls_batch_graph_used(stls_batch_handle b);

/* Work-item shapes and launch geometry of the batched kernels (one int each,
 * in this order).  Results do not depend on them except through the order
 * of the partial sums of dot products (rounding). */
typedef enum stls_batch_tune_field {
  STLS_TUNE_VEC_CHUNK = 0,   /* elements per vector work item: 256..2^20, multiple of 256 */
  STLS_TUNE_INNER_STEPS = 1, /* column steps per inner-stage (d = 2) work item: 1..64 */
  STLS_TUNE_OUTER_CHUNK = 2, /* time slices per outer-stage work item (at most): 1..65536 */
  STLS_TUNE_GRID_FD = 3,     /* workgroups per launch (caps): FD passes, */
  STLS_TUNE_GRID_INNER = 4,  /*   inner stage, */
  STLS_TUNE_GRID_OUTER = 5,  /*   outer stage, */
  STLS_TUNE_GRID_VEC = 6,    /*   vector kernels: 1..65536 */
  STLS_TUNE_GRAPH_DEPTH = 7, /* PCG iterations per captured graph launch (host checks
                                convergence once per launch; never more than maxit): 1..64 */
  STLS_TUNE_COUNT = 8
} stls_batch_tune_field;

/* vals: STLS_TUNE_COUNT ints. */
int stls_batch_get_tuning(stls_batch_handle b, int* vals);
/* Validates every value (STLS_EINVAL if out of range), waits for the
 * batch's streams and rebuilds the work lists.  Synchronises. */
int stls_batch_set_tuning(stls_batch_handle b, const int* vals);

/* Autotuner: picks the tuning fields for this batch by timing candidates
 * with HIP events on the batch's stream, one group of fields at a time
 * (vector chunk and grid; inner steps and grid; outer time chunk and grid;
 * FD grid; then the graph depth by timing whole solves of a right-hand side
 * of ones on scratch vectors), and applies the fastest.  With cache_path
 * (a JSON file, created if missing) a choice stored under the same key (the
 * batch kernels' source hash, the device architecture and a hash of every
 * problem's sizes and degree) is applied without measuring, and a new choice
 * is stored.  *measured (may be NULL) = 1 if timings were taken, 0 if the
 * cache supplied the choice.  The batch's work vectors and PCG scalars are
 * overwritten; synchronises.  STLS_EINVAL for an unreadable or malformed
 * cache file. */
int stls_batch_autotune(stls_batch_handle b, const char* cache_path, int* measured);

/* Per-kernel timing with HIP events on the handle's stream (0 = off). */
int stls_set_profiling(stls_handle h, int on);
/* Kernel class names and accumulated (launches, milliseconds) since the last
 * reset.  idx in [0, stls_profile_count()); name receives a static string. */
int stls_profile_count(void);
int stls_profile_get(stls_handle h, int idx, const char** name, int64_t* launches, double* ms);
int stls_profile_reset(stls_handle h);

/* Human-readable status text (static storage). */
const char* stls_status_string(int status);
/* Text of the last error recorded on this thread (static per-thread storage). */
const char* stls_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STLS_H */
