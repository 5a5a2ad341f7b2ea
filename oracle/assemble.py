"""Univariate matrices and loads by element-wise Gauss quadrature.  Oracle.

The system and preconditioner factors of §4.1-4.2 (eq. A_kron, eq.
preconditioner) are one-dimensional integrals of products of B-splines and
their derivatives; with p + 1 Gauss-Legendre points per non-empty span they
are integrated exactly (integrands are piecewise polynomials of degree <= 2p).
The paper does not state its quadrature; loads of non-polynomial forcing use
p + 3 points per span.
"""
from __future__ import annotations

import numpy as np

from .bspline import eval_basis_points, nonempty_spans, num_basis


def gauss_points(xi, nq):
    """Gauss-Legendre nodes and weights mapped to each non-empty span."""
    t, w = np.polynomial.legendre.leggauss(nq)
    pts, wts = [], []
    for a, b in nonempty_spans(xi):
        pts.append(0.5 * (b - a) * t + 0.5 * (a + b))
        wts.append(0.5 * (b - a) * w)
    return np.concatenate(pts), np.concatenate(wts)


def full_matrices(xi, p, nq=None):
    """Full m x m matrices over all basis functions of the knot vector.

    M = int b_i b_j, K = int b'_i b'_j, J = int b''_i b''_j,
    G = int b''_i b_j (row index carries the second derivative).
    """
    nq = p + 1 if nq is None else nq
    x, w = gauss_points(xi, nq)
    B = eval_basis_points(xi, p, x, nder=2)  # (3, nx, m)
    b0, b1, b2 = B[0], B[1], B[2]
    M = b0.T @ (w[:, None] * b0)
    K = b1.T @ (w[:, None] * b1)
    J = b2.T @ (w[:, None] * b2)
    G = b2.T @ (w[:, None] * b0)
    return dict(M=M, K=K, J=J, G=G)


def space_index(m):
    """Restricted space indices: homogeneous Dirichlet drops the first and
    last function (eq. basis_par: i = 2..m-1, 1-based), n_s = m - 2."""
    return np.arange(1, m - 1)


def time_index(m):
    """Restricted time indices: zero initial value drops the first function
    (eq. basis_par: i = 2..m, 1-based), n_t = m - 1."""
    return np.arange(1, m)


def space_matrices(xi, p):
    """M_k, K_k, J_k, G_k restricted to the Dirichlet space (§4.1-4.2)."""
    F = full_matrices(xi, p)
    idx = space_index(num_basis(xi, p))
    return {k: v[np.ix_(idx, idx)] for k, v in F.items()}


def time_matrices(xi, p, T=1.0):
    """K_t, M_t, W_t restricted to the zero-initial-value space (eq. A_kron).

    With t = T tau the physical matrices are K_t = K_hat / T and
    M_t = T M_hat (Remark of §4.4); W_t[i, j] = b_i(T) b_j(T) is a point
    evaluation at the final time.
    """
    F = full_matrices(xi, p)
    m = num_basis(xi, p)
    idx = time_index(m)
    end = eval_basis_points(xi, p, [1.0], nder=0)[0, 0]  # b_i(1), all i
    e = end[idx]
    return dict(K=F["K"][np.ix_(idx, idx)] / T, M=T * F["M"][np.ix_(idx, idx)],
                W=np.outer(e, e), Khat=F["K"][np.ix_(idx, idx)], Mhat=F["M"][np.ix_(idx, idx)])


def load_1d(xi, p, g, nder, index, nq=None):
    """Vector v_i = int g(x) b_i^{(nder)}(x) dx over the restricted indices."""
    nq = p + 3 if nq is None else nq
    x, w = gauss_points(xi, nq)
    B = eval_basis_points(xi, p, x, nder=max(nder, 0))
    return (B[nder].T @ (w * g(x)))[index]


def load_separable(knots, degrees, terms, kappa=1.0):
    """Load vector F_i = int int f (d_t B_i - kappa Lap B_i) (§3.2, eq. a-form).

    f = sum over ``terms`` of c * prod_k g_k(x_k) * h(t), each term given as
    (c, [g_1, ..., g_d], h).  With B_i = prod_k b_{i_k}(x_k) b_{i_t}(t):
      d_t B_i  = b'_{i_t}(t) prod_k b_{i_k}(x_k)
      Lap B_i  = b_{i_t}(t) sum_k b''_{i_k}(x_k) prod_{l != k} b_{i_l}(x_l)
    so F is a sum of Kronecker products of 1-D loads.  Returned as a tensor
    of shape (n_1, ..., n_d, n_t) (vec = Fortran-order ravel).
    """
    d = len(knots) - 1
    shape = [len(space_index(num_basis(knots[k], degrees[k]))) for k in range(d)]
    shape.append(len(time_index(num_basis(knots[d], degrees[d]))))
    F = np.zeros(shape)
    for c, gs, h in terms:
        it = time_index(num_basis(knots[d], degrees[d]))
        ht1 = load_1d(knots[d], degrees[d], h, 1, it)
        ht0 = load_1d(knots[d], degrees[d], h, 0, it)
        g0, g2 = [], []
        for k in range(d):
            isp = space_index(num_basis(knots[k], degrees[k]))
            g0.append(load_1d(knots[k], degrees[k], gs[k], 0, isp))
            g2.append(load_1d(knots[k], degrees[k], gs[k], 2, isp))
        term = _outer([*g0, ht1])
        for k in range(d):
            fac = [g2[l] if l == k else g0[l] for l in range(d)]
            term = term - kappa * _outer([*fac, ht0])
        F += c * term
    return F


def _outer(vecs):
    """Outer product tensor T[i_1, ..., i_n] = prod_k v_k[i_k]."""
    out = np.asarray(vecs[0])
    for v in vecs[1:]:
        out = np.multiply.outer(out, v)
    return out
