"""Non-zero initial data by lifting (§2, the paragraph after the parabolic
regularity theorem).  Oracle: test use only.

The paper lifts an initial value u0 in H^1_0(Omega) to a function ~u0 of
space and time; w = u - ~u0 then has zero initial and boundary data and
solves the heat equation with forcing f - d_t ~u0 + kappa Lap ~u0.

Discretely ~u0 = u0_h(x) b_1(t): u0_h in the restricted (Dirichlet) spatial
spline space and b_1 the first time B-spline, the only one that is non-zero
at t = 0 on an open knot vector.  The least-squares equations (§3.2) for
w_h in the zero-data space are

    A w = F(f) - a(~u0, B_i),
    a(u, v) = int int (d_t u - kappa Lap u)(d_t v - kappa Lap v),

and u_h = w_h + ~u0.  Here a(~u0, B_i) is expanded term by term, with no
integration by parts, for B_i = b_i(x) b_j(t), j >= 2:

      int b_1' b_j'            * int u0_h b_i
    + kappa^2 int b_1 b_j      * int Lap u0_h Lap b_i
    - kappa   int b_1' b_j     * int u0_h Lap b_i
    - kappa   int b_1 b_j'     * int Lap u0_h b_i.

The last two terms cancel (their time factors add up to [b_1 b_j] between
0 and T, which is zero, and the space factors agree for H^1_0 functions);
they are kept so that the cancellation is checked rather than assumed.
"""
from __future__ import annotations

import numpy as np

from . import assemble
from .bspline import eval_basis_points, num_basis
from .system import kron_apply


def time_columns(xi, p):
    """Couplings of the first time function b_1 with the restricted ones:
    K1[j] = int b_1' b_j', M1[j] = int b_1 b_j, C1[j] = int b_1' b_j,
    C2[j] = int b_1 b_j' (Gauss quadrature with p + 1 points per span, exact
    for these piecewise polynomials)."""
    x, w = assemble.gauss_points(xi, p + 1)
    B = eval_basis_points(xi, p, x, nder=1)  # (2, nx, m)
    b0, b1 = B[0], B[1]
    idx = assemble.time_index(num_basis(xi, p))
    K1 = (w * b1[:, 0]) @ b1[:, idx]
    M1 = (w * b0[:, 0]) @ b0[:, idx]
    C1 = (w * b1[:, 0]) @ b0[:, idx]
    C2 = (w * b0[:, 0]) @ b1[:, idx]
    return dict(K1=K1, M1=M1, C1=C1, C2=C2)


def _space_parts(P, U0):
    """Spatial factors applied to the initial coefficients U0 (restricted
    spatial shape): int u0 b_i, int Lap u0 Lap b_i (literal sum over k, l),
    int u0 Lap b_i and int Lap u0 b_i."""
    d, S = P.d, P.space
    MU = kron_apply([S[k]["M"] for k in range(d)], U0)
    JU = 0.0
    for _, fac in P.system_terms():
        if fac[d] is P.time["M"]:  # spatial parts of the kappa^2 M_t x J_s terms (without kappa^2)
            JU = JU + kron_apply(fac[:d], U0)
    # G = int b''_i b_j (row index carries the second derivative): the test
    # function's Laplacian is G in direction k, the trial function's G^T
    GU = sum(kron_apply([S[m]["G"] if m == k else S[m]["M"] for m in range(d)], U0) for k in range(d))
    GTU = sum(kron_apply([S[m]["G"].T if m == k else S[m]["M"] for m in range(d)], U0) for k in range(d))
    return MU, JU, GU, GTU


def initial_coupling(P, U0):
    """a(u0_h b_1, B_i) for every restricted B_i, as a tensor of P.shape."""
    U0 = np.asarray(U0, dtype=float).reshape(P.shape[:-1], order="F")
    tc = time_columns(P.knots[P.d], P.degrees[P.d])
    MU, JU, GU, GTU = _space_parts(P, U0)
    kap = P.kappa

    def outer(S, c):
        return S[..., None] * np.asarray(c)[(None,) * S.ndim]

    return (outer(MU, tc["K1"]) + kap * kap * outer(JU, tc["M1"])
            - kap * outer(GU, tc["C1"]) - kap * outer(GTU, tc["C2"]))


def lifted_rhs(P, F, U0):
    """Right-hand side of the zero-data problem: F - a(u0_h b_1, B_i)."""
    return np.asarray(F).reshape(P.shape, order="F") - initial_coupling(P, U0)


def combine(P, U0, W):
    """Coefficients of u_h over every time function: u0_h first, then w_h."""
    U0 = np.asarray(U0, dtype=float).reshape(P.shape[:-1], order="F")
    W = np.asarray(W, dtype=float).reshape(P.shape, order="F")
    return np.concatenate([U0[..., None], W], axis=-1)


def l2_projection(P, gs):
    """Coefficients of the L^2 projection of u0 = prod_k g_k(x_k) onto the
    restricted spatial space: (M_1^-1 g_1) x ... x (M_d^-1 g_d) with
    g_k[i] = int g_k b_i."""
    d = P.d
    vecs = []
    for k in range(d):
        isp = assemble.space_index(num_basis(P.knots[k], P.degrees[k]))
        gk = assemble.load_1d(P.knots[k], P.degrees[k], gs[k], 0, isp)
        vecs.append(np.linalg.solve(P.space[k]["M"], gk))
    out = vecs[0]
    for v in vecs[1:]:
        out = np.multiply.outer(out, v)
    return out


# ---------------------------------------------------------------------------
# General data: a lifting u_B anywhere in the full spline space (non-zero
# boundary coefficients in space and/or the initial time coefficients).
# For such a trial function the spatial integrations by parts behind the
# system matrix leave boundary terms, so a(u_B, B_i) is assembled from the
# four products of the least-squares form directly:
#   int int d_t u d_t v            -> K_t (x) M_s
#   kappa^2 int int Lap u Lap v    -> M_t (x) sum_{k,l} int d_kk u d_ll v
#   -kappa int int d_t u Lap v     -> (int b_i b'_j)_t (x) sum_k (int b''_i b_j)_k
#   -kappa int int Lap u d_t v     -> (int b'_i b_j)_t (x) sum_k (int b_i b''_j)_k
# with every factor over test functions i (rows) and trial functions j
# (columns) of the full space; the rows are then restricted.

def _full_factors(xi, p):
    """Full m x m matrices, rows test i, columns trial j: M, K (b' b'),
    J (b'' b''), Gt (int b''_i b_j: test second derivative), Gs (int b_i
    b''_j: trial second derivative), Ct (int b'_i b_j: test derivative),
    Cs (int b_i b'_j: trial derivative)."""
    x, w = assemble.gauss_points(xi, p + 1)
    B = eval_basis_points(xi, p, x, nder=2)
    b0, b1, b2 = B[0], B[1], B[2]
    ip = lambda a, b: a.T @ (w[:, None] * b)
    return dict(M=ip(b0, b0), K=ip(b1, b1), J=ip(b2, b2), Gt=ip(b2, b0), Gs=ip(b0, b2),
                Ct=ip(b1, b0), Cs=ip(b0, b1))


def full_terms(P):
    """(coefficient, factors per mode, time last) of a(u, B_i) over the full
    space, before the restriction of the rows."""
    d, kap = P.d, P.kappa
    S = [_full_factors(P.knots[k], P.degrees[k]) for k in range(d)]
    T = _full_factors(P.knots[d], P.degrees[d])
    terms = [(1.0, [S[k]["M"] for k in range(d)] + [T["K"]])]
    for k in range(d):
        for l in range(d):
            fac = [S[m]["M"] for m in range(d)]
            if k == l:
                fac[k] = S[k]["J"]
            else:
                fac[k] = S[k]["Gs"]  # trial function differentiated twice in x_k
                fac[l] = S[l]["Gt"]  # test function differentiated twice in x_l
            terms.append((kap * kap, fac + [T["M"]]))
    for k in range(d):
        fac = [S[m]["Gt"] if m == k else S[m]["M"] for m in range(d)]
        terms.append((-kap, fac + [T["Cs"]]))
    for k in range(d):
        fac = [S[m]["Gs"] if m == k else S[m]["M"] for m in range(d)]
        terms.append((-kap, fac + [T["Ct"]]))
    return terms


def _restricted_rows(P):
    d = P.d
    idx = [assemble.space_index(num_basis(P.knots[k], P.degrees[k])) for k in range(d)]
    idx.append(assemble.time_index(num_basis(P.knots[d], P.degrees[d])))
    return np.ix_(*idx)


def general_coupling(P, UB):
    """a(u_B, B_i) for every restricted B_i; UB over the full space
    (shape P.full_shape), result of shape P.shape."""
    UB = np.asarray(UB, dtype=float).reshape(P.full_shape, order="F")
    full = sum(c * kron_apply(f, UB) for c, f in full_terms(P))
    return full[_restricted_rows(P)]


def embed(P, W):
    """The restricted coefficients W placed in the full space (zeros on the
    boundary and initial coefficients)."""
    out = np.zeros(P.full_shape)
    out[_restricted_rows(P)] = np.asarray(W, dtype=float).reshape(P.shape, order="F")
    return out


def full_projection(P, gs, h):
    """L^2 projection of u = prod_k g_k(x_k) h(t) onto the full space:
    (M_1^-1 g_1) x ... x (M_d^-1 g_d) x (M_t^-1 h), full mass matrices."""
    vecs = []
    for k in range(P.d + 1):
        xi, p = P.knots[k], P.degrees[k]
        f = gs[k] if k < P.d else h
        m = num_basis(xi, p)
        rhs = assemble.load_1d(xi, p, f, 0, np.arange(m))
        vecs.append(np.linalg.solve(_full_factors(xi, p)["M"], rhs))
    out = vecs[0]
    for v in vecs[1:]:
        out = np.multiply.outer(out, v)
    return out


def boundary_part(P, U):
    """U (full space) with its restricted coefficients set to zero."""
    out = np.array(U, dtype=float).reshape(P.full_shape, order="F")
    out[_restricted_rows(P)] = 0.0
    return out
