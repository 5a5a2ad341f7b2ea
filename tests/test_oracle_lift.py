"""Pins of the lifting oracle (non-zero initial data, §2 paragraph after the
parabolic regularity theorem; least-squares form §3.2).

- a(u0_h b_1, B_i) agrees with the bilinear form evaluated from its
  definition on a space-time Gauss grid (brute force, no Kronecker
  factorisation), d = 1 and d = 2, kappa != 1;
- the two cross terms cancel (time factors add to [b_1 b_j] from 0 to T = 0;
  int u0 Lap b_i = int Lap u0 b_i for H^1_0 splines);
- a manufactured solution with non-zero initial value converges at the
  rates of the homogeneous problem (V0 ~ h^{p-1}, H1 ~ h^p, L2 ~ h^{p+1}),
  and dropping the lifting term (a planted mistake) destroys convergence;
- general data (boundary and initial coefficients, term-by-term form): brute
  force, reproduction of the system matrix on zero-data trial functions
  (whose cross terms were integrated by parts), the initial-data special
  case, optimal rates with non-zero boundary values, and a planted dropped
  cross term.
"""
import numpy as np
import pytest

from oracle import assemble, lift, norms as onorms, system as osys
from oracle.bspline import eval_basis_points, num_basis
from stls_inputs import problem_knots

PI = np.pi


def _brute_coupling(P, U0):
    """int int (d_t u_L - kappa Lap u_L)(d_t B_i - kappa Lap B_i) on the tensor
    Gauss grid, u_L = u0_h(x) b_1(t), for every restricted B_i."""
    d, kap = P.d, P.kappa
    B, W = [], []
    for k in range(d + 1):
        x, w = assemble.gauss_points(P.knots[k], P.degrees[k] + 1)
        B.append(eval_basis_points(P.knots[k], P.degrees[k], x, nder=2))
        W.append(w)
    isp = [assemble.space_index(num_basis(P.knots[k], P.degrees[k])) for k in range(d)]
    itm = assemble.time_index(num_basis(P.knots[d], P.degrees[d]))

    def field(coef, ders):  # sum_i coef_i prod_k b_{i_k}^{(ders_k)} on the spatial grid
        X = coef
        for k in range(d):
            X = osys.mode_product(X, B[k][ders[k]][:, isp[k]], k)
        return X

    u0 = field(U0, [0] * d)
    lap0 = sum(field(U0, [2 if l == k else 0 for l in range(d)]) for k in range(d))
    b1, db1 = B[d][0][:, 0], B[d][1][:, 0]
    RL = np.multiply.outer(u0, db1) - kap * np.multiply.outer(lap0, b1)  # (x grid..., t grid)
    Wt = W[0]
    for w in W[1:]:
        Wt = np.multiply.outer(Wt, w)
    out = np.zeros(P.shape)
    # test functions: loop over the restricted multi-indices (tiny sizes)
    for idx in np.ndindex(*P.shape):
        phi = [B[k][0][:, isp[k][idx[k]]] for k in range(d)]
        phi2 = [B[k][2][:, isp[k][idx[k]]] for k in range(d)]
        psi, dpsi = B[d][0][:, itm[idx[d]]], B[d][1][:, itm[idx[d]]]
        sp = phi[0]
        for v in phi[1:]:
            sp = np.multiply.outer(sp, v)
        lap = 0.0
        for k in range(d):
            t = phi2[0] if k == 0 else phi[0]
            for l in range(1, d):
                t = np.multiply.outer(t, phi2[l] if l == k else phi[l])
            lap = lap + t
        LB = np.multiply.outer(sp, dpsi) - kap * np.multiply.outer(lap, psi)
        out[idx] = np.sum(Wt * RL * LB)
    return out


@pytest.mark.parametrize("d,nel,p,kappa", [(1, [4, 5], 2, 0.6), (1, [3, 4], 4, 2.0), (2, [3, 2, 3], 3, 1.3)])
def test_coupling_matches_brute_force(d, nel, p, kappa):
    P = osys.Problem(*problem_knots(d, nel, p), kappa=kappa)
    U0 = np.random.default_rng(7).standard_normal(P.shape[:-1])
    got = lift.initial_coupling(P, U0)
    ref = _brute_coupling(P, U0)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # only the first p time rows couple to b_1
    assert np.abs(got[..., p:]).max() == 0.0


@pytest.mark.parametrize("nel,p", [(5, 2), (7, 3), (9, 5)])
def test_cross_terms_cancel(nel, p):
    P = osys.Problem(*problem_knots(2, nel, p), kappa=1.7)
    tc = lift.time_columns(P.knots[2], P.degrees[2])
    assert np.abs(tc["C1"] + tc["C2"]).max() < 1e-14 * np.abs(tc["C1"]).max()
    U0 = np.random.default_rng(3).standard_normal(P.shape[:-1])
    _, _, GU, GTU = lift._space_parts(P, U0)
    assert np.abs(GU - GTU).max() < 1e-12 * np.abs(GU).max()


def _manufactured(d, nel, p, kappa, with_lift=True):
    """u = prod sin(pi x_k) cos(pi t): u(., 0) = prod sin(pi x_k) in H^1_0."""
    knots, degs = problem_knots(d, nel, p)
    P = osys.Problem(knots, degs, kappa=kappa)
    s = lambda x: np.sin(PI * x)
    F = assemble.load_separable(knots, degs, [(-PI, [s] * d, lambda t: np.sin(PI * t)),
                                              (kappa * d * PI * PI, [s] * d, lambda t: np.cos(PI * t))], kappa)
    U0 = lift.l2_projection(P, [s] * d)
    rhs = lift.lifted_rhs(P, F, U0) if with_lift else F
    Wsol = np.linalg.solve(P.dense_A(), osys.vec(rhs))
    Ufull = lift.combine(P, U0, Wsol)

    def prod_sin(X):
        out = 1.0
        for x in X:
            out = out * np.sin(PI * x)
        return out

    def grad_k(k):
        return lambda *G: PI * np.cos(PI * G[k]) * prod_sin([G[l] for l in range(d) if l != k]) * np.cos(PI * G[d])

    ex = dict(u=lambda *G: prod_sin(G[:d]) * np.cos(PI * G[d]),
              ut=lambda *G: -PI * prod_sin(G[:d]) * np.sin(PI * G[d]),
              lap=lambda *G: -d * PI * PI * prod_sin(G[:d]) * np.cos(PI * G[d]),
              grad=[grad_k(k) for k in range(d)])
    return onorms.error_norms(Ufull, knots, degs, ex, full_time=True)


@pytest.mark.parametrize("d,nels,p,kappa", [(1, (8, 16), 3, 1.0), (1, (8, 16), 4, 0.5), (2, (6, 12), 3, 1.0)])
def test_manufactured_nonzero_initial_value_rates(d, nels, p, kappa):
    e = [_manufactured(d, n, p, kappa) for n in nels]
    rate = {k: np.log2(e[0][k] / e[1][k]) for k in e[0]}
    assert abs(rate["V0"] - (p - 1)) < 0.3, rate
    assert abs(rate["H1"] - p) < 0.3, rate
    assert abs(rate["L2"] - (p + 1)) < 0.4, rate
    assert e[1]["L2"] < 1e-3


def test_dropping_the_lift_is_caught():
    """Planted mistake: keep u0_h as the first time coefficient but leave the
    right-hand side unlifted.  The error then stays O(1) under refinement."""
    e = [_manufactured(1, n, 3, 1.0, with_lift=False) for n in (8, 16)]
    assert e[1]["L2"] > 0.05 and e[0]["L2"] / e[1]["L2"] < 2.0


# --- general data (boundary and initial coefficients) -----------------------

def _brute_general(P, UB):
    """int int (d_t u_B - kappa Lap u_B)(d_t B_i - kappa Lap B_i) on the tensor
    Gauss grid for u_B over the full space, every restricted B_i."""
    d, kap = P.d, P.kappa
    B, W = [], []
    for k in range(d + 1):
        x, w = assemble.gauss_points(P.knots[k], P.degrees[k] + 1)
        B.append(eval_basis_points(P.knots[k], P.degrees[k], x, nder=2))
        W.append(w)

    def field(ders):  # u_B and its derivatives on the space-time grid
        X = UB
        for k in range(d + 1):
            X = osys.mode_product(X, B[k][ders[k]], k)
        return X

    RL = field([0] * d + [1]) - kap * sum(field([2 if l == k else 0 for l in range(d)] + [0]) for k in range(d))
    Wt = W[0]
    for w in W[1:]:
        Wt = np.multiply.outer(Wt, w)
    isp = [assemble.space_index(num_basis(P.knots[k], P.degrees[k])) for k in range(d)]
    itm = assemble.time_index(num_basis(P.knots[d], P.degrees[d]))
    out = np.zeros(P.shape)
    for idx in np.ndindex(*P.shape):
        cols = [isp[k][idx[k]] for k in range(d)] + [itm[idx[d]]]

        def test(ders):
            t = B[0][ders[0]][:, cols[0]]
            for k in range(1, d + 1):
                t = np.multiply.outer(t, B[k][ders[k]][:, cols[k]])
            return t

        LB = test([0] * d + [1]) - kap * sum(test([2 if l == k else 0 for l in range(d)] + [0]) for k in range(d))
        out[idx] = np.sum(Wt * RL * LB)
    return out


@pytest.mark.parametrize("d,nel,p,kappa", [(1, [4, 5], 3, 0.6), (2, [3, 2, 3], 2, 1.3)])
def test_general_coupling_matches_brute_force(d, nel, p, kappa):
    P = osys.Problem(*problem_knots(d, nel, p), kappa=kappa)
    UB = np.random.default_rng(11).standard_normal(P.full_shape)
    got = lift.general_coupling(P, UB)
    ref = _brute_general(P, UB)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("d,nel,p,kappa", [(1, [5, 6], 3, 0.7), (2, [4, 3, 5], 2, 1.6), (3, [3, 3, 3, 4], 3, 1.0)])
def test_general_coupling_reproduces_system_matrix(d, nel, p, kappa):
    """On trial functions of the zero-data space the term-by-term form must
    equal the system matrix, whose cross terms were integrated by parts into
    the final-time term kappa W_t x L_s (§4.1)."""
    P = osys.Problem(*problem_knots(d, nel, p), kappa=kappa)
    X = np.random.default_rng(12).standard_normal(P.shape)
    got = lift.general_coupling(P, lift.embed(P, X))
    ref = P.matvec(X)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("d", [1, 2, 3])
def test_general_coupling_initial_data_special_case(d):
    P = osys.Problem(*problem_knots(d, 3, 3), kappa=0.9)
    U0 = np.random.default_rng(13).standard_normal(P.shape[:-1])
    UB = np.zeros(P.full_shape)
    inner = np.ix_(*[np.arange(1, P.full_shape[m] - 1) for m in range(d)])
    UB[..., 0][inner] = U0
    got = lift.general_coupling(P, UB)
    ref = lift.initial_coupling(P, U0)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def _boundary_manufactured(d, nel, p, kappa):
    """u = prod cos(pi x_k) (1 + t): non-zero boundary and initial values.
    u_B = boundary and initial coefficients of the full L^2 projection."""
    knots, degs = problem_knots(d, nel, p)
    P = osys.Problem(knots, degs, kappa=kappa)
    c = lambda x: np.cos(PI * x)
    F = assemble.load_separable(knots, degs, [(1.0, [c] * d, np.ones_like),
                                              (kappa * d * PI * PI, [c] * d, lambda t: 1 + t)], kappa)
    UB = lift.boundary_part(P, lift.full_projection(P, [c] * d, lambda t: 1 + t))
    W = np.linalg.solve(P.dense_A(), osys.vec(F - lift.general_coupling(P, UB)))
    U = UB + lift.embed(P, W)

    def pc(X):
        out = 1.0
        for x in X:
            out = out * np.cos(PI * x)
        return out

    def gk(k):
        return lambda *G: -PI * np.sin(PI * G[k]) * pc([G[l] for l in range(d) if l != k]) * (1 + G[d])

    ex = dict(u=lambda *G: pc(G[:d]) * (1 + G[d]), ut=lambda *G: pc(G[:d]),
              lap=lambda *G: -d * PI * PI * pc(G[:d]) * (1 + G[d]), grad=[gk(k) for k in range(d)])
    return onorms.error_norms(U, knots, degs, ex, full_time=True, full_space=True)


@pytest.mark.parametrize("d,nels,p,kappa", [(1, (8, 16), 3, 1.0), (1, (8, 16), 4, 0.5), (2, (6, 12), 3, 1.0)])
def test_manufactured_boundary_data_rates(d, nels, p, kappa):
    e = [_boundary_manufactured(d, n, p, kappa) for n in nels]
    rate = {k: np.log2(e[0][k] / e[1][k]) for k in e[0]}
    assert abs(rate["V0"] - (p - 1)) < 0.3, rate
    assert abs(rate["H1"] - p) < 0.3, rate
    assert abs(rate["L2"] - (p + 1)) < 0.4, rate


def test_dropping_a_cross_term_is_caught(monkeypatch):
    """Planted mistake: without the -kappa int int Lap u d_t v terms the general
    form no longer reproduces the system matrix."""
    orig = lift.full_terms

    def without_last(P):
        terms = orig(P)
        return terms[:len(terms) - P.d]

    monkeypatch.setattr(lift, "full_terms", without_last)
    P = osys.Problem(*problem_knots(2, [4, 3, 5], 2), kappa=1.6)
    X = np.random.default_rng(12).standard_normal(P.shape)
    got = lift.general_coupling(P, lift.embed(P, X))
    ref = P.matvec(X)
    assert np.abs(got - ref).max() > 1e-3 * np.abs(ref).max()
