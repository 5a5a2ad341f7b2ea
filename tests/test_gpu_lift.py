"""Lifting of non-zero initial data on the GPU (§2, the paragraph after the
parabolic regularity theorem; least-squares form §3.2) against the oracle.

- the coupling a(u0_h b_1, B_i) of stls_lift_initial against the oracle's
  term-by-term expansion (no integration by parts), d = 1, 2, 3, kappa != 1:
  both sides are sums of products of O(1)-conditioned banded factors, so the
  bound is rounding level (1e-12 relative);
- the lifted solve u_h = w_h + u0_h b_1 against the oracle's dense solve of
  the same lifted system (solve tolerance 1e-12; bound 1e-8 relative);
- the GPU error norms of the lifted solution of u = sin(pi x) sin(pi y)
  cos(pi t) (non-zero initial value) against the oracle's norms of the same
  quantity (the oracle's optimal rates are pinned in its own tests).
"""
import numpy as np
import pytest

from stls_inputs import problem_knots, uniform_pm1

pytestmark = pytest.mark.gpu

try:
    import paper_1809_10026_amd as stls
except ImportError:  # library not built: GPU tests must fail loudly, not skip
    stls = None

from oracle import assemble, lift, system as osys  # noqa: E402
from oracle.bspline import eval_basis_points, num_basis  # noqa: E402
from tests.gpu_util import rel_err, to_dev, to_host  # noqa: E402

PI = np.pi


def _lib():
    assert stls is not None, "libstls.so is not built; run python paper_1809_10026_amd/build.py"
    return stls


@pytest.mark.parametrize("d,nel,p,kappa", [(1, [7, 9], 2, 1.0), (1, [12, 5], 5, 0.3), (2, [5, 6, 7], 3, 2.5),
                                           (2, [9, 4, 3], 4, 1.0), (3, [3, 4, 5, 4], 2, 0.8), (3, 4, 3, 1.0),
                                           # linear time splines (one coupled row); a single time element
                                           (2, [5, 6, 7], [3, 3, 1], 1.4), (1, [8, 1], [4, 2], 0.9)])
def test_lift_coupling_matches_oracle(d, nel, p, kappa):
    knots, degs = problem_knots(d, nel, p)
    S = _lib().Solver(knots, degs, kappa=kappa)
    P = osys.Problem(knots, degs, kappa=kappa)
    u0 = uniform_pm1(S.ns, 71)
    F = uniform_pm1(S.ndof, 72)
    Fd = to_dev(F)
    S.lift_initial(to_dev(u0), Fd)
    got = F - to_host(Fd)
    ref = osys.vec(lift.initial_coupling(P, u0))
    assert rel_err(got, ref) < 1e-12


def test_zero_initial_value_leaves_rhs_unchanged():
    knots, degs = problem_knots(2, 6, 3)
    S = _lib().Solver(knots, degs)
    F = uniform_pm1(S.ndof, 73)
    Fd = to_dev(F)
    S.lift_initial(to_dev(np.zeros(S.ns)), Fd)
    assert np.array_equal(to_host(Fd), F)


def _manufactured_rhs(knots, degs, d, kappa):
    s = lambda x: np.sin(PI * x)
    F = assemble.load_separable(knots, degs, [(-PI, [s] * d, lambda t: np.sin(PI * t)),
                                              (kappa * d * PI * PI, [s] * d, lambda t: np.cos(PI * t))], kappa)
    return F, [s] * d


@pytest.mark.parametrize("d,nel,p,kappa", [(1, 12, 3, 1.0), (2, 8, 3, 0.7)])
def test_lifted_solve_matches_oracle(d, nel, p, kappa):
    knots, degs = problem_knots(d, nel, p)
    S = _lib().Solver(knots, degs, kappa=kappa)
    P = osys.Problem(knots, degs, kappa=kappa)
    F, gs = _manufactured_rhs(knots, degs, d, kappa)
    U0 = lift.l2_projection(P, gs)
    u0d = to_dev(osys.vec(U0))
    Fd = to_dev(osys.vec(F))
    S.lift_initial(u0d, Fd)
    w, it, rel = S.solve(Fd, rtol=1e-12, maxit=300)
    u = to_host(S.lift_combine(u0d, w))
    ref = osys.vec(lift.combine(P, U0, np.linalg.solve(P.dense_A(), osys.vec(lift.lifted_rhs(P, F, U0)))))
    assert rel <= 1e-12 and rel_err(u, ref) < 1e-8


def _spline_factors(xi, p, coef, x):
    """(value, first, second derivative) at x of the spline sum_i coef_i b_i
    over the restricted spatial functions."""
    B = eval_basis_points(xi, p, x, nder=2)
    idx = assemble.space_index(num_basis(xi, p))
    return np.stack([B[r][:, idx] @ coef for r in range(3)])


@pytest.mark.parametrize("nel,p", [(6, 3), (9, 4)])
def test_lifted_error_norms_match_oracle(nel, p):
    """d = 2: u = sin(pi x) sin(pi y) cos(pi t).  The GPU norms see w_h against
    u - u0_h b_1 (two separable terms), whose error is the error of u_h; the
    oracle evaluates the same quantity with its own basis evaluation (its
    convergence at the optimal rates is pinned in the oracle tests).  Bound as
    for the homogeneous norms: 1e-8 relative plus 1e-12 absolute."""
    from oracle import norms as onorms
    d, kappa = 2, 1.0
    knots, degs = problem_knots(d, nel, p)
    S = _lib().Solver(knots, degs, kappa=kappa)
    P = osys.Problem(knots, degs, kappa=kappa)
    F, gs = _manufactured_rhs(knots, degs, d, kappa)
    isp = [assemble.space_index(num_basis(knots[k], p)) for k in range(d)]
    vecs = [np.linalg.solve(P.space[k]["M"], assemble.load_1d(knots[k], p, gs[k], 0, isp[k])) for k in range(d)]
    U0 = lift.l2_projection(P, gs)
    u0d = to_dev(osys.vec(U0))
    Fd = to_dev(osys.vec(F))
    S.lift_initial(u0d, Fd)
    w, _, _ = S.solve(Fd, rtol=1e-12, maxit=300)
    xs = [S.norm_points(k)[0] for k in range(d + 1)]
    sinf = lambda x: np.stack([np.sin(PI * x), PI * np.cos(PI * x), -PI * PI * np.sin(PI * x)])
    cosf = lambda t: np.stack([np.cos(PI * t), -PI * np.sin(PI * t), -PI * PI * np.cos(PI * t)])
    b1f = lambda t: eval_basis_points(knots[d], p, t, nder=2)[:, :, 0]
    spl = [lambda x, k=k: _spline_factors(knots[k], p, vecs[k], x) for k in range(d)]
    fac = [[sinf(xs[0]), sinf(xs[1]), cosf(xs[2])], [spl[0](xs[0]), spl[1](xs[1]), -b1f(xs[2])]]
    got = S.error_norms(w, fac)

    def sep(G, der):  # u - u0_h b_1 and derivatives on the oracle's meshgrid
        x, y, t = G[0][:, 0, 0], G[1][0, :, 0], G[2][0, 0, :]
        f1 = [sinf(x), sinf(y), cosf(t)]
        f2 = [spl[0](x), spl[1](y), -b1f(t)]
        return sum(np.einsum("i,j,k->ijk", a[der[0]], b[der[1]], c[der[2]]) for a, b, c in (f1, f2))

    ex = dict(u=lambda *G: sep(G, (0, 0, 0)), ut=lambda *G: sep(G, (0, 0, 1)),
              lap=lambda *G: sep(G, (2, 0, 0)) + sep(G, (0, 2, 0)),
              grad=[lambda *G: sep(G, (1, 0, 0)), lambda *G: sep(G, (0, 1, 0))])
    ref = onorms.error_norms(osys.unvec(to_host(w), S.shape), knots, degs, ex)
    for key in ("V0", "L2", "H1"):
        assert abs(got[key] - ref[key]) <= 1e-8 * ref[key] + 1e-12, (key, got[key], ref[key])


def test_lift_rejects_null_pointers():
    knots, degs = problem_knots(1, 4, 2)
    S = _lib().Solver(knots, degs)
    rc = stls._lib.stls_lift_initial(S._h, None, None)
    assert rc != 0


# --- general data (boundary and initial coefficients) -----------------------

@pytest.mark.parametrize("d,nel,p,kappa", [(1, [6, 9], 3, 0.4), (2, [5, 4, 6], 2, 1.7), (3, [3, 4, 3, 5], 3, 1.0),
                                           (2, [5, 6, 7], [3, 3, 1], 1.4), (1, [8, 1], [4, 2], 0.9)])
def test_general_lift_matches_oracle(d, nel, p, kappa):
    knots, degs = problem_knots(d, nel, p)
    S = _lib().Solver(knots, degs, kappa=kappa)
    P = osys.Problem(knots, degs, kappa=kappa)
    nfull = int(np.prod(P.full_shape))
    ub = uniform_pm1(nfull, 81)
    F = uniform_pm1(S.ndof, 82)
    Fd = to_dev(F)
    S.lift_apply(to_dev(ub), Fd)
    got = F - to_host(Fd)
    ref = osys.vec(lift.general_coupling(P, ub))
    assert rel_err(got, ref) < 1e-12


@pytest.mark.parametrize("d,nel,p,kappa", [(1, 11, 4, 0.8), (2, [7, 6, 5], 3, 1.0), (3, 4, 2, 2.0)])
def test_general_lift_of_zero_data_function_is_the_matvec(d, nel, p, kappa):
    """On a trial function of the zero-data space the term-by-term form equals
    the system matrix (two independent GPU code paths)."""
    import torch
    knots, degs = problem_knots(d, nel, p)
    S = _lib().Solver(knots, degs, kappa=kappa)
    nfull = S.forcing_shape[1]
    x = to_dev(uniform_pm1(S.ndof, 83))
    ub = S.lift_embed(torch.zeros(nfull, dtype=torch.float64, device="cuda"), x)
    F = torch.zeros(S.ndof, dtype=torch.float64, device="cuda")
    S.lift_apply(ub, F)
    assert rel_err(-to_host(F), to_host(S.matvec(x))) < 1e-12


def test_lift_embed_is_exact():
    knots, degs = problem_knots(2, [5, 4, 6], 3)
    S = _lib().Solver(knots, degs)
    P = osys.Problem(knots, degs)
    nfull = int(np.prod(P.full_shape))
    ub, w = uniform_pm1(nfull, 84), uniform_pm1(S.ndof, 85)
    got = to_host(S.lift_embed(to_dev(ub), to_dev(w)))
    ref = osys.vec(ub.reshape(P.full_shape, order="F") + lift.embed(P, w))
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("d,nel,p,kappa", [(1, 12, 3, 1.0), (2, 7, 3, 0.6)])
def test_boundary_lifted_solve_matches_oracle(d, nel, p, kappa):
    """u = prod cos(pi x_k) (1 + t): non-zero boundary and initial values; u_B
    from the full L^2 projection (oracle input).  Bound as for the
    initial-data solve."""
    knots, degs = problem_knots(d, nel, p)
    S = _lib().Solver(knots, degs, kappa=kappa)
    P = osys.Problem(knots, degs, kappa=kappa)
    c = lambda x: np.cos(PI * x)
    F = assemble.load_separable(knots, degs, [(1.0, [c] * d, np.ones_like),
                                              (kappa * d * PI * PI, [c] * d, lambda t: 1 + t)], kappa)
    UB = lift.boundary_part(P, lift.full_projection(P, [c] * d, lambda t: 1 + t))
    ubd = to_dev(osys.vec(UB))
    Fd = to_dev(osys.vec(F))
    S.lift_apply(ubd, Fd)
    w, it, rel = S.solve(Fd, rtol=1e-12, maxit=300)
    u = to_host(S.lift_embed(ubd, w))
    W = np.linalg.solve(P.dense_A(), osys.vec(F - lift.general_coupling(P, UB)))
    ref = osys.vec(UB + lift.embed(P, W))
    assert rel <= 1e-12 and rel_err(u, ref) < 1e-8
