"""Pins of the oracle's diagonally scaled FD preconditioner (§4.4, closing
definition: P^G = D^{1/2} P D^{1/2}, D_ii = A_ii / P_ii)."""
import numpy as np
import pytest

from oracle import fd, pcg, system
from stls_inputs import problem_knots, uniform_pm1

CASES = [(1, 5, 2, 1.0), (1, 4, 4, 0.3), (2, 3, 3, 1.0), (2, 3, 2, 10.0), (3, 2, 2, 1.0), (3, 2, 3, 0.5)]


@pytest.mark.parametrize("d,nel,p,kappa", CASES)
def test_kronecker_diagonals_equal_explicit_diagonals(d, nel, p, kappa):
    """Term-by-term diagonals of the Kronecker forms against the diagonals of
    the explicitly assembled matrices (np.kron of the full factors)."""
    knots, degs = problem_knots(d, nel, p)
    P = system.Problem(knots, degs, kappa=kappa)
    a = system.vec(P.kron_diagonal(P.system_terms()))
    b = system.vec(P.kron_diagonal(P.prec_terms()))
    assert np.allclose(a, np.diag(P.dense_A()), rtol=1e-13, atol=0)
    assert np.allclose(b, np.diag(P.dense_P()), rtol=1e-13, atol=0)


@pytest.mark.parametrize("d,nel,p,kappa", CASES)
def test_scaling_is_at_least_one(d, nel, p, kappa):
    """A - P is positive semidefinite on the unit box (cross terms of J_s and
    the final-time term), so its diagonal is >= 0 and D_ii >= 1."""
    knots, degs = problem_knots(d, nel, p)
    P = system.Problem(knots, degs, kappa=kappa)
    D = fd.ScaledFD(P).D
    assert D.min() >= 1.0 - 1e-14
    if d >= 2:  # the cross terms reach every entry
        assert D[..., 0].min() > 1.0


@pytest.mark.parametrize("nel,p,kappa", [(5, 2, 1.0), (6, 4, 2.0)])
def test_scaling_in_one_dimension_touches_only_the_final_slice(nel, p, kappa):
    """d = 1 has no cross terms: A and P differ only by kappa W_t x K_1, whose
    single time entry sits at the final time, so D = 1 elsewhere (exactly:
    the same products are summed) and D > 1 on the final slice."""
    knots, degs = problem_knots(1, nel, p)
    P = system.Problem(knots, degs, kappa=kappa)
    D = fd.ScaledFD(P).D
    assert np.array_equal(D[:, :-1], np.ones_like(D[:, :-1]))
    assert D[:, -1].min() > 1.0


@pytest.mark.parametrize("d,nel,p,kappa", CASES)
def test_scaled_fd_equals_dense_scaled_solve(d, nel, p, kappa):
    """(D^1/2 P D^1/2)^{-1} r by a dense solve with D from the explicit
    matrices, against D^-1/2 (Algorithm 1) D^-1/2 r."""
    knots, degs = problem_knots(d, nel, p)
    P = system.Problem(knots, degs, kappa=kappa)
    Pd = P.dense_P()
    S = np.diag(np.sqrt(np.diag(P.dense_A()) / np.diag(Pd)))
    r = uniform_pm1(P.ndof, 3)
    ref = np.linalg.solve(S @ Pd @ S, r)
    got = system.vec(fd.ScaledFD(P).apply(r))
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("d,nel,p,kappa", [(1, 6, 3, 1.0), (2, 3, 3, 1.0), (3, 2, 2, 0.5)])
def test_scaled_preconditioner_is_symmetric_and_pcg_converges(d, nel, p, kappa):
    knots, degs = problem_knots(d, nel, p)
    P = system.Problem(knots, degs, kappa=kappa)
    G = fd.ScaledFD(P)
    prec = lambda v: system.vec(G.apply(v))
    u, v = uniform_pm1(P.ndof, 4), uniform_pm1(P.ndof, 5)
    assert abs(u @ prec(v) - v @ prec(u)) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(prec(v))
    b = uniform_pm1(P.ndof, 6)
    x, info = pcg.pcg(lambda y: system.vec(P.matvec(y)), prec, b, rtol=1e-11, maxit=200)
    xd = np.linalg.solve(P.dense_A(), b)
    assert info["converged"]
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
