"""Pins of the oracle's univariate matrices (§4.1-4.2) and load vectors."""
import numpy as np
import pytest
import scipy.interpolate

from oracle import assemble, bspline, system
from stls_inputs import uniform_open_knots, problem_knots

CASES = [(uniform_open_knots(n, p), p) for n, p in [(4, 2), (6, 3), (5, 4), (7, 5), (3, 2)]]
CASES.append((np.array([0, 0, 0, 0, 0.2, 0.45, 0.45, 0.8, 1, 1, 1, 1.0]), 3))


@pytest.mark.parametrize("xi,p", CASES)
def test_full_mass_sums_to_domain_measure(xi, p):
    M = assemble.full_matrices(xi, p)["M"]
    assert abs(M.sum() - 1.0) < 1e-14
    m = M.shape[0]
    row_ref = np.array([(xi[i + p + 1] - xi[i]) / (p + 1) for i in range(m)])
    assert np.allclose(M.sum(axis=1), row_ref, atol=1e-15)


@pytest.mark.parametrize("xi,p", CASES)
def test_stiffness_and_bilaplacian_kill_constants_and_lines(xi, p):
    F = assemble.full_matrices(xi, p)
    m = F["M"].shape[0]
    one, g = np.ones(m), bspline.greville(xi, p)
    scaleK, scaleJ = np.abs(F["K"]).max(), np.abs(F["J"]).max()
    assert np.abs(F["K"] @ one).max() < 1e-12 * scaleK
    assert np.abs(F["J"] @ one).max() < 1e-12 * scaleJ
    assert np.abs(F["J"] @ g).max() < 1e-12 * scaleJ
    # (K g)_i = int b_i' * 1 = b_i(1) - b_i(0)
    e = np.zeros(m)
    e[-1], e[0] = 1.0, -1.0
    assert np.allclose(F["K"] @ g, e, atol=1e-12 * scaleK)


@pytest.mark.parametrize("n", [3, 5, 8])
def test_linear_time_matrices_match_fem_closed_form(n):
    h = 1.0 / n
    Tm = assemble.time_matrices(uniform_open_knots(n, 1), 1)
    K, M = Tm["K"], Tm["M"]
    Kref = (2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)) / h
    Mref = h / 6 * (4 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1))
    Kref[-1, -1], Mref[-1, -1] = 1 / h, h / 3  # free end at t = T
    assert np.allclose(K, Kref, atol=1e-13 / h) and np.allclose(M, Mref, atol=1e-15)


@pytest.mark.parametrize("xi,p", [c for c in CASES if c[1] >= 2])
def test_restricted_second_derivative_coupling_is_minus_stiffness(xi, p):
    S = assemble.space_matrices(xi, p)
    assert np.allclose(S["G"], -S["K"], atol=1e-12 * np.abs(S["K"]).max())


@pytest.mark.parametrize("n,p", [(4, 1), (6, 3), (5, 5)])
def test_final_time_matrix_single_unit_entry(n, p):
    W = assemble.time_matrices(uniform_open_knots(n, p), p)["W"]
    ref = np.zeros_like(W)
    ref[-1, -1] = 1.0
    assert np.array_equal(W, ref)


def _spline1d(xi, p, coef_restricted, index):
    m = bspline.num_basis(xi, p)
    c = np.zeros(m)
    c[index] = coef_restricted
    return scipy.interpolate.BSpline(xi, c, p)


@pytest.mark.parametrize("d,nel,p,kappa", [(1, 5, 2, 1.0), (1, 4, 3, 0.3), (2, 3, 3, 2.0), (2, 4, 2, 1.0)])
def test_load_of_a_discrete_solution_equals_A_times_its_coefficients(d, nel, p, kappa):
    """If u_h = prod_k a_k(x_k) c(t) lies in the discrete space and
    f = d_t u_h - kappa Lap u_h, the least-squares load F(v) = A(u_h, v)
    exactly: a consistency pin of the load assembly against A."""
    knots, degs = problem_knots(d, nel, p)
    P = system.Problem(knots, degs, kappa=kappa)
    rng = np.random.default_rng(3)
    facs = []
    for k in range(d + 1):
        m = bspline.num_basis(knots[k], degs[k])
        idx = assemble.space_index(m) if k < d else assemble.time_index(m)
        facs.append((rng.uniform(-1, 1, len(idx)), idx))
    sp = [_spline1d(knots[k], degs[k], facs[k][0], facs[k][1]) for k in range(d + 1)]
    terms = [(1.0, [sp[k] for k in range(d)], sp[d].derivative(1))]
    for k in range(d):
        gs = [sp[l].derivative(2) if l == k else sp[l] for l in range(d)]
        terms.append((-kappa, gs, sp[d]))
    F = assemble.load_separable(knots, degs, terms, kappa=kappa)
    U = facs[0][0]
    for k in range(1, d + 1):
        U = np.multiply.outer(U, facs[k][0])
    AU = P.matvec(U)
    assert np.allclose(F, AU, atol=1e-11 * np.abs(AU).max())
