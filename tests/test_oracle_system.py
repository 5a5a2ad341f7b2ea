"""Pins of the oracle's system matrix, preconditioner, FD and PCG (§4-§5)."""
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import assemble, bspline, fd, pcg, system, norms
from stls_inputs import problem_knots, uniform_pm1

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tensor_basis(knots, degs, nq_extra=1):
    """Basis values/derivatives on a tensor Gauss grid (restricted indices)."""
    d = len(knots) - 1
    out = []
    for k in range(d + 1):
        x, w = assemble.gauss_points(knots[k], degs[k] + nq_extra)
        B = bspline.eval_basis_points(knots[k], degs[k], x, nder=2)
        m = bspline.num_basis(knots[k], degs[k])
        idx = assemble.space_index(m) if k < d else assemble.time_index(m)
        out.append((w, B[:, :, idx]))
    return out


def _bruteforce_A(knots, degs, kappa, with_cross_terms):
    """A by quadrature of the bilinear form on the (d+1)-D grid.

    with_cross_terms=True: the definition int int (v_t - k Lap v)(w_t - k Lap w)
    (eq. a-form with kappa); False: the equivalent form with the final-time
    gradient term (eq. equivalent_A with kappa)."""
    d = len(knots) - 1
    tb = _tensor_basis(knots, degs)
    W = tb[0][0]
    for w, _ in tb[1:]:
        W = np.multiply.outer(W, w)
    Wf = W.ravel(order="F")

    def field(ders):
        # columns: basis functions (colex), rows: grid points (colex)
        mats = [tb[k][1][ders[k]] for k in range(d + 1)]
        out = mats[0]
        for Mk in mats[1:]:
            out = np.kron(Mk, out)
        return out

    Bt = field([0] * d + [1])
    Lap = sum(field([2 if l == k else 0 for l in range(d)] + [0]) for k in range(d))
    if with_cross_terms:
        R = Bt - kappa * Lap
        return R.T @ (Wf[:, None] * R)
    A = Bt.T @ (Wf[:, None] * Bt) + kappa ** 2 * Lap.T @ (Wf[:, None] * Lap)
    # final time term: kappa int grad v(T) . grad w(T)
    end = bspline.eval_basis(knots[d], degs[d], 1.0, nder=0)[0][assemble.time_index(bspline.num_basis(knots[d], degs[d]))]
    sp = [tb[k] for k in range(d)]
    Ws = sp[0][0]
    for w, _ in sp[1:]:
        Ws = np.multiply.outer(Ws, w)
    Wsf = np.atleast_1d(Ws).ravel(order="F")
    grad = 0
    for k in range(d):
        mats = [sp[l][1][1 if l == k else 0] for l in range(d)]
        G = mats[0]
        for Mk in mats[1:]:
            G = np.kron(Mk, G)
        grad = grad + G.T @ (Wsf[:, None] * G)
    return A + kappa * np.kron(np.outer(end, end), grad)


@pytest.mark.parametrize("d,nel,p,kappa", [(1, 4, 2, 1.0), (1, 3, 4, 0.5), (2, 2, 3, 1.0), (2, 3, 2, 3.0)])
def test_kronecker_sum_equals_bilinear_form(d, nel, p, kappa):
    knots, degs = problem_knots(d, nel, p)
    A = system.Problem(knots, degs, kappa=kappa).dense_A()
    A1 = _bruteforce_A(knots, degs, kappa, with_cross_terms=True)
    A2 = _bruteforce_A(knots, degs, kappa, with_cross_terms=False)
    s = np.abs(A).max()
    assert np.allclose(A, A1, atol=1e-11 * s) and np.allclose(A, A2, atol=1e-11 * s)
    assert np.allclose(A, A.T, atol=1e-13 * s)
    assert np.linalg.eigvalsh(A).min() > 0


@pytest.mark.parametrize("d,nel,p", [(1, 5, 3), (2, 3, 2), (3, 2, 2)])
def test_mode_chain_equals_explicit_kronecker(d, nel, p):
    knots, degs = problem_knots(d, nel, p)
    P = system.Problem(knots, degs, kappa=0.7)
    x = uniform_pm1(P.ndof, 1)
    assert np.allclose(system.vec(P.matvec(x)), P.dense_A() @ x, rtol=0, atol=1e-11 * np.abs(P.dense_A()).max())
    assert np.allclose(system.vec(P.prec_matvec(x)), P.dense_P() @ x, rtol=0, atol=1e-11 * np.abs(P.dense_P()).max())


@pytest.mark.parametrize("nel,p", [(6, 2), (8, 3), (10, 5)])
def test_eigendecomposition_normalisation_and_limits(nel, p):
    knots, degs = problem_knots(1, nel, p)
    P = system.Problem(knots, degs)
    F = fd.FD(P)
    (ls, Us), (lt, Ut) = F.eig_space[0], F.eig_time
    S, Tm = P.space[0], P.time
    assert np.allclose(Us.T @ S["M"] @ Us, np.eye(len(ls)), atol=1e-12)
    assert np.allclose(Us.T @ S["J"] @ Us, np.diag(ls), atol=1e-9 * ls.max())
    assert np.allclose(Ut.T @ Tm["Mhat"] @ Ut, np.eye(len(lt)), atol=1e-12)
    assert np.allclose(Ut.T @ Tm["Khat"] @ Ut, np.diag(lt), atol=1e-10 * lt.max())
    # smallest eigenvalues approach (k pi)^4 (space, Dirichlet) and ((k-1/2) pi)^2 (time)
    err_s, err_t = abs(ls[0] / np.pi ** 4 - 1), abs(lt[0] / (np.pi ** 2 / 4) - 1)
    assert err_s < 0.03 and err_t < 0.03
    # the discrete eigenvalues converge to the continuous ones under refinement
    knots2, degs2 = problem_knots(1, 2 * nel, p)
    F2 = fd.FD(system.Problem(knots2, degs2))
    assert abs(F2.eig_space[0][0][0] / np.pi ** 4 - 1) <= max(err_s / 2, 1e-8)
    assert abs(F2.eig_time[0][0] / (np.pi ** 2 / 4) - 1) <= max(err_t / 2, 1e-8)


@pytest.mark.parametrize("d,nel,p,kappa", [(1, 6, 3, 1.0), (2, 3, 2, 0.1), (2, 3, 3, 10.0), (3, 2, 2, 1.0)])
def test_fd_apply_equals_dense_preconditioner_solve(d, nel, p, kappa):
    knots, degs = problem_knots(d, nel, p)
    P = system.Problem(knots, degs, kappa=kappa)
    r = uniform_pm1(P.ndof, 2)
    s_fd = system.vec(fd.FD(P).apply(r))
    s_ref = np.linalg.solve(P.dense_P(), r)
    assert np.linalg.norm(s_fd - s_ref) <= 1e-12 * np.linalg.norm(s_ref)


@pytest.mark.parametrize("d,nel,p,kappa", [(1, 5, 2, 1.0), (1, 6, 4, 1.0), (2, 3, 3, 1.0), (2, 3, 2, 0.1), (2, 3, 2, 10.0)])
def test_spectral_bounds_of_preconditioned_system(d, nel, p, kappa):
    """On the unit box A - P = kappa^2 M_t x (cross terms) + kappa W_t x L_s is
    PSD, so lambda_min(P^-1 A) >= 1; continuity (factor 2) and the norm
    equivalence with factor d (§4.2.1) give lambda_max <= 2 d."""
    knots, degs = problem_knots(d, nel, p)
    P = system.Problem(knots, degs, kappa=kappa)
    ev = scipy.linalg.eigh(P.dense_A(), P.dense_P(), eigvals_only=True)
    assert ev.min() >= 1 - 1e-10 and ev.max() <= 2 * d + 1e-10


@pytest.mark.parametrize("d,nel,p,kappa", [(1, 6, 3, 1.0), (2, 3, 3, 1.0), (2, 4, 2, 2.5)])
def test_pcg_matches_dense_cholesky(d, nel, p, kappa):
    knots, degs = problem_knots(d, nel, p)
    P = system.Problem(knots, degs, kappa=kappa)
    b = uniform_pm1(P.ndof, 4)
    A = P.dense_A()
    x_ref = scipy.linalg.cho_solve(scipy.linalg.cho_factor(A), b)
    F = fd.FD(P)
    x, info = pcg.pcg(lambda v: system.vec(P.matvec(v)), lambda v: system.vec(F.apply(v)), b, rtol=1e-12)
    assert info["converged"] and info["true_relres"] < 1e-11
    cond = np.linalg.cond(A)
    assert np.linalg.norm(x - x_ref) <= 1e-12 * cond * np.linalg.norm(x_ref)
    lo, hi = pcg.lanczos_extremes(info["alphas"], info["betas"])
    assert lo >= 1 - 1e-6 and hi <= 2 * d + 1e-6


def _table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1_iterations.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(tuple(int(v) for v in line.split()))
    return rows


@pytest.mark.parametrize("nsub,p,its", [r for r in _table1() if r[0] <= 16])
def test_table1_iteration_counts(nsub, p, its):
    pi = np.pi
    s = lambda x: np.sin(pi * x)
    knots, degs = problem_knots(3, nsub, p)
    P = system.Problem(knots, degs)
    F = assemble.load_separable(knots, degs, [(1.0, [s, s, s], np.cos), (3 * pi * pi, [s, s, s], np.sin)])
    f = fd.FD(P)
    _, info = pcg.pcg(lambda v: system.vec(P.matvec(v)), lambda v: system.vec(f.apply(v)), system.vec(F), 1e-8)
    assert info["iters"] == its


def test_convergence_rates_of_least_squares_solution():
    """Manufactured u = sin(pi x) sin(pi t), d = 1: V_0 error O(h^{p-1})
    (a-priori estimate, §3.3), H^1 O(h^p), L^2 O(h^{p+1}) for p >= 3 and
    O(h^2) at p = 2 (§5.1)."""
    pi = np.pi
    ex = dict(u=lambda x, t: np.sin(pi * x) * np.sin(pi * t), ut=lambda x, t: pi * np.sin(pi * x) * np.cos(pi * t),
              lap=lambda x, t: -pi * pi * np.sin(pi * x) * np.sin(pi * t),
              grad=[lambda x, t: pi * np.cos(pi * x) * np.sin(pi * t)])
    s = lambda x: np.sin(pi * x)
    for p in (2, 3, 4):
        errs = []
        for nel in (8, 16):
            knots, degs = problem_knots(1, nel, p)
            P = system.Problem(knots, degs)
            F = assemble.load_separable(knots, degs, [(pi, [s], lambda t: np.cos(pi * t)), (pi * pi, [s], lambda t: np.sin(pi * t))])
            u = np.linalg.solve(P.dense_A(), system.vec(F))
            errs.append(norms.error_norms(system.unvec(u, P.shape), knots, degs, ex))
        rate = {k: np.log2(errs[0][k] / errs[1][k]) for k in errs[0]}
        assert abs(rate["V0"] - (p - 1)) < 0.25
        assert abs(rate["H1"] - p) < 0.25
        assert abs(rate["L2"] - (p + 1 if p >= 3 else 2)) < 0.35
