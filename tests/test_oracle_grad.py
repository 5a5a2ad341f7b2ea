"""Pins of the oracle's load operator and adjoint gradients."""
import numpy as np
import pytest
import scipy.interpolate

from oracle import assemble, bspline, grad, system
from stls_inputs import problem_knots, uniform_pm1


@pytest.mark.parametrize("d,nel,p,kappa", [(1, 5, 2, 1.0), (2, 3, 3, 0.7), (2, 4, 2, 2.0)])
def test_load_of_spline_forcing_matches_quadrature_of_callables(d, nel, p, kappa):
    """For a separable spline forcing f = prod_k a_k(x_k) c(t) the load
    B_kappa f equals the quadrature load of the same callables."""
    knots, degs = problem_knots(d, nel, p)
    P = system.Problem(knots, degs, kappa=kappa)
    G = grad.Misfit(P)
    rng = np.random.default_rng(5)
    coefs = [rng.uniform(-1, 1, bspline.num_basis(knots[k], degs[k])) for k in range(d + 1)]
    spl = [scipy.interpolate.BSpline(knots[k], coefs[k], degs[k]) for k in range(d + 1)]
    F_cb = assemble.load_separable(knots, degs, [(1.0, spl[:d], spl[d])], kappa=kappa)
    f = coefs[0]
    for c in coefs[1:]:
        f = np.multiply.outer(f, c)
    F = G.load_apply(f)
    assert np.allclose(F, F_cb, atol=1e-11 * np.abs(F).max())
    # transpose is the adjoint
    lam = uniform_pm1(P.ndof, 3).reshape(P.shape, order="F")
    assert np.isclose(np.sum(lam * F), np.sum(G.load_apply_T(lam) * f), rtol=1e-12)


def _dense_setup(d, nel, p, kappa):
    knots, degs = problem_knots(d, nel, p)
    P = system.Problem(knots, degs, kappa=kappa)
    return P, grad.Misfit(P)


def _loss(d, nel, p, kappa, f, ustar):
    P, G = _dense_setup(d, nel, p, kappa)
    A = P.dense_A()
    u = np.linalg.solve(A, G.load_apply(f).ravel(order="F"))
    e = u - ustar
    return float(e @ G.mass_apply(e).ravel(order="F"))


@pytest.mark.parametrize("d,nel,p,kappa", [(1, 6, 3, 1.0), (2, 4, 3, 1.0), (2, 3, 2, 0.5)])
def test_adjoint_gradient_matches_central_differences(d, nel, p, kappa):
    """The loss is quadratic in f: central differences are exact up to
    rounding; in kappa the step is small enough for 1e-6 agreement."""
    P, G = _dense_setup(d, nel, p, kappa)
    nf = int(np.prod(G.fshape))
    f = uniform_pm1(nf, 7).reshape(G.fshape, order="F")
    ustar = 0.1 * uniform_pm1(P.ndof, 8)
    A = P.dense_A()
    solve = lambda b: np.linalg.solve(A, b)
    L, gf, dk, _ = G.loss_and_grad(f, ustar, solve)
    assert np.isclose(L, _loss(d, nel, p, kappa, f, ustar), rtol=1e-12)
    direction = uniform_pm1(nf, 9).reshape(G.fshape, order="F")
    h = 1e-3
    fd = (_loss(d, nel, p, kappa, f + h * direction, ustar) - _loss(d, nel, p, kappa, f - h * direction, ustar)) / (2 * h)
    assert np.isclose(np.sum(gf * direction), fd, rtol=1e-8)
    hk = 1e-6
    fdk = (_loss(d, nel, p, kappa + hk, f, ustar) - _loss(d, nel, p, kappa - hk, f, ustar)) / (2 * hk)
    assert np.isclose(dk, fdk, rtol=1e-6)
