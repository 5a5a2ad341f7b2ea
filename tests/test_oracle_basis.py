"""Pins of the oracle's B-spline basis (§2.1) and quadrature."""
import numpy as np
import pytest
import scipy.interpolate

from oracle import bspline, assemble
from stls_inputs import uniform_open_knots

KNOTS = [
    (uniform_open_knots(5, 2), 2),
    (uniform_open_knots(7, 3), 3),
    (uniform_open_knots(4, 5), 5),
    (uniform_open_knots(6, 1), 1),
    # non-uniform with a double interior knot (C^{p-2} there)
    (np.array([0, 0, 0, 0, 0.15, 0.4, 0.4, 0.7, 1, 1, 1, 1.0]), 3),
]


@pytest.mark.parametrize("xi,p", KNOTS)
def test_partition_of_unity_closed_interval(xi, p):
    pts = np.concatenate([[0.0, 1.0], np.linspace(0, 1, 37), np.unique(xi)])
    B = bspline.eval_basis_points(xi, p, pts, nder=0)[0]
    assert np.allclose(B.sum(axis=1), 1.0, atol=1e-14, rtol=0)
    assert (B >= -1e-15).all()
    # only the last function is nonzero at the right end (closed last span)
    last = bspline.eval_basis(xi, p, 1.0, nder=0)[0]
    assert last[-1] == 1.0 and np.all(last[:-1] == 0.0)


@pytest.mark.parametrize("xi,p", KNOTS)
def test_values_and_derivatives_match_scipy(xi, p):
    m = bspline.num_basis(xi, p)
    rng = np.random.default_rng(0)
    pts = rng.uniform(0, 1, 25)
    ours = bspline.eval_basis_points(xi, p, pts, nder=2)
    for i in range(m):
        c = np.zeros(m)
        c[i] = 1.0
        spl = scipy.interpolate.BSpline(xi, c, p, extrapolate=False)
        for k in range(min(2, p) + 1):
            ref = spl.derivative(k)(pts) if k else spl(pts)
            assert np.allclose(ours[k, :, i], ref, atol=1e-10 * (1 + np.abs(ref).max()), rtol=1e-12)


@pytest.mark.parametrize("xi,p", KNOTS)
def test_greville_linear_reproduction(xi, p):
    g = bspline.greville(xi, p)
    pts = np.linspace(0, 1, 23)
    B = bspline.eval_basis_points(xi, p, pts, nder=1)
    assert np.allclose(B[0] @ g, pts, atol=1e-14)
    assert np.allclose(B[1] @ g, 1.0, atol=1e-12)


@pytest.mark.parametrize("nq", [1, 2, 4, 6])
def test_gauss_points_exact_on_monomials(nq):
    xi = uniform_open_knots(3, 2)
    x, w = assemble.gauss_points(xi, nq)
    for k in range(2 * nq):
        assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-14
