"""Pins of the oracle's error norms (§3.1 eq. norm_V0, §5.1) by closed forms.

The discrete function is u_h = prod_k q(x_k) * t with q(x) = x (1 - x): a
polynomial that lies in every restricted spline space of space degree >= 2
and time degree >= 1 (it vanishes on the spatial boundary and at t = 0).
Its B-spline coefficients come from the blossoming (Marsden) identity, not
from the oracle: for a degree-p spline with knots xi, the coefficient of
B_i is the blossom of the polynomial at xi_{i+1}, ..., xi_{i+p}; for x that
is the knot average, for x^2 the average of the pairwise knot products.

The exact solution is u = prod_k sin(pi x_k) * sin(pi t).  Every integral
of e = u - u_h and of u over (0,1)^d x (0,1) then factors into 1-D
integrals with closed forms, e.g. int_0^1 x (1-x) sin(pi x) dx = 4/pi^3.
Non-uniform knots with repeated interior knots are used on purpose.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import norms

PI = math.pi


def _blossom_coeffs(xi, p, which):
    """Coefficients of x (which = 1) or x^2 (which = 2) in the degree-p
    B-spline basis of the knot vector xi (all m = len(xi) - p - 1 functions)."""
    m = len(xi) - p - 1
    out = np.empty(m)
    for i in range(m):
        t = xi[i + 1:i + p + 1]
        if which == 1:
            out[i] = sum(t) / p
        else:
            pairs = list(itertools.combinations(t, 2))
            out[i] = sum(a * b for a, b in pairs) / len(pairs)
    return out


def _q_coeffs_restricted(xi, p):
    c = _blossom_coeffs(xi, p, 1) - _blossom_coeffs(xi, p, 2)
    assert abs(c[0]) < 1e-15 and abs(c[-1]) < 1e-15  # q vanishes at 0 and 1
    return c[1:-1]


def _t_coeffs_restricted(xi, p):
    c = _blossom_coeffs(xi, p, 1)
    assert abs(c[0]) < 1e-15  # t vanishes at t = 0
    return c[1:]


SPACE_KNOTS = [
    (np.array([0, 0, 0, 0, 0.2, 0.35, 0.35, 0.6, 0.9, 1, 1, 1, 1.0]), 3),
    (np.array([0, 0, 0, 0.15, 0.4, 0.55, 0.7, 1, 1, 1.0]), 2),
]
TIME_KNOTS = (np.array([0, 0, 0, 0.3, 0.5, 0.5, 0.8, 1, 1, 1.0]), 2)


def _case(d):
    knots = [SPACE_KNOTS[k][0] for k in range(d)] + [TIME_KNOTS[0]]
    degs = [SPACE_KNOTS[k][1] for k in range(d)] + [TIME_KNOTS[1]]
    coef = _t_coeffs_restricted(*TIME_KNOTS)
    for k in reversed(range(d)):
        coef = np.multiply.outer(coef, _q_coeffs_restricted(*SPACE_KNOTS[k]))
    coef = np.transpose(coef, list(reversed(range(d + 1))))  # (n_1, .., n_d, n_t)

    def prod_sin(X):
        out = 1.0
        for x in X:
            out = out * np.sin(PI * x)
        return out

    def u(*G):
        return prod_sin(G[:d]) * np.sin(PI * G[d])

    def ut(*G):
        return prod_sin(G[:d]) * PI * np.cos(PI * G[d])

    def lap(*G):
        return -d * PI * PI * u(*G)

    def grad_k(k):
        def g(*G):
            return PI * np.cos(PI * G[k]) * prod_sin([G[l] for l in range(d) if l != k]) * np.sin(PI * G[d])
        return g

    exact = dict(u=u, ut=ut, lap=lap, grad=[grad_k(k) for k in range(d)])
    return knots, degs, coef, exact


def _closed_forms(d):
    """(err, ref) integrals for e = u - u_h, u as in the module docstring."""
    ss = 0.5              # int sin^2(pi x)
    sq = 4 / PI ** 3      # int sin(pi x) q
    qq = 1 / 30           # int q^2
    q1q1 = 1 / 3          # int q'^2
    q2q2 = 4.0            # int q''^2
    qq2 = -1 / 3          # int q q''
    sq2 = -4 / PI         # int sin(pi x) q''
    cq1 = 4 / PI          # int pi cos(pi x) q'
    st = 1 / PI           # int sin(pi t) t
    tt = 1 / 3            # int t^2
    ct = 0.0              # int pi cos(pi t) * 1
    cc = PI * PI / 2      # int (pi cos(pi t))^2
    ref = dict(val=ss ** (d + 1), dt=ss ** d * cc, lap=(d * PI * PI) ** 2 * ss ** (d + 1),
               grad=d * (PI * PI / 2) * ss ** (d - 1) * ss)
    uh_val = qq ** d * tt
    uh_dt = qq ** d * 1.0
    uh_lap = (d * q2q2 * qq ** (d - 1) + d * (d - 1) * qq2 ** 2 * qq ** max(d - 2, 0)) * tt
    uh_grad = d * q1q1 * qq ** (d - 1) * tt
    x_val = sq ** d * st
    x_dt = sq ** d * ct
    x_lap = (-d * PI * PI) * d * sq2 * sq ** (d - 1) * st
    x_grad = d * cq1 * sq ** (d - 1) * st
    err = dict(val=ref["val"] - 2 * x_val + uh_val, dt=ref["dt"] - 2 * x_dt + uh_dt,
               lap=ref["lap"] - 2 * x_lap + uh_lap, grad=ref["grad"] - 2 * x_grad + uh_grad)
    return err, ref


@pytest.mark.parametrize("d", [1, 2])
def test_error_integrals_match_closed_forms(d):
    knots, degs, coef, exact = _case(d)
    err, ref = norms.error_integrals(coef, knots, degs, exact)
    cerr, cref = _closed_forms(d)
    for key in ("val", "dt", "lap", "grad"):
        # Gauss quadrature (p + 3 points per span) of the sine factors on
        # spans up to 0.3 wide: relative error ~5e-11
        assert abs(ref[key] - cref[key]) <= 1e-9 * cref[key], (key, ref[key], cref[key])
        assert abs(err[key] - cerr[key]) <= 1e-9 * cref[key], (key, err[key], cerr[key])
    # the four error integrals differ from each other and from the reference
    assert len({round(v, 6) for v in cerr.values()}) == 4


@pytest.mark.parametrize("d", [1, 2])
def test_relative_norms_match_closed_forms(d):
    knots, degs, coef, exact = _case(d)
    got = norms.error_norms(coef, knots, degs, exact)
    e, r = _closed_forms(d)
    want = dict(V0=math.sqrt((e["dt"] + e["lap"]) / (r["dt"] + r["lap"])),
                L2=math.sqrt(e["val"] / r["val"]),
                H1=math.sqrt((e["val"] + e["dt"] + e["grad"]) / (r["val"] + r["dt"] + r["grad"])))
    for key, v in want.items():
        assert abs(got[key] - v) <= 1e-9 * v, (key, got[key], v)


@pytest.mark.parametrize("d", [1, 2])
def test_exact_discrete_solution_has_zero_error(d):
    """u = u_h exactly (the polynomial itself as the exact solution)."""
    knots, degs, coef, _ = _case(d)

    def qprod(X):
        out = 1.0
        for x in X:
            out = out * x * (1 - x)
        return out

    def lap(*G):
        tot = 0.0
        for k in range(d):
            tot = tot - 2 * qprod([G[l] for l in range(d) if l != k]) * G[d]
        return tot

    def gk(k):
        return lambda *G: (1 - 2 * G[k]) * qprod([G[l] for l in range(d) if l != k]) * G[d]

    exact = dict(u=lambda *G: qprod(G[:d]) * G[d], ut=lambda *G: qprod(G[:d]) + 0 * G[d], lap=lap,
                 grad=[gk(k) for k in range(d)])
    err, ref = norms.error_integrals(coef, knots, degs, exact)
    for key in ("val", "dt", "lap", "grad"):
        assert err[key] <= 1e-24, (key, err[key])
    assert abs(ref["val"] - (1 / 30) ** d / 3) < 1e-14


def test_zero_coefficients_give_the_solution_integrals():
    knots, degs, coef, exact = _case(1)
    err, ref = norms.error_integrals(0 * coef, knots, degs, exact)
    assert err == ref
    assert norms.error_norms(0 * coef, knots, degs, exact) == dict(V0=1.0, L2=1.0, H1=1.0)
