"""Error norms of a discrete space-time solution (§3.1 eq. norm_V0, §5.1).
Oracle: test use only.

u_h = sum_i u_i B_i is evaluated on a tensor grid of Gauss points with
p + 3 points per span (the paper uses element-wise Gauss quadrature without
stating the count) and compared with an exact solution given by callables.

``error_integrals`` returns the unnormalised space-time integrals of the
error e = u - u_h and of the exact solution, term by term; ``error_norms``
composes them into the relative V_0, L^2 and H^1 errors.  Both are pinned
by closed-form integrals of polynomial splines against trigonometric
solutions (tests/test_oracle_norms.py).
"""
from __future__ import annotations

import numpy as np

from .assemble import gauss_points, space_index, time_index
from .bspline import eval_basis_points, num_basis
from .system import mode_product


def _grid(knots, degrees, full_time=False, full_space=False):
    d = len(knots) - 1
    pts, wts, mats = [], [], []
    for k in range(d + 1):
        x, w = gauss_points(knots[k], degrees[k] + 3)
        B = eval_basis_points(knots[k], degrees[k], x, nder=2)
        m = num_basis(knots[k], degrees[k])
        if k < d:
            idx = np.arange(m) if full_space else space_index(m)
        else:
            idx = np.arange(m) if full_time else time_index(m)
        pts.append(x)
        wts.append(w)
        mats.append(B[:, :, idx])  # (3, nq, n)
    return pts, wts, mats


def _eval(coef, mats, ders):
    X = coef
    for m, B in enumerate(mats):
        X = mode_product(X, B[ders[m]], m)
    return X


def error_integrals(coef, knots, degrees, exact, full_time=False, full_space=False):
    """Space-time integrals of e = u - u_h and of u, unnormalised.

    ``coef`` is indexed by the restricted spaces; with ``full_time`` by every
    time function (the first one carries non-zero initial data), with
    ``full_space`` by every spatial function (boundary data).

    ``exact`` is a dict of callables on meshgrid arrays (x_1, .., x_d, t):
    'u', 'ut' (time derivative), 'lap' (spatial Laplacian) and 'grad'
    (list of spatial first derivatives).

    Returns two dicts, (err, ref), each with the keys
      'val'  int int v^2,          'dt'  int int (d_t v)^2,
      'lap'  int int (Lap v)^2,    'grad' int int |grad_x v|^2,
    for v = e (err) and v = u (ref).
    """
    d = len(knots) - 1
    pts, wts, mats = _grid(knots, degrees, full_time, full_space)
    G = np.meshgrid(*pts, indexing="ij")
    W = wts[0]
    for w in wts[1:]:
        W = np.multiply.outer(W, w)
    zero = [0] * (d + 1)
    uh = _eval(coef, mats, zero)
    uth = _eval(coef, mats, zero[:d] + [1])
    laph = sum(_eval(coef, mats, [2 if l == k else 0 for l in range(d)] + [0]) for k in range(d))
    gradh = [_eval(coef, mats, [1 if l == k else 0 for l in range(d)] + [0]) for k in range(d)]
    u, ut, lap = exact["u"](*G), exact["ut"](*G), exact["lap"](*G)
    grad = [g(*G) for g in exact["grad"]]

    def integ(f):
        return float(np.sum(W * f))

    err = dict(val=integ((u - uh) ** 2), dt=integ((ut - uth) ** 2), lap=integ((lap - laph) ** 2),
               grad=sum(integ((g - gh) ** 2) for g, gh in zip(grad, gradh)))
    ref = dict(val=integ(u ** 2), dt=integ(ut ** 2), lap=integ(lap ** 2), grad=sum(integ(g ** 2) for g in grad))
    return err, ref


def compose_norms(err, ref):
    """Relative errors from the integrals of ``error_integrals``:
    V_0 (||v||^2 = int int (d_t v)^2 + (Lap v)^2, eq. norm_V0), L^2 and the
    space-time H^1 norm (||v||^2 = int int v^2 + (d_t v)^2 + |grad_x v|^2)."""
    def v0(a):
        return a["dt"] + a["lap"]

    def h1(a):
        return a["val"] + a["dt"] + a["grad"]

    return dict(V0=np.sqrt(v0(err) / v0(ref)), L2=np.sqrt(err["val"] / ref["val"]), H1=np.sqrt(h1(err) / h1(ref)))


def error_norms(coef, knots, degrees, exact, kappa=1.0, full_time=False, full_space=False):
    """Relative errors of u_h against ``exact`` in the V_0, L^2 and H^1
    norms (arguments as in ``error_integrals``; ``kappa`` is accepted for
    call compatibility and does not enter the norms)."""
    err, ref = error_integrals(coef, knots, degrees, exact, full_time, full_space)
    return compose_norms(err, ref)
