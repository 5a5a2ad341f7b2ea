"""B-spline basis by the Cox-de Boor recursion (§2.1).  Oracle: test use only.

Indices are 0-based: a knot vector xi[0..m+p] of an open knot vector on
[0, 1] carries m basis functions b_0..b_{m-1} of degree p.
"""
from __future__ import annotations

import numpy as np


def _safe_div(num, den):
    """num / den with the paper's convention 0/0 = 0 (a zero-length span)."""
    return 0.0 if den == 0.0 else num / den


def num_basis(xi, p):
    """m = len(xi) - p - 1 (the knot vector has m + p + 1 entries, §2.1)."""
    return len(xi) - p - 1


def _last_nonempty_span(xi):
    """Index s of the last span [xi_s, xi_{s+1}) with positive length."""
    for s in range(len(xi) - 2, -1, -1):
        if xi[s + 1] > xi[s]:
            return s
    raise ValueError("knot vector has no non-empty span")


def basis_degree0(xi, eta):
    """Degree-0 functions at one point eta: indicator of [xi_i, xi_{i+1}).

    §2.1 uses half-open spans, so every function would vanish at eta = 1.
    Reading adopted: the last non-empty span is closed on the right, so the
    basis is a partition of unity on the closed interval [0, 1].
    """
    n0 = len(xi) - 1
    b = np.zeros(n0)
    for i in range(n0):
        if xi[i] <= eta < xi[i + 1]:
            b[i] = 1.0
    if eta == xi[-1]:
        b[_last_nonempty_span(xi)] = 1.0
    return b


def basis_all_degrees(xi, p, eta):
    """Table B[q][i] = b_{i,q}(eta) for q = 0..p by the recursion of §2.1.

    b_{i,q} = (eta - xi_i)/(xi_{i+q} - xi_i) b_{i,q-1}
            + (xi_{i+q+1} - eta)/(xi_{i+q+1} - xi_{i+1}) b_{i+1,q-1}, 0/0 = 0.
    """
    tables = [basis_degree0(xi, eta)]
    for q in range(1, p + 1):
        prev = tables[-1]
        cur = np.zeros(len(xi) - q - 1)
        for i in range(len(cur)):
            left = _safe_div(eta - xi[i], xi[i + q] - xi[i]) * prev[i]
            right = _safe_div(xi[i + q + 1] - eta, xi[i + q + 1] - xi[i + 1]) * prev[i + 1]
            cur[i] = left + right
        tables.append(cur)
    return tables


def derivative_coeffs(xi, q, lower):
    """Derivative of degree-q functions from degree-(q-1) values.

    Differentiating the recursion gives the standard identity
      b'_{i,q} = q/(xi_{i+q} - xi_i) b_{i,q-1} - q/(xi_{i+q+1} - xi_{i+1}) b_{i+1,q-1}
    (0/0 = 0); ``lower`` holds the degree-(q-1) values (or derivatives).
    """
    out = np.zeros(len(xi) - q - 1)
    for i in range(len(out)):
        out[i] = (q * _safe_div(lower[i], xi[i + q] - xi[i])
                  - q * _safe_div(lower[i + 1], xi[i + q + 1] - xi[i + 1]))
    return out


def eval_basis(xi, p, eta, nder=2):
    """Values and derivatives 0..nder of all m functions of degree p at eta.

    Returns an array of shape (nder + 1, m).  The k-th derivative of the
    degree-p functions is obtained by applying the derivative identity k
    times to the degree-(p-k) table.
    """
    tables = basis_all_degrees(xi, p, eta)
    m = num_basis(xi, p)
    out = np.zeros((nder + 1, m))
    out[0] = tables[p]
    for k in range(1, nder + 1):
        if k > p:
            continue  # a degree-p polynomial piece has zero (p+1)-th derivative
        cur = tables[p - k]
        for q in range(p - k + 1, p + 1):
            cur = derivative_coeffs(xi, q, cur)
        out[k] = cur
    return out


def eval_basis_points(xi, p, etas, nder=2):
    """eval_basis at many points: array of shape (nder + 1, len(etas), m)."""
    etas = np.asarray(etas, dtype=np.float64)
    res = np.zeros((nder + 1, len(etas), num_basis(xi, p)))
    for a, eta in enumerate(etas):
        res[:, a, :] = eval_basis(xi, p, float(eta), nder)
    return res


def nonempty_spans(xi):
    """List of (left, right) of the non-empty knot spans."""
    return [(xi[s], xi[s + 1]) for s in range(len(xi) - 1) if xi[s + 1] > xi[s]]


def greville(xi, p):
    """Greville abscissae: average of p consecutive interior knots.

    The spline with these coefficients reproduces the identity x -> x,
    used as a pin of the assembled matrices (linear reproduction).
    """
    m = num_basis(xi, p)
    return np.array([np.mean(xi[i + 1:i + p + 1]) for i in range(m)])
