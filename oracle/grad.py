"""Adjoint gradients of a space-time misfit.  Oracle: test use only.

Not in the paper: the least-squares discretisation (§3.2-3.3, §4.1) is
differentiated with respect to the forcing and the diffusivity.  Readings:
  * the forcing is a spline in the FULL tensor space (no boundary or initial
    restriction), f = sum_j f_j Bbar_j, coefficient tensor of shape
    (m_1, ..., m_d, m_t);
  * the load F_i = int int f (d_t B_i - kappa Lap B_i) (§3.2 with kappa) is
    F = B_kappa f,  B_kappa = C_t x Mbar_s - kappa Mbar_t x Dbar_s, with the
    rectangular (restricted x full) matrices Mbar = int b_i bbar_j,
    C = int b'_i bbar_j, Gbar = int b''_i bbar_j and
    Dbar_s = sum_k (Gbar_k in direction k, Mbar elsewhere);
  * the misfit is L = e^T M_Q e with e = u - u*, M_Q = M_t x M_s (squared
    L2 norm of u_h - u*_h over the space-time cylinder).
Gradients (A_kappa symmetric): g = 2 M_Q e, lambda = A_kappa^{-1} g,
  dL/df = B_kappa^T lambda,
  dL/dkappa = lambda^T (dF/dkappa - dA/dkappa u),
  dF/dkappa = -(Mbar_t x Dbar_s) f,  dA/dkappa = 2 kappa M_t x J_s + W_t x L_s.
"""
from __future__ import annotations

import numpy as np

from . import assemble
from .bspline import eval_basis_points, num_basis
from .system import kron_apply, kron_dense


def rect_matrices(xi, p, restricted_index, nq=None):
    """Mbar, C, Gbar: rows = restricted functions, columns = all functions."""
    nq = p + 1 if nq is None else nq
    x, w = assemble.gauss_points(xi, nq)
    B = eval_basis_points(xi, p, x, nder=2)
    full = B[0]
    rows = B[:, :, restricted_index]
    return dict(Mbar=rows[0].T @ (w[:, None] * full), C=rows[1].T @ (w[:, None] * full),
                Gbar=rows[2].T @ (w[:, None] * full))


class Misfit:
    """Load operator, misfit and adjoint gradient for a Problem."""

    def __init__(self, prob):
        self.prob = prob
        d = prob.d
        self.rect = []
        for k in range(d + 1):
            m = num_basis(prob.knots[k], prob.degrees[k])
            idx = assemble.space_index(m) if k < d else assemble.time_index(m)
            self.rect.append(rect_matrices(prob.knots[k], prob.degrees[k], idx))
        self.fshape = tuple(num_basis(prob.knots[k], prob.degrees[k]) for k in range(d + 1))

    def load_terms(self, kappa=None):
        kappa = self.prob.kappa if kappa is None else kappa
        d, R = self.prob.d, self.rect
        terms = [(1.0, [R[k]["Mbar"] for k in range(d)] + [R[d]["C"]])]
        for k in range(d):
            fac = [R[m]["Mbar"] for m in range(d)]
            fac[k] = R[k]["Gbar"]
            terms.append((-kappa, fac + [R[d]["Mbar"]]))
        return terms

    def load_apply(self, f, kappa=None):
        f = np.asarray(f).reshape(self.fshape, order="F")
        return sum(c * kron_apply(fac, f) for c, fac in self.load_terms(kappa))

    def load_apply_T(self, lam):
        lam = np.asarray(lam).reshape(self.prob.shape, order="F")
        return sum(c * kron_apply([W.T for W in fac], lam) for c, fac in self.load_terms())

    def dense_load(self, kappa=None):
        return sum(c * kron_dense(fac) for c, fac in self.load_terms(kappa))

    def mass_apply(self, x):
        P = self.prob
        fac = [S["M"] for S in P.space] + [P.time["M"]]
        return kron_apply(fac, np.asarray(x).reshape(P.shape, order="F"))

    def dA_dkappa_apply(self, u):
        """(2 kappa M_t x J_s + W_t x L_s) u: derivative of the kappa^2 and
        kappa terms of A_kappa (J_s expanded literally as in system_terms)."""
        P = self.prob
        kap = P.kappa
        u = np.asarray(u).reshape(P.shape, order="F")
        out = np.zeros(P.shape)
        for c, fac in P.system_terms():
            if c == 1.0 and fac[-1] is P.time["K"]:
                continue  # K_t x M_s carries no kappa
            if fac[-1] is P.time["M"]:
                out += 2.0 * kap * kron_apply(fac, u)
            else:  # W_t terms
                out += kron_apply(fac, u)
        return out

    def dF_dkappa(self, f):
        d, R = self.prob.d, self.rect
        f = np.asarray(f).reshape(self.fshape, order="F")
        out = 0.0
        for k in range(d):
            fac = [R[m]["Mbar"] for m in range(d)]
            fac[k] = R[k]["Gbar"]
            out = out - kron_apply(fac + [R[d]["Mbar"]], f)
        return out

    def loss_and_grad(self, f, ustar, solve):
        """L, dL/df (full-space tensor), dL/dkappa; ``solve(b)`` returns A^{-1} b
        (flat vectors)."""
        F = self.load_apply(f)
        u = solve(F.ravel(order="F"))
        e = u - np.asarray(ustar).ravel(order="F")
        Me = self.mass_apply(e).ravel(order="F")
        L = float(e @ Me)
        lam = solve(2.0 * Me)
        gf = self.load_apply_T(lam)
        dk = float(lam @ (self.dF_dkappa(f).ravel(order="F") - self.dA_dkappa_apply(u).ravel(order="F")))
        return L, gf, dk, u
