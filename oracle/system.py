"""Kronecker-sum system matrix and preconditioner matrix (§4, §4.1-4.2). Oracle.

Tensors have shape (n_1, ..., n_d, n_t) and vec(X) = X.ravel(order="F"),
the colexicographic ordering of §2.2 / eq. kron_vec_multi (first space
index fastest, time slowest).  A Kronecker product W_{d+1} x ... x W_1 acts
on vec(X) as the chain of m-mode products X x_1 W_1 ... x_{d+1} W_{d+1}
(eq. kron_vec_multi), which is how every operator here is applied.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from functools import reduce

import numpy as np

from . import assemble
from .bspline import num_basis


def mode_product(X, W, m):
    """m-mode product (X x_m W)[.., i_m, ..] = sum_j X[.., j, ..] W[i_m, j] (§4)."""
    Y = np.tensordot(W, X, axes=([1], [m]))
    return np.moveaxis(Y, 0, m)


def kron_apply(factors, X):
    """(W_{d+1} x ... x W_1) vec(X) via eq. kron_vec_multi; factors[m] = W_{m+1}."""
    for m, W in enumerate(factors):
        X = mode_product(X, W, m)
    return X


def kron_dense(factors):
    """Explicit W_{d+1} x ... x W_1 (np.kron puts its first argument slowest)."""
    return reduce(np.kron, list(reversed(factors)))


@dataclass
class Problem:
    """Discrete heat problem on the unit box (0,1)^d x (0,T).

    knots/degrees: d + 1 entries, time last.  kappa scales the Laplacian in
    d_t u - kappa Lap u = f; kappa = 1 is the paper's model problem
    (eq. heat_eq).  With kappa the least-squares form reads
      A_kappa = K_t x M_s + kappa^2 M_t x J_s + kappa W_t x L_s,
    because the cross terms of the expanded square integrate to the final-
    time gradient term scaled by kappa (Lemma of §4.1).
    """
    knots: list
    degrees: list
    kappa: float = 1.0
    T: float = 1.0
    space: list = field(init=False)
    time: dict = field(init=False)
    shape: tuple = field(init=False)

    def __post_init__(self):
        self.d = len(self.knots) - 1
        self.space = [assemble.space_matrices(self.knots[k], self.degrees[k]) for k in range(self.d)]
        self.time = assemble.time_matrices(self.knots[self.d], self.degrees[self.d], self.T)
        self.shape = tuple([S["M"].shape[0] for S in self.space] + [self.time["M"].shape[0]])
        self.full_shape = tuple(num_basis(self.knots[k], self.degrees[k]) for k in range(self.d + 1))

    @property
    def ndof(self):
        return int(np.prod(self.shape))

    # --- Kronecker terms ------------------------------------------------
    def system_terms(self):
        """(coefficient, factors) of A_kappa (eq. A_kron with kappa).

        J_s = int Lap B_i Lap B_j is expanded literally as
        sum_{k,l} int d_kk B_i d_ll B_j: the k = l terms carry J_k, the
        k != l terms carry G_k in direction k and G_l^T in direction l
        (G = int b'' b), and M elsewhere.  L_s = sum_k (K_k, M elsewhere).
        """
        d, S, Tm, kap = self.d, self.space, self.time, self.kappa
        terms = [(1.0, [S[k]["M"] for k in range(d)] + [Tm["K"]])]
        for k in range(d):
            for l in range(d):
                fac = [S[m]["M"] for m in range(d)]
                if k == l:
                    fac[k] = S[k]["J"]
                else:
                    fac[k] = S[k]["G"]
                    fac[l] = S[l]["G"].T
                terms.append((kap * kap, fac + [Tm["M"]]))
        for k in range(d):
            fac = [S[m]["M"] for m in range(d)]
            fac[k] = S[k]["K"]
            terms.append((kap, fac + [Tm["W"]]))
        return terms

    def prec_terms(self):
        """(coefficient, factors) of P_kappa = K_t x M_s + kappa^2 M_t x J~_s
        with J~_s = sum_k (J_k, M elsewhere) (eq. preconditioner, §4.2),
        built from the parametric (hatted) time matrices."""
        d, S, Tm, kap = self.d, self.space, self.time, self.kappa
        terms = [(1.0, [S[k]["M"] for k in range(d)] + [Tm["Khat"]])]
        for k in range(d):
            fac = [S[m]["M"] for m in range(d)]
            fac[k] = S[k]["J"]
            terms.append((kap * kap, fac + [Tm["Mhat"]]))
        return terms

    def kron_diagonal(self, terms):
        """Diagonal of sum_c c (W_{d+1} x ... x W_1) as a tensor of self.shape.

        The diagonal of a Kronecker product is the Kronecker product of the
        factors' diagonals, so each term contributes c times the outer product
        of diag(W_m) over the modes m."""
        D = np.zeros(self.shape)
        for c, facs in terms:
            t = np.ones(self.shape)
            for m, W in enumerate(facs):
                sh = [1] * (self.d + 1)
                sh[m] = W.shape[0]
                t = t * np.diag(W).reshape(sh)
            D = D + c * t
        return D

    # --- operators ------------------------------------------------------
    def matvec(self, X):
        """A_kappa vec(X) as a sum of mode-product chains (tensor in, tensor out)."""
        X = np.asarray(X).reshape(self.shape, order="F")
        return sum(c * kron_apply(f, X) for c, f in self.system_terms())

    def prec_matvec(self, X):
        """P_kappa vec(X) (tensor in, tensor out)."""
        X = np.asarray(X).reshape(self.shape, order="F")
        return sum(c * kron_apply(f, X) for c, f in self.prec_terms())

    def dense_A(self):
        """Explicit A_kappa (tiny sizes only)."""
        return sum(c * kron_dense(f) for c, f in self.system_terms())

    def dense_P(self):
        """Explicit P_kappa (tiny sizes only)."""
        return sum(c * kron_dense(f) for c, f in self.prec_terms())


def vec(X):
    """Colexicographic vectorisation (§4)."""
    return np.asarray(X).ravel(order="F")


def unvec(v, shape):
    return np.asarray(v).reshape(shape, order="F")
