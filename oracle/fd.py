"""Fast diagonalization (FD) application of the preconditioner (§4.3,
Algorithm 1, eq. eig_dec).  Oracle: test use only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .system import mode_product


def eig_pencil(Kmat, Mmat):
    """Generalized eigendecomposition Kmat U = Mmat U Lambda with U^T Mmat U = I
    (eq. eig_dec).  The library routine (LAPACK through scipy) is one step."""
    lam, U = scipy.linalg.eigh(Kmat, Mmat)
    return lam, U


class FD:
    """Step 1 of Algorithm 1 at construction, steps 2-4 in ``apply``."""

    def __init__(self, prob):
        self.prob = prob
        self.d = prob.d
        self.eig_space = [eig_pencil(S["J"], S["M"]) for S in prob.space]
        self.eig_time = eig_pencil(prob.time["Khat"], prob.time["Mhat"])

    def eigenvalue_tensor(self):
        """Lambda[i_1..i_d, i_t] = lambda_t[i_t] + kappa^2 sum_k lambda_k[i_k],
        the diagonal of Lambda_t x I + I x Lambda_s in the colex layout (step 3)."""
        k2 = self.prob.kappa ** 2
        lam = np.zeros(self.prob.shape)
        for k, (lk, _) in enumerate(self.eig_space):
            sh = [1] * (self.d + 1)
            sh[k] = len(lk)
            lam = lam + k2 * lk.reshape(sh)
        sh = [1] * (self.d + 1)
        sh[self.d] = len(self.eig_time[0])
        return lam + self.eig_time[0].reshape(sh)

    def apply(self, R):
        """s = P_kappa^{-1} r: forward chain with U^T (step 2), division by the
        eigenvalue tensor (step 3), backward chain with U (step 4)."""
        X = np.asarray(R).reshape(self.prob.shape, order="F")
        Us = [U for _, U in self.eig_space] + [self.eig_time[1]]
        for m, U in enumerate(Us):
            X = mode_product(X, U.T, m)
        X = X / self.eigenvalue_tensor()
        for m, U in enumerate(Us):
            X = mode_product(X, U, m)
        return X


class ScaledFD:
    """Diagonally scaled FD preconditioner (§4.4, closing definition):
    P^G = D^{1/2} Pbar D^{1/2} with D_ii = A_ii / Pbar_ii.

    On the unit box the coefficient functions of §4.4 are constant, the
    separated univariate weights are 1, and Pbar^G is the plain P_kappa of
    §4.2; so (P^G)^{-1} r = D^{-1/2} P^{-1} D^{-1/2} r, with P^{-1} applied by
    Algorithm 1 and both diagonals taken term by term from the Kronecker
    forms of A_kappa and P_kappa."""

    def __init__(self, prob, fd=None):
        self.prob = prob
        self.fd = fd if fd is not None else FD(prob)
        self.D = prob.kron_diagonal(prob.system_terms()) / prob.kron_diagonal(prob.prec_terms())

    def apply(self, R):
        X = np.asarray(R).reshape(self.prob.shape, order="F")
        s = 1.0 / np.sqrt(self.D)
        return s * self.fd.apply(s * X)
