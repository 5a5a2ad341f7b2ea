"""Preconditioned conjugate gradient (§4.2: A is SPD, so PCG; §5: tolerance,
zero initial guess).  Oracle: test use only.

The paper runs CG with a relative tolerance and x_0 = 0 but does not state
the stopping norm.  Reading adopted: stop when the recurrence residual
satisfies ||r_k||_2 / ||b||_2 <= rtol; the true residual is reported too.
"""
from __future__ import annotations

import numpy as np


def pcg(matvec, prec, b, rtol=1e-8, maxit=1000):
    """Hestenes-Stiefel PCG from x_0 = 0 on flat FP64 vectors.

    Returns (x, info) with info = dict(iters, relres, true_relres, history,
    alphas, betas, converged).
    """
    b = np.asarray(b, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return x, dict(iters=0, relres=0.0, true_relres=0.0, history=[0.0],
                       alphas=[], betas=[], converged=True)
    r = b.copy()
    z = prec(r)
    p = z.copy()
    rho = float(r @ z)
    hist, alphas, betas = [1.0], [], []
    converged = False
    k = 0
    for k in range(1, maxit + 1):
        q = matvec(p)
        alpha = rho / float(p @ q)
        x = x + alpha * p
        r = r - alpha * q
        rel = float(np.linalg.norm(r)) / bnorm
        hist.append(rel)
        alphas.append(alpha)
        if rel <= rtol:
            converged = True
            break
        z = prec(r)
        rho_new = float(r @ z)
        beta = rho_new / rho
        betas.append(beta)
        p = z + beta * p
        rho = rho_new
    true_rel = float(np.linalg.norm(b - matvec(x))) / bnorm
    return x, dict(iters=k, relres=hist[-1], true_relres=true_rel, history=hist,
                   alphas=alphas, betas=betas, converged=converged)


def lanczos_extremes(alphas, betas):
    """Extreme eigenvalues of P^{-1} A estimated from the PCG coefficients
    (the Lanczos tridiagonal matrix built from alpha_k, beta_k)."""
    n = len(alphas)
    if n == 0:
        return np.nan, np.nan
    Tm = np.zeros((n, n))
    for j in range(n):
        Tm[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < n:
            off = np.sqrt(betas[j]) / alphas[j]
            Tm[j, j + 1] = Tm[j + 1, j] = off
    ev = np.linalg.eigvalsh(Tm)
    return float(ev[0]), float(ev[-1])
