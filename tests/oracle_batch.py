"""Oracle side of the full batched-solve test, run in worker processes
(numpy and the oracle only: no GPU and no library in the workers).

For one problem of the uneven batch: the oracle's matvec and FD
preconditioner applied to the GPU's inputs, and the quantities the test
bounds: relative matvec difference; FD backward error ||P s - r|| /
(||P|| ||s||) with ||P|| bounded above through the factors' eigenvalues
(every term of P is a Kronecker product of symmetric positive semidefinite
factors); FD forward difference and the first-order bound of two
backward-stable FD applications, eps * max over the pencils of
lambda_max / lambda_min; true relative residual of the batched solution.
"""
import numpy as np

from oracle import fd as ofd, system as osys
from stls_inputs import batch_problem_knots


def check_problem(args):
    nel_row, p, kappa, x, y_gpu, s_gpu, b, xsol = args
    knots, degs = batch_problem_knots(nel_row, p)
    P = osys.Problem(knots, degs, kappa=kappa)
    F = ofd.FD(P)
    y = osys.vec(P.matvec(x))
    s = osys.vec(F.apply(x))
    normP = sum(c * np.prod([np.linalg.eigvalsh(W).max() for W in f]) for c, f in P.prec_terms())
    spread = max(l.max() / l.min() for l, _ in F.eig_space + [F.eig_time])
    return {
        "ndof": P.ndof,
        "matvec": float(np.linalg.norm(y_gpu - y) / np.linalg.norm(y)),
        "fd_backward": float(np.linalg.norm(osys.vec(P.prec_matvec(s_gpu)) - x) / (normP * np.linalg.norm(s_gpu))),
        "fd_forward": float(np.linalg.norm(s_gpu - s) / np.linalg.norm(s)),
        "fd_bound": float(4 * np.finfo(float).eps * spread),
        "true_relres": float(np.linalg.norm(b - osys.vec(P.matvec(xsol))) / np.linalg.norm(b)),
    }
