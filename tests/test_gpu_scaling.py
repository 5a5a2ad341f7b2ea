"""GPU parity of the diagonally scaled FD preconditioner (§4.4, closing
definition: P^G = D^1/2 P D^1/2, D_ii = A_ii / P_ii) against the oracle.

Tolerances as for the unscaled preconditioner: FP64 within
max(1e-12, 10 eps cond(P^G)) of the oracle with a backward error at rounding
level; FP32 products 2e-5; BF16x3 products 5e-4 (sigma itself is formed in
FP64 on the FP64 path and in FP32 with the FP32 / BF16x3 products, 1e-7
relative).  The BF16x3 cases include shapes on the five-pass path (d = 3,
n_1 even, every n <= 64: sigma fused into the slab passes) and off it (n_1
odd: separate scaling passes).
"""
import numpy as np
import pytest

from stls_inputs import problem_knots, uniform_pm1

pytestmark = pytest.mark.gpu

try:
    import paper_1809_10026_amd as stls
except ImportError:  # library not built: GPU tests must fail loudly, not skip
    stls = None

from oracle import fd as ofd, pcg as opcg, system as osys  # noqa: E402
from tests.gpu_util import rel_err, to_dev, to_host  # noqa: E402

CASES = [
    (1, 7, 2, 1.0),
    (1, 20, 3, 2.0),
    (2, 5, 3, 1.0),
    (2, 13, 2, 0.3),
    (3, 4, 2, 1.0),   # n_1 = 4: five-pass BF16x3
    (3, 6, 3, 1.0),   # n_1 = 7: general BF16x3 chain
    (3, 9, 5, 0.7),   # n_1 = 12: five-pass BF16x3
]


def _lib():
    assert stls is not None, "libstls.so is not built; run python paper_1809_10026_amd/build.py"
    return stls


def _power(apply, n, its=60, seed=0):
    v = np.random.default_rng(seed).standard_normal(n)
    lam = 0.0
    for _ in range(its):
        w = apply(v)
        lam = float(np.linalg.norm(w) / np.linalg.norm(v))
        v = w / np.linalg.norm(w)
    return lam


def _setup(d, nel, p, kappa, mode):
    knots, degs = problem_knots(d, nel, p)
    S = _lib().Solver(knots, degs, kappa=kappa)
    S.set_fd_precision(mode)
    S.set_fd_scaling(True)
    P = osys.Problem(knots, degs, kappa=kappa)
    return S, P


@pytest.mark.parametrize("d,nel,p,kappa", CASES)
def test_scaled_prec_apply_fp64_matches_oracle(d, nel, p, kappa):
    S, P = _setup(d, nel, p, kappa, _lib().STLS_FD_FP64)
    G = ofd.ScaledFD(P)
    r = uniform_pm1(P.ndof, 31)
    s = to_host(S.prec_apply(to_dev(r)))
    s_ref = osys.vec(G.apply(r))
    sq = osys.vec(np.sqrt(G.D))
    PG = lambda v: sq * osys.vec(P.prec_matvec(sq * v))  # D^1/2 P D^1/2 v
    norm = _power(PG, P.ndof)
    cond = norm * _power(lambda v: osys.vec(G.apply(v)), P.ndof)
    assert np.linalg.norm(PG(s) - r) / (norm * np.linalg.norm(s)) < 1e-14
    assert rel_err(s, s_ref) < max(1e-12, 10 * np.finfo(float).eps * cond)


@pytest.mark.parametrize("mode,tol", [(1, 2e-5), (2, 5e-4)])
@pytest.mark.parametrize("d,nel,p,kappa", CASES)
def test_scaled_prec_apply_low_precision_error_bound(d, nel, p, kappa, mode, tol):
    S, P = _setup(d, nel, p, kappa, mode)
    r = uniform_pm1(P.ndof, 32)
    s = to_host(S.prec_apply(to_dev(r)))
    assert rel_err(s, osys.vec(ofd.ScaledFD(P).apply(r))) < tol


@pytest.mark.parametrize("mode", [0, 2])
def test_scaling_off_restores_plain_preconditioner(mode):
    """Index and control work: switching the scaling off gives exactly the
    plain preconditioner's result (same kernels, same inputs)."""
    knots, degs = problem_knots(3, 8, 4)
    a = _lib().Solver(knots, degs)
    b = _lib().Solver(knots, degs)
    for S in (a, b):
        S.set_fd_precision(mode)
    r = to_dev(uniform_pm1(a.ndof, 33))
    b.set_fd_scaling(True)
    scaled = to_host(b.prec_apply(r))
    b.set_fd_scaling(False)
    assert np.array_equal(to_host(b.prec_apply(r)), to_host(a.prec_apply(r)))
    assert not np.array_equal(scaled, to_host(a.prec_apply(r)))


@pytest.mark.parametrize("mode", [0, 2])
def test_scaling_follows_kappa(mode):
    knots, degs = problem_knots(3, 8, 4)
    S = _lib().Solver(knots, degs, kappa=1.0)
    S.set_fd_precision(mode)
    S.set_fd_scaling(True)
    S.set_kappa(5.0)
    P = osys.Problem(knots, degs, kappa=5.0)
    r = uniform_pm1(S.ndof, 34)
    s = to_host(S.prec_apply(to_dev(r)))
    assert rel_err(s, osys.vec(ofd.ScaledFD(P).apply(r))) < (1e-12 if mode == 0 else 5e-4)


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("d,nel,p", [(2, 16, 3), (3, 8, 4), (3, 7, 4)])
def test_scaled_pcg_matches_oracle(mode, d, nel, p):
    """PCG with P^G: the true residual reaches the tolerance, the iteration
    count is the oracle's (FP64 products: within one; lower-precision
    products: a few more are allowed) and the solutions agree to the solve
    tolerance times the preconditioned condition bound."""
    knots, degs = problem_knots(d, nel, p)
    P = osys.Problem(knots, degs)
    b = uniform_pm1(P.ndof, 35)
    S = _lib().Solver(knots, degs)
    S.set_fd_precision(mode)
    S.set_fd_scaling(True)
    x, it, rel = S.solve(to_dev(b), rtol=1e-8, maxit=300)
    xo = to_host(x)
    assert rel <= 1e-8
    assert np.linalg.norm(b - osys.vec(P.matvec(xo))) / np.linalg.norm(b) < 2e-8
    G = ofd.ScaledFD(P)
    x_ref, info = opcg.pcg(lambda v: osys.vec(P.matvec(v)), lambda v: osys.vec(G.apply(v)), b, 1e-8)
    if mode == 0:
        assert abs(it - info["iters"]) <= 1
    else:
        assert it <= info["iters"] + 6
    assert rel_err(xo, x_ref) < 2 * d * 10 * 1e-8
