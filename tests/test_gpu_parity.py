"""GPU parity of the HIP path against the FP64 oracle (through the C ABI).

Tolerances.  Setup factors: quadrature of the same polynomials in a different
order, <= 1e-13 relative to the matrix scale.  Matvec: a sum of banded
products, <= 1e-13 relative (2-norm).  FD apply in FP64: both sides compute
U D^-1 U^T r with different (equally valid) eigenvectors from different
eigensolvers; the error bound is a small multiple of eps * cond(P) in the
worst case, and <= 1e-12 holds at the sizes tested here (the dense-solve pin
of the oracle uses the same bound).  PCG: both sides stop on the recurrence
residual at rtol; iteration counts agree within one and the solutions agree
to the solve tolerance times the condition number estimate of the
preconditioned system (<= 2d, spectral bound of §4.2.1).
"""
import numpy as np
import pytest

from stls_inputs import problem_knots, uniform_pm1

pytestmark = pytest.mark.gpu

try:
    import paper_1809_10026_amd as stls
except ImportError:  # library not built: GPU tests must fail loudly, not skip
    stls = None

from oracle import assemble, fd as ofd, pcg as opcg, system as osys  # noqa: E402
from tests.gpu_util import rel_err, to_dev, to_host  # noqa: E402


def _lib():
    assert stls is not None, "libstls.so is not built; run python paper_1809_10026_amd/build.py"
    return stls


CASES = [
    # d, n_el, p, kappa  (ragged tails: n not a multiple of 16 / panel widths)
    (1, 7, 2, 1.0),
    (1, 32, 2, 1.0),
    (2, 5, 3, 1.0),
    (2, 13, 2, 0.3),
    (2, 19, 4, 4.0),
    (3, 4, 2, 1.0),
    (3, 6, 3, 1.0),
    (3, 9, 5, 0.7),
]


@pytest.mark.parametrize("d,nel,p,kappa", CASES)
def test_setup_factors_and_shape(d, nel, p, kappa):
    S = _lib().Solver(*problem_knots(d, nel, p), kappa=kappa)
    P = osys.Problem(*problem_knots(d, nel, p), kappa=kappa)
    assert S.shape == P.shape and S.ndof == P.ndof  # index work: exact
    for k in range(d + 1):
        pk = p
        bw = 2 * pk + 1
        if k < d:
            ref = P.space[k]
            mats = {0: ref["M"], 1: ref["K"], 2: ref["J"]}
        else:
            mats = {0: P.time["M"], 1: P.time["K"]}
        n = mats[0].shape[0]
        for what, R in mats.items():
            band = S.factor(k, what).reshape(n, bw)
            dense = np.zeros((n, n))
            for i in range(n):
                for o in range(bw):
                    j = i + o - pk
                    if 0 <= j < n:
                        dense[i, j] = band[i, o]
            # sparsity is exact: entries outside the band are structurally absent
            assert np.abs(R - dense).max() <= 1e-13 * np.abs(R).max()
        U = S.factor(k, 3).reshape(n, n, order="F")
        lam = S.factor(k, 4)
        Mk = mats[0]
        Kk = mats[2] if k < d else mats[1]
        assert np.abs(U.T @ Mk @ U - np.eye(n)).max() < 1e-11
        assert np.abs(U.T @ Kk @ U - np.diag(lam)).max() < 1e-10 * lam.max()
        lam_ref = ofd.eig_pencil(Kk, Mk)[0]
        assert np.allclose(np.sort(lam), lam_ref, rtol=1e-10, atol=1e-12 * lam_ref.max())
    assert S.factor(d, 5)[0] == 1.0  # W_t: b_last(1)^2 = 1 for open knots


@pytest.mark.parametrize("d,nel,p,kappa", CASES)
def test_matvec_matches_oracle(d, nel, p, kappa):
    S = _lib().Solver(*problem_knots(d, nel, p), kappa=kappa)
    P = osys.Problem(*problem_knots(d, nel, p), kappa=kappa)
    x = uniform_pm1(P.ndof, 11)
    y = to_host(S.matvec(to_dev(x)))
    y_ref = osys.vec(P.matvec(x))
    assert rel_err(y, y_ref) < 1e-13


def _power(apply, n, its=60, seed=0):
    v = np.random.default_rng(seed).standard_normal(n)
    lam = 0.0
    for _ in range(its):
        w = apply(v)
        lam = float(np.linalg.norm(w) / np.linalg.norm(v))
        v = w / np.linalg.norm(w)
    return lam


@pytest.mark.parametrize("d,nel,p,kappa", CASES)
def test_prec_apply_fp64_matches_oracle(d, nel, p, kappa):
    """s = P^-1 r in FP64.  Backward error ||P s - r|| / (||P|| ||s||) must be
    at rounding level; the forward difference to the oracle (and to a dense
    solve) is bounded by max(1e-12, 10 eps cond(P)): two backward-stable
    solves of a system with condition number cond(P) can differ by that much
    (the oracle itself differs from LU by ~eps cond(P))."""
    S = _lib().Solver(*problem_knots(d, nel, p), kappa=kappa)
    P = osys.Problem(*problem_knots(d, nel, p), kappa=kappa)
    r = uniform_pm1(P.ndof, 12)
    s = to_host(S.prec_apply(to_dev(r)))
    fdo = ofd.FD(P)
    s_ref = osys.vec(fdo.apply(r))
    Pv = lambda v: osys.vec(P.prec_matvec(v))
    normP = _power(Pv, P.ndof)
    cond = normP * _power(lambda v: osys.vec(fdo.apply(v)), P.ndof)
    backward = np.linalg.norm(Pv(s) - r) / (normP * np.linalg.norm(s))
    assert backward < 1e-14
    tol = max(1e-12, 10 * np.finfo(float).eps * cond)
    assert rel_err(s, s_ref) < tol
    if P.ndof <= 3000:
        s_dense = np.linalg.solve(P.dense_P(), r)
        assert rel_err(s, s_dense) < tol


@pytest.mark.parametrize("d,nel,p,kappa", CASES)
def test_prec_apply_fp32_error_bound(d, nel, p, kappa):
    S = _lib().Solver(*problem_knots(d, nel, p), kappa=kappa)
    P = osys.Problem(*problem_knots(d, nel, p), kappa=kappa)
    S.set_fd_precision(stls.STLS_FD_FP32)
    r = uniform_pm1(P.ndof, 13)
    s = to_host(S.prec_apply(to_dev(r)))
    s_ref = osys.vec(ofd.FD(P).apply(r))
    # 2(d+1) FP32 products of length <= n with well-conditioned U (cond <= ~15)
    assert rel_err(s, s_ref) < 2e-5


@pytest.mark.parametrize("d,nel,p,kappa", CASES)
def test_prec_apply_bf16x3_error_bound(d, nel, p, kappa):
    """BF16x3 products: each operand split into bf16 hi + lo, three MFMA
    products with FP32 accumulation; the dropped lo*lo term and the lo
    rounding are 2^-18 relative, so 2(d+1) products with cond(U) <= ~15
    stay below 5e-4 relative."""
    S = _lib().Solver(*problem_knots(d, nel, p), kappa=kappa)
    P = osys.Problem(*problem_knots(d, nel, p), kappa=kappa)
    S.set_fd_precision(stls.STLS_FD_BF16X3)
    r = uniform_pm1(P.ndof, 14)
    s = to_host(S.prec_apply(to_dev(r)))
    s_ref = osys.vec(ofd.FD(P).apply(r))
    assert rel_err(s, s_ref) < 5e-4


@pytest.mark.parametrize("d,nel,p,kappa", CASES)
def test_prec_apply_asymmetric_error_bound(d, nel, p, kappa):
    """Asymmetric FD: the d forward space products in FP32, the time pass
    and the backward products in FP64; the error is that of the FP32 forward
    half (the FP32 bound above)."""
    S = _lib().Solver(*problem_knots(d, nel, p), kappa=kappa)
    P = osys.Problem(*problem_knots(d, nel, p), kappa=kappa)
    S.set_fd_precision(stls.STLS_FD_ASYM)
    r = uniform_pm1(P.ndof, 15)
    s = to_host(S.prec_apply(to_dev(r)))
    s_ref = osys.vec(ofd.FD(P).apply(r))
    assert rel_err(s, s_ref) < 2e-5


@pytest.mark.parametrize("mode", [1, 2, 3])
@pytest.mark.parametrize("d,nel,p", [(2, 16, 3), (3, 8, 4)])
def test_pcg_mixed_precision_reaches_fp64_tolerance(mode, d, nel, p):
    """Low-precision FD inside the FP64 PCG still reaches rtol = 1e-8 on the
    true residual; the solution matches the oracle's to the solve tolerance."""
    knots, degs = problem_knots(d, nel, p)
    P = osys.Problem(knots, degs)
    b = uniform_pm1(P.ndof, 21)
    S = _lib().Solver(knots, degs)
    S.set_fd_precision(mode)
    x, it, rel = S.solve(to_dev(b), rtol=1e-8, maxit=300)
    xo = to_host(x)
    true_rel = np.linalg.norm(b - osys.vec(P.matvec(xo))) / np.linalg.norm(b)
    assert rel <= 1e-8 and true_rel < 2e-8
    fdo = ofd.FD(P)
    x_ref, info = opcg.pcg(lambda v: osys.vec(P.matvec(v)), lambda v: osys.vec(fdo.apply(v)), b, 1e-8)
    assert it <= info["iters"] + 6
    assert rel_err(xo, x_ref) < 2 * d * 10 * 1e-8


def _manufactured_rhs(d, knots, degs, kappa=1.0):
    pi = np.pi
    s = lambda x: np.sin(pi * x)
    # u = prod sin(pi x_k) sin(pi t): f = prod sin * (pi cos(pi t) + d kappa pi^2 sin(pi t))
    return assemble.load_separable(knots, degs, [(pi, [s] * d, lambda t: np.cos(pi * t)),
                                                 (d * kappa * pi * pi, [s] * d, lambda t: np.sin(pi * t))],
                                   kappa=kappa)


@pytest.mark.parametrize("d,nel,p,rtol", [(1, 32, 2, 1e-10), (2, 16, 3, 1e-8), (3, 8, 4, 1e-8), (2, 11, 5, 1e-8)])
def test_pcg_matches_oracle_manufactured(d, nel, p, rtol):
    knots, degs = problem_knots(d, nel, p)
    P = osys.Problem(knots, degs)
    F = osys.vec(_manufactured_rhs(d, knots, degs))
    S = _lib().Solver(knots, degs)
    x, it, rel = S.solve(to_dev(F), rtol=rtol, maxit=200)
    xo = to_host(x)
    fdo = ofd.FD(P)
    x_ref, info = opcg.pcg(lambda v: osys.vec(P.matvec(v)), lambda v: osys.vec(fdo.apply(v)), F, rtol)
    assert abs(it - info["iters"]) <= 1 and rel <= rtol
    true_rel = np.linalg.norm(F - osys.vec(P.matvec(xo))) / np.linalg.norm(F)
    assert true_rel < 10 * rtol
    assert rel_err(xo, x_ref) < 2 * d * 10 * rtol


@pytest.mark.parametrize("nsub,p,its", [(8, 2, 9), (8, 3, 11), (8, 4, 11), (8, 5, 11), (16, 3, 11)])
def test_table1_iteration_counts_on_gpu(nsub, p, its):
    pi = np.pi
    s = lambda x: np.sin(pi * x)
    knots, degs = problem_knots(3, nsub, p)
    F = osys.vec(assemble.load_separable(knots, degs, [(1.0, [s, s, s], np.cos), (3 * pi * pi, [s, s, s], np.sin)]))
    S = _lib().Solver(knots, degs)
    _, it, rel = S.solve(to_dev(F), rtol=1e-8, maxit=100)
    assert it == its


def test_pcg_zero_rhs_and_noconv():
    knots, degs = problem_knots(2, 6, 3)
    S = _lib().Solver(knots, degs)
    import torch
    b = torch.zeros(S.ndof, dtype=torch.float64, device="cuda")
    x, it, rel = S.solve(b)
    assert it == 0 and float(x.abs().max()) == 0.0
    b = to_dev(uniform_pm1(S.ndof, 3))
    with pytest.raises(stls.StlsError) as ei:
        S.solve(b, rtol=1e-14, maxit=2)
    assert ei.value.status == stls.STLS_ENOCONV
    b[5] = float("nan")
    with pytest.raises(stls.StlsError) as ei:
        S.solve(b)
    assert ei.value.status == stls.STLS_ENAN


@pytest.mark.parametrize("mode", [0, 2])
def test_pcg_output_alignment_and_history(mode):
    """The solution vector may be any 8-byte-aligned device buffer (here a view
    one element into a larger tensor, so not 16-byte aligned): same iterate as
    an aligned output; the residual history starts at 1, has one entry per
    iteration and ends at the returned relative residual."""
    import torch
    knots, degs = problem_knots(3, 8, 4)
    S = _lib().Solver(knots, degs)
    S.set_fd_precision(mode)
    b = to_dev(uniform_pm1(S.ndof, 31))
    x_al, it_al, rel_al = S.solve(b, rtol=1e-9)
    buf = torch.zeros(S.ndof + 1, dtype=torch.float64, device="cuda")
    x_un = buf[1:]
    _, it_un, rel_un = S.solve(b, rtol=1e-9, out=x_un)
    assert it_un == it_al and rel_un == rel_al
    assert float((x_un - x_al).abs().max()) == 0.0
    hist = S.history()
    assert len(hist) == it_al + 1 and hist[0] == 1.0 and hist[-1] == rel_un <= 1e-9
