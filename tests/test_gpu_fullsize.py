"""Parity at the benchmark workload's full size, in the launch configuration
the benchmark times: d = 3, p = 4, 48 elements per direction, N = 6,375,000,
right-hand side U[-1, 1] with the benchmark's seed.

The oracle applies the matvec, the FD preconditioner and the initial-data
lifting to the whole vector in a few seconds, so those are compared entry by
entry; the general lifting is checked by its identity with the matvec on
zero-data functions; the solves of every FD precision are compared with the
oracle's own FP64 FD-PCG solution (about 17 s on the host cores) and their
true residuals are taken with the oracle's matvec.  Tolerances as in the
small-size parity tests.
"""
import numpy as np
import pytest

from stls_inputs import CONFIGS, problem_knots, uniform_pm1

pytestmark = pytest.mark.gpu

try:
    import paper_1809_10026_amd as stls
except ImportError:  # library not built: GPU tests must fail loudly, not skip
    stls = None

from oracle import fd as ofd, system as osys  # noqa: E402
from tests.gpu_util import rel_err, to_dev, to_host  # noqa: E402

CFG = CONFIGS["d3_p4_nel48"]


@pytest.fixture(scope="module")
def full():
    assert stls is not None, "libstls.so is not built; run python paper_1809_10026_amd/build.py"
    knots, degs = problem_knots(CFG["d"], CFG["n_el"], CFG["p"])
    S = stls.Solver(knots, degs)
    P = osys.Problem(knots, degs)
    F = ofd.FD(P)
    return S, P, F


def test_fullsize_shape(full):
    S, P, _ = full
    assert S.shape == P.shape == (50, 50, 50, 51) and S.ndof == 6375000


def test_fullsize_matvec(full):
    S, P, _ = full
    x = uniform_pm1(S.ndof, 41)
    assert rel_err(to_host(S.matvec(to_dev(x))), osys.vec(P.matvec(x))) < 1e-13


def _eig_bounds(P):
    """Every term of P is a Kronecker product of symmetric positive
    semidefinite factors, whose eigenvalues are the products of the factors'
    eigenvalues: lambda_max(P) <= sum c prod max, lambda_min(P) >= sum c prod min."""
    hi = sum(c * np.prod([np.linalg.eigvalsh(W).max() for W in f]) for c, f in P.prec_terms())
    lo = sum(c * np.prod([np.linalg.eigvalsh(W).min() for W in f]) for c, f in P.prec_terms())
    return hi, lo


@pytest.mark.parametrize("mode,scaled,tol", [(0, False, None), (1, False, 2e-5), (2, False, 5e-4),
                                             (0, True, None), (2, True, 5e-4)])
def test_fullsize_prec_apply(full, mode, scaled, tol):
    """FP64: the backward error ||P s - r|| / (||P|| ||s||) is at rounding
    level (||P|| bounded above through the factors' eigenvalues), and the
    forward difference to the oracle is within 4 eps max_k lambda_max /
    lambda_min over the univariate pencils (5.6e-8 here; measured 3.9e-11).
    Both sides apply U Lambda^-1 U^T with eigenpairs from backward-stable
    eigensolvers, whose eigenvalues carry absolute errors ~eps lambda_max;
    after the division the low modes carry relative errors up to
    eps lambda_max / lambda_min, which bounds the forward difference to first
    order (an FP32 product anywhere in the chain, ~1e-6, fails it).
    FP32 / BF16x3: the product error bounds of the small-size tests."""
    S, P, F = full
    S.set_fd_precision(mode)
    S.set_fd_scaling(scaled)
    try:
        r = uniform_pm1(S.ndof, 42)
        s = to_host(S.prec_apply(to_dev(r)))
        G = ofd.ScaledFD(P, F) if scaled else None
        ref = osys.vec(G.apply(r) if scaled else F.apply(r))
        if tol is not None:
            assert rel_err(s, ref) < tol
            return
        hi, lo = _eig_bounds(P)
        if scaled:  # P^G = D^1/2 P D^1/2
            sq = osys.vec(np.sqrt(G.D))
            Ps = sq * osys.vec(P.prec_matvec(sq * s))
            hi, lo = hi * G.D.max(), lo * G.D.min()
        else:
            Ps = osys.vec(P.prec_matvec(s))
        backward = np.linalg.norm(Ps - r) / (hi * np.linalg.norm(s))
        spread = max(l.max() / l.min() for l, _ in F.eig_space + [F.eig_time])
        bound = 4 * np.finfo(float).eps * spread
        print(f"backward {backward:.2e} forward {rel_err(s, ref):.2e} first-order bound {bound:.2e} "
              f"(cond(P) bound {hi / lo:.2e})", flush=True)
        assert backward < 1e-14
        assert rel_err(s, ref) < bound
    finally:
        S.set_fd_precision(0)
        S.set_fd_scaling(False)


def test_fullsize_pcg(full):
    """The benchmark's solve in every mode: true residual by the oracle's
    matvec, and every solution compared entry by entry with the oracle's own
    FP64 FD-PCG solution of the same system (about 17 s on the host cores)."""
    from oracle import pcg as opcg
    S, P, F = full
    b = uniform_pm1(S.ndof, CFG["seed"])
    bd = to_dev(b)
    sols = {}
    try:
        for mode, scaled in [(0, False), (1, False), (2, False), (2, True)]:
            S.set_fd_precision(mode)
            S.set_fd_scaling(scaled)
            x, it, rel = S.solve(bd, rtol=CFG["rtol"], maxit=200)
            xo = to_host(x)
            true_rel = np.linalg.norm(b - osys.vec(P.matvec(xo))) / np.linalg.norm(b)
            print(f"mode {mode} scaled {scaled}: {it} iterations, relres {rel:.2e}, true {true_rel:.2e}", flush=True)
            assert rel <= CFG["rtol"] and true_rel < 2 * CFG["rtol"]
            sols[(mode, scaled)] = xo
    finally:
        S.set_fd_precision(0)
        S.set_fd_scaling(False)
    x_ref, info = opcg.pcg(lambda v: osys.vec(P.matvec(v)), lambda v: osys.vec(F.apply(v)), b, CFG["rtol"])
    assert abs(info["iters"] - 17) <= 1
    for key, xo in sols.items():
        err = rel_err(xo, x_ref)
        print(f"mode {key}: vs oracle solution rel {err:.2e} max abs {np.abs(xo - x_ref).max():.2e}", flush=True)
        assert err < 2 * 3 * 10 * CFG["rtol"], key


@pytest.mark.parametrize("rhs", ["manufactured", "random"])
def test_fullsize_d2_workload_against_oracle(rhs):
    """The 2-D workload at full size (p = 3, 64 elements per direction,
    N = 278,850): manufactured sin(pi x) sin(pi y) sin(pi t) and the
    U[-1, 1] right-hand side (seed 1809), FP64 FD.  The oracle's own FD-PCG
    runs at this size in seconds: iteration counts within one, solutions to
    the solve tolerance times the preconditioned condition bound (2d), true
    residual by the oracle's matvec."""
    from oracle import assemble, pcg as opcg
    c = CONFIGS["d2_p3_nel64"]
    knots, degs = problem_knots(c["d"], c["n_el"], c["p"])
    P = osys.Problem(knots, degs)
    if rhs == "manufactured":
        pi = np.pi
        s = lambda x: np.sin(pi * x)
        F = osys.vec(assemble.load_separable(knots, degs, [(pi, [s, s], lambda t: np.cos(pi * t)),
                                                           (2 * pi * pi, [s, s], lambda t: np.sin(pi * t))]))
    else:
        F = uniform_pm1(P.ndof, c["seed"])
    S = stls.Solver(knots, degs)
    assert S.ndof == 278850
    x, it, rel = S.solve(to_dev(F), rtol=c["rtol"], maxit=200)
    xo = to_host(x)
    fdo = ofd.FD(P)
    x_ref, info = opcg.pcg(lambda v: osys.vec(P.matvec(v)), lambda v: osys.vec(fdo.apply(v)), F, c["rtol"])
    true_rel = np.linalg.norm(F - osys.vec(P.matvec(xo))) / np.linalg.norm(F)
    print(f"d2 {rhs}: {it} iterations (oracle {info['iters']}), true relres {true_rel:.2e}", flush=True)
    assert abs(it - info["iters"]) <= 1 and rel <= c["rtol"] and true_rel < 2 * c["rtol"]
    assert rel_err(xo, x_ref) < 2 * 2 * 10 * c["rtol"]


def test_fullsize_lift_initial(full):
    """Lifting of initial data at the benchmark shape: the whole coupling
    against the oracle's term-by-term expansion (it takes the oracle well
    under a second); bound as in the small-size lifting tests."""
    from oracle import lift
    S, P, _ = full
    u0 = uniform_pm1(S.ns, 91)
    F = uniform_pm1(S.ndof, 92)
    Fd = to_dev(F)
    S.lift_initial(to_dev(u0), Fd)
    assert rel_err(F - to_host(Fd), osys.vec(lift.initial_coupling(P, u0))) < 1e-12


def test_fullsize_general_lift_of_zero_data_function_is_the_matvec(full):
    """General lifting at the benchmark shape (52^4 full space), by the
    property that holds at any size: on an embedded zero-data vector the
    term-by-term form equals the system matrix (independent GPU paths)."""
    import torch
    S, _, _ = full
    x = to_dev(uniform_pm1(S.ndof, 93))
    ub = S.lift_embed(torch.zeros(S.forcing_shape[1], dtype=torch.float64, device="cuda"), x)
    F = torch.zeros(S.ndof, dtype=torch.float64, device="cuda")
    S.lift_apply(ub, F)
    assert rel_err(-to_host(F), to_host(S.matvec(x))) < 1e-12
