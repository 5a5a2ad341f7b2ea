"""GPU parity on mapped domains (§2.2, §4.4, §5.1-5.2): the quarter annulus
(d = 2) and the rotated quarter annulus (d = 3) against oracle/geometry.py.

Tolerances as on the unit box: matvec 1e-13 (sums of stencil products in a
different order); the preconditioners in FP64 within the first-order bound
4 eps max lambda_max / lambda_min of their (weighted) pencils, FP32 2e-5,
BF16x3 5e-4; PCG iteration counts within one of the oracle's, solutions
within the tolerance times 2d times 10.
"""
import numpy as np
import pytest

from stls_inputs import problem_knots, uniform_pm1

pytestmark = pytest.mark.gpu

try:
    import paper_1809_10026_amd as stls
except ImportError:  # library not built: GPU tests must fail loudly, not skip
    stls = None

from oracle import geometry as geo, pcg as opcg  # noqa: E402
from tests.gpu_util import rel_err, to_dev, to_host  # noqa: E402

PI = np.pi
CASES = [
    # d, n_el, p, kappa
    (2, 6, 3, 1.0),
    (2, 9, 2, 0.6),
    (2, 13, 4, 1.0),
    (3, 4, 2, 1.0),
    (3, 6, 3, 1.0),
    (3, 8, 2, 1.3),   # n = 8 per space direction: the five-pass FD
]


def _geom(d):
    return stls.STLS_GEOM_QUARTER_ANNULUS if d == 2 else stls.STLS_GEOM_ROTATED_QUARTER_ANNULUS


def _map(d):
    return geo.QuarterAnnulus() if d == 2 else geo.RotatedQuarterAnnulus()


def _pair(d, nel, p, kappa, prec):
    assert stls is not None, "libstls.so is not built; run python paper_1809_10026_amd/build.py"
    knots, degs = problem_knots(d, nel, p)
    S = stls.Solver(knots, degs, kappa=kappa, geometry=_geom(d), prec=prec)
    MP = geo.MappedProblem(_map(d), knots, degs, kappa=kappa)
    return S, MP


@pytest.mark.parametrize("d,nel,p,kappa", CASES)
def test_mapped_matvec(d, nel, p, kappa):
    S, MP = _pair(d, nel, p, kappa, 0)
    assert S.ndof == MP.ndof
    x = uniform_pm1(MP.ndof, 301)
    assert rel_err(to_host(S.matvec(to_dev(x))), MP.matvec(x)) < 1e-13


@pytest.mark.parametrize("geometry", [False, True], ids=["P", "PG"])
@pytest.mark.parametrize("d,nel,p,kappa", CASES)
def test_mapped_preconditioners(d, nel, p, kappa, geometry):
    S, MP = _pair(d, nel, p, kappa, 1 if geometry else 0)
    pre = geo.GeometryPreconditioner(MP, geometry=geometry)
    r = uniform_pm1(MP.ndof, 302)
    ref = pre.apply(r)
    spread = max(l.max() / l.min() for l, _ in pre.fd.eig_space + [pre.fd.eig_time])
    bound = max(1e-12, 4 * np.finfo(float).eps * spread)
    err = rel_err(to_host(S.prec_apply(to_dev(r))), ref)
    assert err < bound, (err, bound)
    for mode, tol in ((stls.STLS_FD_FP32, 2e-5), (stls.STLS_FD_BF16X3, 5e-4)):
        S.set_fd_precision(mode)
        err = rel_err(to_host(S.prec_apply(to_dev(r))), ref)
        assert err < tol, (mode, err)


@pytest.mark.parametrize("geometry", [False, True], ids=["P", "PG"])
@pytest.mark.parametrize("d,nel,p,kappa", CASES)
def test_mapped_pcg(d, nel, p, kappa, geometry):
    S, MP = _pair(d, nel, p, kappa, 1 if geometry else 0)
    pre = geo.GeometryPreconditioner(MP, geometry=geometry)
    b = uniform_pm1(MP.ndof, 303)
    x_ref, info = opcg.pcg(MP.matvec, pre.apply, b, 1e-10, maxit=3000)
    x, it, rel = S.solve(to_dev(b), rtol=1e-10, maxit=3000)
    assert abs(it - info["iters"]) <= 1 and rel <= 1e-10, (it, info["iters"])
    assert rel_err(to_host(x), x_ref) < 2 * d * 10 * 1e-10


# Uneven sizes and degrees per direction (time last): row blocks of 32 and of
# 16 rows along direction 1 with several blocks and ragged edges in every
# direction, direction-1 stencil widths 5 and 7 (unrolled line loops) and 11
# (the generic offset loop), mixed degrees, several chunks of time slices.
SHAPES = [
    (3, (20, 6, 9, 12), (2, 2, 2, 2)),   # n_1 = 20: 32-row blocks
    (3, (36, 5, 6, 10), (2, 2, 2, 2)),   # n_1 = 36: 16-row blocks
    (3, (10, 4, 3, 5), (3, 2, 2, 2)),    # width 7 along direction 1, mixed degrees
    (3, (6, 3, 3, 3), (5, 2, 2, 2)),     # width 11: generic loop
    (2, (30, 5, 4), (2, 2, 2)),          # 2-D, 32-row blocks
    (2, (40, 5, 6), (2, 3, 2)),          # 2-D, 16-row blocks, mixed degrees
]


@pytest.mark.parametrize("d,nel,p", SHAPES, ids=[f"d{s[0]}-{'x'.join(map(str, s[1]))}-p{''.join(map(str, s[2]))}"
                                                 for s in SHAPES])
def test_mapped_block_shapes(d, nel, p):
    assert stls is not None, "libstls.so is not built; run python paper_1809_10026_amd/build.py"
    knots, degs = problem_knots(d, nel, p)
    S = stls.Solver(knots, degs, geometry=_geom(d), prec=stls.STLS_PREC_GEOMETRY)
    MP = geo.MappedProblem(_map(d), knots, degs)
    assert S.ndof == MP.ndof
    x = uniform_pm1(MP.ndof, 307)
    assert rel_err(to_host(S.matvec(to_dev(x))), MP.matvec(x)) < 1e-13
    pre = geo.GeometryPreconditioner(MP)
    ref = pre.apply(x)
    spread = max(l.max() / l.min() for l, _ in pre.fd.eig_space + [pre.fd.eig_time])
    err = rel_err(to_host(S.prec_apply(to_dev(x))), ref)
    assert err < max(1e-12, 4 * np.finfo(float).eps * spread), err


def test_kappa_change_rescales_pg():
    S, MP = _pair(2, 7, 3, 1.0, 1)
    S.set_kappa(2.5)
    MP2 = geo.MappedProblem(geo.QuarterAnnulus(), *problem_knots(2, 7, 3), kappa=2.5)
    r = uniform_pm1(MP2.ndof, 304)
    ref = geo.GeometryPreconditioner(MP2).apply(r)
    assert rel_err(to_host(S.prec_apply(to_dev(r))), ref) < 1e-11
    x = uniform_pm1(MP2.ndof, 305)
    assert rel_err(to_host(S.matvec(to_dev(x))), MP2.matvec(x)) < 1e-13


def test_mixed_precision_pg_solve_reaches_the_tolerance():
    S, MP = _pair(3, 8, 3, 1.0, 1)
    b = uniform_pm1(MP.ndof, 306)
    x_ref, info = opcg.pcg(MP.matvec, geo.GeometryPreconditioner(MP).apply, b, 1e-8, maxit=3000)
    for mode in (stls.STLS_FD_FP32, stls.STLS_FD_BF16X3):
        S.set_fd_precision(mode)
        x, it, rel = S.solve(to_dev(b), rtol=1e-8, maxit=3000)
        xo = to_host(x)
        true_rel = np.linalg.norm(b - MP.matvec(xo)) / np.linalg.norm(b)
        assert rel <= 1e-8 and true_rel < 2e-8 and it <= info["iters"] + 6, (mode, it, info["iters"])
        assert rel_err(xo, x_ref) < 2 * 3 * 10 * 1e-8


def test_table2_pg_against_p_on_the_gpu():
    """Rotated quarter annulus, n_sub = 8, p = 2 and 3 (Table 2): the GPU
    counts equal the oracle's within one; P^G needs at least three times
    fewer iterations than P."""
    for p in (2, 3):
        its = []
        for prec in (stls.STLS_PREC_PARAMETRIC, stls.STLS_PREC_GEOMETRY):
            S, MP = _pair(3, 8, p, 1.0, prec)
            b = uniform_pm1(MP.ndof, 1)
            _, it, rel = S.solve(to_dev(b), rtol=1e-8, maxit=3000)
            ref = opcg.pcg(MP.matvec, geo.GeometryPreconditioner(MP, geometry=prec == 1).apply, b, 1e-8,
                           maxit=3000)[1]["iters"]
            assert abs(it - ref) <= 1 and rel <= 1e-8
            its.append(it)
        print(f"rotated quarter annulus n_sub 8 p {p}: P {its[0]}, P^G {its[1]} (paper: 107, 24)", flush=True)
        assert its[0] >= 3 * its[1]


@pytest.mark.parametrize("nsub", [16, 32])
def test_table2_sizes_pg_against_p(nsub):
    """Rotated quarter annulus at Table 2's n_sub = 16 and 32, p = 2, on the
    GPU alone (the oracle's mapped solve is out of reach at 1.1 M unknowns):
    both preconditioners reach the tolerance on the true residual, and P^G
    needs at least three times fewer iterations than P (paper: 126 vs 35 and
    142 vs 42; our parametrisation is not the paper's NURBS, so the counts
    agree in ratio, not exactly)."""
    import torch
    its = []
    for prec in (stls.STLS_PREC_PARAMETRIC, stls.STLS_PREC_GEOMETRY):
        knots, degs = problem_knots(3, nsub, 2)
        S = stls.Solver(knots, degs, geometry=stls.STLS_GEOM_ROTATED_QUARTER_ANNULUS, prec=prec)
        b = to_dev(uniform_pm1(S.ndof, 1))
        x, it, rel = S.solve(b, rtol=1e-8, maxit=3000)
        true_rel = float(torch.linalg.norm(b - S.matvec(x)) / torch.linalg.norm(b))
        assert rel <= 1e-8 and true_rel < 2e-8, (prec, rel, true_rel)
        its.append(it)
    print(f"rotated quarter annulus n_sub {nsub} p 2: P {its[0]}, P^G {its[1]}", flush=True)
    assert its[0] >= 3 * its[1]


def _q(x):
    X, Y = x[:, 0], x[:, 1]
    s = X * X + Y * Y
    return -(s - 1) * (s - 4) * X * Y * Y


def _lapq(x):
    X, Y = x[:, 0], x[:, 1]
    s = X * X + Y * Y
    F, Fp = -(s * s - 5 * s + 4), -(2 * s - 5)
    return 2 * X * F + X * Y * Y * (-16 * s + 20) + 12 * Fp * X * Y * Y


def _gradq(x):
    X, Y = x[:, 0], x[:, 1]
    s = X * X + Y * Y
    F, Fp = -(s * s - 5 * s + 4), -(2 * s - 5)
    g = X * Y * Y
    return [Fp * 2 * X * g + F * Y * Y, Fp * 2 * Y * g + F * 2 * X * Y]


def test_quarter_annulus_convergence_on_the_gpu():
    """§5.1 on the GPU: the manufactured solution of the quarter annulus
    solved with P^G-PCG on the device (load and error norms by the oracle)
    converges at the paper's rates for p = 3: V0 2, H1 3, L2 4."""
    exact = dict(u=lambda x, t: np.multiply.outer(_q(x), np.sin(PI * t)),
                 ut=lambda x, t: np.multiply.outer(_q(x), PI * np.cos(PI * t)),
                 lap=lambda x, t: np.multiply.outer(_lapq(x), np.sin(PI * t)),
                 grad=[lambda x, t: np.multiply.outer(_gradq(x)[0], np.sin(PI * t)),
                       lambda x, t: np.multiply.outer(_gradq(x)[1], np.sin(PI * t))])
    terms = [(lambda x: PI * _q(x), lambda t: np.cos(PI * t)), (lambda x: -_lapq(x), lambda t: np.sin(PI * t))]
    errs = []
    for n in (8, 16):
        S, MP = _pair(2, n, 3, 1.0, 1)
        F = geo.mapped_load(MP, terms)
        x, it, rel = S.solve(to_dev(F), rtol=1e-13, maxit=3000)
        errs.append(geo.mapped_error_norms(MP, to_host(x), exact))
    for key, r in dict(V0=2.0, H1=3.0, L2=4.0).items():
        got = np.log2(errs[0][key] / errs[1][key])
        assert abs(got - r) < 0.15, (key, got)


def test_unit_box_only_calls_refuse_mapped_handles():
    S, _ = _pair(2, 5, 2, 1.0, 1)
    import torch
    with pytest.raises(stls.StlsError) as ei:
        S.set_fd_scaling(True)
    assert ei.value.status == stls.STLS_EINVAL
    f = torch.zeros(S.forcing_shape[1], dtype=torch.float64, device="cuda")
    with pytest.raises(stls.StlsError) as ei:
        S.load_apply(f)
    assert ei.value.status == stls.STLS_EINVAL
