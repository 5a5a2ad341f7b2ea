"""GPU parity on the problem descriptions that stls_setup accepts beyond the
uniform, equal-degree benchmark shapes (§2.1 open knot vectors with uneven
elements and repeated interior knots; §2.2 spaces with a space degree other
than the time degree, as studied in §5.1 with p_s = p_t + 1; different
degrees and sizes per space direction).  These route the matvec, the FD
chain and the batched kernels through their general instances, and a long
time direction (n_t > 128) through the two-launch BF16x3 time pass.

Knots: uneven elements from ``graded_open_knots`` with one interior knot of
multiplicity p - 1 in space (C^1, the least regularity the least-squares
method admits) and p in time (C^0).  Tolerances are those of the uniform
parity tests: matvec 1e-13; FD in FP64 by its backward error (1e-14) and a
forward difference within max(1e-12, 10 eps cond(P)); FP32 products 2e-5;
BF16x3 products 5e-4 (cond(U) stays below ~20 here); the asymmetric mode
(FP32 forward products) 2e-5; PCG iteration counts
within one of the oracle's and solutions within the tolerance times the
condition bound 2d of the preconditioned system (§4.2.1).
"""
import numpy as np
import pytest

from stls_inputs import graded_open_knots, uniform_open_knots, uniform_pm1

pytestmark = pytest.mark.gpu

try:
    import paper_1809_10026_amd as stls
except ImportError:  # library not built: GPU tests must fail loudly, not skip
    stls = None

from oracle import fd as ofd, pcg as opcg, system as osys  # noqa: E402
from tests.gpu_util import rel_err, to_dev, to_host  # noqa: E402


def _knots(spec, seed):
    """spec: list of (n_el, p, graded) per direction, time last."""
    knots, degs = [], []
    for k, (nel, p, graded) in enumerate(spec):
        is_time = k == len(spec) - 1
        if graded:
            mult = p if is_time else p - 1
            knots.append(graded_open_knots(nel, p, mult=mult, seed=seed + k))
        else:
            knots.append(uniform_open_knots(nel, p))
        degs.append(p)
    return knots, degs


CASES = {
    # d = 1: p_s = 3 on graded knots with a double knot, linear time (p_t = 1)
    "d1_ps3_pt1_graded": ([(9, 3, True), (11, 1, True)], 1.0),
    # d = 2: p_s = p_t + 1 (§5.1), graded knots, unequal n per direction
    "d2_ps3_pt2_graded": ([(11, 3, True), (9, 3, True), (10, 2, True)], 0.6),
    # d = 2: time degree above the space degree
    "d2_ps2_pt4_graded": ([(8, 2, True), (12, 2, False), (7, 4, True)], 2.5),
    # d = 3: a different degree in every space direction
    "d3_p2_4_3_pt2_graded": ([(7, 2, True), (6, 4, True), (5, 3, True), (8, 2, True)], 1.0),
    # d = 3: equal space degree, p_s = p_t + 1, unequal n, n_1 even (the
    # five-pass FD and slab matvec instances), uniform knots
    "d3_ps4_pt3_uneven_n": ([(8, 4, False), (6, 4, False), (7, 4, False), (9, 3, False)], 1.0),
    # d = 3: the same with graded knots and repeated interior knots
    "d3_ps4_pt3_graded": ([(8, 4, True), (6, 4, True), (7, 4, True), (9, 3, True)], 0.4),
    # d = 2: a long time direction (n_t = 141 > 128: the BF16x3 time pass
    # splits into a forward product with the division and a backward product,
    # since both time operators no longer fit in LDS together)
    "d2_long_time": ([(6, 2, False), (5, 3, True), (139, 2, True)], 1.0),
}


def _case(name):
    assert stls is not None, "libstls.so is not built; run python paper_1809_10026_amd/build.py"
    spec, kappa = CASES[name]
    knots, degs = _knots(spec, seed=100 + len(name))
    S = stls.Solver(knots, degs, kappa=kappa)
    P = osys.Problem(knots, degs, kappa=kappa)
    return S, P, knots, degs, kappa


def _power(apply, n, its=60, seed=0):
    v = np.random.default_rng(seed).standard_normal(n)
    lam = 0.0
    for _ in range(its):
        w = apply(v)
        lam = float(np.linalg.norm(w) / np.linalg.norm(v))
        v = w / np.linalg.norm(w)
    return lam


@pytest.mark.parametrize("name", list(CASES))
def test_setup_factors_general(name):
    S, P, knots, degs, _ = _case(name)
    d = P.d
    assert S.shape == P.shape and S.ndof == P.ndof
    for k in range(d + 1):
        pk = degs[k]
        bw = 2 * pk + 1
        ref = P.space[k] if k < d else P.time
        mats = {0: ref["M"], 1: ref["K"]}
        if k < d:
            mats[2] = ref["J"]
        n = mats[0].shape[0]
        for what, R in mats.items():
            band = S.factor(k, what).reshape(n, bw)
            dense = np.zeros((n, n))
            for i in range(n):
                for o in range(bw):
                    j = i + o - pk
                    if 0 <= j < n:
                        dense[i, j] = band[i, o]
            assert np.abs(R - dense).max() <= 1e-13 * np.abs(R).max(), (k, what)


@pytest.mark.parametrize("name", list(CASES))
def test_matvec_general(name):
    S, P, *_ = _case(name)
    x = uniform_pm1(P.ndof, 201)
    assert rel_err(to_host(S.matvec(to_dev(x))), osys.vec(P.matvec(x))) < 1e-13


@pytest.mark.parametrize("scaled", [False, True])
@pytest.mark.parametrize("name", list(CASES))
def test_prec_apply_general(name, scaled):
    S, P, *_ = _case(name)
    fdo = ofd.FD(P)
    G = ofd.ScaledFD(P, fdo) if scaled else None
    r = uniform_pm1(P.ndof, 202)
    ref = osys.vec(G.apply(r) if scaled else fdo.apply(r))
    S.set_fd_scaling(scaled)
    # FP64: backward error and forward difference
    s = to_host(S.prec_apply(to_dev(r)))
    if scaled:
        sq = osys.vec(np.sqrt(G.D))
        Pv = lambda v: sq * osys.vec(P.prec_matvec(sq * v))
    else:
        Pv = lambda v: osys.vec(P.prec_matvec(v))
    normP = _power(Pv, P.ndof)
    cond = normP * _power(lambda v: osys.vec(G.apply(v) if scaled else fdo.apply(v)), P.ndof)
    assert np.linalg.norm(Pv(s) - r) / (normP * np.linalg.norm(s)) < 1e-14
    assert rel_err(s, ref) < max(1e-12, 10 * np.finfo(float).eps * cond)
    for mode, tol in ((stls.STLS_FD_FP32, 2e-5), (stls.STLS_FD_BF16X3, 5e-4), (stls.STLS_FD_ASYM, 2e-5)):
        S.set_fd_precision(mode)
        err = rel_err(to_host(S.prec_apply(to_dev(r))), ref)
        assert err < tol, (mode, err)
    S.set_fd_precision(stls.STLS_FD_FP64)


@pytest.mark.parametrize("name", list(CASES))
def test_pcg_general(name):
    S, P, *_ = _case(name)
    d = P.d
    b = uniform_pm1(P.ndof, 203)
    fdo = ofd.FD(P)
    x_ref, info = opcg.pcg(lambda v: osys.vec(P.matvec(v)), lambda v: osys.vec(fdo.apply(v)), b, 1e-10)
    x, it, rel = S.solve(to_dev(b), rtol=1e-10, maxit=300)
    xo = to_host(x)
    assert abs(it - info["iters"]) <= 1 and rel <= 1e-10
    assert rel_err(xo, x_ref) < 2 * d * 10 * 1e-10
    for mode in (stls.STLS_FD_FP32, stls.STLS_FD_BF16X3, stls.STLS_FD_ASYM):
        S.set_fd_precision(mode)
        x, it_m, rel = S.solve(to_dev(b), rtol=1e-8, maxit=300)
        xo = to_host(x)
        true_rel = np.linalg.norm(b - osys.vec(P.matvec(xo))) / np.linalg.norm(b)
        assert rel <= 1e-8 and true_rel < 2e-8, (mode, rel, true_rel)
        assert rel_err(xo, x_ref) < 2 * d * 10 * 1e-8
    S.set_fd_precision(stls.STLS_FD_FP64)


def test_batch_general_knots():
    """A d = 2 batch (one degree per problem, the batch's constraint) on
    graded knots with repeated interior knots and unequal sizes: batched
    matvec and FD against the oracle, batched solve against the oracle's PCG."""
    specs = [
        ([(9, 3, True), (7, 3, True), (11, 3, True)], 0.5),
        ([(6, 2, True), (10, 2, True), (5, 2, True)], 3.0),
        ([(5, 5, True), (6, 5, True), (7, 5, True)], 1.0),
        ([(13, 4, False), (9, 4, True), (8, 4, True)], 0.15),
    ]
    probs = []
    for i, (spec, kappa) in enumerate(specs):
        knots, degs = _knots(spec, seed=300 + 10 * i)
        probs.append((knots, degs, kappa))
    B = stls.Batch(probs)
    off = B.offsets
    x = uniform_pm1(B.total, 204)
    y = to_host(B.matvec(to_dev(x)))
    s = to_host(B.prec_apply(to_dev(x)))
    b = uniform_pm1(B.total, 205)
    xb, its, rels = B.solve(to_dev(b), rtol=1e-10, maxit=300)
    xb = to_host(xb)
    for i, (knots, degs, kappa) in enumerate(probs):
        P = osys.Problem(knots, degs, kappa=kappa)
        sl = slice(off[i], off[i + 1])
        assert rel_err(y[sl], osys.vec(P.matvec(x[sl]))) < 1e-13
        fdo = ofd.FD(P)
        Pv = lambda v: osys.vec(P.prec_matvec(v))
        normP = _power(Pv, P.ndof)
        cond = normP * _power(lambda v: osys.vec(fdo.apply(v)), P.ndof)
        assert np.linalg.norm(Pv(s[sl]) - x[sl]) / (normP * np.linalg.norm(s[sl])) < 1e-14
        assert rel_err(s[sl], osys.vec(fdo.apply(x[sl]))) < max(1e-12, 10 * np.finfo(float).eps * cond)
        x_ref, info = opcg.pcg(lambda v: osys.vec(P.matvec(v)), lambda v: osys.vec(fdo.apply(v)), b[sl], 1e-10)
        assert abs(its[i] - info["iters"]) <= 1 and rels[i] <= 1e-10
        assert rel_err(xb[sl], x_ref) < 2 * 2 * 10 * 1e-10
