"""Batched PCG over many uneven problems (one launch per PCG step).

Invariant: each problem of a batch gives the same result as its standalone
solve on the same factors (batched kernels reduce in a different order:
operators agree to 1e-12 relative, solves to the tolerance, iteration counts
within one).  The smallest problem is also compared with the oracle.
"""
import numpy as np
import pytest

from stls_inputs import batch_params, batch_problem_knots, problem_knots, uniform_pm1

pytestmark = pytest.mark.gpu

try:
    import paper_1809_10026_amd as stls
except ImportError:
    stls = None

from oracle import fd as ofd, pcg as opcg, system as osys  # noqa: E402
from tests.gpu_util import rel_err, to_dev, to_host  # noqa: E402

SMALL = [
    ((7, 9, 8), 2, 0.3),
    ((12, 5, 10), 3, 1.0),
    ((6, 6, 13), 4, 5.0),
    ((9, 11, 7), 5, 0.12),
    ((16, 18, 17), 3, 2.2),
]


def _batch(specs):
    assert stls is not None, "libstls.so is not built"
    probs = []
    for nel, p, kappa in specs:
        knots, degs = problem_knots(2, list(nel), p)
        probs.append((knots, degs, kappa))
    return stls.Batch(probs), probs


def _power(apply, n, its=60):
    """Largest eigenvalue of a symmetric positive definite operator (power iteration)."""
    v = np.random.default_rng(5).standard_normal(n)
    lam = 0.0
    for _ in range(its):
        w = apply(v)
        lam = float(np.linalg.norm(w) / np.linalg.norm(v))
        v = w / np.linalg.norm(w)
    return lam


def _single(B, i, probs):
    knots, degs, kappa = probs[i]
    return stls.Solver(knots, degs, kappa=kappa)


def test_batched_operators_match_single_problem():
    import torch
    B, probs = _batch(SMALL)
    off = B.offsets
    x = to_dev(uniform_pm1(B.total, 61))
    y = B.matvec(x)
    s = B.prec_apply(x)
    for i in range(len(probs)):
        S = _single(B, i, probs)
        xi = x[off[i]:off[i + 1]].contiguous()
        assert rel_err(to_host(y[off[i]:off[i + 1]]), to_host(S.matvec(xi))) < 1e-13
        # same factors would need the batch's own handle: compare with the oracle FD instead
        P = osys.Problem(*problem_knots(2, list(SMALL[i][0]), SMALL[i][1]), kappa=SMALL[i][2])
        s_ref = osys.vec(ofd.FD(P).apply(to_host(xi)))
        assert rel_err(to_host(s[off[i]:off[i + 1]]), s_ref) < 1e-10


def test_batched_solve_matches_single_and_oracle():
    B, probs = _batch(SMALL)
    off = B.offsets
    b = to_dev(uniform_pm1(B.total, 62))
    x, its, rels = B.solve(b, rtol=1e-8, maxit=300)
    assert all(r <= 1e-8 for r in rels)
    for i in range(len(probs)):
        S = _single(B, i, probs)
        xs, it_s, rel_s = S.solve(b[off[i]:off[i + 1]].contiguous(), rtol=1e-8)
        assert abs(its[i] - it_s) <= 1
        assert rel_err(to_host(x[off[i]:off[i + 1]]), to_host(xs)) < 1e-7
    # smallest problem against the oracle
    i = 0
    P = osys.Problem(*problem_knots(2, list(SMALL[i][0]), SMALL[i][1]), kappa=SMALL[i][2])
    bi = to_host(b[off[i]:off[i + 1]])
    fdo = ofd.FD(P)
    xr, info = opcg.pcg(lambda v: osys.vec(P.matvec(v)), lambda v: osys.vec(fdo.apply(v)), bi, 1e-8)
    assert abs(its[i] - info["iters"]) <= 1
    assert rel_err(to_host(x[off[i]:off[i + 1]]), xr) < 1e-6


SMALL_D1 = [
    ((9, 8), 2, 0.5),
    ((20, 13), 3, 1.7),
    ((14, 30), 6, 0.2),
    ((40, 35), 4, 3.0),
]


def test_d1_batch_matches_single_problems():
    """d = 1 batches (the outer stage reads x alone), degrees up to 6: the
    operators agree with the standalone ones (matvec) and the oracle (FD),
    solves with the standalone solves."""
    probs = []
    for nel, p, kappa in SMALL_D1:
        knots, degs = problem_knots(1, list(nel), p)
        probs.append((knots, degs, kappa))
    assert stls is not None, "libstls.so is not built"
    B = stls.Batch(probs)
    off = B.offsets
    x = to_dev(uniform_pm1(B.total, 64))
    y = B.matvec(x)
    s = B.prec_apply(x)
    for i, (knots, degs, kappa) in enumerate(probs):
        S = stls.Solver(knots, degs, kappa=kappa)
        xi = x[off[i]:off[i + 1]].contiguous()
        assert rel_err(to_host(y[off[i]:off[i + 1]]), to_host(S.matvec(xi))) < 1e-13
        si = to_host(s[off[i]:off[i + 1]])
        # same host factors as the standalone handle: kernels differ only in rounding order
        assert rel_err(si, to_host(S.prec_apply(xi))) < 1e-12
        # against the oracle's own eigendecomposition: backward error at rounding
        # level, forward difference within 10 eps cond(P)
        P = osys.Problem(knots, degs, kappa=kappa)
        r = to_host(xi)
        Pv = lambda v: osys.vec(P.prec_matvec(v))
        fdo = ofd.FD(P)
        normP = _power(Pv, P.ndof)
        cond = normP * _power(lambda v: osys.vec(fdo.apply(v)), P.ndof)
        assert np.linalg.norm(Pv(si) - r) / (normP * np.linalg.norm(si)) < 1e-14
        assert rel_err(si, osys.vec(fdo.apply(r))) < max(1e-12, 10 * np.finfo(float).eps * cond)
    b = to_dev(uniform_pm1(B.total, 65))
    xb, its, rels = B.solve(b, rtol=1e-8, maxit=300)
    assert all(r <= 1e-8 for r in rels)
    for i, (knots, degs, kappa) in enumerate(probs):
        S = stls.Solver(knots, degs, kappa=kappa)
        xs, it_s, _ = S.solve(b[off[i]:off[i + 1]].contiguous(), rtol=1e-8)
        assert abs(its[i] - it_s) <= 1
        assert rel_err(to_host(xb[off[i]:off[i + 1]]), to_host(xs)) < 1e-7


def test_full_uneven_batch_converges():
    """256 problems: n_el per direction uniform on 16..96, p uniform on {2..5},
    kappa log-uniform on [0.1, 10], right-hand sides U[-1,1] (seeds 20180927 + i).
    Every problem's batched matvec and FD application is compared with the
    oracle's (FD: backward error at rounding level, forward difference within
    the first-order bound eps * max lambda_max / lambda_min of the pencils),
    and every batched solution's true residual is taken with the oracle's
    matvec; three problems are also solved standalone."""
    nel, p, kappa = batch_params()
    probs = []
    for i in range(len(p)):
        knots, degs = batch_problem_knots(nel[i], p[i])
        probs.append((knots, degs, float(kappa[i])))
    B = stls.Batch(probs)
    off = B.offsets
    b = np.concatenate([uniform_pm1(off[i + 1] - off[i], 20180927 + i) for i in range(len(probs))])
    bt = to_dev(b)
    x, its, rels = B.solve(bt, rtol=1e-8, maxit=500)
    assert len(its) == 256 and max(rels) <= 1e-8 and min(its) >= 1
    # every problem against the oracle: matvec and FD applied to a seeded
    # vector, and the true residual of the batched solution (oracle workers
    # in separate processes: its assembly takes ~0.4 s per problem)
    import multiprocessing as mp
    import os

    from tests.oracle_batch import check_problem
    v = uniform_pm1(B.total, 68)
    vd = to_dev(v)
    yb = to_host(B.matvec(vd))
    sb = to_host(B.prec_apply(vd))
    xh = to_host(x)
    jobs = [(nel[i], int(p[i]), float(kappa[i]), v[off[i]:off[i + 1]], yb[off[i]:off[i + 1]], sb[off[i]:off[i + 1]],
             b[off[i]:off[i + 1]], xh[off[i]:off[i + 1]]) for i in range(len(probs))]
    workers = max(1, min(16, os.cpu_count() or 1))
    # one BLAS thread per worker (the workers start with this environment):
    # a worker pool of multi-threaded BLAS libraries oversubscribes the cores
    blas = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in blas}
    os.environ.update({k: "1" for k in blas})
    try:
        pool = mp.get_context("spawn").Pool(workers)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    res = []
    with pool:
        for r in pool.imap(check_problem, jobs, chunksize=2):
            res.append(r)
            if len(res) % 32 == 0:
                print(f"oracle checks: {len(res)} of {len(jobs)} problems", flush=True)
    worst = {k: max(r[k] for r in res) for k in ("matvec", "fd_backward", "true_relres")}
    fwd = max(r["fd_forward"] / r["fd_bound"] for r in res)
    print(f"256 problems vs oracle: matvec {worst['matvec']:.2e}, FD backward {worst['fd_backward']:.2e}, "
          f"FD forward / bound {fwd:.2e}, true relres {worst['true_relres']:.2e}", flush=True)
    for i, r in enumerate(res):
        assert r["matvec"] < 1e-13, (i, r)
        assert r["fd_backward"] < 1e-14, (i, r)
        assert r["fd_forward"] < max(1e-12, r["fd_bound"]), (i, r)
        assert r["true_relres"] < 2e-8, (i, r)
    # batch invariant on sampled problems: standalone solves agree
    for i in (0, 97, 255):
        knots, degs, kap = probs[i]
        S = stls.Solver(knots, degs, kappa=kap)
        xs, it_s, _ = S.solve(bt[off[i]:off[i + 1]].contiguous(), rtol=1e-8)
        assert abs(its[i] - it_s) <= 1
        assert rel_err(to_host(x[off[i]:off[i + 1]]), to_host(xs)) < 1e-6


@pytest.mark.parametrize("full", [False, True])
def test_graph_replay_matches_direct_launches(full):
    """The batched solve replays one captured iteration as a hipGraph.  It
    must give exactly (bitwise) what direct launches of the same kernels
    give, on repeated solves with eager batch work between them."""
    import time

    import torch
    if full:
        nel, p, kappa = batch_params()
        probs = [(*batch_problem_knots(nel[i], p[i]), float(kappa[i])) for i in range(len(p))]
        B = stls.Batch(probs)
    else:
        B, probs = _batch(SMALL)
    b = to_dev(uniform_pm1(B.total, 63))
    B.set_graph(False)
    torch.cuda.synchronize()
    t = time.perf_counter()
    x0, its0, rel0 = B.solve(b, rtol=1e-8, maxit=500)
    torch.cuda.synchronize()
    t_direct = time.perf_counter() - t
    assert not B.graph_used
    x0 = to_host(x0)
    B.set_graph(True)
    for rep in range(2):
        y = B.matvec(b)  # eager work between the graph solves
        torch.cuda.synchronize()
        t = time.perf_counter()
        x1, its1, rel1 = B.solve(b, rtol=1e-8, maxit=500)
        torch.cuda.synchronize()
        t_graph = time.perf_counter() - t
        assert B.graph_used  # the captured iteration was replayed
        assert its1 == its0 and rel1 == rel0
        assert np.array_equal(to_host(x1), x0)
        assert np.isfinite(to_host(y)).all()
    print(f"{len(probs)} problems, {max(its0)} iterations: direct {t_direct * 1e3:.1f} ms, graph {t_graph * 1e3:.1f} ms",
          flush=True)


def test_degree_six_batch_matches_single_problems():
    """d = 2 batch with the largest supported degree (p = 6) next to p = 2:
    the p = 6 instances of the inner and outer matvec stages and of the FD
    kernels against the standalone operators and solves."""
    specs = [((9, 8, 10), 6, 0.8), ((7, 12, 5), 2, 1.9), ((5, 6, 4), 6, 3.0)]
    B, probs = _batch(specs)
    off = B.offsets
    x = to_dev(uniform_pm1(B.total, 66))
    y = B.matvec(x)
    s = B.prec_apply(x)
    b = to_dev(uniform_pm1(B.total, 67))
    xb, its, rels = B.solve(b, rtol=1e-8, maxit=300)
    assert all(r <= 1e-8 for r in rels)
    for i in range(len(probs)):
        S = _single(B, i, probs)
        xi = x[off[i]:off[i + 1]].contiguous()
        assert rel_err(to_host(y[off[i]:off[i + 1]]), to_host(S.matvec(xi))) < 1e-13
        assert rel_err(to_host(s[off[i]:off[i + 1]]), to_host(S.prec_apply(xi))) < 1e-12
        xs, it_s, _ = S.solve(b[off[i]:off[i + 1]].contiguous(), rtol=1e-8)
        assert abs(its[i] - it_s) <= 1
        assert rel_err(to_host(xb[off[i]:off[i + 1]]), to_host(xs)) < 1e-7
