"""Batch autotuner and the tuning it sets (work-item shapes and launch
geometry of the batched kernels, PCG iterations per graph launch).

Invariants: the batched matvec and FD application do not depend on the
tuning at all (bit for bit: every output entry is computed by the same
arithmetic in the same order, only the assignment of entries to work items
changes); solves differ only through the order of the dot products' partial
sums, so iteration counts agree within one and solutions to the solve
tolerance; the graph depth changes nothing (bit for bit), and maxit is never
exceeded.  The autotuner's choice is valid, stored in its JSON cache and
reused from it without measuring.
"""
import json

import numpy as np
import pytest

from stls_inputs import problem_knots, uniform_pm1

pytestmark = pytest.mark.gpu

try:
    import paper_1809_10026_amd as stls
except ImportError:
    stls = None

from tests.gpu_util import rel_err, to_dev, to_host  # noqa: E402

SPECS = [((7, 9, 8), 2, 0.3), ((12, 5, 10), 3, 1.0), ((6, 6, 13), 4, 5.0), ((9, 11, 7), 5, 0.12),
         ((16, 18, 17), 3, 2.2), ((30, 21, 40), 2, 0.7)]

ODD = {"vec_chunk": 1024, "inner_steps": 3, "outer_chunk": 7, "grid_fd": 5, "grid_inner": 3, "grid_outer": 11,
       "grid_vec": 2, "graph_depth": 1}


def _batch():
    assert stls is not None, "libstls.so is not built"
    probs = [(*problem_knots(2, list(nel), p), kappa) for nel, p, kappa in SPECS]
    return stls.Batch(probs)


def test_operators_do_not_depend_on_the_tuning():
    B = _batch()
    x = to_dev(uniform_pm1(B.total, 71))
    y0, s0 = to_host(B.matvec(x)), to_host(B.prec_apply(x))
    default = B.tuning
    B.tuning = ODD
    assert B.tuning == ODD
    y1, s1 = to_host(B.matvec(x)), to_host(B.prec_apply(x))
    assert np.array_equal(y0, y1) and np.array_equal(s0, s1)
    b = to_dev(uniform_pm1(B.total, 72))
    xo, it1, rel1 = B.solve(b, rtol=1e-9)
    B.tuning = default
    xd, it0, rel0 = B.solve(b, rtol=1e-9)
    assert max(rel1) <= 1e-9 and max(rel0) <= 1e-9
    assert all(abs(a - c) <= 1 for a, c in zip(it0, it1))
    off = B.offsets
    for i in range(len(SPECS)):
        assert rel_err(to_host(xo[off[i]:off[i + 1]]), to_host(xd[off[i]:off[i + 1]])) < 1e-7


@pytest.mark.parametrize("depth", [2, 4, 7])
def test_graph_depth_gives_the_same_solve(depth):
    B = _batch()
    b = to_dev(uniform_pm1(B.total, 73))
    x1, it1, rel1 = B.solve(b, rtol=1e-9)
    x1 = to_host(x1)
    B.tuning = {"graph_depth": depth}
    xk, itk, relk = B.solve(b, rtol=1e-9)
    assert B.graph_used
    assert itk == it1 and relk == rel1 and np.array_equal(to_host(xk), x1)
    # maxit is honoured exactly although a graph launch covers several iterations
    _, its, _ = B.solve(b, rtol=1e-14, maxit=depth + 2, raise_on_noconv=False)
    assert max(its) == depth + 2


def test_invalid_tuning_is_refused():
    B = _batch()
    before = B.tuning
    for bad in ({"vec_chunk": 1000}, {"inner_steps": 0}, {"graph_depth": 65}, {"grid_fd": 0}):
        with pytest.raises(stls.StlsError) as ei:
            B.tuning = bad
        assert ei.value.status == stls.STLS_EINVAL
    assert B.tuning == before


def test_autotune_measures_caches_and_reuses(tmp_path):
    cache = tmp_path / "tune.json"
    B = _batch()
    b = to_dev(uniform_pm1(B.total, 74))
    xd, itd, _ = B.solve(b, rtol=1e-9)
    xd = to_host(xd)
    assert B.autotune(str(cache)) is True
    chosen = B.tuning
    data = json.loads(cache.read_text())
    assert len(data) == 1
    (key, entry), = data.items()
    assert entry == chosen
    print(f"autotuned {key}: {chosen}", flush=True)
    xt, itt, relt = B.solve(b, rtol=1e-9)
    assert max(relt) <= 1e-9 and all(abs(a - c) <= 1 for a, c in zip(itd, itt))
    off = B.offsets
    for i in range(len(SPECS)):
        assert rel_err(to_host(xt[off[i]:off[i + 1]]), xd[off[i]:off[i + 1]]) < 1e-7
    # a second batch of the same problems takes the stored choice without timing
    B2 = _batch()
    assert B2.autotune(str(cache)) is False
    assert B2.tuning == chosen
    # a different problem set gets its own entry
    B3 = stls.Batch([(*problem_knots(2, [8, 8, 8], 3), 1.0)])
    assert B3.autotune(str(cache)) is True
    assert len(json.loads(cache.read_text())) == 2
