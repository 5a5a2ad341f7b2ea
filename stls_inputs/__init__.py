"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module holds no arithmetic of the method: it only draws the data a
user of the solver would hand over (knot vectors, degrees, diffusivities,
right-hand sides, forcing coefficients).  Random tensors are generated with
``numpy.random.default_rng(seed)`` and flattened in colexicographic order
(first space index fastest, time index slowest; Fortran order of the shape
``(n_1, ..., n_d, n_t)``), the ordering of the paper's vec operator (§4,
eq. kron_vec_multi).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "uniform_open_knots",
    "graded_open_knots",
    "problem_knots",
    "uniform_pm1",
    "CONFIGS",
    "batch_params",
    "batch_problem_knots",
]


def uniform_open_knots(n_el: int, p: int) -> np.ndarray:
    """Open uniform knot vector on [0, 1] with ``n_el`` elements (§2.1).

    The first and last ``p + 1`` knots are 0 and 1; interior knot ``i`` is
    the single correctly rounded IEEE division ``i / n_el`` (never an
    accumulated step), so every consumer gets byte-identical knots.
    Simple interior knots give C^{p-1} splines.
    """
    if n_el < 1 or p < 0:
        raise ValueError("n_el >= 1 and p >= 0 required")
    inner = [float(i) / float(n_el) for i in range(1, n_el)]
    return np.array([0.0] * (p + 1) + inner + [1.0] * (p + 1), dtype=np.float64)


def graded_open_knots(n_el: int, p: int, mult: int = 1, seed: int = 0) -> np.ndarray:
    """Open knot vector on [0, 1] with ``n_el`` non-empty elements of uneven
    length and one interior knot of multiplicity ``mult`` (§2.1: the
    regularity at a knot is p minus its multiplicity).

    Element lengths are drawn from U[0.4, 1.6] with ``default_rng(seed)``
    and normalised to sum to one; the breakpoints are their cumulative sums
    (the last one set to 1 exactly).  The interior breakpoint nearest to the
    middle is repeated ``mult`` times.
    """
    if n_el < 2 or p < 0 or mult < 1:
        raise ValueError("n_el >= 2, p >= 0 and mult >= 1 required")
    rng = np.random.default_rng(seed)
    h = rng.uniform(0.4, 1.6, size=n_el)
    b = np.cumsum(h / h.sum())
    b[-1] = 1.0
    inner = [float(v) for v in b[:-1]]
    mid = n_el // 2 - 1
    inner = inner[:mid] + [inner[mid]] * mult + inner[mid + 1:]
    return np.array([0.0] * (p + 1) + inner + [1.0] * (p + 1), dtype=np.float64)


def problem_knots(d: int, n_el, p):
    """Knot vectors and degrees for a unit box in space times (0, 1).

    ``n_el`` and ``p`` are either scalars (same in every direction) or
    sequences of length d + 1 with time last.  Returns (knots, degrees).
    """
    n_el = [int(n_el)] * (d + 1) if np.isscalar(n_el) else [int(v) for v in n_el]
    p = [int(p)] * (d + 1) if np.isscalar(p) else [int(v) for v in p]
    if len(n_el) != d + 1 or len(p) != d + 1:
        raise ValueError("need d + 1 entries (space directions, then time)")
    return [uniform_open_knots(e, q) for e, q in zip(n_el, p)], p


def uniform_pm1(n: int, seed: int) -> np.ndarray:
    """``n`` i.i.d. uniform[-1, 1] FP64 values from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=int(n))


# Workload shapes of the paper-sized configurations (unit box, T = 1,
# p_s = p_t = p, uniform open knots, homogeneous data).
CONFIGS = {
    "d1_p2_nel32_manufactured": dict(d=1, n_el=32, p=2, rtol=1e-10),
    "d2_p3_nel64": dict(d=2, n_el=64, p=3, rtol=1e-8, seed=1809),
    "d3_p4_nel48": dict(d=3, n_el=48, p=4, rtol=1e-8, seed=10026),
    "d2_p3_nel128_gradient": dict(d=2, n_el=128, p=3, rtol=1e-8, seed_f=5, seed_target=6, seed_dir=7),
}


def batch_params(nprob: int = 256, seed: int = 20180926):
    """Uneven batch of 2-D-space heat problems.

    Draw order from one generator: ``nel`` of shape (nprob, 3) uniform on
    16..96 (x, y, t drawn independently), ``p`` of shape (nprob,) uniform on
    {2, 3, 4, 5} (one degree per problem), ``logk`` of shape (nprob,)
    uniform on [-1, 1] with kappa = 10**logk (log-uniform in [0.1, 10]).
    The right-hand side of problem i is drawn with seed ``seed + 1 + i``.
    """
    rng = np.random.default_rng(seed)
    nel = rng.integers(16, 97, size=(nprob, 3))
    p = rng.integers(2, 6, size=nprob)
    logk = rng.uniform(-1.0, 1.0, size=nprob)
    return nel, p, 10.0 ** logk


def batch_problem_knots(nel_row, p):
    """Knots and degrees of one batch problem (d = 2, time last)."""
    return problem_knots(2, [int(v) for v in nel_row], int(p))
