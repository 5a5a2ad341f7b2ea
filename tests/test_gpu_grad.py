"""GPU parity of the differentiation operators and the adjoint gradient.

Operators (load, transpose, mass, d/dkappa): sums of banded Kronecker
products evaluated in a different order than the oracle: <= 1e-12 relative.
Gradients: GPU solves to rtol 1e-12 against dense oracle solves, <= 1e-8
relative at the small size.  At the differentiation workload's full size the
gradient is checked by central differences (step 1e-6, solves to rtol 1e-12,
the loss is quadratic in f so the difference is exact up to rounding) to
1e-6 relative.
"""
import numpy as np
import pytest

from stls_inputs import problem_knots, uniform_pm1

pytestmark = pytest.mark.gpu

try:
    import paper_1809_10026_amd as stls
    from paper_1809_10026_amd import autograd as sag
except ImportError:
    stls = None

from oracle import grad as ograd, system as osys  # noqa: E402
from tests.gpu_util import rel_err, to_dev, to_host  # noqa: E402

CASES = [(1, 6, 2, 1.0), (2, 5, 3, 0.8), (2, 9, 2, 2.0), (3, 3, 3, 1.0)]


def _setup(d, nel, p, kappa):
    assert stls is not None, "libstls.so is not built"
    knots, degs = problem_knots(d, nel, p)
    S = stls.Solver(knots, degs, kappa=kappa)
    P = osys.Problem(knots, degs, kappa=kappa)
    return S, P, ograd.Misfit(P)


@pytest.mark.parametrize("d,nel,p,kappa", CASES)
def test_forcing_shape_and_load_operators(d, nel, p, kappa):
    S, P, G = _setup(d, nel, p, kappa)
    m, nf = S.forcing_shape
    assert m == G.fshape and nf == int(np.prod(G.fshape))
    f = uniform_pm1(nf, 31)
    F = to_host(S.load_apply(to_dev(f)))
    assert rel_err(F, osys.vec(G.load_apply(f))) < 1e-12
    lam = uniform_pm1(P.ndof, 32)
    gf = to_host(S.load_apply_T(to_dev(lam)))
    assert rel_err(gf, G.load_apply_T(lam).ravel(order="F")) < 1e-12
    x = uniform_pm1(P.ndof, 33)
    assert rel_err(to_host(S.mass_apply(to_dev(x))), osys.vec(G.mass_apply(x))) < 1e-12


@pytest.mark.parametrize("d,nel,p,kappa", CASES)
def test_dkappa_and_misfit(d, nel, p, kappa):
    S, P, G = _setup(d, nel, p, kappa)
    nf = S.forcing_shape[1]
    f, u, lam = uniform_pm1(nf, 41), uniform_pm1(P.ndof, 42), uniform_pm1(P.ndof, 43)
    fd, ud, ld = to_dev(f), to_dev(u), to_dev(lam)
    dk = S.dkappa(fd, ud, ld)
    ref = float(lam @ (G.dF_dkappa(f).ravel(order="F") - G.dA_dkappa_apply(u).ravel(order="F")))
    assert abs(dk - ref) <= 1e-11 * max(abs(ref), 1.0)
    # the same entry point under its second name: bit-identical
    import ctypes
    out = ctypes.c_double()
    assert stls._lib.stls_dkappa_terms(S._h, ctypes.c_void_p(fd.data_ptr()), ctypes.c_void_p(ud.data_ptr()),
                                       ctypes.c_void_p(ld.data_ptr()), ctypes.byref(out)) == 0
    assert out.value == dk
    us = uniform_pm1(P.ndof, 44)
    loss, q = S.misfit(to_dev(u), to_dev(us))
    e = u - us
    Me = osys.vec(G.mass_apply(e))
    assert abs(loss - e @ Me) <= 1e-12 * abs(e @ Me)
    assert rel_err(to_host(q), Me) < 1e-12
    assert abs(S.dot(to_dev(u), to_dev(lam)) - u @ lam) <= 1e-12 * np.abs(u).sum()


@pytest.mark.parametrize("d,nel,p,kappa", [(2, 6, 3, 1.0), (1, 10, 3, 0.5)])
def test_autograd_matches_oracle_dense_gradient(d, nel, p, kappa):
    import torch
    S, P, G = _setup(d, nel, p, kappa)
    nf = S.forcing_shape[1]
    f = uniform_pm1(nf, 51)
    ustar = 0.2 * uniform_pm1(P.ndof, 52)
    A = P.dense_A()
    L_ref, gf_ref, dk_ref, _ = G.loss_and_grad(f, ustar, lambda b: np.linalg.solve(A, b))
    ft = to_dev(f).requires_grad_(True)
    kt = torch.tensor(kappa, dtype=torch.float64, device="cuda", requires_grad=True)
    u = sag.heat_solve(ft, kt, S, rtol=1e-13)
    L = sag.misfit(u, to_dev(ustar), S)
    L.backward()
    assert abs(L.item() - L_ref) <= 1e-9 * abs(L_ref)
    assert rel_err(to_host(ft.grad), gf_ref.ravel(order="F")) < 1e-8
    assert abs(float(kt.grad) - dk_ref) <= 1e-8 * abs(dk_ref)


def test_gradient_central_differences_full_size():
    """d = 2, p = 3, 128 elements per direction (ndof 2,163,330; forcing 131^3).

    kappa: central difference with step 1e-6, <= 1e-6 relative.
    f: the misfit is exactly quadratic in f, so a central difference is exact
    at any step and only rounding limits it.  The loss carries about 1e-13
    relative FP64 rounding (solves at the 1e-15 residual floor, cancellation
    in u - u*); with step 1e-6 the loss changes by only ~1e-7 relative, so
    that step is checked against 1e-5, and step 1e-4 against 1e-6."""
    import torch
    knots, degs = problem_knots(2, 128, 3)
    S = stls.Solver(knots, degs, kappa=1.0)
    m, nf = S.forcing_shape
    assert nf == 131 ** 3 and S.ndof == 129 * 129 * 130
    rtol = 1e-13
    fstar = to_dev(uniform_pm1(nf, 6))
    kappa1 = torch.tensor(1.0, dtype=torch.float64, device="cuda")
    ustar = sag.heat_solve(fstar, kappa1, S, rtol=rtol).detach()
    f = to_dev(uniform_pm1(nf, 5)).requires_grad_(True)
    kt = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    L = sag.misfit(sag.heat_solve(f, kt, S, rtol=rtol), ustar, S)
    L.backward()
    direction = to_dev(uniform_pm1(nf, 7))
    g_dir = float(torch.dot(f.grad, direction))

    def loss(fv, kv):
        with torch.no_grad():
            u = sag.heat_solve(fv, torch.tensor(kv, dtype=torch.float64, device="cuda"), S, rtol=rtol)
            return float(sag.misfit(u, ustar, S))

    for h, tol in ((1e-4, 1e-6), (1e-6, 1e-5)):
        fd = (loss(f.detach() + h * direction, 1.0) - loss(f.detach() - h * direction, 1.0)) / (2 * h)
        assert abs(g_dir - fd) <= tol * abs(fd), (h, g_dir, fd)
    h = 1e-6
    fdk = (loss(f.detach(), 1.0 + h) - loss(f.detach(), 1.0 - h)) / (2 * h)
    assert abs(float(kt.grad) - fdk) <= 1e-6 * abs(fdk)
