"""GPU parity of the differentiation operators and the adjoint gradient.

Operators (load, transpose, mass, d/dkappa): sums of banded Kronecker
products evaluated in a different order than the oracle: <= 1e-12 relative.
Gradients: GPU solves to rtol 1e-12 against dense oracle solves, <= 1e-8
relative at the small size.  At the differentiation workload's full size the
gradient is checked by central differences (step 1e-6, solves to rtol 1e-13,
the loss is quadratic in f so the difference is exact up to rounding, and
the loss difference is formed without cancellation) to 1e-6 relative.
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
    assert rel_err(to_host(q), 2.0 * Me) < 1e-12  # the loss's gradient with respect to u
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

    Central differences with step 1e-6 on the forcing (along a seeded
    direction) and on kappa, each within 1e-6 relative of the adjoint
    gradient (step 1e-4 on the forcing as well).  The misfit is exactly
    quadratic in f, so the difference quotient is exact up to rounding; two
    sources of cancellation are avoided.  (1) L(f+hd) - L(f-hd) is formed as
    (u+ - u-)^T M_Q (u+ + u- - 2u*) (M_Q symmetric).  (2) u+ - u- is ~1e-6
    of u while an independent solve of u+ carries ~1e-13 of u, so u- is
    refined by one correction solve (its own error would otherwise enter
    L-), u+ is obtained from u- by another, u+ = u- + A^-1 (F+ - A u-), and
    u+ - u- is that correction itself (all solves to rtol 1e-13)."""
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

    def pair(fm, km, fp, kp):
        """u- = u(fm, km), refined once, and the correction u+ - u- towards u(fp, kp)."""
        S.set_kappa(km)
        Fm = S.load_apply(fm)
        um, _, _ = S.solve(Fm, rtol=rtol)
        dm, _, _ = S.solve(Fm - S.matvec(um), rtol=rtol)
        um = um + dm
        S.set_kappa(kp)
        r0 = S.load_apply(fp) - S.matvec(um)
        du, _, _ = S.solve(r0, rtol=rtol)
        S.set_kappa(1.0)
        return um, du

    def loss_difference(um, du):
        # L+ - L- = (u+ - u-)^T M_Q (u+ + u- - 2 u*) with library mass and dot
        return S.dot(du, S.mass_apply((2.0 * um + du - 2.0 * ustar).contiguous()))

    with torch.no_grad():
        for h in (1e-4, 1e-6):
            um, du = pair(f.detach() - h * direction, 1.0, f.detach() + h * direction, 1.0)
            fd = loss_difference(um, du) / (2 * h)
            print(f"f-gradient step {h:g}: adjoint {g_dir:.15e} central {fd:.15e} "
                  f"rel {abs(g_dir - fd) / abs(fd):.2e}", flush=True)
            assert abs(g_dir - fd) <= 1e-6 * abs(fd), (h, g_dir, fd)
        h = 1e-6
        um, du = pair(f.detach(), 1.0 - h, f.detach(), 1.0 + h)
        fdk = loss_difference(um, du) / (2 * h)
        print(f"kappa-gradient step {h:g}: adjoint {float(kt.grad):.15e} central {fdk:.15e} "
              f"rel {abs(float(kt.grad) - fdk) / abs(fdk):.2e}", flush=True)
        assert abs(float(kt.grad) - fdk) <= 1e-6 * abs(fdk)
