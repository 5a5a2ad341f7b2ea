"""Mapped spatial domains and the geometry-aware preconditioner (§2.2
isoparametric spaces, §4.1, §4.4, Appendix A.3 Algorithm 2, §5.1-5.2).
Oracle: test use only.

The spatial domain is Omega = G((0,1)^d) for a smooth map G; the discrete
functions are the restricted tensor B-splines composed with G^{-1}.  With
kappa and T = 1 the least-squares matrix keeps its time Kronecker structure
(the cross terms integrate by parts in time and space exactly as on the
unit box, since every trial function vanishes on the spatial boundary):

    A = K_t (x) M_s + kappa^2 M_t (x) J_s + kappa W_t (x) L_s,
    M_s = int_Omega B_i B_j,  L_s = int_Omega grad B_i . grad B_j,
    J_s = int_Omega Lap B_i Lap B_j,

but the spatial factors are no longer Kronecker products.  They are
assembled here by tensor Gauss quadrature in the parametric domain, p + 3
points per non-empty span (the integrands are not polynomial), with the
physical derivatives of a pulled-back function v = v^ o G^{-1}:

    grad v = J^{-T} grad_eta v^,
    Lap v  = sum_ab g^{ab} d_a d_b v^ + sum_j (Lap eta_j) d_j v^,

g^{ab} = grad eta_a . grad eta_b (rows of J^{-1}), and the Laplacian of the
coordinate functions Lap eta_j = -sum_ab g^{ab} [J^{-1} d_a d_b G]_j.

Preconditioners on a mapped domain (§4.4):
  P    the unit-box preconditioner of §4.2 built from the parametric
       matrices (it ignores G);
  Pbar^G = Khat^G_t (x) Mhat^G_s + kappa^2 Mhat^G_t (x) Jtilde^G_s, the
       univariate matrices weighted by the separable approximations mu_k,
       omega_k of the coefficients c_k (eq. coefficients-c) interpolated at
       the element barycentres, computed by Algorithm 2 with maxit = 2;
  P^G  = D^{1/2} Pbar^G D^{1/2}, D = diag(A) / diag(Pbar^G).
"""
from __future__ import annotations

from types import SimpleNamespace

import numpy as np
import scipy.sparse as sp

from .assemble import gauss_points, space_index, time_matrices
from .bspline import eval_basis_points, nonempty_spans, num_basis
from .fd import FD

# ---------------------------------------------------------------------------
# maps


class IdentityMap:
    """G(eta) = eta: the unit box itself."""

    def __init__(self, d):
        self.d = d

    def __call__(self, eta):
        return np.asarray(eta, dtype=np.float64)

    def jacobian(self, eta):
        n = np.asarray(eta).shape[0]
        return np.broadcast_to(np.eye(self.d), (n, self.d, self.d)).copy()

    def hessian(self, eta):
        n = np.asarray(eta).shape[0]
        return np.zeros((n, self.d, self.d, self.d))


class QuarterAnnulus:
    """Quarter of the annulus 1 < r < 2 in the first quadrant (§5.1):
    x = r cos(theta), y = r sin(theta), r = 1 + eta_1, theta = (pi/2) eta_2."""

    d = 2
    A = np.pi / 2

    def _polar(self, eta):
        eta = np.asarray(eta, dtype=np.float64)
        return 1.0 + eta[:, 0], self.A * eta[:, 1]

    def __call__(self, eta):
        r, th = self._polar(eta)
        return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)

    def jacobian(self, eta):
        r, th = self._polar(eta)
        c, s, A = np.cos(th), np.sin(th), self.A
        J = np.empty((len(r), 2, 2))
        J[:, 0, 0], J[:, 0, 1] = c, -A * r * s
        J[:, 1, 0], J[:, 1, 1] = s, A * r * c
        return J

    def hessian(self, eta):
        r, th = self._polar(eta)
        c, s, A = np.cos(th), np.sin(th), self.A
        H = np.zeros((len(r), 2, 2, 2))  # H[:, i, a, b] = d^2 x_i / d eta_a d eta_b
        H[:, 0, 0, 1] = H[:, 0, 1, 0] = -A * s
        H[:, 0, 1, 1] = -A * A * r * c
        H[:, 1, 0, 1] = H[:, 1, 1, 0] = A * c
        H[:, 1, 1, 1] = -A * A * r * s
        return H


class RotatedQuarterAnnulus:
    """The quarter annulus of the (x, y) plane revolved by pi/2 about the
    line y = -1, z = 0 (§5.2): with (x0, y0) the quarter-annulus point of
    (eta_1, eta_2), rho = y0 + 1 and phi = (pi/2) eta_3,
    x = x0, y = -1 + rho cos(phi), z = rho sin(phi)."""

    d = 3
    A = np.pi / 2

    def __init__(self):
        self.base = QuarterAnnulus()

    def __call__(self, eta):
        eta = np.asarray(eta, dtype=np.float64)
        p0 = self.base(eta[:, :2])
        rho, ph = p0[:, 1] + 1.0, self.A * eta[:, 2]
        return np.stack([p0[:, 0], -1.0 + rho * np.cos(ph), rho * np.sin(ph)], axis=1)

    def jacobian(self, eta):
        eta = np.asarray(eta, dtype=np.float64)
        p0 = self.base(eta[:, :2])
        J0 = self.base.jacobian(eta[:, :2])
        rho, ph, A = p0[:, 1] + 1.0, self.A * eta[:, 2], self.A
        c, s = np.cos(ph), np.sin(ph)
        J = np.zeros((len(rho), 3, 3))
        J[:, 0, :2] = J0[:, 0, :]
        J[:, 1, :2] = J0[:, 1, :] * c[:, None]
        J[:, 2, :2] = J0[:, 1, :] * s[:, None]
        J[:, 1, 2] = -A * rho * s
        J[:, 2, 2] = A * rho * c
        return J

    def hessian(self, eta):
        eta = np.asarray(eta, dtype=np.float64)
        p0 = self.base(eta[:, :2])
        J0 = self.base.jacobian(eta[:, :2])
        H0 = self.base.hessian(eta[:, :2])
        rho, ph, A = p0[:, 1] + 1.0, self.A * eta[:, 2], self.A
        c, s = np.cos(ph), np.sin(ph)
        H = np.zeros((len(rho), 3, 3, 3))
        H[:, 0, :2, :2] = H0[:, 0]
        H[:, 1, :2, :2] = H0[:, 1] * c[:, None, None]
        H[:, 2, :2, :2] = H0[:, 1] * s[:, None, None]
        for a in range(2):  # mixed eta_a, eta_3 (rho depends on eta_1, eta_2 through y0)
            H[:, 1, a, 2] = H[:, 1, 2, a] = -A * J0[:, 1, a] * s
            H[:, 2, a, 2] = H[:, 2, 2, a] = A * J0[:, 1, a] * c
        H[:, 1, 2, 2] = -A * A * rho * c
        H[:, 2, 2, 2] = -A * A * rho * s
        return H


def metric_terms(G, eta):
    """|det J|, J^{-1} (rows: grad eta_a), g^{ab} and Lap eta_j at the points."""
    J = G.jacobian(eta)
    H = G.hessian(eta)
    det = np.abs(np.linalg.det(J))
    Jinv = np.linalg.inv(J)  # Jinv[:, a, i] = d eta_a / d x_i
    ginv = np.einsum("pai,pbi->pab", Jinv, Jinv)
    lap_eta = -np.einsum("pab,pji,piab->pj", ginv, Jinv, H)
    return det, Jinv, ginv, lap_eta


def physical_laplacian(ginv, lap_eta, d1, d2):
    """Lap v at points from the parametric derivatives of v^:
    d1[:, a] = d_a v^, d2[:, a, b] = d_a d_b v^."""
    return np.einsum("pab,pab->p", ginv, d2) + np.einsum("pj,pj->p", lap_eta, d1)


# ---------------------------------------------------------------------------
# spatial factors by quadrature


def _tensor_points(knots, degrees, d, nq_extra=3, full=False):
    """Parametric Gauss grid (colex: direction 1 fastest) and the 1-D
    evaluation matrices (values, first, second derivatives) per direction,
    restricted to the Dirichlet space unless ``full``."""
    pts, wts, E = [], [], []
    for k in range(d):
        x, w = gauss_points(knots[k], degrees[k] + nq_extra)
        B = eval_basis_points(knots[k], degrees[k], x, nder=2)
        m = num_basis(knots[k], degrees[k])
        idx = np.arange(m) if full else space_index(m)
        pts.append(x)
        wts.append(w)
        E.append([sp.csr_matrix(B[r][:, idx]) for r in range(3)])
    grid = np.stack([g.ravel(order="F") for g in np.meshgrid(*pts, indexing="ij")], axis=1)
    w = wts[0]
    for wk in wts[1:]:
        w = np.multiply.outer(w, wk)
    return grid, w.ravel(order="F"), E


def _kron_eval(E, orders):
    """Evaluation matrix of prod_k b^{(orders[k])}(eta_k) on the colex grid:
    E_d (x) ... (x) E_1 (the first Kronecker argument is the slowest)."""
    out = E[0][orders[0]]
    for k in range(1, len(E)):
        out = sp.kron(E[k][orders[k]], out, format="csr")
    return out


def spatial_factors(G, knots, degrees, full=False):
    """M_s, L_s, J_s on Omega = G((0,1)^d) as sparse matrices over the
    restricted tensor basis (colex), by p + 3 Gauss points per span."""
    d = G.d
    grid, w, E = _tensor_points(knots, degrees, d, full=full)
    det, Jinv, ginv, lap_eta = metric_terms(G, grid)
    wd = w * det
    phi = _kron_eval(E, [0] * d)
    d1 = [_kron_eval(E, [1 if l == a else 0 for l in range(d)]) for a in range(d)]
    d2 = [[_kron_eval(E, [(1 if l == a else 0) + (1 if l == b else 0) for l in range(d)]) for b in range(d)]
          for a in range(d)]
    M = (phi.T @ sp.diags(wd) @ phi).tocsr()
    L = sum(d1[a].T @ sp.diags(wd * ginv[:, a, b]) @ d1[b] for a in range(d) for b in range(d)).tocsr()
    lap = sum(sp.diags(ginv[:, a, b]) @ d2[a][b] for a in range(d) for b in range(d))
    lap = (lap + sum(sp.diags(lap_eta[:, j]) @ d1[j] for j in range(d))).tocsr()
    J = (lap.T @ sp.diags(wd) @ lap).tocsr()
    return dict(M=M, L=L, J=J, lap=lap, phi=phi, d1=d1, grid=grid, w=w, det=det, ginv=ginv)


# ---------------------------------------------------------------------------
# coefficients and Algorithm 2


def element_coefficients(G, knots, degrees, T=1.0):
    """c_1..c_{d+1} (eq. coefficients-c) at the element barycentres, as
    tensors over the elements (space directions, then time).

    c_k = |grad eta_k|^4 |det J| T for k <= d, c_{d+1} = |det J| / T.  The
    paper writes the k-th column of J_F^{-1}; read here as the gradient of
    eta_k (row k of d eta / d x), the factor of d^2/d eta_k^2 in the pulled
    back Laplacian whose square times |det J| T multiplies the pure second
    derivatives in K_{s,1}."""
    d = G.d
    mids = [np.array([(a + b) / 2 for a, b in nonempty_spans(knots[k])]) for k in range(d)]
    ne_t = len(nonempty_spans(knots[d]))
    grid = np.stack([g.ravel(order="F") for g in np.meshgrid(*mids, indexing="ij")], axis=1)
    det, _, ginv, _ = metric_terms(G, grid)
    shape = tuple(len(m) for m in mids)
    cs = []
    for k in range(d):
        ck = (ginv[:, k, k] ** 2) * det * T
        cs.append(np.repeat(ck.reshape(shape, order="F")[..., None], ne_t, axis=d))
    cs.append(np.repeat((det / T).reshape(shape, order="F")[..., None], ne_t, axis=d))
    return cs


def separate_variables(C, maxit=2):
    """Separable approximations of positive tensors (Appendix A.3, Algorithm 2):
        C^(k) ~ mu^(1) ... mu^(k-1) omega^(k) mu^(k+1) ... mu^(D),
    balancing min and max of C^(k) / approximation around 1 in the log sense.

    Each sweep sets every omega^(k)_j to the geometric midpoint of the values
    that C^(k) implies for it over the slice i_k = j (the other factors
    fixed), then every mu^(k)_j, in turn, to the geometric midpoint of the
    values that the equations l != k imply for it over the slice i_k = j.
    The listing's W^(k,l) carries the indices of these two roles the other
    way round; read as stated here, the two-variable case decouples into
    independent problems as the appendix says.  Returns (mu, omega)."""
    D = len(C)
    shape = C[0].shape
    mu = [np.ones(shape[l]) for l in range(D)]
    om = [np.ones(shape[l]) for l in range(D)]

    def along(v, l):
        s = [1] * D
        s[l] = len(v)
        return v.reshape(s)

    def slice_minmax(X, k, lo_of, hi_of):
        ax = tuple(a for a in range(D) if a != k)
        return lo_of(X, axis=ax), hi_of(X, axis=ax)

    for _ in range(maxit):
        for k in range(D):
            V = C[k].copy()
            for l in range(D):
                if l != k:
                    V = V / along(mu[l], l)
            m, M = slice_minmax(V, k, np.min, np.max)
            om[k] = np.sqrt(m * M)
        for k in range(D):
            implied = []
            for l in range(D):
                if l == k:
                    continue
                # equation l implies mu^(k) = C^(l) / (omega^(l) prod_{j != k, l} mu^(j))
                V = C[l] / along(om[l], l)
                for j in range(D):
                    if j != k and j != l:
                        V = V / along(mu[j], j)
                implied.append(V)
            Y = np.minimum.reduce(implied)
            Z = np.maximum.reduce(implied)
            m, _ = slice_minmax(Y, k, np.min, np.max)
            _, M = slice_minmax(Z, k, np.min, np.max)
            mu[k] = np.sqrt(m * M)
    return mu, om


def separation_quality(C, mu, om):
    """max over k and entries of |log(C^(k) / approximation)| (the
    functional that Algorithm 2 decreases)."""
    D = len(C)
    worst = 0.0
    for k in range(D):
        approx = np.ones(C[k].shape)
        for l in range(D):
            s = [1] * D
            s[l] = C[k].shape[l]
            approx = approx * (om[l] if l == k else mu[l]).reshape(s)
        worst = max(worst, float(np.max(np.abs(np.log(C[k] / approx)))))
    return worst


# ---------------------------------------------------------------------------
# weighted univariate matrices


def weighted_matrices(xi, p, weight, orders, restrict):
    """int weight(eta) b_i^{(a)} b_j^{(a)} with a piecewise-constant weight
    (one value per non-empty span), p + 1 Gauss points per span (exact)."""
    spans = nonempty_spans(xi)
    t, wq = np.polynomial.legendre.leggauss(p + 1)
    x = np.concatenate([0.5 * (b - a) * t + 0.5 * (a + b) for a, b in spans])
    w = np.concatenate([0.5 * (b - a) * wq * weight[e] for e, (a, b) in enumerate(spans)])
    B = eval_basis_points(xi, p, x, nder=2)
    m = num_basis(xi, p)
    idx = restrict(m)
    return {a: (B[a].T @ (w[:, None] * B[a]))[np.ix_(idx, idx)] for a in orders}


# ---------------------------------------------------------------------------
# the mapped problem


class MappedProblem:
    """Heat problem on G((0,1)^d) x (0, 1) with homogeneous data.

    Attributes follow oracle.system.Problem where they mean the same
    (d, shape, ndof, time, kappa); ``space`` holds the sparse M, L, J."""

    def __init__(self, G, knots, degrees, kappa=1.0):
        self.G, self.knots, self.degrees, self.kappa = G, knots, degrees, float(kappa)
        self.d = G.d
        self.sfac = spatial_factors(G, knots, degrees)
        self.time = time_matrices(knots[self.d], degrees[self.d])
        ns = self.sfac["M"].shape[0]
        self.ns = ns
        self.shape_s = tuple(num_basis(knots[k], degrees[k]) - 2 for k in range(self.d))
        self.shape = self.shape_s + (self.time["M"].shape[0],)

    @property
    def ndof(self):
        return int(np.prod(self.shape))

    def matvec(self, x):
        """A x with x, A x flat (colex: space fastest, time slowest)."""
        X = np.asarray(x).reshape(self.ns, -1, order="F")
        S, Tm, k = self.sfac, self.time, self.kappa
        Y = S["M"] @ X @ Tm["K"].T + k * k * (S["J"] @ X @ Tm["M"].T) + k * (S["L"] @ X @ Tm["W"].T)
        return Y.ravel(order="F")

    def diagonal(self):
        S, Tm, k = self.sfac, self.time, self.kappa
        return (np.multiply.outer(S["M"].diagonal(), np.diag(Tm["K"]))
                + k * k * np.multiply.outer(S["J"].diagonal(), np.diag(Tm["M"]))
                + k * np.multiply.outer(S["L"].diagonal(), np.diag(Tm["W"]))).ravel(order="F")

    def dense_A(self):
        S, Tm, k = self.sfac, self.time, self.kappa
        return (np.kron(Tm["K"], S["M"].toarray()) + k * k * np.kron(Tm["M"], S["J"].toarray())
                + k * np.kron(Tm["W"], S["L"].toarray()))


def _factors(knots, degrees, d, mu=None, om=None, kappa=1.0):
    """Univariate factors of Pbar^G (weights mu, omega per element; None:
    the unweighted parametric matrices, i.e. the plain P), in the form
    oracle.fd.FD reads (space[k]['M'], ['J']; time['Khat'], ['Mhat'])."""
    space = []
    for k in range(d):
        ne = len(nonempty_spans(knots[k]))
        wm = np.ones(ne) if mu is None else mu[k]
        wj = np.ones(ne) if om is None else om[k]
        Mk = weighted_matrices(knots[k], degrees[k], wm, [0], space_index)[0]
        Jk = weighted_matrices(knots[k], degrees[k], wj, [2], space_index)[2]
        space.append({"M": Mk, "J": Jk})
    ne = len(nonempty_spans(knots[d]))
    wm = np.ones(ne) if mu is None else mu[d]
    wk = np.ones(ne) if om is None else om[d]
    tidx = lambda m: np.arange(1, m)
    Mt = weighted_matrices(knots[d], degrees[d], wm, [0], tidx)[0]
    Kt = weighted_matrices(knots[d], degrees[d], wk, [1], tidx)[1]
    shape = tuple(S["M"].shape[0] for S in space) + (Mt.shape[0],)
    return SimpleNamespace(d=d, kappa=kappa, shape=shape, space=space, time={"Khat": Kt, "Mhat": Mt})


def kron_diag(fac):
    """Diagonal of Khat_t (x) Mhat_s + kappa^2 Mhat_t (x) Jtilde_s (colex flat)."""
    d = fac.d
    dm = [np.diag(S["M"]) for S in fac.space]
    dj = [np.diag(S["J"]) for S in fac.space]

    def outer(vs):
        out = vs[0]
        for v in vs[1:]:
            out = np.multiply.outer(out, v)
        return out

    P = outer(dm + [np.diag(fac.time["Khat"])])
    for k in range(d):
        P = P + fac.kappa ** 2 * outer([dj[l] if l == k else dm[l] for l in range(d)] + [np.diag(fac.time["Mhat"])])
    return P.ravel(order="F")


class GeometryPreconditioner:
    """P^G = D^{1/2} Pbar^G D^{1/2} (§4.4) for a MappedProblem; with
    ``geometry=False`` the plain parametric P (no D, unit weights)."""

    def __init__(self, prob, geometry=True, maxit=2):
        d = prob.d
        self.geometry = geometry
        if geometry:
            self.C = element_coefficients(prob.G, prob.knots, prob.degrees)
            self.mu, self.om = separate_variables(self.C, maxit)
            self.fac = _factors(prob.knots, prob.degrees, d, self.mu, self.om, prob.kappa)
            self.D = prob.diagonal() / kron_diag(self.fac)
        else:
            self.fac = _factors(prob.knots, prob.degrees, d, kappa=prob.kappa)
            self.D = None
        self.fd = FD(self.fac)

    def apply_bar(self, r):
        return self.fd.apply(np.asarray(r)).ravel(order="F")

    def apply(self, r):
        r = np.asarray(r, dtype=np.float64)
        if self.D is None:
            return self.apply_bar(r)
        s = 1.0 / np.sqrt(self.D)
        return s * self.apply_bar(s * r)


# ---------------------------------------------------------------------------
# loads and error norms on the mapped domain (§5.1 manufactured solutions)


def mapped_load(prob, terms):
    """F_i = int_0^1 int_Omega f (d_t B_i - kappa Lap B_i) dx dt for
    f(x, t) = sum over ``terms`` of a(x) alpha(t), each term a pair of
    callables (a on physical points of shape (n, d), alpha on times);
    p + 3 Gauss points per span in every direction.  Flat, colex."""
    from .assemble import load_1d, time_index
    S = prob.sfac
    x = prob.G(S["grid"])
    wd = S["w"] * S["det"]
    kt, pt = prob.knots[prob.d], prob.degrees[prob.d]
    it = time_index(num_basis(kt, pt))
    F = np.zeros((prob.ns, len(it)))
    for a, alpha in terms:
        av = a(x) * wd
        sv = S["phi"].T @ av          # int a B_i
        sl = S["lap"].T @ av          # int a Lap B_i
        t1 = load_1d(kt, pt, alpha, 1, it)
        t0 = load_1d(kt, pt, alpha, 0, it)
        F += np.multiply.outer(sv, t1) - prob.kappa * np.multiply.outer(sl, t0)
    return F.ravel(order="F")


def mapped_error_norms(prob, coef, exact):
    """Relative V_0, L^2 and space-time H^1 errors of u_h = sum u_i B_i on
    the mapped domain against ``exact``: dict of callables of (x, t) with x
    of shape (n, d) and t of shape (m,), returning (n, m) arrays: 'u', 'ut',
    'lap', and 'grad' (list of d).  p + 3 Gauss points per span."""
    from .assemble import time_index
    S = prob.sfac
    x = prob.G(S["grid"])
    wd = S["w"] * S["det"]
    kt, pt = prob.knots[prob.d], prob.degrees[prob.d]
    tq, wt = gauss_points(kt, pt + 3)
    Bt = eval_basis_points(kt, pt, tq, nder=1)[:, :, time_index(num_basis(kt, pt))]
    U = np.asarray(coef).reshape(prob.ns, -1, order="F")
    uh = (S["phi"] @ U) @ Bt[0].T
    uth = (S["phi"] @ U) @ Bt[1].T
    laph = (S["lap"] @ U) @ Bt[0].T
    Jinv = np.linalg.inv(prob.G.jacobian(S["grid"]))
    dpar = [(S["d1"][a] @ U) @ Bt[0].T for a in range(prob.d)]
    gradh = [sum(Jinv[:, a, i][:, None] * dpar[a] for a in range(prob.d)) for i in range(prob.d)]
    W = np.multiply.outer(wd, wt)
    u, ut, lap = exact["u"](x, tq), exact["ut"](x, tq), exact["lap"](x, tq)
    grad = [g(x, tq) for g in exact["grad"]]

    def integ(f):
        return float(np.sum(W * f))

    e = dict(val=integ((u - uh) ** 2), dt=integ((ut - uth) ** 2), lap=integ((lap - laph) ** 2),
             grad=sum(integ((g - gh) ** 2) for g, gh in zip(grad, gradh)))
    r = dict(val=integ(u ** 2), dt=integ(ut ** 2), lap=integ(lap ** 2), grad=sum(integ(g ** 2) for g in grad))
    return dict(V0=np.sqrt((e["dt"] + e["lap"]) / (r["dt"] + r["lap"])), L2=np.sqrt(e["val"] / r["val"]),
                H1=np.sqrt((e["val"] + e["dt"] + e["grad"]) / (r["val"] + r["dt"] + r["grad"])))
