"""MI355X-native space-time least-squares heat solver (Python binding).

Thin ctypes binding over ``libstls.so`` (C ABI in ``include/stls.h``).  It only
marshals arguments: every step of the solve (FD preconditioner, matvec, PCG)
runs in the library's HIP kernels.  PyTorch supplies device memory and the
current stream.  If the library has not been built, importing this package
raises ImportError: there is no CPU fallback.

Method: Montardini, Negri, Sangalli, Tani, arXiv:1809.10026 (space-time
least-squares isogeometric discretisation of the heat equation, §3; Kronecker
system, §4.1; FD-preconditioned PCG, §4.2-4.3).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "LIB_PATH", "STLS_OK", "STLS_FD_FP64", "STLS_FD_FP32", "STLS_FD_BF16X3", "STLS_FD_ASYM", "StlsError",
    "stls_setup", "stls_destroy", "stls_get_shape", "stls_get_factor", "stls_set_kappa",
    "stls_set_fd_precision", "stls_set_fd_scaling", "stls_prec_apply", "stls_matvec", "stls_pcg_solve",
    "stls_pcg_history", "stls_norm_points", "stls_error_norms", "stls_set_profiling", "stls_profile", "stls_profile_reset",
    "stls_lift_initial", "stls_lift_combine", "stls_lift_apply", "stls_lift_embed",
    "Solver",
]

# torch first: its HIP runtime (same soname as ROCm's) then also serves the
# library, so the process holds a single runtime and shares device pointers
# and streams with torch.
import torch  # noqa: E402,F401

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libstls.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_1809_10026_amd/build.py` "
        "(there is no CPU fallback)")
_lib = ctypes.CDLL(LIB_PATH)

STLS_OK, STLS_EINVAL, STLS_ENOMEM, STLS_EHIP, STLS_ENOCONV, STLS_ENAN, STLS_EBREAKDOWN = 0, -1, -2, -3, -4, -5, -6
STLS_FD_FP64, STLS_FD_FP32, STLS_FD_BF16X3, STLS_FD_ASYM = 0, 1, 2, 3
STLS_GEOM_UNIT_BOX, STLS_GEOM_QUARTER_ANNULUS, STLS_GEOM_ROTATED_QUARTER_ANNULUS = 0, 1, 2
STLS_PREC_PARAMETRIC, STLS_PREC_GEOMETRY = 0, 1
# batch tuning fields, in the order of enum stls_batch_tune_field
TUNE_FIELDS = ("vec_chunk", "inner_steps", "outer_chunk", "grid_fd", "grid_inner", "grid_outer", "grid_vec",
               "graph_depth")

_c_int_p = ctypes.POINTER(ctypes.c_int)
_c_dbl_p = ctypes.c_void_p
_sig = {
    "stls_setup": (ctypes.c_int, [ctypes.c_int, _c_int_p, ctypes.POINTER(ctypes.c_void_p), _c_int_p,
                                  ctypes.c_double, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "stls_setup_mapped": (ctypes.c_int, [ctypes.c_int, _c_int_p, ctypes.POINTER(ctypes.c_void_p), _c_int_p,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "stls_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "stls_get_shape": (ctypes.c_int, [ctypes.c_void_p, _c_int_p, ctypes.POINTER(ctypes.c_int64)]),
    "stls_get_factor": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_int64)]),
    "stls_set_kappa": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "stls_set_fd_precision": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "stls_set_fd_scaling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "stls_prec_apply": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p]),
    "stls_matvec": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p]),
    "stls_pcg_solve": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p, ctypes.c_double, ctypes.c_int,
                                      _c_int_p, ctypes.POINTER(ctypes.c_double)]),
    "stls_pcg_history": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, _c_int_p]),
    "stls_norm_points": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, _c_int_p]),
    "stls_error_norms": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "stls_set_profiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "stls_profile_count": (ctypes.c_int, []),
    "stls_profile_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_char_p),
                                        ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
    "stls_profile_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "stls_get_forcing_shape": (ctypes.c_int, [ctypes.c_void_p, _c_int_p, ctypes.POINTER(ctypes.c_int64)]),
    "stls_load_apply": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p]),
    "stls_load_apply_noalloc": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p]),
    "stls_load_apply_T": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p]),
    "stls_lift_initial": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p]),
    "stls_lift_combine": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p, _c_dbl_p]),
    "stls_lift_apply": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p]),
    "stls_lift_embed": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p, _c_dbl_p]),
    "stls_mass_apply": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p]),
    "stls_dkappa": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p, _c_dbl_p, ctypes.POINTER(ctypes.c_double)]),
    "stls_dkappa_terms": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p, _c_dbl_p, ctypes.POINTER(ctypes.c_double)]),
    "stls_dot": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]),
    "stls_misfit": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p, _c_dbl_p, ctypes.POINTER(ctypes.c_double)]),
    "stls_batch_setup": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _c_int_p, ctypes.POINTER(ctypes.c_void_p), _c_int_p,
                                        ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "stls_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "stls_batch_offsets": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "stls_batch_problem": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "stls_batch_matvec": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p]),
    "stls_batch_prec_apply": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p]),
    "stls_batch_pcg_solve": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p, ctypes.c_double, ctypes.c_int,
                                            _c_int_p, ctypes.POINTER(ctypes.c_double)]),
    "stls_batch_set_graph": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "stls_batch_graph_used": (ctypes.c_int, [ctypes.c_void_p]),
    "stls_batch_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]),
    "stls_batch_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]),
    "stls_batch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)]),
    "stls_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "stls_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class StlsError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.stls_status_string(status).decode()
        detail = _lib.stls_last_error().decode()
        super().__init__(f"{where}: {msg} ({status}){': ' + detail if detail else ''}")


def _check(status, where, ok=(STLS_OK,)):
    if status not in ok:
        raise StlsError(status, where)
    return status


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, n, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# C ABI mirrors (same names); handles are opaque ctypes.c_void_p values.

def stls_setup(knots, degrees, kappa=1.0, stream=None, geometry=0, prec=0):
    """Handle for one problem; knots: d+1 host arrays (time last).  geometry
    (STLS_GEOM_*) != 0 sets up a mapped domain with preconditioner prec
    (STLS_PREC_PARAMETRIC or STLS_PREC_GEOMETRY)."""
    d = len(knots) - 1
    arrs = [np.ascontiguousarray(k, dtype=np.float64) for k in knots]
    nk = (ctypes.c_int * (d + 1))(*[len(a) for a in arrs])
    ptrs = (ctypes.c_void_p * (d + 1))(*[a.ctypes.data for a in arrs])
    degs = (ctypes.c_int * (d + 1))(*[int(p) for p in degrees])
    h = ctypes.c_void_p()
    if geometry:
        _check(_lib.stls_setup_mapped(d, nk, ptrs, degs, float(kappa), int(geometry), int(prec), _stream_ptr(stream),
                                      ctypes.byref(h)), "stls_setup_mapped")
    else:
        _check(_lib.stls_setup(d, nk, ptrs, degs, float(kappa), _stream_ptr(stream), ctypes.byref(h)), "stls_setup")
    return h


def stls_destroy(h):
    _check(_lib.stls_destroy(h), "stls_destroy")


def stls_get_shape(h, d):
    n = (ctypes.c_int * (d + 1))()
    nd = ctypes.c_int64()
    _check(_lib.stls_get_shape(h, n, ctypes.byref(nd)), "stls_get_shape")
    return tuple(n), int(nd.value)


def stls_get_factor(h, direction, what):
    cnt = ctypes.c_int64()
    _check(_lib.stls_get_factor(h, direction, what, None, ctypes.byref(cnt)), "stls_get_factor")
    out = np.zeros(cnt.value)
    _check(_lib.stls_get_factor(h, direction, what, out.ctypes.data, ctypes.byref(cnt)), "stls_get_factor")
    return out


def stls_set_kappa(h, kappa):
    _check(_lib.stls_set_kappa(h, float(kappa)), "stls_set_kappa")


def stls_set_fd_precision(h, mode):
    _check(_lib.stls_set_fd_precision(h, int(mode)), "stls_set_fd_precision")


def stls_set_fd_scaling(h, on):
    _check(_lib.stls_set_fd_scaling(h, 1 if on else 0), "stls_set_fd_scaling")


def stls_prec_apply(h, ndof, r, s):
    _check(_lib.stls_prec_apply(h, _dev_ptr(r, ndof, "r"), _dev_ptr(s, ndof, "s")), "stls_prec_apply")


def stls_matvec(h, ndof, x, y):
    _check(_lib.stls_matvec(h, _dev_ptr(x, ndof, "x"), _dev_ptr(y, ndof, "y")), "stls_matvec")


def stls_pcg_solve(h, ndof, b, x, rtol, maxit, raise_on_noconv=True):
    it = ctypes.c_int()
    rel = ctypes.c_double()
    ok = (STLS_OK,) if raise_on_noconv else (STLS_OK, STLS_ENOCONV)
    st = _check(_lib.stls_pcg_solve(h, _dev_ptr(b, ndof, "b"), _dev_ptr(x, ndof, "x"), float(rtol), int(maxit),
                                    ctypes.byref(it), ctypes.byref(rel)), "stls_pcg_solve", ok)
    return int(it.value), float(rel.value), st


def stls_norm_points(h, direction):
    """Quadrature points and weights of the error norms in one direction."""
    nq = ctypes.c_int()
    _check(_lib.stls_norm_points(h, int(direction), None, None, ctypes.byref(nq)), "stls_norm_points")
    x, w = np.zeros(nq.value), np.zeros(nq.value)
    _check(_lib.stls_norm_points(h, int(direction), x.ctypes.data, w.ctypes.data, ctypes.byref(nq)),
           "stls_norm_points")
    return x, w


def stls_error_norms(h, ndof, u, factors):
    """factors[s][k]: array (3, nq_k) of g_{s,k}, g', g'' at the direction's
    norm points; returns the relative V0, L2 and H1 errors."""
    arrays = [np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1)) for term in factors for f in term]
    ptrs = (ctypes.c_void_p * len(arrays))(*[a.ctypes.data for a in arrays])
    out = np.zeros(3)
    _check(_lib.stls_error_norms(h, _dev_ptr(u, ndof, "u"), len(factors), ptrs, out.ctypes.data),
           "stls_error_norms")
    return dict(V0=float(out[0]), L2=float(out[1]), H1=float(out[2]))


def stls_pcg_history(h):
    cnt = ctypes.c_int()
    _check(_lib.stls_pcg_history(h, None, 0, ctypes.byref(cnt)), "stls_pcg_history")
    out = np.zeros(cnt.value)
    _check(_lib.stls_pcg_history(h, out.ctypes.data, cnt.value, ctypes.byref(cnt)), "stls_pcg_history")
    return out


def stls_get_forcing_shape(h, d):
    m = (ctypes.c_int * (d + 1))()
    nf = ctypes.c_int64()
    _check(_lib.stls_get_forcing_shape(h, m, ctypes.byref(nf)), "stls_get_forcing_shape")
    return tuple(m), int(nf.value)


def stls_load_apply(h, nfull, ndof, f, F):
    _check(_lib.stls_load_apply(h, _dev_ptr(f, nfull, "f"), _dev_ptr(F, ndof, "F")), "stls_load_apply")


def stls_load_apply_noalloc(h, nfull, ndof, f, F):
    _check(_lib.stls_load_apply_noalloc(h, _dev_ptr(f, nfull, "f"), _dev_ptr(F, ndof, "F")),
           "stls_load_apply_noalloc")


def stls_load_apply_T(h, nfull, ndof, lam, gf):
    _check(_lib.stls_load_apply_T(h, _dev_ptr(lam, ndof, "l"), _dev_ptr(gf, nfull, "gf")), "stls_load_apply_T")


def stls_lift_initial(h, ns, ndof, u0, F):
    _check(_lib.stls_lift_initial(h, _dev_ptr(u0, ns, "u0"), _dev_ptr(F, ndof, "F")), "stls_lift_initial")


def stls_lift_combine(h, ns, ndof, u0, w, u):
    _check(_lib.stls_lift_combine(h, _dev_ptr(u0, ns, "u0"), _dev_ptr(w, ndof, "w"), _dev_ptr(u, ns + ndof, "u")),
           "stls_lift_combine")


def stls_lift_apply(h, nfull, ndof, ub, F):
    _check(_lib.stls_lift_apply(h, _dev_ptr(ub, nfull, "ub"), _dev_ptr(F, ndof, "F")), "stls_lift_apply")


def stls_lift_embed(h, nfull, ndof, ub, w, u):
    _check(_lib.stls_lift_embed(h, _dev_ptr(ub, nfull, "ub"), _dev_ptr(w, ndof, "w"), _dev_ptr(u, nfull, "u")),
           "stls_lift_embed")


def stls_mass_apply(h, ndof, x, y):
    _check(_lib.stls_mass_apply(h, _dev_ptr(x, ndof, "x"), _dev_ptr(y, ndof, "y")), "stls_mass_apply")


def stls_dkappa(h, nfull, ndof, f, u, lam):
    out = ctypes.c_double()
    _check(_lib.stls_dkappa(h, _dev_ptr(f, nfull, "f"), _dev_ptr(u, ndof, "u"), _dev_ptr(lam, ndof, "l"),
                            ctypes.byref(out)), "stls_dkappa")
    return float(out.value)


def stls_dot(h, a, b):
    out = ctypes.c_double()
    n = a.numel()
    _check(_lib.stls_dot(h, _dev_ptr(a, n, "a"), _dev_ptr(b, n, "b"), n, ctypes.byref(out)), "stls_dot")
    return float(out.value)


def stls_misfit(h, ndof, u, ustar, q):
    out = ctypes.c_double()
    _check(_lib.stls_misfit(h, _dev_ptr(u, ndof, "u"), _dev_ptr(ustar, ndof, "ustar"), _dev_ptr(q, ndof, "q"),
                            ctypes.byref(out)), "stls_misfit")
    return float(out.value)


def stls_set_profiling(h, on):
    _check(_lib.stls_set_profiling(h, 1 if on else 0), "stls_set_profiling")


def stls_profile(h):
    """{kernel class: (launches, total ms)} accumulated since the last reset."""
    res = {}
    for i in range(_lib.stls_profile_count()):
        name = ctypes.c_char_p()
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(_lib.stls_profile_get(h, i, ctypes.byref(name), ctypes.byref(n), ctypes.byref(ms)), "stls_profile_get")
        res[name.value.decode()] = (int(n.value), float(ms.value))
    return res


def stls_profile_reset(h):
    _check(_lib.stls_profile_reset(h), "stls_profile_reset")


# ---------------------------------------------------------------------------
class Batch:
    """Many independent problems solved together (one launch per PCG step).

    problems: list of (knots, degrees, kappa) with the same d (1 or 2).
    Vectors are concatenated float64 CUDA tensors; ``offsets[i]:offsets[i+1]``
    is problem i.
    """

    def __init__(self, problems, stream=None):
        self.nprob = len(problems)
        self.d = len(problems[0][0]) - 1
        d1 = self.d + 1
        arrs, nks, degs, kaps = [], [], [], []
        for knots, degrees, kappa in problems:
            if len(knots) != d1:
                raise ValueError("all problems of a batch need the same d")
            for k in knots:
                arrs.append(np.ascontiguousarray(k, dtype=np.float64))
                nks.append(len(arrs[-1]))
            degs.extend(int(p) for p in degrees)
            kaps.append(float(kappa))
        nk = (ctypes.c_int * len(nks))(*nks)
        ptrs = (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
        dg = (ctypes.c_int * len(degs))(*degs)
        kp = (ctypes.c_double * len(kaps))(*kaps)
        h = ctypes.c_void_p()
        _check(_lib.stls_batch_setup(self.nprob, self.d, nk, ptrs, dg, kp, _stream_ptr(stream), ctypes.byref(h)),
               "stls_batch_setup")
        self._h = h
        off = (ctypes.c_int64 * (self.nprob + 1))()
        _check(_lib.stls_batch_offsets(h, off), "stls_batch_offsets")
        self.offsets = [int(v) for v in off]
        self.total = self.offsets[-1]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(_lib.stls_batch_destroy(self._h), "stls_batch_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def problem_handle(self, i):
        h = ctypes.c_void_p()
        _check(_lib.stls_batch_problem(self._h, i, ctypes.byref(h)), "stls_batch_problem")
        return h

    def _empty(self):
        import torch
        return torch.empty(self.total, dtype=torch.float64, device="cuda")

    def matvec(self, x, out=None):
        y = self._empty() if out is None else out
        _check(_lib.stls_batch_matvec(self._h, _dev_ptr(x, self.total, "x"), _dev_ptr(y, self.total, "y")),
               "stls_batch_matvec")
        return y

    def prec_apply(self, r, out=None):
        s = self._empty() if out is None else out
        _check(_lib.stls_batch_prec_apply(self._h, _dev_ptr(r, self.total, "r"), _dev_ptr(s, self.total, "s")),
               "stls_batch_prec_apply")
        return s

    def solve(self, b, rtol=1e-8, maxit=500, out=None, raise_on_noconv=True):
        x = self._empty() if out is None else out
        its = (ctypes.c_int * self.nprob)()
        rel = (ctypes.c_double * self.nprob)()
        ok = (STLS_OK,) if raise_on_noconv else (STLS_OK, STLS_ENOCONV)
        _check(_lib.stls_batch_pcg_solve(self._h, _dev_ptr(b, self.total, "b"), _dev_ptr(x, self.total, "x"),
                                         float(rtol), int(maxit), its, rel), "stls_batch_pcg_solve", ok)
        return x, list(its), list(rel)

    def set_graph(self, on):
        """Replay the PCG iterations from a captured hipGraph (default) or launch directly."""
        _check(_lib.stls_batch_set_graph(self._h, 1 if on else 0), "stls_batch_set_graph")

    @property
    def graph_used(self):
        """Whether the last solve replayed a captured graph."""
        v = _lib.stls_batch_graph_used(self._h)
        _check(min(v, 0), "stls_batch_graph_used")
        return bool(v)

    @property
    def tuning(self):
        """Work-item shapes and launch geometry, a dict keyed by TUNE_FIELDS."""
        vals = (ctypes.c_int * len(TUNE_FIELDS))()
        _check(_lib.stls_batch_get_tuning(self._h, vals), "stls_batch_get_tuning")
        return dict(zip(TUNE_FIELDS, list(vals)))

    @tuning.setter
    def tuning(self, values):
        cur = self.tuning
        cur.update(values)
        vals = (ctypes.c_int * len(TUNE_FIELDS))(*[int(cur[k]) for k in TUNE_FIELDS])
        _check(_lib.stls_batch_set_tuning(self._h, vals), "stls_batch_set_tuning")

    def autotune(self, cache_path=None):
        """Pick the tuning by timing candidates (or reuse the choice stored in
        the JSON file ``cache_path`` under this batch's key).  Returns True if
        timings were taken, False if the cache supplied the choice."""
        measured = ctypes.c_int(0)
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(_lib.stls_batch_autotune(self._h, path, ctypes.byref(measured)), "stls_batch_autotune")
        return bool(measured.value)


# ---------------------------------------------------------------------------
class Solver:
    """One space-time heat problem on the unit box (or, with ``geometry``, on
    a mapped domain: STLS_GEOM_QUARTER_ANNULUS, d = 2, or
    STLS_GEOM_ROTATED_QUARTER_ANNULUS, d = 3, with preconditioner ``prec``
    STLS_PREC_PARAMETRIC or STLS_PREC_GEOMETRY); owns a library handle.

    knots/degrees: d+1 entries (space directions, then time).  Vectors are
    float64 CUDA tensors of ``ndof`` entries in colexicographic order.
    """

    def __init__(self, knots, degrees, kappa=1.0, stream=None, geometry=0, prec=0):
        self.d = len(knots) - 1
        self.geometry = int(geometry)
        self._h = stls_setup(knots, degrees, kappa, stream, geometry, prec)
        self.shape, self.ndof = stls_get_shape(self._h, self.d)
        self.kappa = float(kappa)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            stls_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    def _empty(self):
        import torch
        return torch.empty(self.ndof, dtype=torch.float64, device="cuda")

    def set_kappa(self, kappa):
        stls_set_kappa(self._h, kappa)
        self.kappa = float(kappa)

    def set_fd_precision(self, mode):
        stls_set_fd_precision(self._h, mode)

    def set_fd_scaling(self, on):
        """Diagonally scaled preconditioner D^-1/2 P^-1 D^-1/2 (on) or P^-1 (off)."""
        stls_set_fd_scaling(self._h, on)

    def factor(self, direction, what):
        return stls_get_factor(self._h, direction, what)

    def prec_apply(self, r, out=None):
        s = self._empty() if out is None else out
        stls_prec_apply(self._h, self.ndof, r, s)
        return s

    def matvec(self, x, out=None):
        y = self._empty() if out is None else out
        stls_matvec(self._h, self.ndof, x, y)
        return y

    def solve(self, b, rtol=1e-8, maxit=500, out=None, raise_on_noconv=True):
        x = self._empty() if out is None else out
        it, rel, st = stls_pcg_solve(self._h, self.ndof, b, x, rtol, maxit, raise_on_noconv)
        return x, it, rel

    def history(self):
        return stls_pcg_history(self._h)

    def norm_points(self, direction):
        return stls_norm_points(self._h, direction)

    def error_norms(self, u, factors):
        """Relative V0 / L2 / H1 errors of u against sum_s prod_k g_{s,k}
        (factors[s][k] = (g, g', g'') at norm_points(k))."""
        return stls_error_norms(self._h, self.ndof, u, factors)

    # --- differentiation operators ---------------------------------------
    @property
    def forcing_shape(self):
        return stls_get_forcing_shape(self._h, self.d)

    def load_apply(self, f, out=None):
        import torch
        F = self._empty() if out is None else out
        stls_load_apply(self._h, self.forcing_shape[1], self.ndof, f, F)
        return F

    def load_apply_T(self, lam, out=None):
        import torch
        nf = self.forcing_shape[1]
        gf = torch.empty(nf, dtype=torch.float64, device="cuda") if out is None else out
        stls_load_apply_T(self._h, nf, self.ndof, lam, gf)
        return gf

    # --- lifting of non-zero initial data ---------------------------------
    @property
    def ns(self):
        return self.ndof // self.shape[-1]

    def lift_initial(self, u0, F):
        """F -= a(u0_h b_1, B_i) in place (u0: restricted spatial coefficients
        of the initial value); returns F."""
        stls_lift_initial(self._h, self.ns, self.ndof, u0, F)
        return F

    def lift_combine(self, u0, w, out=None):
        """Coefficients over every time function: [u0, w] (time slowest)."""
        import torch
        u = torch.empty(self.ns + self.ndof, dtype=torch.float64, device="cuda") if out is None else out
        stls_lift_combine(self._h, self.ns, self.ndof, u0, w, u)
        return u

    def lift_apply(self, ub, F):
        """F -= a(u_B, B_i) in place for a lifting u_B over the full space
        (boundary and initial coefficients); returns F."""
        stls_lift_apply(self._h, self.forcing_shape[1], self.ndof, ub, F)
        return F

    def lift_embed(self, ub, w, out=None):
        """Coefficients over the full space: u_B plus w at the restricted ones."""
        import torch
        nf = self.forcing_shape[1]
        u = torch.empty(nf, dtype=torch.float64, device="cuda") if out is None else out
        stls_lift_embed(self._h, nf, self.ndof, ub, w, u)
        return u

    def mass_apply(self, x, out=None):
        y = self._empty() if out is None else out
        stls_mass_apply(self._h, self.ndof, x, y)
        return y

    def dkappa(self, f, u, lam):
        return stls_dkappa(self._h, self.forcing_shape[1], self.ndof, f, u, lam)

    def dot(self, a, b):
        return stls_dot(self._h, a, b)

    def misfit(self, u, ustar):
        """(loss, q): loss = (u - u*)^T M_Q (u - u*) and q = 2 M_Q (u - u*), its gradient."""
        q = self._empty()
        return stls_misfit(self._h, self.ndof, u, ustar, q), q

    def profiling(self, on=True):
        stls_set_profiling(self._h, on)

    def profile(self):
        return stls_profile(self._h)

    def profile_reset(self):
        stls_profile_reset(self._h)
