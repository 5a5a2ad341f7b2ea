"""The C-ABI library loads on a CPU host, exports every function declared in
include/stls.h, and rejects invalid problem descriptions on the host before
any device call (input validation of §2.1 / Assumption 2)."""
import ctypes
import os
import re

import numpy as np
import pytest

from stls_inputs import uniform_open_knots

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1809_10026_amd", "libstls.so")
HDR = os.path.join(ROOT, "include", "stls.h")


def _declared():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stls_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libstls.so is not built (python paper_1809_10026_amd/build.py)")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    lib.stls_status_string.restype = ctypes.c_char_p
    for code in range(0, -7, -1):
        assert lib.stls_status_string(code) and lib.stls_status_string(code) != b"unknown status"


def _setup_status(lib, d, knots, degs, kappa=1.0):
    arrs = [np.ascontiguousarray(k, dtype=np.float64) for k in knots]
    nk = (ctypes.c_int * len(arrs))(*[len(a) for a in arrs])
    ptrs = (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
    dg = (ctypes.c_int * len(degs))(*degs)
    h = ctypes.c_void_p()
    lib.stls_setup.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_void_p),
                               ctypes.POINTER(ctypes.c_int), ctypes.c_double, ctypes.c_void_p,
                               ctypes.POINTER(ctypes.c_void_p)]
    st = lib.stls_setup(d, nk, ptrs, dg, kappa, None, ctypes.byref(h))
    return st, h


BAD = [
    ("d out of range", 4, [uniform_open_knots(4, 2)] * 5, [2] * 5, 1.0),
    ("space degree 1", 1, [uniform_open_knots(4, 1), uniform_open_knots(4, 1)], [1, 1], 1.0),
    ("not open", 1, [np.array([0, 0, 0.1, 0.5, 1, 1, 1.0]), uniform_open_knots(4, 2)], [2, 2], 1.0),
    ("decreasing", 1, [np.array([0, 0, 0, 0.6, 0.4, 1, 1, 1.0]), uniform_open_knots(4, 2)], [2, 2], 1.0),
    ("C0 in space", 1, [np.array([0, 0, 0, 0.5, 0.5, 1, 1, 1.0]), uniform_open_knots(4, 2)], [2, 2], 1.0),
    ("discontinuous in time", 1, [uniform_open_knots(4, 2), np.array([0, 0, 0, 0.5, 0.5, 0.5, 1, 1, 1.0])], [2, 2], 1.0),
    ("end multiplicity p+2", 1, [np.array([0, 0, 0, 0, 0.5, 1, 1, 1.0]), uniform_open_knots(4, 2)], [2, 2], 1.0),
    ("degree above 12", 1, [uniform_open_knots(4, 13), uniform_open_knots(4, 2)], [13, 2], 1.0),
    ("kappa <= 0", 1, [uniform_open_knots(4, 2)] * 2, [2, 2], 0.0),
    ("nan knot", 1, [np.array([0, 0, 0, np.nan, 1, 1, 1.0]), uniform_open_knots(4, 2)], [2, 2], 1.0),
]


@pytest.mark.parametrize("what,d,knots,degs,kappa", BAD, ids=[b[0] for b in BAD])
def test_invalid_problems_rejected_on_host(lib, what, d, knots, degs, kappa):
    st, h = _setup_status(lib, d, knots, degs, kappa)
    assert st == -1 and not h.value
    lib.stls_last_error.restype = ctypes.c_char_p
    assert lib.stls_last_error()
