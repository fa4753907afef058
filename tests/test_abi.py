"""The C-ABI library loads and exports every symbol include/lupp.h declares;
argument checks that need no device return LAPACK-style negative codes."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lupp.h")
LIB = os.path.join(ROOT, "paper_2104_05782_amd", "liblupp.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lupp_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2104_05782_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_entry_points():
    names = _declared()
    for n in ("lupp_create", "lupp_destroy", "lupp_dgetrf", "lupp_sgetrf", "lupp_dgetrs", "lupp_sgetrs"):
        assert n in names


def test_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_null_handle_codes(lib):
    lib.lupp_dgetrf.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                ctypes.c_void_p, ctypes.c_void_p]
    assert lib.lupp_dgetrf(None, 4, 4, None, 4, None, None) == -1
    lib.lupp_create.argtypes = [ctypes.c_void_p]
    assert lib.lupp_create(None) == -1
    lib.lupp_status_string.restype = ctypes.c_char_p
    assert lib.lupp_status_string(0) == b"success"
    assert lib.lupp_status_string(-3) == b"invalid argument"


def test_ir_opts_defaults():
    """lupp_ir_opts_default is host-only: the documented defaults."""
    import paper_2104_05782_amd as lupp
    g = lupp.ir_opts("gmres")
    c = lupp.ir_opts("classical")
    assert (g.factor_prec, g.solver, g.tol, g.max_iter, g.gmres_restart, g.inner_tol, g.nb, g.fallback_fp64) == \
        (lupp.PREC["fp16"], 1, 1e-14, 10, 30, 1e-6, 0, 0)
    assert (c.solver, c.max_iter) == (0, 50)
    assert lupp.ir_opts("gmres", factor_prec="fp8").factor_prec == 3
