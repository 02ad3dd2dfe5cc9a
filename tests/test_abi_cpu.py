"""CPU-side checks of the C ABI library: it builds/loads without a GPU and
exports every function include/inla_bta.h declares (no compute calls)."""
import ctypes
import os

import pytest

from paper_2204_04678_amd import _build, binding


@pytest.fixture(scope="module")
def libpath():
    if not os.path.exists(_build.LIB):
        _build.build()
    return _build.LIB


def test_header_declares_the_six_operations():
    names = binding.header_functions()
    for op in ("inla_assemble", "inla_factor_logdet", "inla_solve", "inla_selinv",
               "inla_eval_f", "inla_eval_f_grad"):
        assert op in names


def test_library_exports_every_declared_symbol(libpath):
    L = ctypes.CDLL(libpath)
    missing = [n for n in binding.header_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings(libpath):
    L = binding.lib(libpath)
    assert L.inla_status_string(0) == b"ok"
    assert L.inla_status_string(-3) == b"item exceeds the HBM budget"
    assert L.inla_last_error() == b""


def test_argument_errors_are_synchronous(libpath):
    """Invalid descriptions are rejected on the host before any device call."""
    L = binding.lib(libpath)
    desc = binding.ModelDesc(0, 1, 0, 1.0, 1e-3, 0, None, None, None, None, None, None)
    h = ctypes.c_void_p()
    assert L.inla_model_create(ctypes.byref(desc), None, ctypes.byref(h)) == -1
    assert b"N >= 1" in L.inla_last_error()
    bad = binding.Bta(0, 1, 0, None, None, None, None)
    assert L.inla_factor_logdet(ctypes.byref(bad), None, None, None) == -1
    assert L.inla_solve(ctypes.byref(bad), None, None, 1, None) == -1
