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


def test_batch_and_shape_errors_are_synchronous(libpath):
    """Empty batches, NULL models, bad options and mismatched shapes are
    rejected with INLA_ERR_ARG before any device call (the pointers below are
    never dereferenced)."""
    L = binding.lib(libpath)
    dummy = ctypes.c_void_p(64)
    empty = (ctypes.c_void_p * 1)()
    assert L.inla_eval_f(empty, 0, dummy, dummy, None, None, None, None, None) == -1
    assert b"n_items >= 1" in L.inla_last_error()
    assert L.inla_eval_f_grad(empty, 0, dummy, dummy, dummy, None, None, None, None,
                              None) == -1
    assert b"n_items >= 1" in L.inla_last_error()
    assert L.inla_eval_f(None, 1, dummy, dummy, None, None, None, None, None) == -1
    holes = (ctypes.c_void_p * 2)(dummy.value, None)
    assert L.inla_eval_f(holes, 2, dummy, dummy, None, None, None, None, None) == -1
    assert b"NULL model" in L.inla_last_error()
    one = (ctypes.c_void_p * 1)(dummy.value)
    for field, value, msg in (("tile", 96, b"tile must be"), ("recompute", 3, b"recompute"),
                              ("keep_sigma", 1, b"keep_sigma")):
        o = binding.Opts()
        setattr(o, field, value)
        assert L.inla_eval_f(one, 1, dummy, dummy, None, None, None, ctypes.byref(o),
                             None) == -1
        assert msg in L.inla_last_error()
    # arrow wider than 64, missing S with nt > 1, missing R/T with a > 0
    for b, nt, a, S, R in ((8, 2, 65, dummy, dummy), (8, 2, 0, None, None),
                           (8, 1, 2, None, None)):
        q = binding.Bta(b, nt, a, dummy, S, R, R)
        assert L.inla_factor_logdet(ctypes.byref(q), dummy, dummy, None) == -1
        assert b"QL" in L.inla_last_error()
    Lq = binding.Bta(8, 2, 1, dummy, dummy, dummy, dummy)
    sig = binding.Bta(8, 3, 1, dummy, dummy, dummy, dummy)
    assert L.inla_selinv(ctypes.byref(Lq), ctypes.byref(sig), None, None) == -1
    assert b"sigma shape" in L.inla_last_error()
    assert L.inla_assemble(None, dummy, 0, ctypes.byref(Lq), None, None) == -1
    assert L.inla_assemble(dummy, dummy, 2, ctypes.byref(Lq), None, None) == -1
    assert b"which" in L.inla_last_error()


def test_build_id_ties_the_library_to_its_sources(libpath, monkeypatch):
    """The library reports the hash of the sources it was built from, and the
    binding refuses a library whose hash differs from the sources beside it."""
    L = ctypes.CDLL(libpath)
    L.inla_build_id.restype = ctypes.c_char_p
    assert L.inla_build_id().decode() == _build.source_hash()
    monkeypatch.setattr(binding, "_LIB", None)
    monkeypatch.setattr(binding, "source_hash", lambda: "0" * 16)
    with pytest.raises(RuntimeError, match="other sources"):
        binding.lib(libpath)


def test_state_and_sigma_argument_errors(libpath):
    """The kept-state calls and keep_sigma reject bad arguments on the host."""
    L = binding.lib(libpath)
    dummy = ctypes.c_void_p(64)
    one = (ctypes.c_void_p * 1)(dummy.value)
    o = binding.Opts()
    o.keep_sigma = 2
    assert L.inla_eval_f(one, 1, dummy, dummy, None, None, None, ctypes.byref(o), None) == -1
    assert b"keep_sigma" in L.inla_last_error()
    st = ctypes.c_void_p()
    assert L.inla_eval_f_keep(one, 1, dummy, dummy, None, None, None, None, None) == -1
    assert b"state_out" in L.inla_last_error()
    assert L.inla_eval_f_keep(one, 0, dummy, dummy, None, None, None, None, ctypes.byref(st)) == -1
    assert st.value is None
    assert L.inla_eval_grad_kept(None, dummy, dummy, None, None, None) == -1
    assert b"state is NULL" in L.inla_last_error()
    assert L.inla_eval_state_kept(None) == 0
    L.inla_eval_state_destroy(None)


def test_integrate_argument_errors(libpath):
    """inla_integrate rejects bad arguments on the host before any device call."""
    L = binding.lib(libpath)
    res = binding.IntegrateResult()
    th = (ctypes.c_double * 4)(0.0, 0.0, 0.0, 0.0)
    assert L.inla_integrate(None, th, None, ctypes.byref(res), None, 0, None, None, None) == -1
    assert b"need model" in L.inla_last_error()
    bad = (ctypes.c_double * 4)(0.0, float("nan"), 0.0, 0.0)
    dummy = ctypes.c_void_p(64)
    assert L.inla_integrate(dummy, bad, None, ctypes.byref(res), None, 0, None, None, None) == -1
    assert b"not finite" in L.inla_last_error()
    o = binding.IntegrateOpts(0.0, 0.0, 0.0, 65, 0, None)
    assert L.inla_integrate(dummy, th, ctypes.byref(o), ctypes.byref(res), None, 0, None, None,
                            None) == -1
    assert b"max_steps" in L.inla_last_error()


def test_poisson_argument_errors(libpath):
    """inla_eval_f_grad_poisson rejects bad arguments on the host."""
    L = binding.lib(libpath)
    res = binding.NewtonResult()
    th = (ctypes.c_double * 4)(0.0, 0.0, 0.0, 0.0)
    assert L.inla_eval_f_grad_poisson(None, th, None, ctypes.byref(res), None, None, None) == -1
    assert b"need model" in L.inla_last_error()
    dummy = ctypes.c_void_p(64)
    bad = (ctypes.c_double * 4)(0.0, 0.0, float("inf"), 0.0)
    assert L.inla_eval_f_grad_poisson(dummy, bad, None, ctypes.byref(res), None, None, None) == -1
    assert b"not finite" in L.inla_last_error()
