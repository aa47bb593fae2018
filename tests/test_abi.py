"""The C-ABI library loads, exports every function include/fmmhp.h declares, and
rejects invalid arguments on the host before touching a GPU (no compute calls)."""
import ctypes
import os

import pytest

import paper_2507_21913_amd as F

pytestmark = pytest.mark.skipif(not os.path.exists(F.LIB_PATH),
                                reason="libfmmhp.so not built (python -m paper_2507_21913_amd.build)")


def test_exports_every_declared_symbol():
    names = F.header_functions()
    assert len(names) >= 9
    L = ctypes.CDLL(F.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    # and the binding wires each of them
    assert set(names) <= set(F._SIGNATURES)


def test_status_strings():
    L = F.lib()
    for k, v in F.STATUS.items():
        assert L.fmmhp_status_string(k).decode() == v


def _status(fn, *args):
    return fn(*args)


def test_plan_create_validation():
    L = F.lib()
    h = ctypes.c_void_p()
    good = F.Opts(20, 40, 0, 0)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    # NULL plan_out
    assert L.fmmhp_plan_create(10, fake, fake, None, None, 1.0, 0.0, ctypes.byref(good), None, None) == 1
    # sizes
    assert L.fmmhp_plan_create(0, fake, fake, None, None, 1.0, 0.0, ctypes.byref(good), None, ctypes.byref(h)) == 1
    assert L.fmmhp_plan_create(1 << 31, fake, fake, None, None, 1.0, 0.0, ctypes.byref(good), None,
                               ctypes.byref(h)) == 1
    # NULL coordinates, unpaired image arrays
    assert L.fmmhp_plan_create(10, None, fake, None, None, 1.0, 0.0, ctypes.byref(good), None, ctypes.byref(h)) == 1
    assert L.fmmhp_plan_create(10, fake, fake, fake, None, 1.0, 0.0, ctypes.byref(good), None, ctypes.byref(h)) == 1
    # impedance domain (Re > 0, Im >= 0) and finiteness
    for re, im, st in ((0.0, 0.0, 2), (-1.0, 0.5, 2), (1.0, -0.1, 2), (float("nan"), 0.0, 1), (float("inf"), 0, 1)):
        assert L.fmmhp_plan_create(10, fake, fake, None, None, re, im, ctypes.byref(good), None,
                                   ctypes.byref(h)) == st
    # options
    for o in (F.Opts(0, 40, 0, 0), F.Opts(41, 40, 0, 0), F.Opts(20, 0, 0, 0), F.Opts(20, 40, 31, 0),
              F.Opts(20, 40, -1, 0), F.Opts(20, 40, 0, 128), F.Opts(20, 40, 0, 12), F.Opts(20, 40, 0, 96),
              F.Opts(20, 40, 0, 0, 5, 0),
              F.Opts(20, 40, 0, 0, -1, 0),
              F.Opts(20, 40, 0, 0, 0, 17), F.Opts(20, 40, 0, 0, 1, -2)):
        assert L.fmmhp_plan_create(10, fake, fake, None, None, 1.0, 0.0, ctypes.byref(o), None,
                                   ctypes.byref(h)) == 1
    assert h.value is None
    assert "options" in L.fmmhp_last_error_message().decode()


def test_plan_create_targets_validation():
    L = F.lib()
    h = ctypes.c_void_p()
    good = F.Opts(20, 40, 0, 0)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    f = L.fmmhp_plan_create_targets
    assert f(10, fake, fake, 10, fake, fake, 1.0, 0.0, ctypes.byref(good), None, None) == 1  # NULL plan_out
    for ns, nt in ((0, 10), (10, 0), (1 << 30, 1 << 30)):
        assert f(ns, fake, fake, nt, fake, fake, 1.0, 0.0, ctypes.byref(good), None, ctypes.byref(h)) == 1
    assert f(10, fake, fake, 10, None, fake, 1.0, 0.0, ctypes.byref(good), None, ctypes.byref(h)) == 1
    assert f(10, fake, None, 10, fake, fake, 1.0, 0.0, ctypes.byref(good), None, ctypes.byref(h)) == 1
    assert f(10, fake, fake, 10, fake, fake, 1.0, -0.5, ctypes.byref(good), None, ctypes.byref(h)) == 2
    assert h.value is None


def test_null_and_dead_plans():
    L = F.lib()
    assert L.fmmhp_eval(None, 1, None, None, None) == 5
    assert L.fmmhp_plan_info(None, None) == 5
    assert L.fmmhp_plan_destroy(None) == 0
    # a block of host memory that is not a plan (wrong magic)
    junk = (ctypes.c_uint64 * 64)()
    assert L.fmmhp_eval(ctypes.cast(junk, ctypes.c_void_p), 1, None, None, None) == 5
    assert L.fmmhp_plan_destroy(ctypes.cast(junk, ctypes.c_void_p)) == 5


def test_direct_and_integrals_validation():
    L = F.lib()
    fake = ctypes.c_void_p(0x1000)
    assert L.fmmhp_direct_eval(0, fake, fake, 1, fake, 1, fake, fake, 1.0, 0.0, fake, None) == 1
    assert L.fmmhp_direct_eval(1, fake, fake, 1, fake, 1, fake, fake, 1.0, -1.0, fake, None) == 2
    assert L.fmmhp_reaction_integrals(1, fake, fake, 81, 1.0, 0.0, fake, None) == 1
    assert L.fmmhp_reaction_integrals(1, fake, fake, 5, 0.0, 0.0, fake, None) == 2


def test_binding_refuses_cpu_tensors():
    import torch
    x = torch.rand(10, dtype=torch.float64)
    with pytest.raises(TypeError):
        F.HalfPlaneFMM(x, x + 0.1, 1.0)
    with pytest.raises(TypeError):
        F.direct(x, x + 0.1, x, 1.0)


def test_batch_plan_create_validation():
    """Host-side validation of fmmhp_batch_plan_create: no device work happens before it fails."""
    L = F.lib()
    h = ctypes.c_void_p()
    good = F.Opts(20, 40, 0, 0)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first

    def call(n_inst, offs, lam, opts=good):
        o = (ctypes.c_int64 * len(offs))(*offs) if offs is not None else None
        la = (ctypes.c_double * len(lam))(*lam) if lam is not None else None
        return L.fmmhp_batch_plan_create(n_inst, o, fake, fake, la, ctypes.byref(opts), None, ctypes.byref(h))

    assert call(0, [0], []) == 1                              # no instance
    assert call(513, list(range(514)), [1.0, 0.0] * 513) == 1  # too many
    assert call(2, None, [1.0, 0.0] * 2) == 1                 # NULL offsets
    assert call(2, [1, 5, 9], [1.0, 0.0] * 2) == 1            # offsets[0] != 0
    assert call(2, [0, 5, 5], [1.0, 0.0] * 2) == 1            # empty instance
    assert call(2, [0, 5, 3], [1.0, 0.0] * 2) == 1            # decreasing
    assert call(2, [0, 5, 1 << 31], [1.0, 0.0] * 2) == 1      # total too large
    assert call(2, [0, 5, 9], [1.0, 0.0, -1.0, 0.0]) == 2     # impedance outside Re > 0
    assert call(2, [0, 5, 9], [1.0, 0.0, 1.0, -0.5]) == 2     # Im < 0
    assert call(2, [0, 5, 9], [1.0, 0.0, 1.0, 0.0], F.Opts(20, 40, 28, 0)) == 1  # max_level > 27 in a forest
    assert h.value is None


def test_backward_validation_without_plan():
    L = F.lib()
    fake = ctypes.c_void_p(0x1000)
    assert L.fmmhp_backward(None, fake, fake, None, None, None, None, None) == 5  # FMMHP_ESTATE
