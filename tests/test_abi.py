"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/pint.h declares, and rejects invalid problems
before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2007_13125_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "pint.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pint_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = _declared()
    assert "pint_solve" in names and "pint_sweeps" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(B.EXPORTS), "binding and header disagree"


def _create(grid, params):
    h = ctypes.c_void_p()
    st = B.lib().pint_plan_create(ctypes.byref(h), ctypes.byref(grid), ctypes.byref(params), None)
    return st, h


@pytest.mark.parametrize("change,status", [
    (dict(k=0), B.PINT_E_ARG), (dict(k=7), B.PINT_E_ARG), (dict(alpha=0.0), B.PINT_E_ARG),
    (dict(alpha=1.5), B.PINT_E_ARG), (dict(kappa=0.0), B.PINT_E_ARG), (dict(kappa=1.0), B.PINT_E_ARG),
    (dict(T=-1.0), B.PINT_E_ARG), (dict(tol=0.0), B.PINT_E_ARG), (dict(max_sweeps=0), B.PINT_E_ARG),
    (dict(N=4, k=4), B.PINT_E_ARG), (dict(N=101), B.PINT_E_ARG), (dict(N=2050), B.PINT_E_UNSUPPORTED),
    (dict(N=4096), B.PINT_E_UNSUPPORTED),
])
def test_invalid_params_rejected(change, status):
    base = dict(k=2, alpha=1.0, T=1.0, N=64, kappa=1e-3)
    base.update(change)
    p = B.make_params(**base)
    st, h = _create(B.make_grid((63,)), p)
    assert st == status
    assert not h.value
    assert len(B.lib().pint_last_error()) > 0


def test_mixed_direct_rejected():
    # the direct form's right-hand side would carry FP32 rounding into the fixed point
    p = B.make_params(2, 1.0, 1.0, 64, 1e-3, precision="mixed", form="direct")
    st, h = _create(B.make_grid((63,)), p)
    assert st == B.PINT_E_UNSUPPORTED and not h.value
    assert b"residual" in B.lib().pint_last_error()


@pytest.mark.parametrize("m,status", [((0,), B.PINT_E_ARG), ((4096,), B.PINT_E_UNSUPPORTED), ((2048,), B.PINT_E_UNSUPPORTED),
                                      ((5, 0), B.PINT_E_ARG), ((2048, 15), B.PINT_E_UNSUPPORTED),
                                      ((15, 15, 2048), B.PINT_E_UNSUPPORTED), ((1023, 1023, 511), B.PINT_E_UNSUPPORTED)])
def test_invalid_grids_rejected(m, status):
    st, h = _create(B.make_grid(m), B.make_params(2, 1.0, 1.0, 64, 1e-3))
    assert st == status


def test_bad_enum_and_null_plan():
    p = B.make_params(2, 1.0, 1.0, 64, 1e-3)
    p.precision = 7
    st, _ = _create(B.make_grid((63,)), p)
    assert st == B.PINT_E_ARG
    g, p = B.make_grid((63,)), B.make_params(2, 1.0, 1.0, 64, 1e-3)
    assert B.lib().pint_plan_create(None, ctypes.byref(g), ctypes.byref(p), None) == B.PINT_E_ARG
    assert B.lib().pint_plan_destroy(None) == B.PINT_OK
    assert B.lib().pint_plan_workspace_bytes(None) == 0
    assert B.lib().pint_status_str(B.PINT_E_DIVERGED) == b"PINT_E_DIVERGED"


def test_batch_rejects_unsupported_instance():
    grids = [B.make_grid((63,)), B.make_grid((2048, 127))]
    params = [B.make_params(2, 1.0, 1.0, 64, 1e-3), B.make_params(2, 1.0, 1.0, 64, 1e-3)]
    G = (B.pint_grid * 2)(*grids)
    Pm = (B.pint_params * 2)(*params)
    h = ctypes.c_void_p()
    st = B.lib().pint_batch_plan_create(ctypes.byref(h), 2, G, Pm, None)
    assert st == B.PINT_E_UNSUPPORTED
    assert b"instance 1" in B.lib().pint_last_error()


def test_autotune_entry_points_reject_bad_arguments():
    L = B.lib()
    c = (ctypes.c_int * 4)()
    assert L.pint_plan_set_autotune(None, 3) == B.PINT_E_ARG
    assert L.pint_plan_tune(None, None, 3) == B.PINT_E_ARG
    assert L.pint_plan_get_variants(None, 0, c) == B.PINT_E_ARG
    assert L.pint_plan_set_variants(None, 0, c) == B.PINT_E_ARG


def test_fem_validation():
    # P1 elements are implemented for 1D grids; a bad space value is an argument error;
    # batches take finite differences
    p = B.make_params(2, 1.0, 1.0, 64, 1e-3, space="fem")
    st, h = _create(B.make_grid((15, 15)), p)
    assert st == B.PINT_E_UNSUPPORTED and not h.value
    assert b"1D" in B.lib().pint_last_error()
    p = B.make_params(2, 1.0, 1.0, 64, 1e-3)
    p.space = 5
    st, _ = _create(B.make_grid((63,)), p)
    assert st == B.PINT_E_ARG
    G = (B.pint_grid * 1)(B.make_grid((63,)))
    Pm = (B.pint_params * 1)(B.make_params(2, 1.0, 1.0, 64, 1e-3, space="fem"))
    h = ctypes.c_void_p()
    assert B.lib().pint_batch_plan_create(ctypes.byref(h), 1, G, Pm, None) == B.PINT_E_UNSUPPORTED
