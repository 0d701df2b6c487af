"""C-ABI checks that need no GPU: the library loads, exports every call that include/spgm.h
declares, and rejects invalid arguments on the host before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2509_00774_amd import binding as bd
from paper_2509_00774_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(spgm_\w+)\s*\(", text, flags=re.M))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(bd.LIB_PATH):
        from paper_2509_00774_amd import build
        build.build()
    return bd.load_library()


def test_header_declares_the_calls():
    assert set(bd.EXPORTED) <= declared_symbols()


def test_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_null_and_range_errors(lib):
    assert lib.spgm_plan_create(None, None, 0) == bd.SPGM_E_INVALID
    h = C.c_void_p()
    assert lib.spgm_plan_create(C.byref(h), None, 0) == bd.SPGM_E_INVALID
    assert b"NULL" in lib.spgm_last_error()
    assert lib.spgm_forward(None, C.c_void_p(8), 4, C.c_void_p(8), C.c_void_p(8), None) == bd.SPGM_E_INVALID
    assert lib.spgm_adjoint(None, C.c_void_p(8), 4, C.c_void_p(8), C.c_void_p(8), None) == bd.SPGM_E_INVALID
    assert lib.spgm_step(None, C.c_void_p(8), 4, C.c_void_p(8), C.c_void_p(8), 1.0, 0.0, None) == bd.SPGM_E_INVALID
    assert lib.spgm_solve(None, C.c_void_p(8), 1, 4, C.c_void_p(8), C.c_void_p(8), 1.0, 0.0, None) == bd.SPGM_E_INVALID
    reg = bd.SpgmRegularizer(bd.REG_TV_MAGNITUDE, 0.0, 4)
    assert lib.spgm_prox(None, C.byref(reg), C.c_void_p(8), 0.1, None) == bd.SPGM_E_INVALID
    assert lib.spgm_step_reg(None, C.byref(reg), C.c_void_p(8), 4, C.c_void_p(8), C.c_void_p(8), 1.0, 0.0,
                             None) == bd.SPGM_E_INVALID
    assert lib.spgm_solve_reg(None, C.byref(reg), C.c_void_p(8), 1, 4, C.c_void_p(8), C.c_void_p(8), 1.0, 0.0,
                              None) == bd.SPGM_E_INVALID
    assert lib.spgm_plan_dims(None, None, None) == bd.SPGM_E_INVALID
    st = C.c_int32()
    assert lib.spgm_plan_status(None, C.byref(st)) == bd.SPGM_E_INVALID
    assert lib.spgm_plan_destroy(None) == bd.SPGM_OK


def _create(lib, geom, mode=0):
    g, keep = bd.make_geometry_struct(geom)
    h = C.c_void_p()
    rc = lib.spgm_plan_create(C.byref(h), C.byref(g), mode)
    return rc, h


@pytest.mark.parametrize("mutate,code", [
    (lambda g: g.update(grid=(0, 4, 4)), bd.SPGM_E_INVALID),
    (lambda g: g.update(pitch=np.array([5e-3, 0.0, 5e-3])), bd.SPGM_E_INVALID),
    (lambda g: g.update(c=-1.0), bd.SPGM_E_INVALID),
    (lambda g: g.update(c=float("nan")), bd.SPGM_E_INVALID),
    (lambda g: g["freq"].__setitem__(0, 0.0), bd.SPGM_E_INVALID),
    (lambda g: g["tx"].__setitem__((0, 0), float("inf")), bd.SPGM_E_INVALID),
    # an antenna placed on a voxel centre makes Eq. 2 singular
    (lambda g: g["rx"].__setitem__(1, g["centre"] + np.array([0.5 * 5e-3, 0.5 * 5e-3, 0.5 * 5e-3])), bd.SPGM_E_INVALID),
    (lambda g: g.update(tx=np.zeros((70, 3)), rx=np.zeros((70, 3))), bd.SPGM_E_UNSUPPORTED),
])
def test_plan_create_rejects_bad_geometry(lib, mutate, code):
    geom = W.make_geometry(4, 5, 3, (20e9, 30e9), (4, 4, 4), 5e-3, 0.25, 0.2, seed=1)
    mutate(geom)
    rc, _ = _create(lib, geom)
    assert rc == code, lib.spgm_last_error()


def test_plan_create_rejects_unknown_phase_mode(lib):
    geom = W.make_geometry(4, 5, 3, (20e9, 30e9), (4, 4, 4), 5e-3, 0.25, 0.2, seed=1)
    rc, _ = _create(lib, geom, mode=7)
    assert rc == bd.SPGM_E_INVALID


def test_product_path_refuses_to_run_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(bd, "_LIB", None)
    with pytest.raises(RuntimeError, match="not built"):
        bd.load_library(str(tmp_path / "missing.so"))


def test_autotune_rejects_null_plan(lib):
    assert lib.spgm_plan_autotune(None, 16, None, None, None) == bd.SPGM_E_INVALID
