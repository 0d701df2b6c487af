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


def test_phase_window_bound(lib):
    """1/2 + 2 (f_max/c) h, h the half-diagonal of the 8 x 8 x 4 brick: 0.5 + 2 (30 GHz / c) *
    sqrt(2 (17.5 mm)^2 + (7.5 mm)^2) = 5.675 turns for the 5 mm, 20-30 GHz geometry."""
    geom = W.make_geometry(8, 8, 16, (20e9, 30e9), (16, 16, 8), 5e-3, 0.25, 0.2, seed=1)
    h = np.sqrt(2 * 17.5e-3 ** 2 + 7.5e-3 ** 2)
    assert abs(bd.phase_window(geom) - (0.5 + 2 * 100.0 * h)) < 1e-12
    # anisotropic pitch: each axis's half-extent uses its own pitch (3.5, 3.5, 1.5 pitches)
    geom["pitch"] = np.array([2e-3, 3e-3, 4e-3])
    h = np.sqrt((3.5 * 2e-3) ** 2 + (3.5 * 3e-3) ** 2 + (1.5 * 4e-3) ** 2)
    assert abs(bd.phase_window(geom) - (0.5 + 2 * 100.0 * h)) < 1e-12
    # only the highest frequency matters, whatever the order
    geom["freq"] = np.array([30e9, 20e9, 25e9])
    assert abs(bd.phase_window(geom) - (0.5 + 2 * 100.0 * h)) < 1e-12
    g, keep = bd.make_geometry_struct(geom)
    assert lib.spgm_phase_window(C.byref(g), None) == bd.SPGM_E_INVALID
    assert lib.spgm_phase_window(None, C.byref(C.c_double())) == bd.SPGM_E_INVALID
    geom["c"] = 0.0
    g, keep = bd.make_geometry_struct(geom)
    assert lib.spgm_phase_window(C.byref(g), C.byref(C.c_double())) == bd.SPGM_E_INVALID


@pytest.mark.parametrize("name", ["c0", "c1", "c2", "c4"])
def test_benchmark_geometries_fit_the_compensated_window(lib, name):
    assert bd.phase_window(W.config_geometry(name)) <= bd.COMP32_WINDOW_TURNS


def test_compensated_plan_refused_beyond_the_window(lib):
    """7.5 mm pitch at 30 GHz: 0.5 + 2 * 100 * sqrt(2 (26.25 mm)^2 + (11.25 mm)^2) = 8.26 turns,
    beyond the 8-turn window: COMP32 plans are refused on the host (before any device call);
    the float64-phase policy is not (it then needs a device)."""
    geom = W.make_geometry(8, 8, 4, (20e9, 30e9), (16, 16, 8), 7.5e-3, 0.25, 0.2, seed=1)
    assert bd.phase_window(geom) > bd.COMP32_WINDOW_TURNS
    rc, _ = _create(lib, geom, mode=bd.PHASE_COMP32)
    assert rc == bd.SPGM_E_UNSUPPORTED
    assert b"SPGM_PHASE_F64" in lib.spgm_last_error()
    rc, h = _create(lib, geom, mode=bd.PHASE_F64)
    assert rc != bd.SPGM_E_UNSUPPORTED
    if rc == bd.SPGM_OK:
        lib.spgm_plan_destroy(h)


def test_plan_create_ex_rejects_bad_options(lib):
    geom = W.make_geometry(4, 5, 3, (20e9, 30e9), (4, 4, 4), 5e-3, 0.25, 0.2, seed=1)
    g, keep = bd.make_geometry_struct(geom)
    h = C.c_void_p()
    assert lib.spgm_plan_create_ex(C.byref(h), C.byref(g), None) == bd.SPGM_E_INVALID
    o = bd.SpgmPlanOpts()
    assert lib.spgm_plan_opts_init(C.byref(o)) == bd.SPGM_OK
    assert (o.phase_mode, o.device, o.tune_cache) == (bd.PHASE_COMP32, -1, None)
    o.phase_mode = 9
    assert lib.spgm_plan_create_ex(C.byref(h), C.byref(g), C.byref(o)) == bd.SPGM_E_INVALID
    o.phase_mode = bd.PHASE_COMP32
    o.device = 1 << 20  # no such device (and none at all without a GPU)
    assert lib.spgm_plan_create_ex(C.byref(h), C.byref(g), C.byref(o)) == bd.SPGM_E_INVALID
    assert b"not present" in lib.spgm_last_error()


def test_solve_opts_defaults(lib):
    o = bd.SpgmSolveOpts()
    assert lib.spgm_solve_opts_init(C.byref(o)) == bd.SPGM_OK
    assert o.check_every == 50 and o.iters == 0 and o.B == 0 and not o.rows_d and o.tol == 0.0
    assert lib.spgm_solve_ex(None, None, None, C.byref(o), None) == bd.SPGM_E_INVALID
