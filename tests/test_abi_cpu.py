"""CPU-side checks of the C ABI: the built library loads, exports every entry point
that include/xrt.h declares, and rejects invalid arguments before touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xrt.h")
LIB = os.path.join(ROOT, "paper_2006_00686_amd", "libxrt.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(xrt_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libxrt.so is not built (python -m paper_2006_00686_amd.build)")
    from paper_2006_00686_amd import xrt
    return xrt.library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("xrt_plan_create", "xrt_plan_destroy", "xrt_forward", "xrt_adjoint", "xrt_ray_hits",
              "xrt_ray_hit_counts", "xrt_status_str", "xrt_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_status_strings(lib):
    assert lib.xrt_status_str(0).decode() == "XRT_OK"
    assert "geometry" in lib.xrt_status_str(-2).decode()
    assert lib.xrt_status_str(12345).decode() == "unknown xrt_status"


def _create(lib, grid_kw, scan_kw):
    from paper_2006_00686_amd import xrt
    g = xrt.Grid(**grid_kw)
    s = xrt.Scan()
    keep = []
    for k, v in scan_kw.items():
        if isinstance(v, (list, np.ndarray)):
            a = np.ascontiguousarray(v, dtype=np.float64)
            keep.append(a)
            setattr(s, k, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        else:
            setattr(s, k, v)
    h = ctypes.c_void_p()
    st = lib.xrt_plan_create(ctypes.byref(g), ctypes.byref(s), 0, ctypes.byref(h))
    return st, h


GOOD_GRID = dict(nx=16, ny=16, nz=0, dx=1.0, dy=1.0, dz=1.0)


@pytest.mark.parametrize("grid_kw,scan_kw,expect", [
    (dict(GOOD_GRID, nx=0), dict(kind=1, n_views=1, n_rows=1, n_cols=4, du=1.0, view_angle=[0.0]), -2),
    (dict(GOOD_GRID, dx=-1.0), dict(kind=1, n_views=1, n_rows=1, n_cols=4, du=1.0, view_angle=[0.0]), -2),
    (GOOD_GRID, dict(kind=99, n_views=1, n_rows=1, n_cols=4, du=1.0, view_angle=[0.0]), -1),
    (GOOD_GRID, dict(kind=1, n_views=1, n_rows=1, n_cols=4, du=1.0), -1),                 # no angles
    (GOOD_GRID, dict(kind=1, n_views=0, n_rows=1, n_cols=4, du=1.0, view_angle=[0.0]), -2),
    (GOOD_GRID, dict(kind=1, n_views=1, n_rows=2, n_cols=4, du=1.0, view_angle=[0.0]), -2),  # 2D, 2 rows
    (GOOD_GRID, dict(kind=5, n_views=1, n_rows=2, n_cols=4, du=1.0, dv=1.0, sod=50.0, sdd=80.0,
                     view_angle=[0.0]), -2),                                                  # 3D kind, 2D grid
    (GOOD_GRID, dict(kind=2, n_views=1, n_rows=1, n_cols=4, du=1.0, sod=0.0, sdd=80.0, view_angle=[0.0]), -2),
    (GOOD_GRID, dict(kind=2, n_views=1, n_rows=1, n_cols=4, du=1.0, sod=50.0, sdd=-1.0, view_angle=[0.0]), -2),
    (GOOD_GRID, dict(kind=2, n_views=1, n_rows=1, n_cols=4, du=1.0, sod=50.0, sdd=80.0,
                     view_angle=[float("nan")]), -2),
    (GOOD_GRID, dict(kind=3, n_views=1, n_rows=1, n_cols=4, du=2.0, sod=50.0, view_angle=[0.0]), -2),  # |gamma| >= pi/2
    (GOOD_GRID, dict(kind=7, n_rays=0, ray_params=[0.0, 0.0]), -2),
    (dict(nx=2048, ny=2048, nz=1024, dx=1.0, dy=1.0, dz=1.0),
     dict(kind=4, n_views=1, n_rows=1, n_cols=1, du=1.0, dv=1.0, view_angle=[0.0], view_phi2=[0.0]), -3),
])
def test_validation_rejects_before_any_gpu_work(lib, grid_kw, scan_kw, expect):
    st, h = _create(lib, grid_kw, scan_kw)
    assert st == expect, lib.xrt_last_error().decode()
    assert not h.value
    assert lib.xrt_last_error().decode() != ""


def test_null_arguments(lib):
    vp = ctypes.c_void_p
    assert lib.xrt_forward(None, vp(1), vp(1), 1, None) == -1
    assert lib.xrt_adjoint(None, vp(1), vp(1), 1, 0, None) == -1
    assert lib.xrt_plan_destroy(None) == 0
    assert lib.xrt_plan_create(None, None, 0, None) == -1
