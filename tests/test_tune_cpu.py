"""Autotuner cache handling (host logic): corrupt or missing caches and invalid entries
fall back to the default launch shape; signatures separate geometry classes."""
import json

import numpy as np

from paper_2006_00686_amd import tune


def _geom(nx=64, helical=False):
    grid = dict(nx=nx, ny=nx, nz=nx, dx=1.0, dy=1.0, dz=1.0)
    scan = dict(kind="cone_flat", angles=np.arange(36) * 0.1, ncols=80, nrows=60, du=1.0, dv=1.0, sod=500.0,
                sdd=800.0, view_z=np.linspace(-5, 5, 36) if helical else None)
    return grid, scan


def test_missing_and_corrupt_cache(tmp_path):
    p = tmp_path / "c.json"
    assert tune.load_cache(str(p)) == {}
    p.write_text("{ not json")
    assert tune.load_cache(str(p)) == {}
    p.write_text("[1, 2, 3]")
    assert tune.load_cache(str(p)) == {}


def test_invalid_entries_fall_back():
    assert tune.valid_entry(None) is None
    assert tune.valid_entry({"packet_cols": 48, "xcd_remap": 0}) is None
    assert tune.valid_entry({"packet_cols": 32, "xcd_remap": 2}) is None
    assert tune.valid_entry({"packet_cols": "32", "xcd_remap": 0}) is None
    assert tune.valid_entry({"packet_cols": 32, "xcd_remap": 1, "ms": 1.0}) == {"packet_cols": 32, "xcd_remap": 1}
    assert all(tune.valid_entry({"packet_cols": pc, "xcd_remap": xr}) == {"packet_cols": pc, "xcd_remap": xr}
               for pc, xr in tune.CANDIDATES)


def test_signature_separates_geometry_classes():
    a = tune.signature(*_geom(64), "dev")
    assert a == tune.signature(*_geom(64), "dev")
    assert a != tune.signature(*_geom(96), "dev")
    assert a != tune.signature(*_geom(64, helical=True), "dev")
    assert a != tune.signature(*_geom(64), "other")


def test_save_and_reload(tmp_path):
    p = str(tmp_path / "sub" / "c.json")
    assert tune.save_cache({"k": {"packet_cols": 16, "xcd_remap": 1}}, p)
    assert tune.valid_entry(tune.load_cache(p)["k"]) == {"packet_cols": 16, "xcd_remap": 1}
    assert json.load(open(p))["k"]["packet_cols"] == 16
