"""CPU run of the GPU path's own per-ray code (xrt_walk.h + the plan's FP64 table
expansion, compiled for the host): every index the forward kernel dereferences is in
range, and its hit lists and line integrals agree with the FP64 oracle.  This checks the
kernels' indexing and the geometry expansion before any GPU launch."""
import math
import os
import struct
import subprocess

import numpy as np
import pytest

from oracle import core as ocore
from oracle import geometry as ogeom
from paper_2006_00686_amd import build as xbuild
from paper_2006_00686_amd import inputs
from tests import helpers as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host_walk", "walk_check.cpp")
KIND = {"par2d": 1, "fan2d_flat": 2, "fan2d_arc": 3, "par3d": 4, "cone_flat": 5, "cone_arc": 6,
        "raylist2d": 7, "raylist3d": 8}
PI = math.pi


@pytest.fixture(scope="session")
def walker(tmp_path_factory):
    objs = [os.path.join(xbuild.BUILD, os.path.splitext(src)[0] + ".o") for src in xbuild.SOURCES]
    if not all(os.path.exists(o) for o in objs):
        xbuild.build()
    exe = str(tmp_path_factory.mktemp("walk") / "walk_check")
    cmd = [xbuild._hipcc(), "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
           "-fno-honor-nans", "-I" + os.path.join(ROOT, "include"), SRC, "-x", "none"] + objs + ["-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


def run_walk(exe, tmpdir, grid, scan, eps=0.0, simplex=False):
    kind = scan["kind"]
    vals = [KIND[kind], grid["nx"], grid["ny"], grid.get("nz", 0), grid.get("dx", 1.0), grid.get("dy", 1.0),
            grid.get("dz", 1.0), grid.get("cx", 0.0), grid.get("cy", 0.0), grid.get("cz", 0.0)]
    if kind.startswith("raylist"):
        rays = np.asarray(scan["rays"], dtype=np.float64).ravel()
        w = 2 if kind == "raylist2d" else 4
        head2 = [0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, rays.size // w, eps]
        body = [rays]
    else:
        ang = np.asarray(scan["angles"], dtype=np.float64)
        hz = scan.get("view_z") is not None
        hp = scan.get("phi2") is not None
        head2 = [ang.size, scan.get("nrows", 1), scan["ncols"], scan["du"], scan.get("dv", 1.0), scan.get("u0", 0.0),
                 scan.get("v0", 0.0), scan.get("sod", 0.0), scan.get("sdd", 0.0), int(hz), int(hp), 0, eps]
        body = [ang] + ([np.asarray(scan["view_z"], float)] if hz else []) + ([np.asarray(scan["phi2"], float)] if hp else [])
    sp = os.path.join(tmpdir, "scan.txt")
    hp_ = os.path.join(tmpdir, "hits.bin")
    with open(sp, "w") as f:
        f.write(" ".join(repr(float(v)) if isinstance(v, float) else str(v) for v in vals) + "\n")
        f.write(" ".join(repr(float(v)) if isinstance(v, float) else str(v) for v in head2) + "\n")
        for b in body:
            f.write(" ".join(repr(float(x)) for x in b) + "\n")
    res = subprocess.run([exe, sp, hp_] + (["simplex"] if simplex else []), capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    rows = []
    with open(hp_, "rb") as f:
        data = f.read()
    off = 0
    while off < len(data):
        (n,) = struct.unpack_from("<i", data, off)
        off += 4
        idx = np.empty(n, np.int64)
        ln = np.empty(n, np.float64)
        for k in range(n):
            idx[k], ln[k] = struct.unpack_from("<id", data, off)
            off += 12
        rows.append((idx, ln))
    return rows


def dense_forward(rows, img):
    f = img.astype(np.float64).ravel()
    return np.array([float(np.dot(f[i], l)) for i, l in rows])


SCANS = H.small_scans()


@pytest.mark.parametrize("name,grid,scan", SCANS, ids=[s[0] for s in SCANS])
def test_host_walk_in_bounds_and_matches_oracle(walker, tmp_path, name, grid, scan):
    rows = run_walk(walker, str(tmp_path), grid, scan)
    img = inputs.random_image(inputs.image_shape(grid), 3)
    ref, scl = H.forward_bar(grid, scan, img)
    got = dense_forward(rows, img)
    # FP64 end to end: far inside the 1e-5 bar
    H.assert_within_bar(got, ref, scl, rtol=1e-9, what=f"host walk {name}")


@pytest.mark.parametrize("d3", [False, True])
def test_host_walk_random_and_grid_aligned_rays(walker, tmp_path, d3):
    grid = dict(nx=9, ny=8, nz=(7 if d3 else 0), dx=1.0, dy=1.0, dz=1.0)
    rng = np.random.default_rng(17)
    rays = (inputs.random_rays3d if d3 else inputs.random_rays2d)(1500, 6.0, 5 + d3)
    # grid-aligned rays: axis-parallel and on grid lines / planes, including the border
    al = []
    for s in np.arange(-5, 5.5, 0.5):
        if d3:
            for s2 in (-3.5, -1.0, 0.0, 2.5, 3.5):
                al += [[s, s2, 0.0, 0.0], [s, s2, PI / 2, 0.0], [s, s2, 0.0, PI / 2], [s, s2, 0.0, PI / 4],
                       [s, s2, PI, 0.0], [s, s2, 3 * PI / 2, -PI / 4]]
        else:
            al += [[s, 0.0], [s, PI / 2], [s, PI], [s, 3 * PI / 2], [s, PI / 4], [s, 3 * PI / 4]]
    rays = np.concatenate([rays, np.array(al)], axis=0)
    kind = "raylist3d" if d3 else "raylist2d"
    rows = run_walk(walker, str(tmp_path), grid, dict(kind=kind, rays=rays))
    p, th = (ogeom.par3d_lines(*rays.T) if d3 else ogeom.par2d_lines(*rays.T))
    img = inputs.random_image(inputs.image_shape(grid), 4)
    f = img.astype(np.float64).ravel()
    for r in range(len(rays)):
        oi, ol = ocore.ray_hits_line(grid, p[r], th[r], 1e-9)
        gi, gl = rows[r]
        o = np.argsort(gi)
        keep = gl[o] > 1e-9
        np.testing.assert_array_equal(gi[o][keep], oi, err_msg=f"ray {r} {rays[r]}")
        np.testing.assert_allclose(gl[o][keep], ol, atol=1e-9)
        ref = ocore.forward_lines(grid, p[r:r + 1], th[r:r + 1], f.reshape(img.shape))[0]
        assert abs(np.dot(f[gi], gl) - ref) < 1e-9 * max(1.0, abs(ref))
    del rng


def test_host_walk_worked_examples(walker, tmp_path, golden_dir):
    from tests.test_oracle_pins import read_table
    from tests.test_gpu_parity import WORKED_SCANS
    for fname, grid, scan in WORKED_SCANS:
        (idx, ln), = run_walk(walker, str(tmp_path), grid, scan, eps=1e-9)
        gi, gl = read_table(os.path.join(golden_dir, fname))
        o = np.argsort(idx)
        np.testing.assert_array_equal(idx[o], gi)
        np.testing.assert_allclose(ln[o], gl, rtol=6e-6, atol=1e-6)


def test_host_walk_par2d_128_full(walker, tmp_path):
    cfg = inputs.workload("par2d_128")
    rows = run_walk(walker, str(tmp_path), cfg["grid"], cfg["scan"])
    img = inputs.make_image(cfg)
    ref, scl = H.forward_bar(cfg["grid"], cfg["scan"], img)
    H.assert_within_bar(dense_forward(rows, img), ref, scl, rtol=1e-9, what="par2d_128 host walk")


# ------------------------------------------------------------------ simplex basis

def dense_rows(rows, n):
    """Dense per-ray vectors from hit lists (repeated indices summed)."""
    out = np.zeros((len(rows), n))
    for r, (i, l) in enumerate(rows):
        np.add.at(out[r], i, l)
    return out


@pytest.mark.parametrize("name,grid,scan", SCANS, ids=[s[0] for s in SCANS])
def test_host_simplex_walk_matches_oracle(walker, tmp_path, name, grid, scan):
    """The kernels' simplex cutting (xrt_simplex.h) run on the host over every scan kind:
    every simplex index in range, and line integrals of a random simplex image equal to
    the FP64 simplex oracle's."""
    rows = run_walk(walker, str(tmp_path), grid, scan, simplex=True)
    img = np.random.default_rng(8).uniform(size=ocore.simplex_image_shape(grid))
    p, th = ogeom.expand(scan)
    ref = ocore.forward_simplex_lines(grid, p, th, img)
    scl = ocore.forward_simplex_lines(grid, p, th, np.abs(img))
    got = np.array([float(np.dot(img.ravel()[i], l)) for i, l in rows])
    H.assert_within_bar(got, ref, scl, rtol=1e-9, what=f"host simplex walk {name}")


@pytest.mark.parametrize("d3", [False, True])
def test_host_simplex_walk_random_and_aligned_rays(walker, tmp_path, d3):
    """Per-simplex lengths against the oracle's, ray by ray, on random rays and on rays
    along the grid and diagonal planes (the resolution of Sec. 4.1 on both kinds of
    face)."""
    grid = dict(nx=7, ny=6, nz=(5 if d3 else 0), dx=1.0, dy=1.0, dz=1.0)
    rays = (inputs.random_rays3d if d3 else inputs.random_rays2d)(800, 5.0, 15 + d3)
    al = []
    for s in np.arange(-4, 4.5, 0.5):
        if d3:
            for s2 in (-2.5, -1.0, 0.0, 1.5, 2.5):
                al += [[s, s2, 0.0, 0.0], [s, s2, PI / 2, 0.0], [s, s2, 0.0, PI / 2], [s, s2, PI / 4, 0.0],
                       [s, s2, 3 * PI / 4, 0.0], [s, s2, 0.0, PI / 4]]
        else:
            al += [[s, 0.0], [s, PI / 2], [s, PI / 4], [s, 3 * PI / 4], [s, -PI / 4]]
    rays = np.concatenate([rays, np.array(al)], axis=0)
    kind = "raylist3d" if d3 else "raylist2d"
    rows = run_walk(walker, str(tmp_path), grid, dict(kind=kind, rays=rays), simplex=True)
    p, th = (ogeom.par3d_lines(*rays.T) if d3 else ogeom.par2d_lines(*rays.T))
    n = int(np.prod(ocore.simplex_image_shape(grid)))
    got = dense_rows(rows, n)
    for r in range(len(rays)):
        want = np.zeros(n)
        oi, ol = ocore.ray_hits_simplex_line(grid, p[r], th[r], 0.0)
        np.add.at(want, oi, ol)
        np.testing.assert_allclose(got[r], want, atol=1e-9, err_msg=f"ray {r} {rays[r]}")
