"""Shared helpers of the test suite (comparison bars, small scans)."""
from __future__ import annotations

import numpy as np

from oracle import core as ocore
from oracle import geometry as ogeom

# Line integrals within 1e-5 relative: |g_gpu - g_ref| <= RTOL * sum_I |f_I| len(r, I)
RTOL = 1e-5
# Plus an absolute floor at the oracle's own FP64 length resolution: a ray through a unit's
# edge or corner touches it with zero length in exact arithmetic (Sec. 2.2.1: the overlap
# "is just a point"), but FP64 rounding of the crossing parameters (magnitudes up to
# ~1e3) can leave a sliver of ~1e-13 on either side.  1e-9 * max|input| is four orders
# above such slivers and far below any real error.
ABS_FLOOR = 1e-9


def forward_bar(grid, scan, img):
    """Oracle forward of img and of |img| (the per-ray scale of the bar)."""
    p, th = ogeom.expand(scan)
    ref = ocore.forward_lines(grid, p, th, img.astype(np.float64))
    scl = ocore.forward_lines(grid, p, th, np.abs(img).astype(np.float64))
    return ref, scl


def adjoint_bar(grid, scan, sino):
    p, th = ogeom.expand(scan)
    ref = ocore.adjoint_lines(grid, p, th, sino.astype(np.float64))
    scl = ocore.adjoint_lines(grid, p, th, np.abs(sino).astype(np.float64))
    return ref, scl


def assert_within_bar(got, ref, scl, rtol=RTOL, what="", floor=None):
    """|got - ref| <= rtol * scl + floor, with floor = ABS_FLOOR * max|ref| unless given."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    scl = np.asarray(scl, dtype=np.float64).ravel()
    err = np.abs(got - ref)
    if floor is None:
        floor = ABS_FLOOR * float(np.max(scl)) if scl.size else 0.0
    bar = rtol * scl + floor + 1e-30
    bad = np.nonzero(err > bar)[0]
    if bad.size:
        i = bad[np.argmax(err[bad] / bar[bad])]
        raise AssertionError(f"{what}: {bad.size}/{got.size} elements outside the bar; worst #{i}: "
                             f"got {got[i]!r} ref {ref[i]!r} scale {scl[i]!r} err/bar {err[i] / bar[i]:.3g}")


def generic_rays(grid, p, th, mu=1e-3):
    """Indices of rays whose every hit has length >= mu (no near-vertex/edge passage)."""
    keep = []
    for r in range(len(p)):
        idx, ln = ocore.ray_hits_line(grid, p[r], th[r], 0.0)
        if ln.size and ln.min() >= mu:
            keep.append(r)
    return np.array(keep, dtype=np.int64)


def small_scans():
    """Small scans of every kind, sized to span several 64-ray packets and a ragged tail."""
    pi = np.pi
    out = []
    g2 = dict(nx=37, ny=29, nz=0, dx=1.0, dy=1.0, cx=0.0, cy=0.0)
    angles = np.concatenate([[0.0, pi / 2], np.linspace(0.01, pi, 21, endpoint=False)])
    out.append(("par2d", g2, dict(kind="par2d", angles=angles, ncols=47, du=1.0, u0=0.0)))
    g2o = dict(nx=40, ny=33, nz=0, dx=0.8, dy=0.8, cx=3.0, cy=-2.5)
    out.append(("fan2d_flat", g2o, dict(kind="fan2d_flat", angles=np.linspace(0, 2 * pi, 30, endpoint=False),
                                         ncols=77, du=1.1, u0=0.2, sod=60.0, sdd=95.0)))
    out.append(("fan2d_arc", g2o, dict(kind="fan2d_arc", angles=np.linspace(0.1, 2 * pi, 25, endpoint=False),
                                        ncols=69, du=0.012, u0=0.0, sod=55.0)))
    g3 = dict(nx=21, ny=19, nz=17, dx=1.0, dy=1.0, dz=1.0, cx=0.0, cy=0.0, cz=0.0)
    out.append(("par3d", g3, dict(kind="par3d", angles=np.linspace(0, 2 * pi, 9, endpoint=False),
                                   phi2=np.linspace(-1.2, 1.2, 9), ncols=31, nrows=27, du=0.9, dv=0.9)))
    g3o = dict(nx=24, ny=20, nz=18, dx=1.1, dy=0.9, dz=1.2, cx=1.5, cy=-0.5, cz=0.7)
    out.append(("cone_flat", g3o, dict(kind="cone_flat", angles=np.linspace(0, 2 * pi, 12, endpoint=False),
                                        ncols=70, nrows=33, du=1.0, dv=1.0, sod=80.0, sdd=120.0)))
    vz = np.linspace(-6, 6, 15)
    out.append(("helical", g3o, dict(kind="cone_flat", angles=np.linspace(0, 3 * 2 * pi, 15, endpoint=False),
                                      ncols=67, nrows=9, du=1.0, dv=1.0, sod=80.0, sdd=120.0, view_z=vz)))
    # odd row count: the central row has v = 0 and its rays run in the grid plane z = 0
    # of an even-nz grid (the Sec. 4.1 resolution in 3D); odd column count: u = 0 rays
    g3e = dict(nx=20, ny=22, nz=16, dx=1.0, dy=1.0, dz=1.0, cx=0.0, cy=0.0, cz=0.0)
    out.append(("cone_zero_row", g3e, dict(kind="cone_flat", angles=np.arange(8) * (pi / 4), ncols=55,
                                            nrows=23, du=1.0, dv=1.0, sod=70.0, sdd=105.0)))
    out.append(("cone_arc", g3, dict(kind="cone_arc", angles=np.linspace(0, 2 * pi, 10, endpoint=False),
                                      ncols=65, nrows=21, du=0.006, dv=0.006, sod=90.0,
                                      view_z=np.linspace(-2, 2, 10))))
    return out
