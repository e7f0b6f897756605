"""CPU: the gathers' candidate detector columns contain every column whose ray crosses the
pixel, with the hardware reciprocal at its documented error bound.

The voxel-driven cone gather and the pixel-driven 2D fan gather find, per view, the
detector columns a pixel's shadow can cover with the hardware FP64 reciprocal (relative
error below 2^-20), then widen the column range by the plan's slack
1e-7 + (max |u| / du + 1) 2^-20 bins; the exact clip decides hits and lengths afterwards,
so a column left out of the range would be a lost hit.  This test writes the range
formulas of both kernels out in FP64 with every reciprocal moved by 2^-20 against the
range (the worst case for containment) and checks, for pixels spread over the image
(corners and edges included) and every view, that each column whose ray crosses the
pixel with positive length lies inside.  The rays are the oracle's lines (the paper's
transforms); the source and detector frame of the range formulas are checked against
them first.  Rows use the refined reciprocal (full FP64 precision), far inside their
1e-7-bin slack, and are not repeated here.
"""
import math

import numpy as np

from oracle import geometry as G
from paper_2006_00686_amd import inputs

EPS = 2.0 ** -20   # relative error bound of the hardware reciprocal estimate


def _bins(n, d, off):
    return (np.arange(n, dtype=np.float64) - (n - 1) / 2.0) * d + off


def _frames(scan):
    """Source S, detector-centre vector E (|E| = sdd) and unit u axis B per view, in xy,
    as the header documents them for flat detectors."""
    a = np.asarray(scan["angles"], dtype=np.float64)
    sod, sdd = float(scan["sod"]), float(scan["sdd"])
    if scan["kind"] == "fan2d_flat":
        S = sod * np.stack([-np.sin(a), np.cos(a)], 1)
    else:   # cone_flat
        S = -sod * np.stack([np.cos(a), np.sin(a)], 1)
    Eh = -S / np.linalg.norm(S, axis=1, keepdims=True)
    B = np.stack([-Eh[:, 1], Eh[:, 0]], 1)
    return S, sdd * Eh, B


def _xy_lines(scan):
    """The oracle's rays of every (view, column), projected onto xy: point and unit
    direction, arrays [views][cols][2]."""
    p, th = G.expand(scan)
    nv, nc = len(scan["angles"]), int(scan["ncols"])
    nr = 1 if scan["kind"] == "fan2d_flat" else int(scan["nrows"])
    p = p.reshape(nv, nr, nc, -1)[:, nr // 2, :, :2]
    th = th.reshape(nv, nr, nc, -1)[:, nr // 2, :, :2]
    th = th / np.linalg.norm(th, axis=-1, keepdims=True)
    return p, th


def _check_frames(scan, S, E, B, p, th):
    u = _bins(int(scan["ncols"]), scan["du"], scan.get("u0", 0.0))
    d = E[:, None, :] + u[None, :, None] * B[:, None, :]
    d = d / np.linalg.norm(d, axis=-1, keepdims=True)
    # parallel directions and the source on the line
    assert np.max(np.abs(d[..., 0] * th[..., 1] - d[..., 1] * th[..., 0])) < 1e-12
    rel = S[:, None, :] - p
    assert np.max(np.abs(rel[..., 0] * th[..., 1] - rel[..., 1] * th[..., 0])) < 1e-9 * np.max(np.abs(S))


def _hit_columns(p, th, xa, xb, ya, yb):
    """[views][cols] bool: the line crosses [xa, xb] x [ya, yb] with positive length."""
    lo = np.full(p.shape[:2], -np.inf)
    hi = np.full(p.shape[:2], np.inf)
    for ax, (a0, a1) in enumerate(((xa, xb), (ya, yb))):
        w = th[..., ax]
        with np.errstate(divide="ignore", invalid="ignore"):
            t0 = (a0 - p[..., ax]) / w
            t1 = (a1 - p[..., ax]) / w
        inside = (p[..., ax] > a0) & (p[..., ax] < a1)
        t0 = np.where(w == 0, np.where(inside, -np.inf, np.inf), t0)
        t1 = np.where(w == 0, np.where(inside, np.inf, -np.inf), t1)
        lo = np.maximum(lo, np.minimum(t0, t1))
        hi = np.minimum(hi, np.maximum(t0, t1))
    return hi - lo > 1e-9


def _uslack(scan):
    nc, du = int(scan["ncols"]), float(scan["du"])
    ubase = -(nc - 1) / 2.0 * du + scan.get("u0", 0.0)
    return 1e-7 + math.ldexp(max(abs(ubase), abs(ubase + (nc - 1) * du)) / du + 1.0, -20), ubase


def _columns(umin, umax, scan):
    nc, du = int(scan["ncols"]), float(scan["du"])
    us, ubase = _uslack(scan)
    c0 = np.maximum(np.ceil(np.clip((umin - ubase) / du - us, -1.0, nc)), 0)
    c1 = np.minimum(np.floor(np.clip((umax - ubase) / du + us, -1.0, nc)), nc - 1)
    return c0, c1


def _pixels(g, n, seed):
    rng = np.random.default_rng(seed)
    nx, ny = g["nx"], g["ny"]
    edge = [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1), (nx // 2, 0), (0, ny // 2)]
    return edge + [(int(rng.integers(nx)), int(rng.integers(ny))) for _ in range(n)]


def _bounds(g, i, j):
    dx, dy = g.get("dx", 1.0), g.get("dy", 1.0)
    xa = g.get("cx", 0.0) + (i - g["nx"] / 2.0) * dx
    yb = g.get("cy", 0.0) + (g["ny"] / 2.0 - j) * dy
    return xa, xa + dx, yb - dy, yb


def _assert_contained(hits, c0, c1, what):
    cols = np.arange(hits.shape[1])[None, :]
    missed = hits & ((cols < c0[:, None]) | (cols > c1[:, None]))
    assert not missed.any(), f"{what}: {int(missed.sum())} hit columns outside the candidate range"
    # the ranges stay tight: at most a few bins beyond the hit columns
    width = np.where(hits.any(1), c1 - c0 + 1 - hits.sum(1), 0)
    assert width.max() <= 4, f"{what}: range {int(width.max())} bins wider than the hits"


def test_cone_gather_corner_ranges_contain_every_hit_column():
    cfg = inputs.workload("cone_256")
    g, scan = cfg["grid"], cfg["scan"]
    S, E, B = _frames(scan)
    p, th = _xy_lines(scan)
    _check_frames(scan, S, E, B, p, th)
    sdd2 = float(scan["sdd"]) ** 2
    for (i, j) in _pixels(g, 40, 11):
        xa, xb, ya, yb = _bounds(g, i, j)
        umin = np.full(S.shape[0], np.inf)
        umax = np.full(S.shape[0], -np.inf)
        for px, py in ((xa, ya), (xb, ya), (xa, yb), (xb, yb)):
            ax, ay = px - S[:, 0], py - S[:, 1]
            u = sdd2 * (ax * B[:, 0] + ay * B[:, 1]) / (ax * E[:, 0] + ay * E[:, 1])
            # the estimate moved against the range: up for the lower end, down for the upper
            umin = np.minimum(umin, u * (1.0 + EPS * np.sign(u)))
            umax = np.maximum(umax, u * (1.0 - EPS * np.sign(u)))
        c0, c1 = _columns(umin, umax, scan)
        _assert_contained(_hit_columns(p, th, xa, xb, ya, yb), c0, c1, f"cone pixel ({i}, {j})")


def test_fan_gather_disc_ranges_contain_every_hit_column():
    cfg = inputs.workload("fan2d_512")
    g, scan = cfg["grid"], cfg["scan"]
    S, E, B = _frames(scan)
    p, th = _xy_lines(scan)
    _check_frames(scan, S, E, B, p, th)
    nc, du = int(scan["ncols"]), float(scan["du"])
    # the plan's disc bound: rho = half the pixel diagonal, dmin = least depth of the image
    # box along E over the views, A = asin(x) / x at x = rho / dmin (widened by 1e-9)
    rho = 0.5 * math.hypot(g["dx"], g["dy"])
    en = np.linalg.norm(E, axis=1)
    dmin = np.inf
    for cx in (0, 1):
        for cy in (0, 1):
            Px = g["cx"] + (cx - 0.5) * g["nx"] * g["dx"]
            Py = g["cy"] + (0.5 - cy) * g["ny"] * g["dy"]
            dmin = min(dmin, float(np.min(((Px - S[:, 0]) * E[:, 0] + (Py - S[:, 1]) * E[:, 1]) / en)))
    x = rho / dmin
    assert x < 0.5
    A = math.asin(x) / x * (1.0 + 1e-9)
    ubase = -(nc - 1) / 2.0 * du + scan.get("u0", 0.0)
    um = max(abs(ubase), abs(ubase + (nc - 1) * du)) + du
    umax2, g2r = um * um, A * rho / du
    e2 = E[:, 0] ** 2 + E[:, 1] ** 2
    for (i, j) in _pixels(g, 40, 12):
        xa, xb, ya, yb = _bounds(g, i, j)
        hits = _hit_columns(p, th, xa, xb, ya, yb)
        px, py = 0.5 * (xa + xb) - S[:, 0], 0.5 * (ya + yb) - S[:, 1]
        for delta in (-EPS, EPS):   # one estimate of 1/depth for the centre and the width
            r = (1.0 + delta) / (px * E[:, 0] + py * E[:, 1])
            uc = e2 * (px * B[:, 0] + py * B[:, 1]) * r
            hw = (e2 + np.maximum(umax2, uc * uc)) * g2r * r * du
            c0, c1 = _columns(uc - hw, uc + hw, scan)
            _assert_contained(hits, c0, c1, f"fan pixel ({i}, {j}), reciprocal error {delta:+.1e}")
