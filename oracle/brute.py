"""Per-unit brute force for tiny grids -- TEST INFRASTRUCTURE.

For every unit of the image, clip the ray's line against that unit's box
(Liang-Barsky slab clipping) and report the length inside it.  This is the plain
definition of the intersection length (Sec. 2.2.1 eq. intersection_length,
Sec. 3.2.1 eq. intersection_length_3D) evaluated unit by unit over all N^d units,
with no ordering or range logic.  Axes along which the ray does not move use the
half-open membership of the ambiguity resolution (Sec. 4.1: the unit with the
bigger 1D index wins): x in [lo, hi), y in (lo, hi], z in (lo, hi].
"""
from __future__ import annotations

import numpy as np


def _axis_bounds(n, d, c, sign):
    """Physical [lo, hi] of the n units along one axis.  sign=+1: index grows with the
    coordinate (x); sign=-1: index grows against it (y, z)."""
    q = np.arange(n, dtype=np.float64)
    if sign > 0:
        lo = c + (q - n / 2.0) * d
        hi = c + (q - n / 2.0 + 1.0) * d
    else:
        lo = c + (n / 2.0 - q - 1.0) * d
        hi = c + (n / 2.0 - q) * d
    return lo, hi


def unit_lengths(g: dict, p, th):
    """Dense array (image shape) of len(ray, unit) for every unit."""
    L, U = unit_intervals(g, p, th)
    return np.maximum(U - L, 0.0)


def unit_intervals(g: dict, p, th):
    """Dense arrays (image shape) of the parameters t where the line p + t th enters and
    leaves every unit (U <= L: not crossed)."""
    p = np.asarray(p, dtype=np.float64).ravel()
    th = np.asarray(th, dtype=np.float64).ravel()
    nz = int(g.get("nz", 0))
    dims = [("nx", "dx", "cx", +1), ("ny", "dy", "cy", -1)]
    if nz > 0:
        dims.append(("nz", "dz", "cz", -1))
    tlo, thi, member = [], [], []
    for a, (kn, kd, kc, sgn) in enumerate(dims):
        n = int(g[kn])
        lo, hi = _axis_bounds(n, float(g.get(kd, 1.0)), float(g.get(kc, 0.0)), sgn)
        if th[a] != 0.0:
            t0 = (lo - p[a]) / th[a]
            t1 = (hi - p[a]) / th[a]
            tlo.append(np.minimum(t0, t1))
            thi.append(np.maximum(t0, t1))
            member.append(np.ones(n, dtype=bool))
        else:
            if sgn > 0:
                m = (lo <= p[a]) & (p[a] < hi)
            else:
                m = (lo < p[a]) & (p[a] <= hi)
            tlo.append(np.full(n, -np.inf))
            thi.append(np.full(n, np.inf))
            member.append(m)
    if nz > 0:
        # axis order of the array: [k][j][i]
        L = np.maximum(np.maximum(tlo[2][:, None, None], tlo[1][None, :, None]), tlo[0][None, None, :])
        U = np.minimum(np.minimum(thi[2][:, None, None], thi[1][None, :, None]), thi[0][None, None, :])
        M = member[2][:, None, None] & member[1][None, :, None] & member[0][None, None, :]
    else:
        L = np.maximum(tlo[1][:, None], tlo[0][None, :])
        U = np.minimum(thi[1][:, None], thi[0][None, :])
        M = member[1][:, None] & member[0][None, :]
    L = np.where(M, L, 0.0)
    U = np.where(M, U, 0.0)
    return L, U


def hits(g: dict, p, th, eps=0.0):
    """(1D indices, lengths) with length > eps, sorted by index."""
    ln = unit_lengths(g, p, th).ravel()
    idx = np.nonzero(ln > eps)[0]
    return idx.astype(np.int64), ln[idx]


def matrix(g: dict, lines_p, lines_th):
    """Dense projection matrix A[ray, unit] (tiny grids only)."""
    rows = [unit_lengths(g, lines_p[r], lines_th[r]).ravel() for r in range(len(lines_p))]
    return np.stack(rows, axis=0)


def one_unit_lengths(g: dict, P, TH, unit):
    """len(ray, unit) of many lines (P, TH: [n][d] points and directions) through one
    unit, (k, j, i) in 3D or (j, i) in 2D: the same slab clip as unit_intervals, for one
    box and many rays (sampled checks of the adjoint at full size)."""
    P = np.asarray(P, dtype=np.float64)
    TH = np.asarray(TH, dtype=np.float64)
    nz = int(g.get("nz", 0))
    dims = [("nx", "dx", "cx", +1), ("ny", "dy", "cy", -1)]
    if nz > 0:
        dims.append(("nz", "dz", "cz", -1))
    q_of_axis = list(unit)[::-1]           # unit is (k, j, i) / (j, i); axes are x, y, z
    n = P.shape[0]
    L = np.full(n, -np.inf)
    U = np.full(n, np.inf)
    member = np.ones(n, dtype=bool)
    for a, (kn, kd, kc, sgn) in enumerate(dims):
        q = int(q_of_axis[a])
        lo, hi = _axis_bounds(int(g[kn]), float(g.get(kd, 1.0)), float(g.get(kc, 0.0)), sgn)
        lo, hi = lo[q], hi[q]
        d = TH[:, a]
        mv = d != 0.0
        with np.errstate(divide="ignore", invalid="ignore"):
            t0 = (lo - P[:, a]) / d
            t1 = (hi - P[:, a]) / d
        L = np.where(mv, np.maximum(L, np.minimum(t0, t1)), L)
        U = np.where(mv, np.minimum(U, np.maximum(t0, t1)), U)
        inside = (lo <= P[:, a]) & (P[:, a] < hi) if sgn > 0 else (lo < P[:, a]) & (P[:, a] <= hi)
        member &= mv | inside
    return np.where(member, np.maximum(U - L, 0.0), 0.0)
