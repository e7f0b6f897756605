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


# ------------------------------------------------------------------ simplex basis
# Simplex s of a unit is the set of points whose local index coordinates (in [0, 1] per
# axis), sorted from largest to smallest, come in the s-th axis order below (Kuhn's
# triangulation of the pixel / voxel in index coordinates).
SIMPLEX_ORDERS = {2: [(0, 1), (1, 0)],
                  3: [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]}


def _index_line(g: dict, p, th):
    """Index coordinates of the line: xi(t) = x0 + t om, t the physical arc length
    (x: (x - cx)/dx + nx/2; y: ny/2 - (y - cy)/dy; z: nz/2 - (z - cz)/dz)."""
    p = np.asarray(p, dtype=np.float64).ravel()
    th = np.asarray(th, dtype=np.float64).ravel()
    d3 = int(g.get("nz", 0)) > 0
    axes = [("nx", "dx", "cx", +1), ("ny", "dy", "cy", -1)] + ([("nz", "dz", "cz", -1)] if d3 else [])
    x0, om = [], []
    for a, (kn, kd, kc, sgn) in enumerate(axes):
        d, c, n = float(g.get(kd, 1.0)), float(g.get(kc, 0.0)), int(g[kn])
        x0.append(sgn * (p[a] - c) / d + n / 2.0)
        om.append(sgn * th[a] / d)
    return np.array(x0), np.array(om)


def simplex_lengths(g: dict, p, th):
    """Dense array (image shape + (S,)) of len(ray, simplex) for every simplex: the line
    clipped against the simplex's half-spaces (closed), one simplex at a time."""
    x0, om = _index_line(g, p, th)
    dim = x0.size
    shape = tuple(int(g[k]) for k in (["nz"] if dim == 3 else []) + ["ny", "nx"])
    orders = SIMPLEX_ORDERS[dim]
    out = np.zeros(shape + (len(orders),))
    for unit in np.ndindex(*shape):
        base = np.array(unit[::-1], dtype=np.float64)          # (i, j[, k]) along x, y[, z]
        a0 = x0 - base                                          # local coordinates at t = 0
        for s, order in enumerate(orders):
            # constraints alpha + beta t >= 0: l_first <= 1, l_o[m] >= l_o[m+1], l_last >= 0
            cons = [(1.0 - a0[order[0]], -om[order[0]])]
            for m in range(dim - 1):
                u, v = order[m], order[m + 1]
                cons.append((a0[u] - a0[v], om[u] - om[v]))
            cons.append((a0[order[-1]], om[order[-1]]))
            lo, hi = -np.inf, np.inf
            for alpha, beta in cons:
                if beta > 0.0:
                    lo = max(lo, -alpha / beta)
                elif beta < 0.0:
                    hi = min(hi, -alpha / beta)
                elif alpha < 0.0:
                    hi = -np.inf
            out[unit + (s,)] = max(0.0, hi - lo)
    return out
