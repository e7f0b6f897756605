"""The paper's closed-form candidate ranges -- TEST INFRASTRUCTURE.

Only tests/ use this module; it shares no code with the HIP path.

For a ray in Case 1 of Sec. 2.2.1 (2D, phi in (0, pi/2)) or of Sec. 3.2.1 (3D,
(phi1, phi2) in (0, pi/2)^2) on the paper's unit grid centred at the origin
(d = 1, unit (k, j, i) = [i - Nx/2, i - Nx/2 + 1] x [Ny/2 - j - 1, Ny/2 - j] x
[Nz/2 - k - 1, Nz/2 - k]), the units with a non-vanishing intersection are listed
slab by slab as the paper does:

* 2D, given i: the valid j satisfy C_1 - tan(phi) - 1 < j < C_1 (eq. restriction_j),
  C_1 = Ny/2 - s cos(phi) - C_x sin(phi), C_x = (i - Nx/2 + s sin(phi)) / cos(phi)
  (eq. C_xC_y);
* 2D, given j: the valid i satisfy C_2 - cot(phi) - 1 < i < C_2 (eq. restriction_i),
  C_2 = Nx/2 - s sin(phi) + C_y cos(phi), C_y = (Ny/2 - j - s cos(phi)) / sin(phi);
* 3D, given i: the valid j by eq. restriction_j_3D, then for each of them the valid k by
  the two inequalities of eq. restriction_k_3D_1 (C_1, C_2, C_3 and C_x, C_y, C_z as in
  eq. C_xC_yC_z);

and the length of each listed unit is C_up - C_low (eqs. range_length,
range_length_3D) with C_low, C_up the bounds of eqs. conditions_2D_1 / conditions_3D_1.
The ranges are intersected with the image's index range, the only step the paper leaves
implicit.  Plain Python loops in FP64: for small grids only.
"""
from __future__ import annotations

import math


def _open_integers(lo: float, hi: float, n: int):
    """Integers q with lo < q < hi and 0 <= q < n."""
    first = max(0, math.floor(lo) + 1)
    last = min(n - 1, math.ceil(hi) - 1)
    return [q for q in range(first, last + 1) if lo < q < hi]


def case1_2d_steps(nx: int, ny: int, s: float, phi: float):
    """The steps of the 2D range computation for every i, as the paper's hand
    computations of Test suite 1 list them: [(i, C_x, C_1, {j: (C_y, length)})]."""
    assert 0.0 < phi < math.pi / 2
    c, sn = math.cos(phi), math.sin(phi)
    steps = []
    for i in range(nx):
        cx = (i - nx / 2 + s * sn) / c
        c1 = ny / 2 - s * c - cx * sn
        js = {}
        for j in _open_integers(c1 - math.tan(phi) - 1.0, c1, ny):
            cy = (ny / 2 - j - s * c) / sn
            c_low = max(cx, cy - 1.0 / sn)
            c_up = min(cx + 1.0 / c, cy)
            js[j] = (cy, c_up - c_low)
        steps.append((i, cx, c1, js))
    return steps


def case1_2d(nx: int, ny: int, s: float, phi: float):
    """Units (j, i) -> length of the 2D ray (s, phi), phi in (0, pi/2), listed by i
    (eq. restriction_j) with C_up - C_low (eq. range_length)."""
    return {(j, i): ln for i, _, _, js in case1_2d_steps(nx, ny, s, phi) for j, (_, ln) in js.items()}


def case1_2d_given_j(nx: int, ny: int, s: float, phi: float):
    """The same units listed by j (eq. restriction_i)."""
    assert 0.0 < phi < math.pi / 2
    c, sn = math.cos(phi), math.sin(phi)
    out = {}
    for j in range(ny):
        cy = (ny / 2 - j - s * c) / sn
        c2 = nx / 2 - s * sn + cy * c
        for i in _open_integers(c2 - 1.0 / math.tan(phi) - 1.0, c2, nx):
            cx = (i - nx / 2 + s * sn) / c
            out[(j, i)] = min(cx + 1.0 / c, cy) - max(cx, cy - 1.0 / sn)
    return out


def case1_3d_steps(nx: int, ny: int, nz: int, s1: float, s2: float, phi1: float, phi2: float):
    """The steps of the 3D range computation for every i, as the paper's hand computations
    of Test suite 3 list them: [(i, C_x, (j_lo, j_hi), {j: (C_y, (k_lo, k_hi),
    {k: length})})], (j_lo, j_hi) and (k_lo, k_hi) the open intervals of eqs.
    restriction_j_3D and restriction_k_3D_1 (the two k intervals intersected)."""
    assert 0.0 < phi1 < math.pi / 2 and 0.0 < phi2 < math.pi / 2
    c1_, s1_ = math.cos(phi1), math.sin(phi1)
    c2_, s2_ = math.cos(phi2), math.sin(phi2)
    wx, wy, wz = 1.0 / (c2_ * c1_), 1.0 / (c2_ * s1_), 1.0 / s2_   # a unit's extent in t
    steps = []
    for i in range(nx):
        cx = (i - nx / 2 + s1 * s1_ + s2 * s2_ * c1_) * wx
        c1 = ny / 2 - s1 * c1_ + s2 * s2_ * s1_ - cx * c2_ * s1_
        c2 = nz / 2 - s2 * c2_ - cx * s2_
        jr = (c1 - math.tan(phi1) - 1.0, c1)
        js = {}
        for j in _open_integers(*jr, ny):
            cy = (ny / 2 - j - s1 * c1_ + s2 * s2_ * s1_) * wy
            c3 = nz / 2 - s2 * c2_ - cy * s2_
            kr = (max(c2 - math.tan(phi2) / c1_ - 1.0, c3 - 1.0), min(c2, c3 + math.tan(phi2) / s1_))
            ks = {}
            for k in _open_integers(*kr, nz):
                cz = (nz / 2 - k - s2 * c2_) * wz
                c_low = max(cx, cy - wy, cz - wz)
                c_up = min(cx + wx, cy, cz)
                ks[k] = c_up - c_low
            js[j] = (cy, kr, ks)
        steps.append((i, cx, jr, js))
    return steps


def case1_3d(nx: int, ny: int, nz: int, s1: float, s2: float, phi1: float, phi2: float):
    """Units (k, j, i) -> length of the 3D ray (s1, s2, phi1, phi2), both angles in
    (0, pi/2), listed by i (eqs. restriction_j_3D, restriction_k_3D_1) with
    C_up - C_low (eq. range_length_3D)."""
    return {(k, j, i): ln for i, _, _, js in case1_3d_steps(nx, ny, nz, s1, s2, phi1, phi2)
            for j, (_, _, ks) in js.items() for k, ln in ks.items()}


def to_1d(units: dict, nx: int, ny: int):
    """{1D index I = (k ny + j) nx + i: length} of a dict keyed by (j, i) or (k, j, i)."""
    res = {}
    for key, ln in units.items():
        k, j, i = key if len(key) == 3 else (0,) + key
        res[(k * ny + j) * nx + i] = ln
    return res
