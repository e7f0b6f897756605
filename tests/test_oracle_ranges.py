"""CPU: the paper's closed-form candidate ranges (eqs. restriction_j, restriction_i,
restriction_j_3D, restriction_k_3D_1, with the lengths of eqs. range_length and
range_length_3D; oracle/ranges.py) pinned by the printed tables of Sec. 5 and by the
per-unit brute-force clip, and then used to check the kernels' slab walk compiled for the
host: for every slab of the driving axis, the units the walk gives a positive length are
exactly the paper's range for that slab, with the paper's length."""
import math
import os

import numpy as np
import pytest

from oracle import brute
from oracle import geometry as G
from oracle import ranges
from tests.test_oracle_pins import read_table
from tests.test_walk_host import run_walk, walker  # noqa: F401  (session fixture)

PI = math.pi


def _generic_case1_rays(d3: bool, n: int, seed: int, dims, smax: float):
    """Random Case-1 rays whose every unit is either missed or crossed for more than
    1e-6 (away from the zero-length contacts where the strict inequalities decide)."""
    rng = np.random.default_rng(seed)
    g = dict(nx=dims[0], ny=dims[1], nz=(dims[2] if d3 else 0))
    out = []
    while len(out) < n:
        if d3:
            r = (rng.uniform(-smax, smax), rng.uniform(-smax, smax), rng.uniform(0.02, PI / 2 - 0.02),
                 rng.uniform(0.02, PI / 2 - 0.02))
            p, th = G.par3d_lines(*r)
        else:
            r = (rng.uniform(-smax, smax), rng.uniform(0.02, PI / 2 - 0.02))
            p, th = G.par2d_lines(*r)
        dense = brute.unit_lengths(g, p, th).ravel()
        if np.any((dense > 0) & (dense < 1e-6)):
            continue
        out.append(r)
    return g, out


def _brute_dict(g, r, d3):
    p, th = (G.par3d_lines(*r) if d3 else G.par2d_lines(*r))
    dense = brute.unit_lengths(g, p, th).ravel()
    return {int(I): float(dense[I]) for I in np.nonzero(dense > 0)[0]}


def _range_dict(g, r, d3):
    if d3:
        u = ranges.case1_3d(g["nx"], g["ny"], g["nz"], *r)
    else:
        u = ranges.case1_2d(g["nx"], g["ny"], *r)
    return ranges.to_1d(u, g["nx"], g["ny"])


def _assert_same(got: dict, ref: dict, tol: float, what: str):
    assert sorted(got) == sorted(ref), f"{what}: units {sorted(set(got) ^ set(ref))} differ"
    for I in ref:
        assert abs(got[I] - ref[I]) <= tol * max(1.0, abs(ref[I])), f"{what}: unit {I} {got[I]} vs {ref[I]}"


# ------------------------------------------------------------------ pins of the ranges

CASE1_TABLES = [
    ("t1_parallel2d.txt", dict(nx=3, ny=3, nz=0), (1.0, PI / 4)),
    ("t3_parallel3d.txt", dict(nx=3, ny=3, nz=3), (0.0, 0.0, PI / 4, PI / 4)),
    ("t4_cone_equiangular.txt", dict(nx=4, ny=4, nz=4), G.cone_equiangular(4.0, PI / 4, PI / 12, PI / 12)),
    ("t5_helical_equiangular.txt", dict(nx=4, ny=4, nz=4), G.cone_equiangular(4.0, PI / 4, PI / 12, PI / 12, 0.5)),
]


@pytest.mark.parametrize("fname,g,ray", CASE1_TABLES, ids=[c[0] for c in CASE1_TABLES])
def test_ranges_reproduce_the_printed_tables(fname, g, ray, golden_dir):
    """Tables of Test suites 1, 3, 4, 5 (all in Case 1): the units the closed-form ranges
    list and their C_up - C_low are the printed ones.  These rays pass through edges of
    the grid, where FP64 leaves slivers of ~1e-16 that exact arithmetic makes zero-length
    contacts; units of length <= 1e-12 are dropped, as in the oracle's table checks."""
    r = tuple(float(v) for v in ray)
    got = {I: v for I, v in _range_dict(g, r, len(r) == 4).items() if v > 1e-12}
    gi, gl = read_table(os.path.join(golden_dir, fname))
    assert sorted(got) == sorted(int(i) for i in gi)
    np.testing.assert_allclose([got[int(i)] for i in gi], gl, rtol=6e-6, atol=1e-6)


@pytest.mark.parametrize("d3", [False, True])
def test_ranges_match_brute_force(d3):
    """Random Case-1 rays over non-square grids: the ranges list exactly the units with a
    positive brute-force length, with the same lengths."""
    dims = (7, 5, 6) if d3 else (9, 6)
    g, rays = _generic_case1_rays(d3, 300, 31 + d3, dims, 4.0)
    hit_rays = 0
    for r in rays:
        ref = _brute_dict(g, r, d3)
        hit_rays += bool(ref)
        _assert_same(_range_dict(g, r, d3), ref, 1e-12, f"ray {r}")
    assert hit_rays > 150


def test_ranges_given_i_and_given_j_agree():
    """eq. restriction_j (slabs of i) and eq. restriction_i (slabs of j) list the same
    units with the same lengths."""
    g, rays = _generic_case1_rays(False, 200, 37, (8, 11), 5.0)
    for r in rays:
        a = ranges.case1_2d(g["nx"], g["ny"], *r)
        b = ranges.case1_2d_given_j(g["nx"], g["ny"], *r)
        assert sorted(a) == sorted(b)
        for key in a:
            assert abs(a[key] - b[key]) <= 1e-12


def test_ranges_width_bound():
    """A slab of i holds at most ceil(tan(phi)) + 1 valid j (the width of the open
    interval of eq. restriction_j is tan(phi) + 1): at most two candidates when the
    ray runs closer to x than to y, the count the kernels' slab walk provides for."""
    g, rays = _generic_case1_rays(False, 200, 41, (12, 12), 5.0)
    for s, phi in rays:
        u = ranges.case1_2d(12, 12, s, phi)
        per_i = {}
        for (j, i) in u:
            per_i[i] = per_i.get(i, 0) + 1
        assert max(per_i.values(), default=0) <= math.ceil(math.tan(phi)) + 1


# ------------------------------------------------------------------ the kernels' walk

@pytest.mark.parametrize("d3", [False, True])
def test_host_walk_slabs_equal_the_paper_ranges(walker, tmp_path, d3):  # noqa: F811
    """The kernels' per-ray walk (compiled for the host) on Case-1 rays given as a ray
    list: grouped by the driving index, its hit units are the paper's ranges slab by slab
    and its lengths are C_up - C_low."""
    dims = (10, 7, 8) if d3 else (11, 8)
    g, rays = _generic_case1_rays(d3, 250, 43 + d3, dims, 4.5)
    kind = "raylist3d" if d3 else "raylist2d"
    rows = run_walk(walker, str(tmp_path), dict(g, dx=1.0, dy=1.0, dz=1.0), dict(kind=kind, rays=np.array(rays)))
    nx = g["nx"]
    for r, (idx, ln) in zip(rays, rows):
        ref = _range_dict(g, r, d3)
        got = {}
        for I, L in zip(idx, ln):
            if L > 0:
                got[int(I)] = got.get(int(I), 0.0) + float(L)
        for i in range(nx):                      # slab by slab along x
            gs = {I: v for I, v in got.items() if I % nx == i}
            rs = {I: v for I, v in ref.items() if I % nx == i}
            _assert_same(gs, rs, 1e-10, f"ray {r} slab i={i}")
        assert len(got) == len(ref)


# ------------------------------------------------------------------ the paper's hand computations

R2, R3 = math.sqrt(2.0), math.sqrt(3.0)


def test_ranges_reproduce_hand_computation_of_test_suite_1():
    """Test suite 1 (2D parallel beam, 3 x 3 image, ray (1, pi/4)) computed by hand slab
    by slab: C_x, C_1, the valid j, C_y and the lengths.  For i = 1 the paper prints
    C_1 = 5/2 - 3 sqrt(2)/2; its own definition gives 2 - sqrt(2) (the range, j = 0, is
    the same either way)."""
    steps = ranges.case1_2d_steps(3, 3, 1.0, PI / 4)
    want = [
        (0, -3 * R2 / 2 + 1, 3 - R2, {0: (3 * R2 / 2 - 1, 2 - R2), 1: (R2 / 2 - 1, 2 * R2 - 2)}),
        (1, -R2 / 2 + 1, 2 - R2, {0: (3 * R2 / 2 - 1, 2 * R2 - 2)}),
        (2, None, None, {}),
    ]
    for (i, cx, c1, js), (wi, wcx, wc1, wjs) in zip(steps, want):
        assert i == wi and sorted(js) == sorted(wjs), (i, js)
        if wcx is not None:
            assert abs(cx - wcx) < 1e-12 and abs(c1 - wc1) < 1e-12
        for j, (cy, ln) in wjs.items():
            assert abs(js[j][0] - cy) < 1e-12 and abs(js[j][1] - ln) < 1e-12


def test_ranges_reproduce_hand_computation_of_test_suite_3():
    """Test suite 3 (3D parallel beam, 3 x 3 x 3 image, ray (0, 0, pi/4, pi/4)) by hand:
    C_x, the interval of j, C_y, the interval of k and the lengths, slab by slab.  The ray
    runs through grid edges, where FP64 puts interval ends within 1e-15 of the integers
    the exact values hit and admits units with slivers of ~1e-16; the exact hand
    computation's sets are those of length > 1e-12 (zero-length contacts are no hits)."""
    steps = ranges.case1_3d_steps(3, 3, 3, 0.0, 0.0, PI / 4, PI / 4)
    steps = [(i, cx, jr, {j: (cy, kr, {k: ln for k, ln in ks.items() if ln > 1e-12})
                          for j, (cy, kr, ks) in js.items() if any(ln > 1e-12 for ln in ks.values())})
             for i, cx, jr, js in steps]
    want = [
        (0, -3.0, (1.0, 3.0), {2: (-1.0, ((1 + R2) / 2, (3 + 3 * R2) / 2), {2: 3 * R2 / 2 - 1})}),
        (1, -1.0, (0.0, 2.0), {1: (1.0, ((1 - R2) / 2, (3 + R2) / 2), {0: 1 - R2 / 2, 1: R2, 2: 1 - R2 / 2})}),
        (2, 1.0, (-1.0, 1.0), {0: (3.0, ((1 - 3 * R2) / 2, (3 - R2) / 2), {0: 3 * R2 / 2 - 1})}),
    ]
    for (i, cx, jr, js), (wi, wcx, wjr, wjs) in zip(steps, want):
        assert i == wi and abs(cx - wcx) < 1e-12
        assert abs(jr[0] - wjr[0]) < 1e-12 and abs(jr[1] - wjr[1]) < 1e-12
        assert sorted(js) == sorted(wjs), (i, js)
        for j, (cy, kr, ks) in wjs.items():
            gcy, gkr, gks = js[j]
            assert abs(gcy - cy) < 1e-12 and abs(gkr[0] - kr[0]) < 1e-12 and abs(gkr[1] - kr[1]) < 1e-12
            assert sorted(gks) == sorted(ks), (i, j, gks)
            for k, ln in ks.items():
                assert abs(gks[k] - ln) < 1e-12
