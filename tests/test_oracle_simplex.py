"""CPU: the FP64 oracle of the transform on the simplex basis (every pixel cut into 2
triangles, every voxel into 6 tetrahedra; the paper's polygonal / polyhedral extension,
Introduction "Contributions" and Sec. 4.2), pinned by hand-computed rays, by a per-simplex
brute force (the line clipped against each simplex's half-spaces), by the pixel / voxel
lengths of the unit oracle (the simplices of a unit partition it), and by the adjoint
identity."""
import os

import numpy as np
import pytest

from oracle import brute, core
from oracle import geometry as G
from paper_2006_00686_amd import inputs


def _read(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "simplex_examples.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, dims, ray, pairs = (x.strip() for x in line.split("|"))
            nx, ny, nz = (int(v) for v in dims.split())
            kind, *kv = ray.split()
            par = {k: np.array([float(c) for c in v.split(",")]) if "," in v else float(v)
                   for k, v in (x.split("=") for x in kv)}
            want = {int(a): float(b) for a, b in (x.split(":") for x in pairs.split())}
            rows.append((name, dict(nx=nx, ny=ny, nz=nz), kind, par, want))
    return rows


def _line(kind, par):
    if kind == "line":
        return par["p"], par["th"]
    if kind == "par2d":
        p, th = G.par2d_lines(np.array([par["s"]]), np.array([par["phi"]]))
    else:
        p, th = G.par3d_lines(np.array([par["s1"]]), np.array([par["s2"]]), np.array([par["phi1"]]),
                              np.array([par["phi2"]]))
    return p[0], th[0]


def test_hand_computed_rays(golden_dir):
    for name, g, kind, par, want in _read(golden_dir):
        p, th = _line(kind, par)
        idx, ln = core.ray_hits_simplex_line(g, p, th, 1e-12)
        assert dict(zip(idx.tolist(), ln.tolist())).keys() == want.keys(), name
        for i, l in zip(idx, ln):
            assert abs(l - want[int(i)]) <= 1e-12, (name, i, l)
        if name != "tie2d":       # the tie is a resolution, not something a closed clip sees
            dense = brute.simplex_lengths(g, p, th).ravel()
            nz = np.nonzero(dense > 1e-12)[0]
            assert set(nz.tolist()) == set(want), name
            for i in nz:
                assert abs(dense[i] - want[int(i)]) <= 1e-12, (name, i)


def _random_grid(rng, d3):
    return dict(nx=int(rng.integers(1, 6)), ny=int(rng.integers(1, 6)), nz=int(rng.integers(1, 5)) if d3 else 0,
                dx=float(rng.uniform(0.5, 2)), dy=float(rng.uniform(0.5, 2)), dz=float(rng.uniform(0.5, 2)),
                cx=float(rng.uniform(-2, 2)), cy=float(rng.uniform(-2, 2)), cz=float(rng.uniform(-2, 2)))


@pytest.mark.parametrize("d3", [False, True])
def test_oracle_matches_simplex_brute_force(d3):
    """Generic rays (every simplex either missed or crossed for at least 1e-3): the
    chord partition and the per-simplex clip give the same lengths."""
    rng = np.random.default_rng(61 + d3)
    checked = 0
    for trial in range(25):
        g = _random_grid(rng, d3)
        rays = (inputs.random_rays3d if d3 else inputs.random_rays2d)(20, 6.0, 700 + trial)
        p, th = (G.par3d_lines(*rays.T) if d3 else G.par2d_lines(*rays.T))
        for r in range(len(p)):
            dense = brute.simplex_lengths(g, p[r], th[r]).ravel()
            if np.any((dense > 0.0) & (dense < 1e-3)):
                continue
            got = np.zeros_like(dense)
            idx, ln = core.ray_hits_simplex_line(g, p[r], th[r], 0.0)
            got[idx] = ln
            np.testing.assert_allclose(got, dense, atol=1e-10)
            checked += 1
    assert checked > 300


@pytest.mark.parametrize("d3", [False, True])
def test_simplices_partition_each_unit(d3):
    """For every ray -- axis-parallel rays on grid planes and rays inside diagonal planes
    included -- the lengths of a unit's simplices add up to the unit's length."""
    rng = np.random.default_rng(71 + d3)
    for trial in range(20):
        g = _random_grid(rng, d3)
        rays = (inputs.random_rays3d if d3 else inputs.random_rays2d)(30, 6.0, 900 + trial)
        rays[:5, -1] = 0.0                          # axis-parallel (phi = 0 / phi2 = 0)
        if d3:
            rays[5:8, 2] = 0.0                      # phi1 = 0 as well: along x
        p, th = (G.par3d_lines(*rays.T) if d3 else G.par2d_lines(*rays.T))
        S = core.simplex_count(g)
        nu = int(np.prod(inputs.image_shape(g)))
        for r in range(len(p)):
            unit = np.zeros(nu)
            ui, ul = core.ray_hits_line(g, p[r], th[r], 0.0)
            unit[ui] = ul
            simp = np.zeros(nu * S)
            si, sl = core.ray_hits_simplex_line(g, p[r], th[r], 0.0)
            simp[si] = sl
            np.testing.assert_allclose(simp.reshape(nu, S).sum(axis=1), unit, atol=1e-12)


def test_diagonal_plane_rays_go_to_the_bigger_index():
    """Rays inside the diagonal planes of a 3x3x3 grid (xi - eta, eta - zeta or
    xi - zeta constant and integer along the whole ray): each unit's length goes to one
    simplex, the bigger of the two that share the face."""
    g = dict(nx=3, ny=3, nz=3)
    # in physical coordinates xi = x + 1.5, eta = 1.5 - y, zeta = 1.5 - z
    cases = [((0.25, -0.25, 0.3), (1.0, 1.0, 0.0), (0, 1)),     # xi - eta = 0: x = -y
             ((0.3, 0.2, 0.2), (0.0, 1.0, 1.0), (1, 2)),        # eta - zeta = 0: z = y
             ((0.2, 0.4, -0.2), (1.0, 0.0, 1.0), (0, 2))]       # xi - zeta = 0: x = -z
    for (x, y, z), (a, b, c), (u, v) in cases:
        th = np.array([a, -b, -c], dtype=np.float64)          # index direction (a, b, c)
        th /= np.linalg.norm(th)
        p = np.array([x, y, z])
        idx, ln = core.ray_hits_simplex_line(g, p, th, 1e-12)
        assert idx.size > 0
        for I, l in zip(idx, ln):
            # the other simplex sharing the face: the axes u and v swapped in its order
            s = int(I % 6)
            order = brute.SIMPLEX_ORDERS[3][s]
            pos = [order.index(u), order.index(v)]
            assert abs(pos[0] - pos[1]) == 1          # u and v adjacent in the order: on the face
            swapped = list(order)
            swapped[pos[0]], swapped[pos[1]] = swapped[pos[1]], swapped[pos[0]]
            assert brute.SIMPLEX_ORDERS[3].index(tuple(swapped)) < s


@pytest.mark.parametrize("d3", [False, True])
def test_simplex_adjoint_identity(d3):
    g = dict(nx=7, ny=6, nz=5 if d3 else 0, dx=1.1, dy=0.9, dz=1.0, cx=0.3, cy=-0.2, cz=0.1)
    rays = (inputs.random_rays3d if d3 else inputs.random_rays2d)(400, 6.0, 55)
    p, th = (G.par3d_lines(*rays.T) if d3 else G.par2d_lines(*rays.T))
    rng = np.random.default_rng(3)
    f = rng.normal(size=core.simplex_image_shape(g))
    w = rng.normal(size=len(p))
    lhs = float(core.forward_simplex_lines(g, p, th, f) @ w)
    rhs = float((f * core.adjoint_simplex_lines(g, p, th, w)).sum())
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


def test_unit_constant_image_is_the_unit_transform():
    """An image constant on each unit (every simplex of a unit carries the unit's value)
    projects like the pixel / voxel image, on a cone scan with offsets."""
    g = dict(nx=9, ny=8, nz=7, dx=1.0, dy=1.2, dz=0.8, cx=0.5, cy=-0.4, cz=0.2)
    scan = dict(kind="cone_flat", angles=np.linspace(0, 2 * np.pi, 5, endpoint=False), ncols=21, nrows=17,
                du=1.0, dv=1.0, sod=40.0, sdd=60.0)
    p, th = G.expand(scan)
    img = np.random.default_rng(4).uniform(size=inputs.image_shape(g))
    simp = np.repeat(img[..., None], 6, axis=-1)
    np.testing.assert_allclose(core.forward_simplex_lines(g, p, th, simp), core.forward_lines(g, p, th, img),
                               rtol=1e-12, atol=1e-12)
