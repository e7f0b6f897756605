"""The FP64 oracle's PET form of the generalised transform (Introduction, eq.
generalizedRadontransform with a weight that depends on the ray only, so the transform is
that weight times the X-ray transform) and its transmission weight exp(-integral of mu)
against what fixes them: unit weights give the plain transform, a uniform medium gives
exp(-mu L) with L the chord of a textbook box clip, brute force over every unit on tiny
grids, a ray along a row of three units computed by hand, and the adjoint identity."""
import numpy as np
import pytest

from oracle import brute, core
from paper_2006_00686_amd import inputs


def _g2(nx=7, ny=5, dx=1.0, dy=1.0, cx=0.0, cy=0.0):
    return dict(nx=nx, ny=ny, nz=0, dx=dx, dy=dy, cx=cx, cy=cy)


def _g3(n=(5, 4, 3), d=(1.0, 1.1, 0.9), c=(0.2, -0.1, 0.3)):
    return dict(nx=n[0], ny=n[1], nz=n[2], dx=d[0], dy=d[1], dz=d[2], cx=c[0], cy=c[1], cz=c[2])


def _rays(rng, n, dim):
    p = np.zeros((n, 3))
    p[:, :dim] = rng.uniform(-3, 3, size=(n, dim))
    th = np.zeros((n, 3))
    th[:, :dim] = rng.normal(size=(n, dim))
    th /= np.linalg.norm(th, axis=1, keepdims=True)
    return p, th


def _box_chord(g, p, th):
    """Length of the line p + t th inside the image box (slab clip of each axis)."""
    dims = [("nx", "dx", "cx"), ("ny", "dy", "cy")] + ([("nz", "dz", "cz")] if g.get("nz", 0) else [])
    t0, t1 = -np.inf, np.inf
    for a, (kn, kd, kc) in enumerate(dims):
        half = g[kn] * g.get(kd, 1.0) / 2.0
        lo, hi = g.get(kc, 0.0) - half, g.get(kc, 0.0) + half
        if th[a] == 0.0:
            if not lo <= p[a] <= hi:
                return 0.0
            continue
        u, v = (lo - p[a]) / th[a], (hi - p[a]) / th[a]
        t0, t1 = max(t0, min(u, v)), min(t1, max(u, v))
    return max(t1 - t0, 0.0)


@pytest.mark.parametrize("g", [_g2(), _g3()])
def test_unit_weights_give_the_transform(g):
    rng = np.random.default_rng(11)
    p, th = _rays(rng, 300, 3 if g["nz"] else 2)
    img = rng.uniform(0, 1, inputs.image_shape(g))
    one = np.ones(len(p))
    np.testing.assert_array_equal(core.forward_weighted_lines(g, p, th, img, one), core.forward_lines(g, p, th, img))
    sino = rng.normal(size=len(p))
    np.testing.assert_array_equal(core.adjoint_weighted_lines(g, p, th, sino, one),
                                  core.adjoint_lines(g, p, th, sino))


@pytest.mark.parametrize("g", [_g2(9, 6, 0.7, 1.3, 0.4, -0.2), _g3()])
def test_uniform_medium_transmission_closed_form(g):
    rng = np.random.default_rng(12)
    p, th = _rays(rng, 400, 3 if g["nz"] else 2)
    mu = 0.29
    got = core.transmission_lines(g, p, th, np.full(inputs.image_shape(g), mu))
    L = np.array([_box_chord(g, p[r], th[r]) for r in range(len(p))])
    assert (L > 0).sum() > 100
    np.testing.assert_allclose(got, np.exp(-mu * L), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("g", [_g2(6, 5, 1.2, 0.8, 0.1, 0.3), _g3((4, 3, 3), (0.9, 1.2, 1.0), (0.0, 0.2, -0.1))])
def test_brute_force_transmission_and_weighted_forward(g):
    rng = np.random.default_rng(13)
    p, th = _rays(rng, 120, 3 if g["nz"] else 2)
    mu = rng.uniform(0, 0.5, inputs.image_shape(g))
    img = rng.uniform(0, 1, inputs.image_shape(g))
    w = rng.uniform(0.2, 1.5, len(p))
    trans = core.transmission_lines(g, p, th, mu)
    fw = core.forward_weighted_lines(g, p, th, img, w)
    for r in range(len(p)):
        ln = brute.unit_lengths(g, p[r], th[r])
        assert abs(trans[r] - np.exp(-(ln * mu).sum())) < 1e-12
        assert abs(fw[r] - w[r] * (ln * img).sum()) < 1e-12 * max(1.0, abs(fw[r]))


def test_row_of_three_units_by_hand():
    # 2D grid 3 x 1 with unit spacing centred at 0: the ray y = 0 along +x crosses the
    # three units over length 1 each
    g = _g2(3, 1, 1.0, 1.0, 0.0, 0.0)
    p = np.array([[-5.0, 0.0, 0.0]])
    th = np.array([[1.0, 0.0, 0.0]])
    mu = np.array([[0.1, 0.4, 0.25]])
    img = np.array([[2.0, 3.0, 5.0]])
    assert abs(core.transmission_lines(g, p, th, mu)[0] - np.exp(-0.75)) < 1e-15
    assert abs(core.forward_weighted_lines(g, p, th, img, [0.5])[0] - 5.0) < 1e-14
    back = core.adjoint_weighted_lines(g, p, th, [2.0], [0.5])
    np.testing.assert_allclose(back.ravel(), [1.0, 1.0, 1.0], atol=1e-15)


@pytest.mark.parametrize("g", [_g2(), _g3()])
def test_weighted_adjoint_identity(g):
    rng = np.random.default_rng(14)
    p, th = _rays(rng, 250, 3 if g["nz"] else 2)
    f = rng.normal(size=inputs.image_shape(g))
    s = rng.normal(size=len(p))
    w = rng.uniform(0.1, 2.0, len(p))
    lhs = np.dot(core.forward_weighted_lines(g, p, th, f, w), s)
    rhs = np.dot(f.ravel(), core.adjoint_weighted_lines(g, p, th, s, w).ravel())
    assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(lhs))
