"""Pins of the FP64 reference CGLS: it reaches the least-squares / minimum-norm solution
that numpy.linalg.lstsq computes, with a monotonically decreasing residual."""
import numpy as np

from oracle import brute
from oracle import geometry as G
from oracle import solvers
from paper_2006_00686_amd import inputs


def _matrix(n_rays, seed):
    g = dict(nx=5, ny=4, nz=0, dx=1.0, dy=1.0)
    rays = inputs.random_rays2d(n_rays, 2.0, seed)
    p, th = G.par2d_lines(*rays.T)
    return brute.matrix(g, p, th)


def test_cgls_overdetermined_matches_lstsq():
    A = _matrix(60, 1)
    rng = np.random.default_rng(2)
    g = rng.normal(size=A.shape[0])
    x, hist = solvers.cgls(lambda v: A @ v, lambda w: A.T @ w, g, 200)
    ref = np.linalg.lstsq(A, g, rcond=None)[0]
    np.testing.assert_allclose(x, ref, rtol=1e-8, atol=1e-8)
    assert all(b <= a + 1e-12 for a, b in zip(hist, hist[1:]))


def test_cgls_underdetermined_reaches_minimum_norm_solution():
    A = _matrix(12, 3)
    rng = np.random.default_rng(4)
    g = A @ rng.uniform(0, 1, A.shape[1])
    x, hist = solvers.cgls(lambda v: A @ v, lambda w: A.T @ w, g, 300)
    ref = np.linalg.lstsq(A, g, rcond=None)[0]     # minimum-norm solution
    np.testing.assert_allclose(x, ref, rtol=1e-7, atol=1e-7)
    assert hist[-1] / hist[0] < 1e-9
    assert solvers.residual(lambda v: A @ v, x, g) < 1e-9
