"""GPU: batched vector kernels, CGLS, Landweber and right-preconditioned CGLS against the
FP64 references."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import core as ocore
from oracle import geometry as ogeom
from oracle import solvers as osolvers
from paper_2006_00686_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_00686_amd import solvers, xrt
    xrt.library()
    return solvers, xrt


DEV = "cuda:0"


def test_vector_kernels(mods):
    _, xrt = mods
    rng = np.random.default_rng(1)
    B, n = 5, 100003
    a = rng.normal(size=(B, n)).astype(np.float32)
    b = rng.normal(size=(B, n)).astype(np.float32)
    ta, tb = torch.from_numpy(a).to(DEV), torch.from_numpy(b).to(DEV)
    out = torch.empty(B, dtype=torch.float64, device=DEV)
    work = torch.empty(64 * B, dtype=torch.float64, device=DEV)
    xrt.vec_dot(ta, tb, B, work, out)
    ref = (a.astype(np.float64) * b.astype(np.float64)).sum(1)
    np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=1e-12, atol=1e-9)
    num = torch.from_numpy(rng.uniform(1, 2, B)).to(DEV)
    den = torch.from_numpy(np.array([2.0, 0.0, 3.0, 4.0, 5.0])).to(DEV)
    y = tb.clone()
    xrt.vec_axpy_ratio(num, den, -1.0, ta, y, B)
    nn, dd = num.cpu().numpy(), den.cpu().numpy()
    coef = np.where(dd != 0, -nn / np.where(dd != 0, dd, 1), 0.0).astype(np.float32)
    np.testing.assert_allclose(y.cpu().numpy(), b + coef[:, None] * a, rtol=1e-6, atol=1e-6)
    p = tb.clone()
    xrt.vec_xpby_ratio(num, den, ta, p, B)
    coef = np.where(dd != 0, nn / np.where(dd != 0, dd, 1), 0.0).astype(np.float32)
    np.testing.assert_allclose(p.cpu().numpy(), a + coef[:, None] * b, rtol=1e-6, atol=1e-6)
    z = tb.clone()
    xrt.vec_axpby(0.5, ta, -2.0, z)
    np.testing.assert_allclose(z.cpu().numpy(), 0.5 * a - 2.0 * b, rtol=1e-6, atol=1e-6)


def _small_problem():
    grid = dict(nx=32, ny=32, nz=0, dx=1.0, dy=1.0)
    scan = dict(kind="fan2d_flat", angles=np.arange(12) * 2 * np.pi / 12, ncols=64, du=0.75, sod=100.0, sdd=150.0)
    imgs = np.stack([inputs.ellipse_phantom(32, 32, 6, s) for s in (11, 12, 13)])
    return grid, scan, imgs


def test_cgls_iterates_match_fp64_reference(mods):
    solvers, xrt = mods
    grid, scan, imgs = _small_problem()
    plan = xrt.Plan(grid, scan)
    op = solvers.PlanOperator(plan)
    g = plan.forward(torch.from_numpy(imgs).to(DEV))
    p, th = ogeom.expand(scan)
    A = lambda v: ocore.forward_lines(grid, p, th, v.reshape(32, 32))
    At = lambda w: ocore.adjoint_lines(grid, p, th, w).ravel()
    gn = g.cpu().numpy().astype(np.float64)
    # The first iterates are compared directly; later iterates of a Krylov recursion on an
    # underdetermined, ill-conditioned system carry growing FP32-vs-FP64 drift, so from
    # there on the residual norms (the solver's stopping quantity) are compared.
    for k, bar in ((1, 1e-5), (2, 1e-4)):
        x, info = solvers.cgls(op, g, iters=k)
        for b in range(3):
            xr, _ = osolvers.cgls(A, At, gn[b].ravel(), k)
            got = x[b].cpu().numpy().ravel()
            assert np.linalg.norm(got - xr) <= bar * np.linalg.norm(xr), (k, b)
    for k in (4, 8, 16):
        x, info = solvers.cgls(op, g, iters=k)
        for b in range(3):
            _, hist = osolvers.cgls(A, At, gn[b].ravel(), k)
            res = np.linalg.norm(A(x[b].cpu().numpy().astype(np.float64)) - gn[b].ravel())
            assert abs(res - hist[-1]) <= 2e-3 * hist[0], (k, b, res, hist[-1])


def test_cgls_reaches_tolerance_confirmed_in_fp64(mods):
    solvers, xrt = mods
    grid, scan, imgs = _small_problem()
    plan = xrt.Plan(grid, scan)
    op = solvers.PlanOperator(plan)
    g = plan.forward(torch.from_numpy(imgs).to(DEV))
    x, info = solvers.cgls(op, g, iters=500, tol=1e-3, check_every=5)
    assert info.converged
    p, th = ogeom.expand(scan)
    A = lambda v: ocore.forward_lines(grid, p, th, v)
    gn = g.cpu().numpy().astype(np.float64)
    for b in range(3):
        assert osolvers.residual(A, x[b].cpu().numpy(), gn[b].ravel()) <= 1.2e-3


def test_landweber_decreases_residual(mods):
    solvers, xrt = mods
    grid, scan, imgs = _small_problem()
    plan = xrt.Plan(grid, scan)
    op = solvers.PlanOperator(plan)
    g = plan.forward(torch.from_numpy(imgs).to(DEV))
    L = solvers.operator_norm_sq(op, plan.image_shape, DEV)
    prev = None
    for k in (5, 10, 20):
        x = solvers.landweber(op, g, k, 1.0 / L)
        res = float(torch.linalg.vector_norm((plan.forward(x) - g).double()) / torch.linalg.vector_norm(g.double()))
        assert prev is None or res < prev
        prev = res


class _Identity:
    def apply(self, x, out=None):
        if out is None:
            return x
        out.copy_(x)
        return out

    adjoint = apply


def test_pcgls_with_identity_is_cgls(mods):
    solvers, xrt = mods
    grid, scan, imgs = _small_problem()
    plan = xrt.Plan(grid, scan)
    op = solvers.PlanOperator(plan)
    g = plan.forward(torch.from_numpy(imgs).to(DEV))
    a, _ = solvers.cgls(op, g, iters=10)
    b, _ = solvers.pcgls(op, _Identity(), g, iters=10)
    # the same sequence of deterministic kernels (the 2D adjoint is the voxel-driven gather)
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_cgls_is_reproducible(mods):
    solvers, xrt = mods
    grid, scan, imgs = _small_problem()
    plan = xrt.Plan(grid, scan)
    op = solvers.PlanOperator(plan)
    g = plan.forward(torch.from_numpy(imgs).to(DEV))
    a, _ = solvers.cgls(op, g, iters=25)
    b, _ = solvers.cgls(op, g, iters=25)
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())


@pytest.mark.parametrize("k", [1, 5])
def test_graph_replayed_cgls_matches_eager(mods, k):
    solvers, xrt = mods
    grid, scan, imgs = _small_problem()
    plan = xrt.Plan(grid, scan)
    op = solvers.PlanOperator(plan)
    g = plan.forward(torch.from_numpy(imgs).to(DEV))
    a, ia = solvers.cgls(op, g, 40, tol=1e-4, check_every=k)
    b, ib = solvers.cgls(op, g, 40, tol=1e-4, check_every=k, graph=True)
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    assert ia.iterations == ib.iterations and ia.rel_residual == ib.rel_residual
    # right-preconditioned, through the graph as well
    from paper_2006_00686_amd.learned import ConvPreconditioner
    P = ConvPreconditioner(DEV, seed=1, init_scale=0.05)
    c, ic = solvers.pcgls(op, P, g, 30, tol=1e-4, check_every=k)
    d, id_ = solvers.pcgls(op, P, g, 30, tol=1e-4, check_every=k, graph=True)
    np.testing.assert_array_equal(c.cpu().numpy(), d.cpu().numpy())
    assert ic.iterations == id_.iterations
