"""GPU: the batch-in-lanes transforms (a batch of problems held interleaved, one ray or
pixel per wavefront for the whole batch) give each problem exactly the result of the
per-image calls, on every 2D scan kind and a 3D forward, for batches of 1, 5 and 64; the
solver operator that uses them gives the same CGLS iterates bit for bit; errors."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import tests.helpers as H
from paper_2006_00686_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def X():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_00686_amd import xrt
    xrt.library()
    return xrt


def _scan(name):
    return {n: (g, s) for n, g, s in H.small_scans()}[name]


def _images(grid, batch, seed):
    return torch.from_numpy(np.stack([inputs.random_image(inputs.image_shape(grid), seed + b)
                                      for b in range(batch)])).to(DEV)


@pytest.mark.parametrize("name", ["par2d", "fan2d_flat", "fan2d_arc"])
@pytest.mark.parametrize("batch", [1, 5, 64])
def test_interleaved_2d_equals_per_image(X, name, batch):
    grid, scan = _scan(name)
    plan = X.Plan(grid, scan)
    imgs = _images(grid, batch, 40)
    ref_f = plan.forward(imgs)
    got_f = X.deinterleave(plan.forward_interleaved(X.interleave(imgs, batch), batch), batch, torch.empty_like(ref_f))
    assert torch.equal(got_f, ref_f)
    sino = torch.from_numpy(np.random.default_rng(41).normal(size=(batch,) + tuple(plan.sino_shape))
                            .astype(np.float32)).to(DEV)
    ref_a = plan.adjoint(sino, mode="gather")
    got_a = X.deinterleave(plan.adjoint_interleaved(X.interleave(sino, batch), batch), batch, torch.empty_like(ref_a))
    assert torch.equal(got_a, ref_a)


def test_interleaved_3d_forward_and_errors(X):
    grid, scan = _scan("cone_flat")
    plan = X.Plan(grid, scan)
    imgs = _images(grid, 3, 50)
    ref = plan.forward(imgs)
    got = X.deinterleave(plan.forward_interleaved(X.interleave(imgs, 3), 3), 3, torch.empty_like(ref))
    assert torch.equal(got, ref)
    with pytest.raises(X.XrtError):
        plan.adjoint_interleaved(torch.zeros((plan.n_rays, 3), device=DEV), 3)
    g2, s2 = _scan("fan2d_flat")
    p2 = X.Plan(g2, s2)
    with pytest.raises(X.XrtError):
        p2.forward_interleaved(torch.zeros((p2.n_units, 65), device=DEV), 65)
    with pytest.raises(ValueError):
        p2.forward_interleaved(torch.zeros((p2.n_units, 2), device=DEV), 3)


def test_solver_operator_batch_in_lanes_matches_plain(X):
    from paper_2006_00686_amd import solvers
    cfg = inputs.workload("fan2d_256_sparse")
    plan = X.Plan(cfg["grid"], cfg["scan"])
    batch = 32   # interleaved forward and adjoint both in use
    imgs = _images(cfg["grid"], batch, 60)
    g = plan.forward(imgs)
    op_il = solvers.PlanOperator(plan)
    op_plain = solvers.PlanOperator(plan, interleave=False)
    assert torch.equal(op_il.apply(imgs), op_plain.apply(imgs))
    assert torch.equal(op_il.adjoint(g), op_plain.adjoint(g))
    x1, _ = solvers.cgls(op_il, g, iters=12, tol=0.0)
    x2, _ = solvers.cgls(op_plain, g, iters=12, tol=0.0)
    assert torch.equal(x1, x2)
