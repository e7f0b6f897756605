"""GPU: the batched uneven workload (16 cone / helical problems, volumes up to
512 x 512 x 256) and the sparse-view fan-beam workload at their full sizes, in the
launches the benchmark times: sampled rays against the oracle and the adjoint identity
for every member; full forward / adjoint parity for the fan-beam workload."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import tests.helpers as H
from oracle import core as ocore
from oracle import geometry as ogeom
from paper_2006_00686_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def xrt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_00686_amd import xrt as X
    X.library()
    return X


def _views_subset(scan, views):
    sub = dict(scan)
    sub["angles"] = np.asarray(scan["angles"])[views]
    if scan.get("view_z") is not None:
        sub["view_z"] = np.asarray(scan["view_z"])[views]
    return sub


def test_batched_cone_helical_full_sampled(xrt):
    cfg = inputs.batched_workload()
    plans = [xrt.Plan(m["grid"], m["scan"]) for m in cfg["members"]]
    batch = xrt.Batch(plans)
    imgs_np = [inputs.random_image(inputs.image_shape(m["grid"]), m["seed"]) for m in cfg["members"]]
    imgs = [torch.from_numpy(a).to(DEV) for a in imgs_np]
    sinos = batch.forward(imgs)
    torch.cuda.synchronize()
    rng = np.random.default_rng(44)
    for k, (m, p) in enumerate(zip(cfg["members"], plans)):
        nv, nr, nc = inputs.sino_shape(m["scan"])
        views = np.sort(rng.choice(nv, 3, replace=False))
        sub = _views_subset(m["scan"], views)
        pl, th = ogeom.expand(sub)
        pick = rng.choice(pl.shape[0], 300, replace=False)
        vloc, rem = np.divmod(pick, nr * nc)
        global_idx = (views[vloc] * nr * nc + rem).astype(np.int64)
        got = sinos[k].reshape(-1)[torch.from_numpy(global_idx).to(DEV)].cpu().numpy()
        ref = ocore.forward_lines(m["grid"], pl[pick], th[pick], imgs_np[k].astype(np.float64))
        scl = ocore.forward_lines(m["grid"], pl[pick], th[pick], np.abs(imgs_np[k]).astype(np.float64))
        H.assert_within_bar(got, ref, scl, what=f"batched member {k} sampled forward")
    # adjoint identity for every member: <A f, w> = <f, A^T w>
    gen = torch.Generator(device=DEV).manual_seed(7)
    ws = [torch.rand(tuple(p.sino_shape), generator=gen, device=DEV) for p in plans]
    backs = batch.adjoint(ws)
    for k in range(len(plans)):
        lhs = float((sinos[k].double() * ws[k].double()).sum())
        rhs = float((imgs[k].double() * backs[k].double()).sum())
        assert abs(lhs - rhs) <= 1e-5 * abs(lhs), (k, lhs, rhs)


def test_fan2d_256_sparse_full_parity(xrt):
    cfg = inputs.workload("fan2d_256_sparse")
    grid, scan = cfg["grid"], cfg["scan"]
    plan = xrt.Plan(grid, scan)
    imgs = np.stack([inputs.ellipse_phantom(256, 256, 10, 5000 + k) for k in range(4)])
    got = plan.forward(torch.from_numpy(imgs).to(DEV)).cpu().numpy()
    for b in range(4):
        ref, scl = H.forward_bar(grid, scan, imgs[b])
        H.assert_within_bar(got[b], ref, scl, what=f"fan2d_256_sparse forward {b}")
    rng = np.random.default_rng(5)
    w = rng.normal(size=(4,) + tuple(plan.sino_shape)).astype(np.float32)
    back = plan.adjoint(torch.from_numpy(w).to(DEV)).cpu().numpy()
    for b in range(4):
        ref, scl = H.adjoint_bar(grid, scan, w[b])
        H.assert_within_bar(back[b], ref, scl, what=f"fan2d_256_sparse adjoint {b}")
