"""GPU: the ray-driven adjoints (plain scatter and attenuated) merge the atomics of
neighbouring lanes that add to the same unit: each run of consecutive lanes with one unit
sums its values and adds them from its first lane.  The workloads' detectors give runs of
one or two lanes; these scans sample the detector ten times finer than the grid (runs of
about ten lanes, so every pass of the run sum is taken), with every seventh sinogram value
zero (lanes that leave before the walk and split runs) and rays that leave the grid in
different slabs.  Against the FP64 oracle's adjoints, element by element; and the plain
scatter of the 256^3 cone workload at full size on three views."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import tests.helpers as H
from oracle import core as ocore
from oracle import geometry as ogeom
from paper_2006_00686_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

G3 = dict(nx=10, ny=9, nz=8, dx=1.0, dy=1.0, dz=1.0, cx=0.3, cy=-0.2, cz=0.1)
CONE = dict(kind="cone_flat", angles=np.array([0.1, 0.9, 2.2, 4.0]), ncols=130, nrows=11, du=0.12, dv=1.1,
            sod=40.0, sdd=60.0)
G2 = dict(nx=12, ny=10, nz=0, dx=1.0, dy=1.0, cx=0.0, cy=0.5)
FAN = dict(kind="fan2d_flat", angles=np.linspace(0.0, 2 * np.pi, 6, endpoint=False), ncols=150, du=0.1,
           sod=40.0, sdd=60.0)


@pytest.fixture(scope="module")
def X():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_00686_amd import xrt
    xrt.library()
    return xrt


def _spacing(grid, scan):
    """Largest distance between the rays of neighbouring columns inside the grid, in units
    of the smallest unit edge: the column spacing scaled to the farthest corner."""
    far = scan["sod"] + 0.5 * np.sqrt(sum((grid[k] * grid["d" + k[1]]) ** 2 for k in ("nx", "ny", "nz") if grid[k]))
    far += np.hypot(grid["cx"], grid["cy"])
    return scan["du"] * far / scan["sdd"] / min(grid["dx"], grid["dy"])


def _sino(scan, seed):
    rng = np.random.default_rng(seed)
    w = rng.normal(size=inputs.sino_shape(scan)).astype(np.float32)
    w.reshape(-1)[::7] = 0.0
    return w


@pytest.mark.parametrize("name,grid,scan", [("cone", G3, CONE), ("fan", G2, FAN)], ids=["cone", "fan"])
def test_scatter_with_long_runs(X, name, grid, scan):
    assert _spacing(grid, scan) < 0.15   # ten or more neighbouring lanes per unit and slab
    w = _sino(scan, 3)
    plan = X.Plan(grid, scan)
    got = plan.adjoint(torch.from_numpy(w).to(DEV), mode="scatter").cpu().numpy()
    ref, scl = H.adjoint_bar(grid, scan, w)
    assert np.count_nonzero(scl) > 0.9 * scl.size
    H.assert_within_bar(got, ref, scl, what=f"scatter {name}")


def test_attenuated_adjoint_with_long_runs(X):
    assert _spacing(G3, CONE) < 0.15
    w = _sino(CONE, 4)
    plan = X.Plan(G3, CONE)
    rng = np.random.default_rng(5)
    mu = rng.uniform(0, 0.3, size=tuple(plan.image_shape)).astype(np.float32)
    got = plan.adjoint_attenuated(torch.from_numpy(w).to(DEV), torch.from_numpy(mu).to(DEV)).cpu().numpy()
    p, th = ogeom.expand(CONE)
    ref = ocore.adjoint_att_lines(G3, p, th, w.astype(np.float64), mu.astype(np.float64))
    scl = ocore.adjoint_att_lines(G3, p, th, np.abs(w).astype(np.float64), mu.astype(np.float64))
    assert np.count_nonzero(scl) > 0.9 * scl.size
    H.assert_within_bar(got, ref, scl, what="attenuated adjoint")


def test_cone_256_scatter_three_views(X):
    """The plain scatter adjoint of the 256^3 cone workload at full size on a sinogram that
    is zero outside three views, against the oracle's adjoint of those views' rays, voxel
    by voxel."""
    cfg = inputs.workload("cone_256")
    plan = X.Plan(cfg["grid"], cfg["scan"])
    rng = np.random.default_rng(17)
    views = np.sort(rng.choice(len(cfg["scan"]["angles"]), 3, replace=False))
    w = np.zeros(tuple(plan.sino_shape), dtype=np.float32)
    w[views] = rng.normal(size=(3,) + tuple(plan.sino_shape)[1:]).astype(np.float32)
    got = plan.adjoint(torch.from_numpy(w).to(DEV), mode="scatter").cpu().numpy()
    sub = dict(cfg["scan"])
    sub["angles"] = np.asarray(cfg["scan"]["angles"])[views]
    p, th = ogeom.expand(sub)
    wv = w[views].reshape(-1).astype(np.float64)
    ref = ocore.adjoint_lines(cfg["grid"], p, th, wv)
    scl = ocore.adjoint_lines(cfg["grid"], p, th, np.abs(wv))
    assert np.count_nonzero(scl) > 0.5 * scl.size
    H.assert_within_bar(got, ref, scl, what="cone_256 scatter, three views")
