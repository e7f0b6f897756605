"""GPU: the attenuated transform (the paper's generalised transform with the SPECT
weight) and its adjoint against the FP64 oracle on every scan kind, the plain transform
when mu = 0, shared and per-image maps, the adjoint identity, and sampled rays of the
256^3 cone workload."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import tests.helpers as H
from oracle import core as ocore
from oracle import geometry as ogeom
from paper_2006_00686_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
KINDS = ["par2d", "fan2d_flat", "fan2d_arc", "par3d", "cone_flat", "helical", "cone_arc"]


@pytest.fixture(scope="module")
def X():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_00686_amd import xrt
    xrt.library()
    return xrt


def _scan(name):
    return {n: (g, s) for n, g, s in H.small_scans()}[name]


def _bar(grid, scan, img, mu):
    p, th = ogeom.expand(scan)
    ref = ocore.forward_att_lines(grid, p, th, img.astype(np.float64), mu.astype(np.float64))
    scl = ocore.forward_att_lines(grid, p, th, np.abs(img).astype(np.float64), mu.astype(np.float64))
    return ref, scl


@pytest.mark.parametrize("name", KINDS)
def test_attenuated_parity(X, name):
    grid, scan = _scan(name)
    plan = X.Plan(grid, scan)
    rng = np.random.default_rng(21)
    shape = tuple(plan.image_shape)
    img = rng.uniform(0, 1, size=(2,) + shape).astype(np.float32)
    mu = rng.uniform(0, 0.3, size=(2,) + shape).astype(np.float32)
    got = plan.forward_attenuated(torch.from_numpy(img).to(DEV), torch.from_numpy(mu).to(DEV)).cpu().numpy()
    for b in range(2):
        ref, scl = _bar(grid, scan, img[b], mu[b])
        H.assert_within_bar(got[b], ref, scl, what=f"attenuated {name} image {b}")
    # one map shared by both images
    shared = plan.forward_attenuated(torch.from_numpy(img).to(DEV), torch.from_numpy(mu[0]).to(DEV)).cpu().numpy()
    ref, scl = _bar(grid, scan, img[1], mu[0])
    H.assert_within_bar(shared[1], ref, scl, what=f"attenuated {name} shared map")
    # adjoint against the oracle's
    w = rng.normal(size=tuple(plan.sino_shape)).astype(np.float32)
    adj = plan.adjoint_attenuated(torch.from_numpy(w).to(DEV), torch.from_numpy(mu[0]).to(DEV)).cpu().numpy()
    p, th = ogeom.expand(scan)
    aref = ocore.adjoint_att_lines(grid, p, th, w.astype(np.float64), mu[0].astype(np.float64))
    ascl = ocore.adjoint_att_lines(grid, p, th, np.abs(w).astype(np.float64), mu[0].astype(np.float64))
    H.assert_within_bar(adj, aref, ascl, what=f"attenuated adjoint {name}")


MANY_ROW_SCANS = [
    ("cone_flat", dict(nx=35, ny=17, nz=40, dx=1.0, dy=1.1, dz=0.9, cx=0.5, cy=-1.0, cz=0.3),
     dict(kind="cone_flat", angles=np.linspace(0.2, 2 * np.pi, 5, endpoint=False), ncols=23, nrows=70, du=1.3,
          dv=0.8, sod=90.0, sdd=140.0)),
    ("cone_arc", dict(nx=21, ny=33, nz=36, dx=1.0, dy=1.0, dz=1.0, cx=0.0, cy=0.0, cz=0.0),
     dict(kind="cone_arc", angles=np.linspace(0.0, 2 * np.pi, 4, endpoint=False), ncols=19, nrows=131,
          du=0.01, dv=0.004, sod=85.0, sdd=130.0, view_z=np.linspace(-3, 3, 4))),
]


@pytest.mark.parametrize("name,grid,scan", MANY_ROW_SCANS, ids=[c[0] for c in MANY_ROW_SCANS])
def test_attenuated_many_rows(X, name, grid, scan):
    """Cone plans of 70 and 131 rows (column packets: a partial packet per column) on grids
    of several 32-unit tiles with a ragged tail.  The forward reads z-fastest (f, mu) pairs;
    the adjoint adds into the y-fastest partial volume with the merged atomics of
    neighbouring lanes.  Against the oracle for two images with their own maps and with one
    shared map, and (adjoint) a view of zeros."""
    plan = X.Plan(grid, scan)
    assert plan.tuning()["packet_cols"] == 1
    rng = np.random.default_rng(41)
    shape = tuple(plan.image_shape)
    mu = rng.uniform(0, 0.3, size=(2,) + shape).astype(np.float32)
    img = rng.uniform(0, 1, size=(2,) + shape).astype(np.float32)
    fwd = plan.forward_attenuated(torch.from_numpy(img).to(DEV), torch.from_numpy(mu).to(DEV)).cpu().numpy()
    fsh = plan.forward_attenuated(torch.from_numpy(img).to(DEV), torch.from_numpy(mu[0]).to(DEV)).cpu().numpy()
    for b in range(2):
        ref, scl = _bar(grid, scan, img[b], mu[b])
        H.assert_within_bar(fwd[b], ref, scl, what=f"many-row forward {name} image {b}")
    ref, scl = _bar(grid, scan, img[1], mu[0])
    H.assert_within_bar(fsh[1], ref, scl, what=f"many-row forward {name} shared map")
    w = rng.normal(size=(2,) + tuple(plan.sino_shape)).astype(np.float32)
    w[1, 1] = 0.0   # a view of zero values (rays that return before walking)
    p, th = ogeom.expand(scan)
    per = plan.adjoint_attenuated(torch.from_numpy(w).to(DEV), torch.from_numpy(mu).to(DEV)).cpu().numpy()
    shared = plan.adjoint_attenuated(torch.from_numpy(w).to(DEV), torch.from_numpy(mu[0]).to(DEV)).cpu().numpy()
    for b in range(2):
        for got, m, what in ((per[b], mu[b], "own map"), (shared[b], mu[0], "shared map")):
            ref = ocore.adjoint_att_lines(grid, p, th, w[b].astype(np.float64), m.astype(np.float64))
            scl = ocore.adjoint_att_lines(grid, p, th, np.abs(w[b]).astype(np.float64), m.astype(np.float64))
            H.assert_within_bar(got, ref, scl, what=f"many-row adjoint {name} image {b} {what}")


def test_attenuated_forward_wide_grid(X):
    """A grid wider than 256 units: the attenuated forward takes the walk's flat form."""
    from tests.test_gpu_parity import WIDE_SCANS
    for name, grid, scan in WIDE_SCANS:
        plan = X.Plan(grid, scan)
        rng = np.random.default_rng(23)
        shape = tuple(plan.image_shape)
        img = rng.uniform(0, 1, size=shape).astype(np.float32)
        mu = rng.uniform(0, 0.05, size=shape).astype(np.float32)
        got = plan.forward_attenuated(torch.from_numpy(img).to(DEV), torch.from_numpy(mu).to(DEV)).cpu().numpy()
        ref, scl = _bar(grid, scan, img, mu)
        H.assert_within_bar(got, ref, scl, what=f"attenuated {name}")


def test_zero_attenuation_is_the_transform(X):
    grid, scan = _scan("cone_flat")
    plan = X.Plan(grid, scan)
    img = torch.from_numpy(inputs.random_image(tuple(plan.image_shape), 5)).to(DEV)
    a = plan.forward_attenuated(img, torch.zeros_like(img)).cpu().numpy()
    b = plan.forward(img).cpu().numpy()
    ref, scl = H.forward_bar(grid, scan, img.cpu().numpy())
    H.assert_within_bar(a, b, scl, rtol=1e-6, what="mu = 0")


def test_attenuated_adjoint_identity(X):
    grid, scan = _scan("helical")
    plan = X.Plan(grid, scan)
    rng = np.random.default_rng(8)
    f = torch.from_numpy(rng.uniform(0, 1, tuple(plan.image_shape)).astype(np.float32)).to(DEV)
    mu = torch.from_numpy(rng.uniform(0, 0.2, tuple(plan.image_shape)).astype(np.float32)).to(DEV)
    w = torch.from_numpy(rng.uniform(0, 1, tuple(plan.sino_shape)).astype(np.float32)).to(DEV)
    lhs = float((plan.forward_attenuated(f, mu).double() * w.double()).sum())
    rhs = float((f.double() * plan.adjoint_attenuated(w, mu).double()).sum())
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_cone_256_attenuated_sampled(X):
    cfg = inputs.workload("cone_256")
    plan = X.Plan(cfg["grid"], cfg["scan"])
    img = inputs.random_image(tuple(plan.image_shape), 9)
    mu = (0.01 * inputs.random_image(tuple(plan.image_shape), 10)).astype(np.float32)
    got = plan.forward_attenuated(torch.from_numpy(img).to(DEV), torch.from_numpy(mu).to(DEV)).cpu().numpy().ravel()
    rng = np.random.default_rng(11)
    views = np.sort(rng.choice(len(cfg["scan"]["angles"]), 3, replace=False))
    sub = dict(cfg["scan"])
    sub["angles"] = np.asarray(cfg["scan"]["angles"])[views]
    p, th = ogeom.expand(sub)
    pick = rng.choice(p.shape[0], 1500, replace=False)
    nr, nc = cfg["scan"]["nrows"], cfg["scan"]["ncols"]
    vloc, rem = np.divmod(pick, nr * nc)
    gidx = views[vloc] * nr * nc + rem
    ref = ocore.forward_att_lines(cfg["grid"], p[pick], th[pick], img.astype(np.float64), mu.astype(np.float64))
    scl = ocore.forward_att_lines(cfg["grid"], p[pick], th[pick], np.abs(img).astype(np.float64),
                                  mu.astype(np.float64))
    H.assert_within_bar(got[gidx], ref, scl, what="cone_256 attenuated sampled")


def test_cone_256_attenuated_adjoint_three_views(X):
    """The 256^3 cone workload's attenuated adjoint (the packet layout, the merged and
    handed-over atomics at full size) on a sinogram that is zero outside three views,
    against the oracle's adjoint of those views' rays, voxel by voxel over the whole
    volume (the zero views' rays return before walking)."""
    cfg = inputs.workload("cone_256")
    plan = X.Plan(cfg["grid"], cfg["scan"])
    mu = (0.01 * inputs.random_image(tuple(plan.image_shape), 12)).astype(np.float32)
    rng = np.random.default_rng(13)
    views = np.sort(rng.choice(len(cfg["scan"]["angles"]), 3, replace=False))
    w = np.zeros(tuple(plan.sino_shape), dtype=np.float32)
    w[views] = rng.normal(size=(3,) + tuple(plan.sino_shape)[1:]).astype(np.float32)
    got = plan.adjoint_attenuated(torch.from_numpy(w).to(DEV), torch.from_numpy(mu).to(DEV)).cpu().numpy()
    sub = dict(cfg["scan"])
    sub["angles"] = np.asarray(cfg["scan"]["angles"])[views]
    p, th = ogeom.expand(sub)
    wv = w[views].reshape(-1).astype(np.float64)
    ref = ocore.adjoint_att_lines(cfg["grid"], p, th, wv, mu.astype(np.float64))
    scl = ocore.adjoint_att_lines(cfg["grid"], p, th, np.abs(wv), mu.astype(np.float64))
    assert np.count_nonzero(scl) > 0.5 * scl.size
    H.assert_within_bar(got, ref, scl, what="cone_256 attenuated adjoint, three views")


def test_attenuated_forward_captured_before_its_workspace(X):
    """A captured call on a plan without the pair workspace allocates nothing and takes the
    unpaired walk; replays equal the paired eager result bit for bit."""
    grid, scan = _scan("cone_flat")
    plan = X.Plan(grid, scan)
    rng = np.random.default_rng(71)
    img = torch.from_numpy(inputs.random_image(inputs.image_shape(grid), 72)).to(DEV)
    mu = torch.from_numpy(rng.uniform(0, 0.2, inputs.image_shape(grid)).astype(np.float32)).to(DEV)
    out = torch.empty(tuple(plan.sino_shape), device=DEV)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.forward_attenuated(img, mu, out=out)
    eager = plan.forward_attenuated(img, mu)   # allocates the workspace: paired walk
    for _ in range(3):
        out.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager)
        _ = plan.forward(img)   # eager work between replays
