"""GPU: the PET form of the generalised transform (a weight per ray times the X-ray
transform) and its adjoint, and the transmission weights exp(-integral of mu), against
the FP64 oracle on every scan kind and adjoint path; unit weights give the plain
transform bit for bit; shared and per-image weights; the adjoint identity."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import tests.helpers as H
from oracle import core as ocore
from oracle import geometry as ogeom
from paper_2006_00686_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
KINDS = ["par2d", "fan2d_flat", "fan2d_arc", "par3d", "cone_flat", "helical", "cone_zero_row", "cone_arc"]


@pytest.fixture(scope="module")
def X():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_00686_amd import xrt
    xrt.library()
    return xrt


def _scan(name):
    return {n: (g, s) for n, g, s in H.small_scans()}[name]


def _weights(scan, seed, n=1):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.05, 2.0, (n,) + tuple(inputs.sino_shape(scan))).astype(np.float32)


@pytest.mark.parametrize("name", KINDS)
def test_weighted_forward_matches_oracle(X, name):
    grid, scan = _scan(name)
    plan = X.Plan(grid, scan)
    img = inputs.random_image(inputs.image_shape(grid), 21)
    w = _weights(scan, 22)[0]
    got = plan.forward_weighted(torch.from_numpy(img).to(DEV), torch.from_numpy(w).to(DEV)).cpu().numpy()
    p, th = ogeom.expand(scan)
    ref = ocore.forward_weighted_lines(grid, p, th, img.astype(np.float64), w)
    scl = ocore.forward_weighted_lines(grid, p, th, np.abs(img).astype(np.float64), w)
    H.assert_within_bar(got, ref, scl, what=f"weighted forward {name}")


@pytest.mark.parametrize("name", KINDS)
def test_weighted_adjoint_matches_oracle_on_every_path(X, name):
    grid, scan = _scan(name)
    plan = X.Plan(grid, scan)
    rng = np.random.default_rng(23)
    sino = rng.normal(size=inputs.sino_shape(scan)).astype(np.float32)
    w = _weights(scan, 24)[0]
    p, th = ogeom.expand(scan)
    ref = ocore.adjoint_weighted_lines(grid, p, th, sino.astype(np.float64), w)
    scl = ocore.adjoint_weighted_lines(grid, p, th, np.abs(sino).astype(np.float64), w)
    ds, dw = torch.from_numpy(sino).to(DEV), torch.from_numpy(w).to(DEV)
    modes = ["auto", "scatter"]
    try:
        plan.adjoint(ds, mode="gather")
        modes.append("gather")
    except X.XrtError:
        pass
    for mode in modes:
        got = plan.adjoint_weighted(ds, dw, mode=mode).cpu().numpy()
        H.assert_within_bar(got, ref, scl, what=f"weighted adjoint {name} ({mode})")


@pytest.mark.parametrize("name", ["par2d", "fan2d_flat", "cone_flat", "helical"])
def test_unit_weights_are_the_plain_transform(X, name):
    grid, scan = _scan(name)
    plan = X.Plan(grid, scan)
    img = torch.from_numpy(inputs.random_image(inputs.image_shape(grid), 25)).to(DEV)
    one = torch.ones(tuple(plan.sino_shape), device=DEV)
    sino = plan.forward(img)
    assert torch.equal(plan.forward_weighted(img, one), sino)
    # the voxel-driven adjoints are deterministic: identical bits
    try:
        plain = plan.adjoint(sino, mode="gather")
    except X.XrtError:
        return
    assert torch.equal(plan.adjoint_weighted(sino, one, mode="gather"), plain)


@pytest.mark.parametrize("name", ["fan2d_arc", "par3d", "cone_flat"])
def test_shared_and_per_image_weights(X, name):
    grid, scan = _scan(name)
    plan = X.Plan(grid, scan)
    imgs = np.stack([inputs.random_image(inputs.image_shape(grid), s) for s in (31, 32)])
    w2 = _weights(scan, 33, 2)
    d_img = torch.from_numpy(imgs).to(DEV)
    per = plan.forward_weighted(d_img, torch.from_numpy(w2).to(DEV)).cpu().numpy()
    shared = plan.forward_weighted(d_img, torch.from_numpy(w2[0]).to(DEV)).cpu().numpy()
    p, th = ogeom.expand(scan)
    for b in range(2):
        ref_p = ocore.forward_weighted_lines(grid, p, th, imgs[b].astype(np.float64), w2[b])
        scl_p = ocore.forward_weighted_lines(grid, p, th, np.abs(imgs[b]).astype(np.float64), w2[b])
        H.assert_within_bar(per[b], ref_p, scl_p, what=f"per-image weights {name} #{b}")
        ref_s = ocore.forward_weighted_lines(grid, p, th, imgs[b].astype(np.float64), w2[0])
        scl_s = ocore.forward_weighted_lines(grid, p, th, np.abs(imgs[b]).astype(np.float64), w2[0])
        H.assert_within_bar(shared[b], ref_s, scl_s, what=f"shared weights {name} #{b}")
    sinos = np.random.default_rng(34).normal(size=(2,) + tuple(inputs.sino_shape(scan))).astype(np.float32)
    back = plan.adjoint_weighted(torch.from_numpy(sinos).to(DEV), torch.from_numpy(w2).to(DEV)).cpu().numpy()
    for b in range(2):
        ref = ocore.adjoint_weighted_lines(grid, p, th, sinos[b].astype(np.float64), w2[b])
        scl = ocore.adjoint_weighted_lines(grid, p, th, np.abs(sinos[b]).astype(np.float64), w2[b])
        H.assert_within_bar(back[b], ref, scl, what=f"per-image weighted adjoint {name} #{b}")
    with pytest.raises(ValueError):
        plan.forward_weighted(d_img, torch.ones(3, device=DEV))


@pytest.mark.parametrize("name", KINDS)
def test_transmission_matches_oracle(X, name):
    grid, scan = _scan(name)
    plan = X.Plan(grid, scan)
    mu = np.random.default_rng(35).uniform(0, 0.3, inputs.image_shape(grid)).astype(np.float32)
    got = plan.ray_transmission(torch.from_numpy(mu).to(DEV)).cpu().numpy().ravel()
    p, th = ogeom.expand(scan)
    line = ocore.forward_lines(grid, p, th, mu.astype(np.float64))
    ref = np.exp(-line)
    # the line integral carries the forward's error bar; exp adds float32 rounding
    err = np.abs(got - ref)
    bar = ref * (H.RTOL * line + 2.5e-7) + 1e-12
    assert np.all(err <= bar), f"transmission {name}: worst err/bar {float(np.max(err / bar)):.3g}"


@pytest.mark.parametrize("name", ["fan2d_flat", "cone_flat"])
def test_weighted_adjoint_identity(X, name):
    grid, scan = _scan(name)
    plan = X.Plan(grid, scan)
    rng = np.random.default_rng(36)
    f = torch.from_numpy(rng.normal(size=inputs.image_shape(grid)).astype(np.float32)).to(DEV)
    g = torch.from_numpy(rng.normal(size=inputs.sino_shape(scan)).astype(np.float32)).to(DEV)
    w = torch.from_numpy(_weights(scan, 37)[0]).to(DEV)
    lhs = float(torch.sum(plan.forward_weighted(f, w).double() * g.double()))
    rhs = float(torch.sum(f.double() * plan.adjoint_weighted(g, w).double()))
    assert abs(lhs - rhs) <= 1e-5 * (abs(lhs) + 1.0)


def test_weighted_transform_many_rows(X):
    """Cone plans of 70 and 131 rows (column packets: the forward reads the z-fastest copy
    and applies the weight there; the adjoint's gather or scatter applies it where it reads
    the sinogram) against the oracle, forward and every adjoint path."""
    from tests.test_gpu_attenuated import MANY_ROW_SCANS
    for name, grid, scan in MANY_ROW_SCANS:
        plan = X.Plan(grid, scan)
        assert plan.tuning()["packet_cols"] == 1
        p, th = ogeom.expand(scan)
        img = inputs.random_image(inputs.image_shape(grid), 31)
        w = _weights(scan, 32)[0]
        got = plan.forward_weighted(torch.from_numpy(img).to(DEV), torch.from_numpy(w).to(DEV)).cpu().numpy()
        ref = ocore.forward_weighted_lines(grid, p, th, img.astype(np.float64), w)
        scl = ocore.forward_weighted_lines(grid, p, th, np.abs(img).astype(np.float64), w)
        H.assert_within_bar(got, ref, scl, what=f"weighted forward {name}")
        rng = np.random.default_rng(33)
        sino = rng.normal(size=inputs.sino_shape(scan)).astype(np.float32)
        ref = ocore.adjoint_weighted_lines(grid, p, th, sino.astype(np.float64), w)
        scl = ocore.adjoint_weighted_lines(grid, p, th, np.abs(sino).astype(np.float64), w)
        ds, dw = torch.from_numpy(sino).to(DEV), torch.from_numpy(w).to(DEV)
        modes = ["auto", "scatter"]
        try:
            plan.adjoint(ds, mode="gather")
            modes.append("gather")
        except X.XrtError:
            pass
        for mode in modes:
            got = plan.adjoint_weighted(ds, dw, mode=mode).cpu().numpy()
            H.assert_within_bar(got, ref, scl, what=f"weighted adjoint {name} ({mode})")
