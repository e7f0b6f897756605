"""GPU: forward launch shapes (packets of detector columns x rows, XCD-aware order), the
batched persistent launch over uneven cone / helical problems, its graph capture and
replay, and the autotuner."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2006_00686_amd import inputs
from tests.helpers import assert_within_bar, forward_bar, small_scans

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SHAPES = [(0, 0), (0, 1), (64, 0), (32, 1), (16, 0), (16, 1), (1, 0), (1, 1)]


@pytest.fixture(scope="module")
def X():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_00686_amd import xrt
    xrt.library()
    return xrt


def _img(grid, seed):
    rng = np.random.default_rng(seed)
    shape = (grid["nz"], grid["ny"], grid["nx"]) if grid.get("nz", 0) else (grid["ny"], grid["nx"])
    return rng.uniform(0.0, 1.0, size=shape).astype(np.float32)


@pytest.mark.parametrize("name", ["par2d", "fan2d_flat", "fan2d_arc", "par3d", "cone_flat", "helical", "cone_arc"])
def test_launch_shapes_give_identical_results(X, name):
    grid, scan = {n: (g, s) for n, g, s in small_scans()}[name]
    plan = X.Plan(grid, scan)
    img = torch.from_numpy(_img(grid, 3)).to(DEV)
    ref = plan.forward(img).cpu().numpy()
    for pc, xr in SHAPES:
        plan.set_tuning(pc, xr)
        assert plan.tuning() == {"packet_cols": pc, "xcd_remap": xr}
        np.testing.assert_array_equal(plan.forward(img).cpu().numpy(), ref, err_msg=f"{pc}x{xr}")
    # and the values are the transform's
    gref, scl = forward_bar(grid, scan, _img(grid, 3))
    assert_within_bar(ref, gref, scl, what=name)


def test_tuning_rejects_bad_values(X):
    grid, scan = {n: (g, s) for n, g, s in small_scans()}["cone_flat"]
    plan = X.Plan(grid, scan)
    for pc, xr in ((48, 0), (32, 2), (-1, 0), (2, 0)):
        with pytest.raises(X.XrtError) as e:
            plan.set_tuning(pc, xr)
        assert e.value.status == -1


def _close_adjoint(got, ref, msg):
    """Adjoints agree to FP32 summation order (a plan whose geometry exceeds the gather's
    row bound uses the atomic scatter, whose order varies from run to run)."""
    np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-6 * float(np.abs(ref).max()), err_msg=msg)


def _members(scale=0.12, count=6):
    return inputs.batched_workload(count=count, scale=scale)["members"]


def test_batch_matches_each_plan(X):
    members = _members()
    plans = [X.Plan(m["grid"], m["scan"]) for m in members]
    plans[1].set_tuning(32, 1)
    plans[2].set_tuning(16, 0)
    imgs = [torch.from_numpy(_img(m["grid"], 10 + k)).to(DEV) for k, m in enumerate(members)]
    batch = X.Batch(plans)
    sinos = batch.forward(imgs)
    backs = batch.adjoint(sinos)
    for k, (p, im) in enumerate(zip(plans, imgs)):
        np.testing.assert_array_equal(sinos[k].cpu().numpy(), p.forward(im).cpu().numpy(), err_msg=f"member {k}")
        _close_adjoint(backs[k].cpu().numpy(), p.adjoint(sinos[k]).cpu().numpy(), f"member {k}")
    # member 1 (helical) against the oracle
    m = members[1]
    gref, scl = forward_bar(m["grid"], m["scan"], _img(m["grid"], 11))
    assert_within_bar(sinos[1].cpu().numpy(), gref, scl, what="batched helical")


def test_batch_graph_replays_match_eager(X):
    from paper_2006_00686_amd.batched import BatchGraph
    members = _members(count=5)
    plans = [X.Plan(m["grid"], m["scan"]) for m in members]
    bg = BatchGraph(X.Batch(plans)).capture()
    for rep in range(3):
        new = [torch.from_numpy(_img(m["grid"], 100 * rep + k)).to(DEV) for k, m in enumerate(members)]
        for dst, src in zip(bg.imgs, new):
            dst.copy_(src)
        bg.replay()
        torch.cuda.synchronize()
        # eager work of the program between replays
        eager_s = [p.forward(im) for p, im in zip(plans, new)]
        eager_b = [p.adjoint(s) for p, s in zip(plans, eager_s)]
        torch.cuda.synchronize()
        for k in range(len(plans)):
            np.testing.assert_array_equal(bg.sinos[k].cpu().numpy(), eager_s[k].cpu().numpy(),
                                          err_msg=f"replay {rep} member {k}")
            _close_adjoint(bg.backs[k].cpu().numpy(), eager_b[k].cpu().numpy(), f"replay {rep} member {k}")


def test_batch_errors(X):
    named = {n: (g, s) for n, g, s in small_scans()}
    cone = X.Plan(*named["cone_flat"])
    par = X.Plan(*named["par3d"])
    with pytest.raises(X.XrtError) as e:
        X.Batch([cone, par])
    assert e.value.status == -6
    with pytest.raises(X.XrtError) as e:
        X.Batch([cone] * 33)
    assert e.value.status == -1


def test_autotune_and_cache(X, tmp_path):
    from paper_2006_00686_amd import tune
    grid, scan = {n: (g, s) for n, g, s in small_scans()}["cone_flat"]
    plan = X.Plan(grid, scan)
    img = torch.from_numpy(_img(grid, 4)).to(DEV)
    ref = plan.forward(img).cpu().numpy()
    path = str(tmp_path / "tune.json")
    res = tune.autotune(plan, img, path=path, repeats=2)
    assert not res["cached"] and len(res["table"]) == len(tune.CANDIDATES)
    np.testing.assert_array_equal(plan.forward(img).cpu().numpy(), ref)
    again = X.Plan(grid, scan)
    assert tune.apply_cached(again, path=path) == {k: res[k] for k in ("packet_cols", "xcd_remap")}
    assert tune.autotune(again, img, path=path)["cached"]
    # a corrupt cache falls back to the shape the library chose for the plan
    open(path, "w").write("corrupt")
    assert tune.apply_cached(again, path=path) == again.default_tuning
    assert again.tuning() == again.default_tuning
