"""GPU: the voxel-driven cone adjoint where a voxel's shadow spans many detector rows
(fine rows: bound of 6-8 candidate rows per column), many detector columns (fine
columns: 32 or 64 column slots per view, and shadows wider than 64 columns that take
further record passes), and on a long helix over a short volume (most views see a band
of z that misses most voxels)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import tests.helpers as H
from paper_2006_00686_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def xrt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_00686_amd import xrt as X
    X.library()
    return X


def _scans():
    g = dict(nx=20, ny=18, nz=12, dx=1.0, dy=1.1, dz=1.0, cx=0.4, cy=-0.3, cz=0.2)
    fine = dict(kind="cone_flat", angles=np.linspace(0.05, 2 * np.pi, 24, endpoint=False), ncols=40, nrows=61,
                du=1.5, dv=0.3, u0=0.1, v0=0.05, sod=100.0, sdd=150.0)
    gh = dict(nx=16, ny=16, nz=8, dx=1.0, dy=1.0, dz=1.0, cx=0.0, cy=0.0, cz=0.0)
    nv = 96
    helix = dict(kind="cone_flat", angles=np.arange(nv) * 2 * np.pi * 4 / nv, ncols=36, nrows=6, du=1.2, dv=1.5,
                 u0=0.0, v0=0.0, sod=60.0, sdd=90.0, view_z=np.linspace(-20.0, 20.0, nv))
    gc = dict(nx=12, ny=10, nz=8, dx=1.0, dy=1.0, dz=1.0, cx=0.3, cy=-0.2, cz=0.1)
    mid_cols = dict(kind="cone_flat", angles=np.linspace(0.1, 2 * np.pi, 10, endpoint=False), ncols=200, nrows=9,
                    du=0.1, dv=1.4, u0=0.03, v0=0.2, sod=100.0, sdd=150.0)
    fine_cols = dict(kind="cone_flat", angles=np.linspace(0.2, 2 * np.pi, 8, endpoint=False), ncols=1000, nrows=9,
                     du=0.02, dv=1.4, u0=0.011, v0=0.2, sod=100.0, sdd=150.0)
    return [("fine_rows", g, fine), ("long_helix", gh, helix), ("mid_cols", gc, mid_cols),
            ("fine_cols", gc, fine_cols)]


@pytest.mark.parametrize("name,grid,scan", _scans(), ids=[s[0] for s in _scans()])
def test_gather_parity(xrt, name, grid, scan):
    rng = np.random.default_rng(12)
    sino = rng.normal(size=inputs.sino_shape(scan)).astype(np.float32)
    plan = xrt.Plan(grid, scan)
    d = torch.from_numpy(sino).to("cuda:0")
    got = plan.adjoint(d, mode="gather").cpu().numpy()
    ref, scl = H.adjoint_bar(grid, scan, sino)
    H.assert_within_bar(got, ref, scl, what=f"gather adjoint {name}")
    sc = plan.adjoint(d, mode="scatter").cpu().numpy()
    H.assert_within_bar(sc, ref, scl, what=f"scatter adjoint {name}")
    np.testing.assert_array_equal(plan.adjoint(d, mode="auto").cpu().numpy(), got)
