"""GPU: the allocation-free dot product xrt_vec_dot_noalloc (partial sums in the library's
static device array) against xrt_vec_dot with a workspace argument: the same kernels in
the same order, so equal bit for bit, on two calls in a row (the second smaller, which
must not see the first call's partial sums), and its size limit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def xrt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_00686_amd import xrt as X
    X.library()
    return X


def _vectors(n, batch, seed):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(batch, n)).astype(np.float32)
    b = rng.uniform(-1, 1, size=(batch, n)).astype(np.float32)
    return a, b


def _both(xrt, a, b):
    batch = a.shape[0]
    da, db = torch.from_numpy(a).to(DEV), torch.from_numpy(b).to(DEV)
    work = torch.empty(64 * batch, dtype=torch.float64, device=DEV)
    ref = torch.empty(batch, dtype=torch.float64, device=DEV)
    xrt.vec_dot(da, db, batch, work, ref)
    got = torch.full((batch,), float("nan"), dtype=torch.float64, device=DEV)
    xrt.vec_dot_noalloc(da, db, batch, got)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_dot_matches_workspace_dot(xrt):
    for n, batch, seed in ((300_001, 37, 1), (1_000, 5, 2)):     # the second call is smaller
        a, b = _vectors(n, batch, seed)
        ref, got = _both(xrt, a, b)
        np.testing.assert_array_equal(got, ref)
        # the definition: an FP64 sum of the FP32 products (order differs: FP64 rounding only)
        exact = (a.astype(np.float64) * b.astype(np.float64)).sum(axis=1)
        scale = (np.abs(a.astype(np.float64) * b.astype(np.float64))).sum(axis=1)
        assert np.all(np.abs(got - exact) <= 1e-13 * scale)


def test_noalloc_dot_size_limit(xrt):
    a, b = _vectors(257, 1024, 3)                  # the largest batch the scratch holds
    ref, got = _both(xrt, a, b)
    np.testing.assert_array_equal(got, ref)
    da = torch.zeros((1025, 4), dtype=torch.float32, device=DEV)
    out = torch.zeros(1025, dtype=torch.float64, device=DEV)
    with pytest.raises(xrt.XrtError) as e:
        xrt.vec_dot_noalloc(da, da, 1025, out)
    assert e.value.status == -3                    # XRT_E_SIZE, nothing written
    assert float(out.abs().sum()) == 0.0
