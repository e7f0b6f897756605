"""GPU: the CNN convolution kernels (BF16 operands, FP32 accumulation, MFMA for 32->32)
against the FP64 reference on identical BF16-rounded operands, and the preconditioner's
operators (P and its adjoint) and gradients."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import conv as oconv

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
LAYERS = [(1, 32), (32, 32), (32, 1)]


@pytest.fixture(scope="module")
def X():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_00686_amd import xrt
    xrt.library()
    return xrt


def _tensor(a, ch):
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
    return (t if ch == 1 else t.to(torch.bfloat16)).to(DEV)


def _rand(rng, B, H, W, ch):
    shape = (B, H, W) if ch == 1 else (B, H, W, 32)
    return oconv.bf16(rng.normal(size=shape))


def _bar(ref_abs, rtol=2e-6):
    return rtol * ref_abs + 1e-6


@pytest.mark.parametrize("cin,cout", LAYERS)
@pytest.mark.parametrize("transposed", [False, True])
@pytest.mark.parametrize("H,W", [(19, 45), (32, 64)])
def test_conv_matches_fp64(X, cin, cout, transposed, H, W):
    rng = np.random.default_rng(cin * 7 + cout + transposed + H)
    B = 3
    ich, och = (cout, cin) if transposed else (cin, cout)
    x = _rand(rng, B, H, W, ich)
    Wt = rng.normal(size=(cout, 3, 3, cin)).astype(np.float32)
    got = X.conv3x3(_tensor(x, ich), torch.from_numpy(Wt).to(DEV), cin, cout, transposed, out_bf16=False)
    got = got.float().cpu().numpy()
    ref = oconv.conv(x, Wt, cin, cout, transposed)
    scl = oconv.conv(np.abs(x), np.abs(oconv.bf16(Wt)), cin, cout, transposed)
    assert np.all(np.abs(got - ref) <= _bar(scl)), np.max(np.abs(got - ref) / _bar(scl))


def test_conv_bf16_output_is_rounded_result(X):
    rng = np.random.default_rng(5)
    x = _rand(rng, 2, 16, 32, 32)
    Wt = rng.normal(size=(32, 3, 3, 32)).astype(np.float32)
    f32 = X.conv3x3(_tensor(x, 32), torch.from_numpy(Wt).to(DEV), 32, 32, out_bf16=False)
    b16 = X.conv3x3(_tensor(x, 32), torch.from_numpy(Wt).to(DEV), 32, 32, out_bf16=True)
    np.testing.assert_array_equal(b16.cpu().float().numpy(), f32.to(torch.bfloat16).float().cpu().numpy())


def test_conv_residual(X):
    rng = np.random.default_rng(6)
    x = _rand(rng, 2, 16, 32, 32)
    r = rng.normal(size=(2, 16, 32)).astype(np.float32)
    Wt = rng.normal(size=(1, 3, 3, 32)).astype(np.float32)
    a = X.conv3x3(_tensor(x, 32), torch.from_numpy(Wt).to(DEV), 32, 1).cpu().numpy()
    b = X.conv3x3(_tensor(x, 32), torch.from_numpy(Wt).to(DEV), 32, 1, residual=torch.from_numpy(r).to(DEV))
    np.testing.assert_allclose(b.cpu().numpy(), a + r, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("cin,cout", LAYERS)
@pytest.mark.parametrize("H,W", [(19, 45), (64, 64)])
def test_wgrad_matches_fp64(X, cin, cout, H, W):
    rng = np.random.default_rng(cin + 3 * cout + H)
    B = 3
    x = _rand(rng, B, H, W, cin)
    d = _rand(rng, B, H, W, cout)
    got = X.conv3x3_wgrad(_tensor(x, cin), _tensor(d, cout), cin, cout).cpu().numpy()
    ref = oconv.wgrad(x, d, cin, cout)
    scl = oconv.wgrad(np.abs(x), np.abs(d), cin, cout)
    assert np.all(np.abs(got - ref) <= 1e-5 * scl + 1e-6), np.max(np.abs(got - ref) / (1e-5 * scl + 1e-6))


def test_preconditioner_adjoint_identity_and_gradients(X):
    from paper_2006_00686_amd.learned import ConvPreconditioner
    P = ConvPreconditioner(DEV, seed=3, init_scale=0.5)
    rng = np.random.default_rng(7)
    x = torch.from_numpy(rng.normal(size=(2, 24, 40)).astype(np.float32)).to(DEV)
    y = torch.from_numpy(rng.normal(size=(2, 24, 40)).astype(np.float32)).to(DEV)
    Px, Pty = P.apply(x), P.adjoint(y)
    lhs = float((Px.double() * y.double()).sum())
    rhs = float((x.double() * Pty.double()).sum())
    # BF16 rounding of the hidden activations differs between P and P^T
    assert abs(lhs - rhs) <= 2e-2 * float((Px - x).double().abs().mul(y.double().abs()).sum()) + 1e-6
    # the differentiable path computes the same operators
    np.testing.assert_allclose(P.apply_diff(x).detach().cpu().numpy(), Px.cpu().numpy(), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(P.adjoint_diff(y).detach().cpu().numpy(), Pty.cpu().numpy(), rtol=1e-6, atol=1e-6)
    # weight gradients of <P x, y> through autograd against the chain rule recomputed in
    # FP64 from the kernels' own BF16 activations (the master weights are rounded to BF16
    # by the kernels, so a finite difference of small size would measure that rounding)
    P.zero_grad()
    (P.apply_diff(x) * y).sum().backward()
    W = [oconv.bf16(w.detach().cpu().numpy()) for w in (P.w1, P.w2, P.w3)]
    h1 = X.conv3x3(x, P.w1.data, 1, 32)
    h2 = X.conv3x3(h1, P.w2.data, 32, 32)
    xn, yn = x.cpu().numpy(), y.cpu().numpy()
    h1n, h2n = h1.float().cpu().numpy(), h2.float().cpu().numpy()
    dh2 = oconv.bf16(oconv.conv(yn, W[2], 32, 1, transposed=True))
    dh1 = oconv.bf16(oconv.conv(dh2, W[1], 32, 32, transposed=True))
    refs = {"w3": (h2n, yn, 32, 1), "w2": (h1n, dh2, 32, 32), "w1": (xn, dh1, 1, 32)}
    for wname, (a, d, ci, co) in refs.items():
        got = getattr(P, wname).grad.cpu().numpy()
        ref = oconv.wgrad(a, d, ci, co)
        scl = oconv.wgrad(np.abs(a), np.abs(d), ci, co)
        # an occasional one-ulp BF16 rounding difference of a recomputed gradient activation
        assert np.all(np.abs(got - ref) <= 8e-3 * scl + 1e-5), (wname, np.max(np.abs(got - ref) / (scl + 1e-9)))
