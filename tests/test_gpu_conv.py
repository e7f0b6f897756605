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


def _exact_operands(rng, B, H, W):
    """Integer-valued operands for which every hidden activation and every sum is exact in
    BF16 / FP32 (|h1| <= 9, |h2| <= 27 * 9 = 243, |y| < 2^24) for P and for P^T: kernels
    and reference must agree bit for bit, whatever the summation order."""
    x = rng.integers(-1, 2, size=(B, H, W)).astype(np.float32)
    w1 = rng.integers(-1, 2, size=(32, 3, 3, 1)).astype(np.float32)
    co, t, ci = np.meshgrid(np.arange(32), np.arange(9), np.arange(32), indexing="ij")
    mask = (co + ci + 5 * t) % 11 == 0          # <= 27 nonzeros per output and per input channel
    assert mask.sum(axis=(1, 2)).max() <= 27 and mask.sum(axis=(0, 1)).max() <= 27
    w2 = (mask * rng.choice([-1.0, 1.0], size=mask.shape)).reshape(32, 3, 3, 32).astype(np.float32)
    w3 = rng.integers(-1, 2, size=(1, 3, 3, 32)).astype(np.float32)
    return x, w1, w2, w3


def _ref_chain(x, w1, w2, w3, transposed):
    if not transposed:
        h = oconv.bf16(oconv.conv(x, w1, 1, 32))
        h = oconv.bf16(oconv.conv(h, w2, 32, 32))
        return x + oconv.conv(h, w3, 32, 1)
    h = oconv.bf16(oconv.conv(x, w3, 32, 1, transposed=True))
    h = oconv.bf16(oconv.conv(h, w2, 32, 32, transposed=True))
    return x + oconv.conv(h, w1, 1, 32, transposed=True)


@pytest.mark.parametrize("transposed", [False, True])
@pytest.mark.parametrize("B,H,W", [(2, 37, 61), (1, 14, 30), (3, 1, 1), (1, 5, 95), (2, 64, 64)])
def test_fused_preconditioner_exact(X, transposed, B, H, W):
    rng = np.random.default_rng(B * 1000 + H * 10 + W + transposed)
    x, w1, w2, w3 = _exact_operands(rng, B, H, W)
    dev = [torch.from_numpy(a).to(DEV) for a in (x, w1, w2, w3)]
    got = X.precond_apply(*dev, transposed=transposed).cpu().numpy()
    ref = _ref_chain(x, w1, w2, w3, transposed)
    assert np.max(np.abs(ref)) > 10 or H * W < 16
    np.testing.assert_array_equal(got, ref.astype(np.float32))
    # the layer-by-layer kernels compute the same values
    from paper_2006_00686_amd.learned import ConvPreconditioner
    P = ConvPreconditioner(DEV)
    with torch.no_grad():
        P.w1.copy_(dev[1]), P.w2.copy_(dev[2]), P.w3.copy_(dev[3])
    lay = (P.adjoint_layers(dev[0]) if transposed else P.apply_layers(dev[0])).cpu().numpy()
    np.testing.assert_array_equal(lay, got)


@pytest.mark.parametrize("transposed", [False, True])
def test_fused_preconditioner_random(X, transposed):
    """Real-valued operands: FP32 sums in a different order may round a hidden activation
    to the neighbouring BF16 value (at most one BF16 spacing, 2^-7 relative)."""
    rng = np.random.default_rng(17 + transposed)
    B, H, W = 2, 45, 77
    x = rng.normal(size=(B, H, W)).astype(np.float32)
    w1, w2, w3 = (rng.normal(size=s).astype(np.float32) * 0.3 for s in ((32, 3, 3, 1), (32, 3, 3, 32), (1, 3, 3, 32)))
    dev = [torch.from_numpy(a).to(DEV) for a in (x, w1, w2, w3)]
    got = X.precond_apply(*dev, transposed=transposed).cpu().numpy()
    ref = _ref_chain(x, w1, w2, w3, transposed)
    a1, a2, a3 = (np.abs(oconv.bf16(w)) for w in (w1, w2, w3))
    ax = np.abs(oconv.bf16(x))
    if not transposed:
        h1 = oconv.conv(ax, a1, 1, 32)
        h2 = oconv.conv(h1, a2, 32, 32)
        s0, s1 = oconv.conv(h2, a3, 32, 1), oconv.conv(oconv.conv(h1, a2, 32, 32), a3, 32, 1)
    else:
        h1 = oconv.conv(ax, a3, 32, 1, transposed=True)
        h2 = oconv.conv(h1, a2, 32, 32, transposed=True)
        s0 = s1 = oconv.conv(h2, a1, 1, 32, transposed=True)
    bar = 2.0 ** -7 * (s0 + s1) + 1e-5 * s0 + 1e-6
    assert np.all(np.abs(got - ref) <= bar), np.max(np.abs(got - ref) / bar)
    # most outputs see no rounding flip at all and agree to FP32 summation accuracy
    tight = np.abs(got - ref) <= 1e-5 * s0 + 1e-6
    assert tight.mean() >= 0.5, tight.mean()


def test_fused_preconditioner_rejects_aliasing(X):
    x = torch.zeros((1, 8, 8), dtype=torch.float32, device=DEV)
    w = [torch.zeros(n, dtype=torch.float32, device=DEV) for n in (288, 9216, 288)]
    with pytest.raises(X.XrtError):
        X.precond_apply(x, *w, out=x)
