"""Pins of the FP64 convolution reference: a per-pixel loop of the definition, the
adjoint identity of the transposed convolution, and the weight gradient."""
import numpy as np

from oracle import conv


def _loop(x, W):
    """direct definition on a [B][H][W][C] input (zero padding)."""
    B, H, Wd, C = x.shape
    co_n = W.shape[0]
    out = np.zeros((B, H, Wd, co_n))
    xp = np.zeros((B, H + 2, Wd + 2, C))
    xp[:, 1:-1, 1:-1] = x
    for kh in range(3):
        for kw in range(3):
            patch = xp[:, kh:kh + H, kw:kw + Wd]                # in[p + (kh-1, kw-1)]
            out += np.einsum("bhwc,oc->bhwo", patch, W[:, kh, kw, :])
    return out


def test_conv_matches_definition_loop():
    rng = np.random.default_rng(0)
    x = conv.bf16(rng.normal(size=(2, 7, 9, 32)))
    W = conv.bf16(rng.normal(size=(32, 3, 3, 32)))
    np.testing.assert_allclose(conv.conv(x, W, 32, 32), _loop(x, W), rtol=1e-12, atol=1e-10)
    x1 = conv.bf16(rng.normal(size=(2, 7, 9)))
    W1 = conv.bf16(rng.normal(size=(32, 3, 3, 1)))
    np.testing.assert_allclose(conv.conv(x1, W1, 1, 32), _loop(x1[..., None], W1), rtol=1e-12, atol=1e-10)


def test_transposed_is_the_adjoint():
    rng = np.random.default_rng(1)
    for cin, cout in ((1, 32), (32, 32), (32, 1)):
        x = conv.bf16(rng.normal(size=(2, 6, 5) + ((cin,) if cin > 1 else ())))
        y = conv.bf16(rng.normal(size=(2, 6, 5) + ((cout,) if cout > 1 else ())))
        W = conv.bf16(rng.normal(size=(cout, 3, 3, cin)))
        lhs = float((conv.conv(x, W, cin, cout) * y).sum())
        rhs = float((x * conv.conv(y, W, cin, cout, transposed=True)).sum())
        assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))


def test_weight_gradient_is_the_derivative():
    rng = np.random.default_rng(2)
    x = conv.bf16(rng.normal(size=(2, 5, 6, 32)))
    d = conv.bf16(rng.normal(size=(2, 5, 6, 32)))
    W = conv.bf16(rng.normal(size=(32, 3, 3, 32)))
    g = conv.wgrad(x, d, 32, 32)
    # <conv(x; W), d> is linear in W: its derivative along V is <conv(x; V), d>
    V = conv.bf16(rng.normal(size=W.shape))
    np.testing.assert_allclose((g * V).sum(), (conv.conv(x, V, 32, 32) * d).sum(), rtol=1e-10)
    # explicit formula at one weight
    co, kh, kw, ci = 3, 0, 2, 5
    xp = np.zeros((2, 7, 8, 32))
    xp[:, 1:-1, 1:-1] = x
    ref = (d[..., co] * xp[:, kh:kh + 5, kw:kw + 6, ci]).sum()
    assert abs(g[co, kh, kw, ci] - ref) < 1e-10
