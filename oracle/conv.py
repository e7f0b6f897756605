"""FP64 reference of the preconditioner's 3x3 convolutions -- TEST INFRASTRUCTURE.

Operands are rounded to BF16 (the kernels' operand type), then convolved in FP64 with
torch's CPU conv2d / conv_transpose2d (a library primitive used as one step).
Layouts: one-channel tensors [B][H][W], 32-channel tensors NHWC; weights [cout][3][3][cin].
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F


def bf16(a) -> np.ndarray:
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _nchw(x):
    x = torch.as_tensor(np.asarray(x, dtype=np.float64))
    return x.unsqueeze(1) if x.dim() == 3 else x.permute(0, 3, 1, 2)


def _back(y, ch):
    return y[:, 0] if ch == 1 else y.permute(0, 2, 3, 1)


def conv(x, W, cin, cout, transposed=False) -> np.ndarray:
    """out[p][co] = sum W[co][t][ci] in[p + t][ci]; transposed: the adjoint."""
    xb = _nchw(bf16(x))
    w = torch.as_tensor(bf16(W)).permute(0, 3, 1, 2)           # [cout][cin][3][3]
    if not transposed:
        y = F.conv2d(xb, w, padding=1)
        return _back(y, cout).numpy()
    y = F.conv_transpose2d(xb, w, padding=1)                    # input cout channels
    return _back(y, cin).numpy()


def wgrad(x, dout, cin, cout) -> np.ndarray:
    """dW[co][kh][kw][ci] = sum_p dout[p][co] in[p + (kh-1, kw-1)][ci] (BF16 operands)."""
    xb = _nchw(bf16(x))
    db = _nchw(bf16(dout))
    w = torch.zeros((cout, cin, 3, 3), dtype=torch.float64, requires_grad=True)
    (F.conv2d(xb, w, padding=1) * db).sum().backward()
    return w.grad.permute(0, 2, 3, 1).numpy()
