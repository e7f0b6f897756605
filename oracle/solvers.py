"""FP64 reference CGLS (Bjorck's formulation) -- TEST INFRASTRUCTURE.

x0 = 0, r = g, s = A^T r, p = s, gamma = ||s||^2; per iteration q = A p,
alpha = gamma / ||q||^2, x += alpha p, r -= alpha q, s = A^T r, beta = ||s||^2 / gamma,
p = s + beta p.  `apply` and `adjoint` are callables (an explicit matrix or the oracle's
FP64 transform).
"""
from __future__ import annotations

import numpy as np


def cgls(apply, adjoint, g, iters: int, x0_shape=None):
    g = np.asarray(g, dtype=np.float64)
    r = g.copy()
    s = adjoint(r)
    x = np.zeros_like(s)
    p = s.copy()
    gamma = float(np.vdot(s, s))
    history = [float(np.linalg.norm(r))]
    for _ in range(iters):
        q = apply(p)
        delta = float(np.vdot(q, q))
        if delta == 0.0:
            break
        alpha = gamma / delta
        x = x + alpha * p
        r = r - alpha * q
        s = adjoint(r)
        gamma_new = float(np.vdot(s, s))
        p = s + (gamma_new / gamma) * p
        gamma = gamma_new
        history.append(float(np.linalg.norm(r)))
    return x, history


def residual(apply, f, g) -> float:
    """||A f - g|| / ||g|| in FP64."""
    g = np.asarray(g, dtype=np.float64)
    return float(np.linalg.norm(apply(np.asarray(f, dtype=np.float64)) - g) / np.linalg.norm(g))
