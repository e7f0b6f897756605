"""Iterative reconstruction on top of the transform: CGLS, Landweber and right-preconditioned
CGLS.  Every arithmetic step runs in the library's kernels (A and A^T, batched FP64 dots,
ratio-scaled updates); this module only sequences the calls.  A check of the recursive
residual (one host synchronisation) happens every `check_every` iterations.

All vectors carry an explicit leading batch dimension; every batch member is an
independent problem with its own step sizes.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import xrt as X


class PlanOperator:
    """A = the plan's forward projection, A^T = its adjoint.

    On a 2D plan with the voxel-driven gather, batches run interleaved ([unit][problem],
    through buffers kept between calls; identical results): the forward from 24 problems
    (one ray per wavefront, the batch in its lanes: 0.27 vs 0.73 ms for 64 sparse-view
    fan-beam problems, slower below ~22), the adjoint from 6 (one pixel per lane, a
    candidate's 8 values in two 16-byte loads: 0.40 vs 0.92 ms at 64)."""

    IL_FORWARD_MIN = 24
    IL_ADJOINT_MIN = 6

    def __init__(self, plan: X.Plan, adjoint_mode: str = "auto", interleave: bool = True):
        self.plan = plan
        self.adjoint_mode = adjoint_mode
        self.domain_shape = tuple(plan.image_shape)
        self.range_shape = tuple(plan.sino_shape)
        self._il_ok = interleave and len(self.domain_shape) == 2 and adjoint_mode in ("auto", "gather")
        self._bufs = {}

    def _buffers(self, batch, dev):
        if batch not in self._bufs:
            self._bufs[batch] = (torch.empty((self.plan.n_units, batch), dtype=torch.float32, device=dev),
                                 torch.empty((self.plan.n_rays, batch), dtype=torch.float32, device=dev))
        return self._bufs[batch]

    def apply(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        batch = x.numel() // int(np.prod(self.domain_shape))
        if not self._il_ok or not self.IL_FORWARD_MIN <= batch <= 64:
            return self.plan.forward(x, out=out)
        if out is None:
            out = torch.empty(tuple(x.shape[:-len(self.domain_shape)]) + self.range_shape, dtype=torch.float32,
                              device=x.device)
        bi, bo = self._buffers(batch, x.device)
        X.interleave(x, batch, out=bi)
        self.plan.forward_interleaved(bi, batch, out=bo)
        return X.deinterleave(bo, batch, out)

    def adjoint(self, y: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        batch = y.numel() // int(np.prod(self.range_shape))
        if self._il_ok and self.IL_ADJOINT_MIN <= batch <= 64:
            if out is None:
                out = torch.empty(tuple(y.shape[:-len(self.range_shape)]) + self.domain_shape, dtype=torch.float32,
                                  device=y.device)
            bi, bo = self._buffers(batch, y.device)
            X.interleave(y, batch, out=bo)
            try:
                self.plan.adjoint_interleaved(bo, batch, out=bi)
            except X.XrtError:
                # no voxel-driven gather for this plan: plain calls from now on
                self._il_ok = False
                return self.plan.adjoint(y, mode=self.adjoint_mode, out=out)
            return X.deinterleave(bi, batch, out)
        return self.plan.adjoint(y, mode=self.adjoint_mode, out=out)


class MatrixOperator:
    """A and A^T as products with the stored projection matrix (xrt.SparseMatrix).

    Batches of 9..64 problems run interleaved ([unit][problem]: each nonzero reads the
    batch's values from contiguous memory) through buffers kept between calls; smaller
    batches use the wavefront-per-row product directly."""

    def __init__(self, A):
        self.A = A
        self.At = A.transpose()
        self.domain_shape = tuple(A.col_shape)
        self.range_shape = tuple(A.row_shape)
        self._bufs = {}

    def _il(self, batch, dev):
        if batch not in self._bufs:
            self._bufs[batch] = (torch.empty((self.A.n_cols, batch), dtype=torch.float32, device=dev),
                                 torch.empty((self.A.n_rows, batch), dtype=torch.float32, device=dev))
        return self._bufs[batch]

    def _product(self, M, x, out, in_shape, out_shape):
        batch = x.numel() // int(np.prod(in_shape))
        if out is None:
            out = torch.empty((batch,) + tuple(out_shape), dtype=torch.float32, device=x.device)
        if batch <= 8 or batch > 64:
            return M.matmul(x, out=out)
        bi, bo = self._il(batch, x.device)
        xi, yo = (bi, bo) if M is self.A else (bo, bi)
        X.interleave(x, batch, out=xi)
        M.matmul_interleaved(xi, batch, out=yo)
        return X.deinterleave(yo, batch, out)

    def apply(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        return self._product(self.A, x, out, self.domain_shape, self.range_shape)

    def adjoint(self, y: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        return self._product(self.At, y, out, self.range_shape, self.domain_shape)


@dataclass
class SolveInfo:
    iterations: int = 0
    converged: bool = False
    rel_residual: list = field(default_factory=list)   # recursive ||r|| / ||g||, per check
    true_residual: list = field(default_factory=list)  # ||g - A f|| / ||g|| (FP64 norms), per confirmation
    seconds: float = 0.0
    failure: str | None = None     # "nonfinite" or "stall" when the iteration was abandoned
    fallback: bool = False         # result comes from plain CGLS after a failed PCGLS


class _Dots:
    def __init__(self, batch: int, device):
        self.batch = batch
        self.work = torch.empty(64 * batch, dtype=torch.float64, device=device)

    def __call__(self, a: torch.Tensor, b: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        return X.vec_dot(a, b, self.batch, self.work, out)


def cgls(op, g: torch.Tensor, iters: int, tol: float | None = None, check_every: int = 5,
         stall_checks: int = 0, stall_ratio: float = 0.999, graph: bool = False, P=None,
         confirm: bool = True) -> tuple[torch.Tensor, SolveInfo]:
    """CGLS (x0 = 0): minimises ||op(x) - g|| for every batch member; with a linear
    preconditioner P (apply / adjoint on the image space), right-preconditioned CGLS:
    min ||op(P z) - g|| with the image f = P z.

    With P the image is accumulated directly, f += alpha (P p), from the same P p whose
    projection q = op(P p) updates the residual r -= alpha q.  So r tracks g - op(f) of
    the returned image up to FP32 rounding even where P is linear only up to rounding
    (BF16 hidden activations); P applied to the accumulated z would not be.

    Stops after `iters` iterations or once every member's residual satisfies
    ||r|| <= tol ||g||.  With confirm=True (and a tolerance), the recursive residual only
    proposes the stop: the true residual ||g - op(f)|| / ||g|| is then computed on the GPU
    (FP32 residual vector, FP64 norms) and the iteration goes on until it satisfies the
    tolerance for every member too (inside the timed region, info.true_residual).  With a
    tolerance, the iteration is abandoned (info.failure) when the worst residual is not
    finite, or, if stall_checks > 0, when it has not dropped below stall_ratio times its
    value stall_checks checks earlier.

    graph=True captures `check_every` iterations in a HIP graph once (after a first
    iteration run directly, which loads every kernel) and replays it between checks: the
    same kernels in the same order, so the same results, without one launch per kernel."""
    batch = g.shape[0]
    dev = g.device
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    dots = _Dots(batch, dev)
    f64 = dict(dtype=torch.float64, device=dev)
    x = torch.zeros((batch,) + tuple(op.domain_shape), dtype=torch.float32, device=dev)
    r = g.clone()
    s = op.adjoint(r)
    if P is not None:
        s = P.adjoint(s)
    p = s.clone()
    q = torch.empty_like(r)
    w = torch.empty_like(x) if P is not None else p      # image of the search direction, P p
    t = torch.empty_like(x) if P is not None else s      # op^T r before P^T
    gamma, gamma_new, delta, rr, gg = (torch.empty(batch, **f64) for _ in range(5))
    dots(s, s, gamma)
    dots(g, g, gg)
    info = SolveInfo()

    def step():
        if P is not None:
            P.apply(p, out=w)
        op.apply(w, out=q)
        dots(q, q, delta)
        X.vec_axpy_ratio(gamma, delta, 1.0, w, x, batch)     # f += (gamma / delta) P p
        X.vec_axpy_ratio(gamma, delta, -1.0, q, r, batch)    # r -= (gamma / delta) q
        op.adjoint(r, out=t)
        if P is not None:
            P.adjoint(t, out=s)
        dots(s, s, gamma_new)
        X.vec_xpby_ratio(gamma_new, gamma, s, p, batch)      # p = s + (gamma' / gamma) p
        torch.mul(gamma_new, 1.0, out=gamma)                  # gamma = gamma' (a kernel)

    def true_worst() -> float:
        op.apply(x, out=q)
        X.vec_axpby(1.0, g, -1.0, q)                          # q = g - op(f)
        dots(q, q, rr)
        worst = float(torch.sqrt(rr / gg).max().item())
        info.true_residual.append(worst)
        return worst

    def check() -> bool:
        """Record the worst residual; True when the iteration ends here."""
        dots(r, r, rr)
        worst = float(torch.sqrt(rr / gg).max().item())
        info.rel_residual.append(worst)
        if worst <= tol and (not confirm or true_worst() <= tol):
            info.converged = True
            return True
        if not math.isfinite(worst):
            info.failure = "nonfinite"
            return True
        h = info.rel_residual
        if stall_checks and len(h) > stall_checks and h[-1] > stall_ratio * h[-1 - stall_checks]:
            info.failure = "stall"
            return True
        return False

    k = max(1, int(check_every))
    it, g_obj = 0, None
    while it < iters:
        n = min(k - it % k, iters - it)        # iterations up to the next check
        if graph and it > 0 and n == k:
            if g_obj is None:
                g_obj = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g_obj):
                    for _ in range(k):
                        step()
            g_obj.replay()
        else:
            for _ in range(n):
                step()
        it += n
        info.iterations = it
        if tol is not None and check():
            break
    torch.cuda.synchronize(dev)
    info.seconds = time.perf_counter() - t0
    return x, info


def pcgls(op, P, g: torch.Tensor, iters: int, tol: float | None = None, check_every: int = 5,
          fallback: bool = True, stall_checks: int = 4, graph: bool = False, confirm: bool = True):
    """Right-preconditioned CGLS: min ||A P z - g||, image f = P z (accumulated directly).

    With a tolerance and fallback=True, a preconditioned run whose worst residual becomes
    non-finite or stalls is discarded and plain CGLS solves the problem from x0 = 0
    (info.fallback and info.failure are set; info.seconds covers both runs)."""
    x, info = cgls(op, g, iters, tol, check_every, stall_checks=stall_checks if tol is not None else 0,
                   graph=graph, P=P, confirm=confirm)
    if info.failure is None or not fallback:
        return x, info
    x, plain = cgls(op, g, iters, tol, check_every, graph=graph, confirm=confirm)
    plain.fallback = True
    plain.failure = info.failure
    plain.seconds += info.seconds
    return x, plain


def operator_norm_sq(op, shape, device, iters: int = 20, seed: int = 0) -> float:
    """Estimate ||A||^2 by power iteration on A^T A (one problem)."""
    gen = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.rand((1,) + tuple(shape), generator=gen).to(device)
    lam = 0.0
    for _ in range(iters):
        y = op.adjoint(op.apply(x))
        lam = float(torch.linalg.vector_norm(y.double()).item() / torch.linalg.vector_norm(x.double()).item())
        x = (y / torch.linalg.vector_norm(y)).contiguous()
    return lam


def landweber(op, g: torch.Tensor, iters: int, omega: float) -> torch.Tensor:
    """x_{k+1} = x_k + omega A^T (g - A x_k), x_0 = 0 (converges for 0 < omega < 2/||A||^2)."""
    batch = g.shape[0]
    x = torch.zeros((batch,) + tuple(op.domain_shape), dtype=torch.float32, device=g.device)
    r = torch.empty_like(g)
    for _ in range(iters):
        op.apply(x, out=r)
        X.vec_axpby(1.0, g, -1.0, r)          # r = g - A x
        X.vec_axpby(omega, op.adjoint(r), 1.0, x)
    return x
