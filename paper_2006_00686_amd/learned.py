"""Learned preconditioner for CGLS: P = I + C3 C2 C1, a three-layer 3x3 CNN
(1 -> 32 -> 32 -> 1 channels, BF16 weights, FP32 accumulation) on the image.

CGLS is a Krylov method for a fixed linear operator, so the preconditioner is linear:
the layers have no bias and no activation (a nonlinear network would change the
operator from one iteration to the next).  Right preconditioning solves
min ||A P z - g|| and returns f = P z; its adjoint is P^T = I + C1^T C2^T C3^T, computed
by the same kernels as transposed convolutions.  Every convolution (and, for training,
its input and weight gradients) runs in the library's kernels.

Training unrolls K iterations of right-preconditioned CGLS on sinograms the projector
itself produces and minimises the relative data residual left after K iterations.  The
projector, its adjoint and all convolutions are the library's kernels; the CGLS scalar
and vector algebra of the unrolled training graph goes through torch autograd.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import autograd as xag
from . import xrt as X


class _Conv(torch.autograd.Function):
    """One layer (cin -> cout), or its adjoint, with input and weight gradients."""

    @staticmethod
    def forward(ctx, x, w, cin, cout, transposed):
        ctx.save_for_backward(x, w)
        ctx.cfg = (cin, cout, transposed)
        return X.conv3x3(x.contiguous(), w, cin, cout, transposed)

    @staticmethod
    def backward(ctx, dout):
        x, w = ctx.saved_tensors
        cin, cout, tr = ctx.cfg
        och = cin if tr else cout
        dout = dout.contiguous().to(torch.float32 if och == 1 else torch.bfloat16)
        dx = X.conv3x3(dout, w, cin, cout, not tr)
        dw = X.conv3x3_wgrad(dout, x, cin, cout) if tr else X.conv3x3_wgrad(x, dout, cin, cout)
        return dx, dw, None, None, None


class ConvPreconditioner(torch.nn.Module):
    SHAPES = ((1, 32), (32, 32), (32, 1))

    def __init__(self, device="cuda:0", seed: int = 0, init_scale: float = 1e-3):
        super().__init__()
        gen = torch.Generator().manual_seed(seed)
        ws = []
        for cin, cout in self.SHAPES:
            w = torch.randn((cout, 3, 3, cin), generator=gen) * init_scale / np.sqrt(9 * cin)
            ws.append(torch.nn.Parameter(w.to(device)))
        self.w1, self.w2, self.w3 = ws

    # -------------------------------------------------------------- operators (no grad)

    @torch.no_grad()
    def apply(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """P x in one fused launch (hidden activations stay on chip)."""
        if out is not None and out.data_ptr() == x.data_ptr():
            out.copy_(X.precond_apply(x, self.w1.data, self.w2.data, self.w3.data))
            return out
        return X.precond_apply(x, self.w1.data, self.w2.data, self.w3.data, out=out)

    @torch.no_grad()
    def adjoint(self, y: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """P^T y in one fused launch."""
        if out is not None and out.data_ptr() == y.data_ptr():
            out.copy_(X.precond_apply(y, self.w1.data, self.w2.data, self.w3.data, transposed=True))
            return out
        return X.precond_apply(y, self.w1.data, self.w2.data, self.w3.data, transposed=True, out=out)

    @torch.no_grad()
    def apply_layers(self, x: torch.Tensor) -> torch.Tensor:
        """P x layer by layer (the activations the training path keeps)."""
        h = X.conv3x3(x, self.w1.data, 1, 32)
        h = X.conv3x3(h, self.w2.data, 32, 32)
        return X.conv3x3(h, self.w3.data, 32, 1, residual=x)

    @torch.no_grad()
    def adjoint_layers(self, y: torch.Tensor) -> torch.Tensor:
        h = X.conv3x3(y, self.w3.data, 32, 1, transposed=True)
        h = X.conv3x3(h, self.w2.data, 32, 32, transposed=True)
        return X.conv3x3(h, self.w1.data, 1, 32, transposed=True, residual=y)

    # -------------------------------------------------------------- differentiable

    def apply_diff(self, x: torch.Tensor) -> torch.Tensor:
        h = _Conv.apply(x, self.w1, 1, 32, False)
        h = _Conv.apply(h, self.w2, 32, 32, False)
        return x + _Conv.apply(h, self.w3, 32, 1, False)

    def adjoint_diff(self, y: torch.Tensor) -> torch.Tensor:
        h = _Conv.apply(y, self.w3, 32, 1, True)
        h = _Conv.apply(h, self.w2, 32, 32, True)
        return y + _Conv.apply(h, self.w1, 1, 32, True)

    def save(self, path: str):
        torch.save({"w1": self.w1.detach().cpu(), "w2": self.w2.detach().cpu(), "w3": self.w3.detach().cpu()}, path)

    def load(self, path: str):
        st = torch.load(path, map_location="cpu", weights_only=True)
        with torch.no_grad():
            self.w1.copy_(st["w1"])
            self.w2.copy_(st["w2"])
            self.w3.copy_(st["w3"])
        return self


def _bdot(a, b):
    return (a.double() * b.double()).flatten(1).sum(1)


def unrolled_pcgls_residuals(plan: X.Plan, P: ConvPreconditioner, g: torch.Tensor, K: int) -> torch.Tensor:
    """Relative recursive residuals ||r_k|| / ||g||, k = 1..K, of right-preconditioned
    CGLS (z0 = 0) per problem ([K][batch]), differentiable in P's weights."""
    shape = (-1,) + (1,) * (g.dim() - 1)
    gg = _bdot(g, g)
    r = g
    s = P.adjoint_diff(xag.backproject(r, plan))
    p = s
    gamma = _bdot(s, s)
    out = []
    for _ in range(K):
        q = xag.project(P.apply_diff(p), plan)
        alpha = (gamma / _bdot(q, q)).float()
        r = r - alpha.view(shape) * q
        out.append(torch.sqrt(_bdot(r, r) / gg))
        s = P.adjoint_diff(xag.backproject(r, plan))
        gnew = _bdot(s, s)
        p = s + (gnew / gamma).float().view(shape) * p
        gamma = gnew
    return torch.stack(out)


def training_batch(cfg: dict, plan: X.Plan, batch: int, seed0: int, device) -> torch.Tensor:
    """Noisy sinograms of fresh random phantoms (seeds seed0 .. seed0 + batch - 1)."""
    from . import inputs
    g = cfg["grid"]
    imgs = np.stack([inputs.ellipse_phantom(g["nx"], g["ny"], cfg["phantom"][1], seed0 + k) for k in range(batch)])
    clean = plan.forward(torch.from_numpy(imgs).to(device)).cpu().numpy()
    noisy = np.stack([inputs.poisson_sinogram(clean[k], cfg.get("photons", 1e5), seed0 + 77777 + k)
                      for k in range(batch)]).astype(np.float32)
    return torch.from_numpy(noisy).to(device)


VAL_SEED0 = 3_000_000      # validation phantoms for model selection


def iterations_to(plan: X.Plan, P, g: torch.Tensor, tol: float, max_iters: int = 400) -> int:
    """PCGLS iterations until every problem's recursive residual is <= tol (max_iters + 1
    when it does not get there)."""
    from . import solvers
    _, info = solvers.pcgls(solvers.PlanOperator(plan), P, g, max_iters, tol, check_every=1, fallback=False)
    return info.iterations if info.converged else max_iters + 1


def train(plan: X.Plan, cfg: dict, steps: int = 300, batch: int = 16, K: int = 10, lr: float = 2e-3,
          seed: int = 0, device="cuda:0", init: str | None = None, clip: float | None = None,
          loss_kind: str = "final", cosine: bool = False, val_every: int = 25, val_batch: int = 16,
          tol: float = 1e-3, log=print) -> tuple[ConvPreconditioner, list]:
    """Adam on the mean relative residual after K unrolled PCGLS iterations (loss_kind
    "final") or on the mean log residual along all K ("trajectory"), optionally with
    gradient-norm clipping and cosine learning-rate decay.  Every val_every steps the
    weights are scored by the PCGLS iterations to `tol` on a fixed validation batch and
    the best weights seen are returned (the starting weights are scored first)."""
    P = ConvPreconditioner(device, seed=seed)
    if init is not None:
        P.load(init)
    opt = torch.optim.Adam(P.parameters(), lr=lr)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, T_max=max(steps, 1)) if cosine else None
    gval = training_batch(cfg, plan, val_batch, VAL_SEED0, device)
    best = (iterations_to(plan, P, gval, tol), {k: v.detach().clone() for k, v in P.state_dict().items()})
    log(f"[train] validation: {best[0]} iterations to {tol:g} at the start")
    history = []
    data_seed = 1_000_000 + 1000 * seed
    t0 = time.perf_counter()
    for step in range(steps):
        g = training_batch(cfg, plan, batch, data_seed + step * batch, device)
        res = unrolled_pcgls_residuals(plan, P, g, K)
        loss = torch.log(res).mean() if loss_kind == "trajectory" else res[-1].mean()
        opt.zero_grad()
        loss.backward()
        if clip is not None:
            torch.nn.utils.clip_grad_norm_(P.parameters(), clip)
        opt.step()
        if sched is not None:
            sched.step()
        history.append(float(res[-1].mean().item()))
        if (step + 1) % val_every == 0 or step == steps - 1:
            it = iterations_to(plan, P, gval, tol)
            if it < best[0]:
                best = (it, {k: v.detach().clone() for k, v in P.state_dict().items()})
            log(f"[train] step {step + 1} residual after {K} PCGLS iterations {history[-1]:.4e}, "
                f"validation {it} iterations (best {best[0]}) ({time.perf_counter() - t0:.1f} s)")
    P.load_state_dict(best[1])
    return P, history


EVAL_SEED0 = 5_000_000     # held-out phantoms; training draws from 1_000_000 + 1000 * seed onwards


def default_weights() -> str:
    import os
    return os.path.join(os.path.dirname(__file__), "weights", "precond_fan256_60views.pt")


def evaluate(plan: X.Plan, P: ConvPreconditioner, g: torch.Tensor, tol: float = 1e-3, max_iters: int = 3000,
             check_every: int = 1, op=None) -> dict:
    """Wall time from data on the device to the first image whose residual satisfies
    ||A f - g|| <= tol ||g|| for every problem of the batch (the recursive residual
    proposes the stop, the true residual with FP64 norms confirms it inside the timed
    region): plain CGLS and CGLS right-preconditioned by P, with the on-the-fly transform
    of the plan or the operator `op` (e.g. the stored matrix).  Both solvers run once
    untimed first (kernel loading)."""
    from . import solvers
    op = op if op is not None else solvers.PlanOperator(plan)
    solvers.cgls(op, g, 2, tol, check_every)
    solvers.pcgls(op, P, g, 2, tol, check_every, fallback=False)
    xc, ic = solvers.cgls(op, g, max_iters, tol, check_every)
    xp, ip = solvers.pcgls(op, P, g, max_iters, tol, check_every)
    def last(h):
        return h[-1] if h else None

    return dict(cgls=dict(seconds=ic.seconds, iterations=ic.iterations, converged=ic.converged,
                          rel_residual=last(ic.rel_residual), true_residual=last(ic.true_residual),
                          confirmations=len(ic.true_residual)),
                pcgls=dict(seconds=ip.seconds, iterations=ip.iterations, converged=ip.converged,
                           rel_residual=last(ip.rel_residual), true_residual=last(ip.true_residual),
                           confirmations=len(ip.true_residual), fallback=ip.fallback, failure=ip.failure),
                speedup=ic.seconds / ip.seconds if ip.seconds > 0 else None,
                images=(xc, xp))
