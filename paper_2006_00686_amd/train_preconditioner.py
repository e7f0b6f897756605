"""Train the learned CGLS preconditioner on the sparse-view fan-beam workload (256 x 256
unit pixels, 60 views over 2 pi, 512 flat-detector bins of 0.75, source-to-centre 1000,
source-to-detector 1500; random-ellipse phantoms, Poisson noise at 1e5 photons per ray)
and report PCGLS against plain CGLS on held-out phantoms.

    python -m paper_2006_00686_amd.train_preconditioner --steps 300 --out weights.pt
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import torch

from . import inputs, learned
from . import xrt as X


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--unroll", type=int, default=10, help="PCGLS iterations unrolled in the loss")
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--clip", type=float, default=None)
    ap.add_argument("--loss", choices=["final", "trajectory"], default="final")
    ap.add_argument("--cosine", action="store_true")
    ap.add_argument("--val-every", type=int, default=25)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=learned.default_weights())
    ap.add_argument("--resume", default=None, help="weights to start from")
    ap.add_argument("--eval-batch", type=int, default=64)
    ap.add_argument("--tol", type=float, default=1e-3)
    args = ap.parse_args(argv)

    dev = "cuda:0"
    cfg = inputs.workload("fan2d_256_sparse")
    plan = X.Plan(cfg["grid"], cfg["scan"], device=0)
    t0 = time.perf_counter()
    P, hist = learned.train(plan, cfg, steps=args.steps, batch=args.batch, K=args.unroll, lr=args.lr,
                            seed=args.seed, device=dev, init=args.resume, clip=args.clip,
                            loss_kind=args.loss, cosine=args.cosine,
                            val_every=args.val_every, tol=args.tol,
                            log=lambda m: print(m, flush=True))
    train_s = time.perf_counter() - t0
    import os
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    P.save(args.out)
    g = learned.training_batch(cfg, plan, args.eval_batch, learned.EVAL_SEED0, dev)
    res = learned.evaluate(plan, P, g, tol=args.tol)
    res.pop("images")
    print(json.dumps(dict(train_seconds=train_s, steps=args.steps, batch=args.batch, unroll=args.unroll,
                          loss_first=hist[0], loss_last=hist[-1], weights=args.out, eval=res)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
