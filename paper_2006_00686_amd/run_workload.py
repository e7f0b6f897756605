"""Run a named workload's forward projection and adjoint a number of times, for a
profiler to trace (the transform only: no oracle, no timing of its own).

    python -m paper_2006_00686_amd.run_workload fan2d_512 --steps 10 [--batch B] [--adjoint auto]
"""
from __future__ import annotations

import argparse
import sys

import torch

from . import inputs, xrt


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["par2d_128", "fan2d_512", "cone_256", "fan2d_256_sparse"])
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--adjoint", default="auto", choices=["auto", "scatter", "gather"])
    args = ap.parse_args(argv)
    cfg = inputs.workload(args.workload)
    plan = xrt.Plan(cfg["grid"], cfg["scan"], 0)
    one = torch.from_numpy(inputs.make_image(cfg)).to("cuda:0")
    img = one.expand((args.batch,) + tuple(one.shape)).contiguous() if args.batch > 1 else one
    sino = plan.forward(img)
    back = plan.adjoint(sino, mode=args.adjoint)
    for k in range(args.steps):
        plan.forward(img, out=sino)
        plan.adjoint(sino, mode=args.adjoint, out=back)
    torch.cuda.synchronize()
    print(f"[run_workload] {cfg['name']}: {args.steps} steps of forward + adjoint ({plan.adjoint_info()})", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
