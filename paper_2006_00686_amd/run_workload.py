"""Run a named workload's forward projection and adjoint a number of times, for a
profiler to trace (the transform only: no oracle, no timing of its own).

    python -m paper_2006_00686_amd.run_workload fan2d_512 --steps 10 [--batch B] [--adjoint auto]
    python -m paper_2006_00686_amd.run_workload batched_cone_helical --steps 1

The batched workload (16 uneven circular and helical cone problems) runs the persistent
forward of all members and then each member's adjoint, on seeded uniform volumes.
"""
from __future__ import annotations

import argparse
import sys

import torch

from . import inputs, xrt


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["par2d_128", "fan2d_512", "cone_256", "fan2d_256_sparse",
                                         "batched_cone_helical"])
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--adjoint", default="auto", choices=["auto", "scatter", "gather"])
    args = ap.parse_args(argv)
    if args.workload == "batched_cone_helical":
        return run_batched(args.steps)
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


def run_batched(steps: int) -> int:
    cfg = inputs.batched_workload()
    plans = [xrt.Plan(m["grid"], m["scan"], 0) for m in cfg["members"]]
    batch = xrt.Batch(plans)
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(4)
    imgs = [torch.empty(p.image_shape, device="cuda:0").uniform_(0.0, 1.0, generator=gen) for p in plans]
    sinos = [torch.empty(p.sino_shape, device="cuda:0") for p in plans]
    backs = [torch.empty(p.image_shape, device="cuda:0") for p in plans]
    for k in range(steps + 1):
        batch.forward(imgs, sinos)
        for p, sn, bk in zip(plans, sinos, backs):
            p.adjoint(sn, out=bk)
    torch.cuda.synchronize()
    print(f"[run_workload] {cfg['name']}: {steps + 1} steps of the batched forward + {len(plans)} adjoints",
          flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
