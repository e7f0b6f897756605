#!/usr/bin/env python3
"""Benchmark of the hot path: forward + adjoint X-ray transform of the 256^3 circular
cone-beam workload (256^3 float32 volume of 20 random ellipsoids, 360 views over 2 pi,
SOD 1000, SDD 1500, flat 512 x 384 detector at spacing 1.0) on one MI355X.

A step is one forward projection and one adjoint of the whole scan, with the volume
already resident in HBM.  Prints ONE JSON line on stdout (everything else on stderr):
metric (Mrays/s of forward + adjoint), the dominant kernel's roofline figures, the
FP64 oracle timed on a bounded sample on the host cores, and the time to a relative
residual of 1e-3 of CGLS with and without the learned preconditioner.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("xrt_walk.h", "xrt_project.hip", "xrt_gather.hip", "xrt_internal.h"):
        with open(os.path.join(ROOT, "paper_2006_00686_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc summary, or
    None when it is absent or was taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def copy_bandwidth(dev, stream, mib: int = 1024, reps: int = 10) -> float:
    """Measured device-to-device copy rate (bytes read + written per second, GB/s) of a
    `mib` MiB buffer: the practical ceiling the datasheet HBM peak is compared with."""
    import torch
    src = torch.empty(mib * (1 << 20) // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        e0.record(stream)
        dst.copy_(src)
        e1.record(stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    del src, dst
    return 2.0 * mib * (1 << 20) / (float(np.median(ts)) * 1e-3) / 1e9


def cpu_baseline(cfg, img, views_every: int):
    """The FP64 oracle, as it stands, on every `views_every`-th view of the scan."""
    from oracle import core as ocore
    from oracle import geometry as ogeom
    scan = dict(cfg["scan"])
    scan["angles"] = np.asarray(cfg["scan"]["angles"])[::views_every]
    p, th = ogeom.expand(scan)
    threads = ocore.default_threads()
    f64 = img.astype(np.float64)
    t0 = time.perf_counter()
    g = ocore.forward_lines(cfg["grid"], p, th, f64, nthreads=threads)
    t1 = time.perf_counter()
    ocore.adjoint_lines(cfg["grid"], p, th, g, nthreads=threads)
    t2 = time.perf_counter()
    m = p.shape[0]
    nv = len(cfg["scan"]["angles"])
    return {"value": m / (t2 - t0) / 1e6, "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "host": ocore.host_info(),
            "sample": f"every {views_every}th view ({scan['angles'].size} of {nv} views, {m} rays; every view "
                      f"has the same work, so the rate is that of the full scan, which would take about "
                      f"{(t2 - t0) * nv / scan['angles'].size:.0f} s), forward {t1 - t0:.2f} s + adjoint "
                      f"{t2 - t1:.2f} s, FP64, {threads} threads (the cores this process may use, capped by "
                      f"OMP_NUM_THREADS)"}


def learned_solve(torch, dev, tol: float = 1e-3):
    """Sparse-view fan-beam workload (64 held-out phantoms, 256^2, 60 views, Poisson noise):
    wall time to relative residual `tol` of plain CGLS and of CGLS right-preconditioned by
    the trained CNN, plus the true data residual of both final images."""
    from paper_2006_00686_amd import inputs, learned, xrt
    cfg = inputs.workload("fan2d_256_sparse")
    plan = xrt.Plan(cfg["grid"], cfg["scan"], 0)
    g = learned.training_batch(cfg, plan, cfg["batch"], learned.EVAL_SEED0, dev)
    P = learned.ConvPreconditioner(dev).load(learned.default_weights())
    r = learned.evaluate(plan, P, g, tol=tol)
    xc, xp = r.pop("images")

    def true_residual(x):
        d = (plan.forward(x) - g).double().flatten(1)
        return float(torch.sqrt((d * d).sum(1) / (g.double().flatten(1) ** 2).sum(1)).max())

    # the same solves with the projection matrix stored (CSR of A and its transpose)
    from paper_2006_00686_amd import solvers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    A = xrt.SparseMatrix.from_plan(plan)
    mop = solvers.MatrixOperator(A)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    rs = learned.evaluate(plan, P, g, tol=tol, op=mop)
    rs.pop("images")
    stored = {"build_s": round(build_s, 5), "nnz": A.nnz, "bytes": 2 * A.bytes(),
              "cgls_s": round(rs["cgls"]["seconds"], 5), "cgls_iterations": rs["cgls"]["iterations"],
              "pcgls_s": round(rs["pcgls"]["seconds"], 5), "pcgls_iterations": rs["pcgls"]["iterations"],
              "speedup": round(rs["speedup"], 3)}

    return {"workload": cfg["name"], "batch": cfg["batch"], "tol": tol,
            "cgls_s": round(r["cgls"]["seconds"], 5), "cgls_iterations": r["cgls"]["iterations"],
            "pcgls_s": round(r["pcgls"]["seconds"], 5), "pcgls_iterations": r["pcgls"]["iterations"],
            "speedup": round(r["speedup"], 3), "fallback": r["pcgls"]["fallback"],
            "true_residual": {"cgls": true_residual(xc), "pcgls": true_residual(xp)},
            "confirmations": {"cgls": r["cgls"]["confirmations"], "pcgls": r["pcgls"]["confirmations"]},
            "weights": os.path.relpath(learned.default_weights(), ROOT), "stored_matrix": stored}


def workloads_2d(torch, dev, steps: int = 20):
    """The 2D workloads: forward + adjoint (AUTO) of one image per step, and the 2D
    parallel case also as 64 images per launch each way; median of `steps` steps."""
    from paper_2006_00686_amd import inputs, xrt
    out = {}
    for name, batch in (("par2d_128", 1), ("par2d_128", 64), ("fan2d_512", 1)):
        cfg = inputs.workload(name)
        plan = xrt.Plan(cfg["grid"], cfg["scan"], 0)
        one = torch.from_numpy(inputs.make_image(cfg)).to(dev)
        img = one.expand((batch,) + tuple(one.shape)).contiguous() if batch > 1 else one
        sino = plan.forward(img)
        back = plan.adjoint(sino)
        torch.cuda.synchronize()
        ts = []
        for _ in range(steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.forward(img, out=sino)
            plan.adjoint(sino, out=back)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        key = cfg["name"] + (f"_batch{batch}" if batch > 1 else "")
        out[key] = {"ms_per_step": round(ms, 4), "images": batch,
                    "mrays_per_s": round(plan.n_rays * batch / (ms * 1e-3) / 1e6, 1)}
        plan.close()
    return out


def batched_bench(torch, dev, steps: int, tuning: dict):
    """16 uneven cone / helical problems: forward of all members in one persistent launch
    plus every member's adjoint, captured once in a graph and replayed; the same work as
    plain per-plan launches for comparison."""
    from paper_2006_00686_amd import inputs, xrt
    from paper_2006_00686_amd.batched import BatchGraph
    cfg = inputs.batched_workload()
    plans = [xrt.Plan(m["grid"], m["scan"], 0) for m in cfg["members"]]
    if tuning is not None:
        for p in plans:
            p.set_tuning(**tuning)
    bg = BatchGraph(xrt.Batch(plans))
    gen = torch.Generator(device=dev)
    for k, im in enumerate(bg.imgs):
        gen.manual_seed(cfg["members"][k]["seed"])
        im.uniform_(0.0, 1.0, generator=gen)
    bg.capture()
    bg.replay()
    torch.cuda.synchronize()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / steps

    t_graph = timed(bg.replay)

    def eager():
        for p, im, sn, bk in zip(plans, bg.imgs, bg.sinos, bg.backs):
            p.forward(im, out=sn)
            p.adjoint(sn, out=bk)

    eager()
    t_eager = timed(eager)

    # the forward alone: one persistent launch over the queue vs one launch per plan
    t_fwd_batch = timed(lambda: bg.batch.forward(bg.imgs, out=bg.sinos))

    def fwd_each():
        for p, im, sn in zip(plans, bg.imgs, bg.sinos):
            p.forward(im, out=sn)

    t_fwd_each = timed(fwd_each)
    rays = sum(p.n_rays for p in plans)
    dims = sorted({tuple(p.image_shape) for p in plans}, key=lambda d: -int(np.prod(d)))
    return {"workload": cfg["name"], "members": len(plans), "rays": rays, "volumes_zyx": [list(d) for d in dims],
            "ms_per_step": round(t_graph, 3), "mrays_per_s": round(rays / (t_graph * 1e-3) / 1e6, 1),
            "per_plan_launches_ms": round(t_eager, 3), "forward_persistent_ms": round(t_fwd_batch, 3),
            "forward_per_plan_ms": round(t_fwd_each, 3),
            "launch": tuning if tuning is not None else "each plan's own",
            "data": "synthetic: seeded uniform volumes"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--adjoint", default="auto", choices=["auto", "scatter", "gather"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner solve comparison")
    ap.add_argument("--no-batched", action="store_true", help="skip the 16-problem batched launch")
    ap.add_argument("--no-2d", dest="w2d", action="store_false", help="skip the 2D workloads")
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="skip the forward launch-shape autotuner (untimed; default on) and keep the plan's own shape")
    ap.add_argument("--launch", default=None, metavar="PC,XR",
                    help="forward launch shape packet_cols,xcd_remap to use instead of the autotuner's")
    ap.add_argument("--cpu-views-every", type=int, default=4,
                    help="time the oracle on every n-th view of the scan (default 4: 90 views, about 10-15 s)")
    ap.add_argument("--copy-reference", action="store_true",
                    help="first run a plain 256 MiB device copy (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported (this build runs the "
              "transform on a single MI355X; sharding across GPUs is a design note, not code).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2006_00686_amd import inputs
    from paper_2006_00686_amd import xrt

    cfg = inputs.workload("cone_256")
    log(f"[bench] building phantom {cfg['name']}")
    img = inputs.make_image(cfg)
    dev = torch.device("cuda:0")
    plan = xrt.Plan(cfg["grid"], cfg["scan"], 0)
    d_img = torch.from_numpy(img).to(dev)
    d_sino = torch.empty(plan.sino_shape, dtype=torch.float32, device=dev)
    d_back = torch.empty(plan.image_shape, dtype=torch.float32, device=dev)
    # hits of physical length > 1e-9 (rays through unit edges leave FP64 slivers of ~1e-13)
    nnz = int(plan.hit_counts(eps=1e-9).to(torch.int64).sum().item())
    M, V = plan.n_rays, plan.n_units
    log(f"[bench] rays {M}, units {V}, nnz {nnz} ({nnz / M:.1f} per ray)")

    tuning = plan.tuning()   # the library's choice for this plan
    if args.launch:
        pc, xr = (int(v) for v in args.launch.split(","))
        plan.set_tuning(pc, xr)
        tuning = plan.tuning()
        log(f"[bench] forward launch shape {tuning} (given)")
    elif args.tune:
        from paper_2006_00686_amd import tune
        res = tune.autotune(plan, d_img, log=log)
        tuning = {"packet_cols": res["packet_cols"], "xcd_remap": res["xcd_remap"]}
        log(f"[bench] forward launch shape {tuning} ({'cached' if res['cached'] else 'tuned'})")

    if args.copy_reference:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        plan.forward(d_img, out=d_sino)
        plan.adjoint(d_sino, mode=args.adjoint, out=d_back)
    torch.cuda.synchronize()
    log(f"[bench] warmup done, timing {args.steps} steps")

    stream = torch.cuda.current_stream(dev)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        plan.forward(d_img, out=d_sino)
        ev[k][1].record(stream)
        plan.adjoint(d_sino, mode=args.adjoint, out=d_back)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    # per-kernel times: median over the timed steps (robust to a stray slow step)
    t_fwd = float(np.median([e[0].elapsed_time(e[1]) for e in ev]))
    t_adj = float(np.median([e[1].elapsed_time(e[2]) for e in ev]))
    log(f"[bench] {ms_step:.3f} ms/step (events: forward {t_fwd:.3f} ms, adjoint {t_adj:.3f} ms)")

    b_fwd = 4.0 * nnz + 4.0 * M        # one 4-byte gather per hit + the ray's output
    b_adj = 4.0 * nnz + 4.0 * V        # one 4-byte operand per hit + the image once
    adj_kernel = "k_scatter" if args.adjoint == "scatter" else "k_cone_gather"
    if t_fwd >= t_adj:
        kname, bytes_, t_k = "k_forward", b_fwd, t_fwd
    else:
        kname, bytes_, t_k = adj_kernel, b_adj, t_adj
    achieved = bytes_ / (t_k * 1e-3) / 1e9
    traffic = measured_traffic(kname)
    # (not in counter runs, whose only large copy must be the 256 MiB reference)
    copy_gbs = None if args.copy_reference else copy_bandwidth(dev, stream)
    if copy_gbs:
        log(f"[bench] device-to-device copy: {copy_gbs:.0f} GB/s (read + write)")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kname,
                "kernel_ms": round(t_k, 4), "algorithmic_bytes": bytes_,
                "fwd_ms": round(t_fwd, 4), "adj_ms": round(t_adj, 4),
                "fwd_plus_adj_frac": round((b_fwd + b_adj) / ((t_fwd + t_adj) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "copy_GBps": round(copy_gbs, 1) if copy_gbs else None,
                "frac_of_copy": round(achieved / copy_gbs, 4) if copy_gbs else None}

    # the attenuated transform (SPECT weight) of the same workload, mu = 0.01 per unit length
    log("[bench] attenuated transform")
    gen = torch.Generator(device=dev).manual_seed(13)
    d_mu = torch.rand(tuple(plan.image_shape), generator=gen, device=dev) * 0.01
    plan.forward_attenuated(d_img, d_mu, out=d_sino)
    plan.adjoint_attenuated(d_sino, d_mu, out=d_back)
    ea = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    ea[0].record(stream)
    for _ in range(2):
        plan.forward_attenuated(d_img, d_mu, out=d_sino)
    ea[1].record(stream)
    for _ in range(2):
        plan.adjoint_attenuated(d_sino, d_mu, out=d_back)
    ea[2].record(stream)
    torch.cuda.synchronize()
    attenuated = {"forward_ms": round(ea[0].elapsed_time(ea[1]) / 2, 3),
                  "adjoint_ms": round(ea[1].elapsed_time(ea[2]) / 2, 3), "adjoint": "scatter",
                  "mu": "uniform [0, 0.01) per unit length"}
    log(f"[bench] attenuated {attenuated}")

    w2d = None
    if args.w2d:
        w2d = workloads_2d(torch, dev)
        log(f"[bench] 2D workloads {w2d}")

    batched = None
    if not args.no_batched:
        log("[bench] batched launch: 16 uneven cone/helical problems")
        batched = batched_bench(torch, dev, 3, None)
        log(f"[bench] batched {batched}")

    learned = None
    if not args.no_learned:
        log("[bench] learned preconditioner vs plain CGLS (sparse-view fan beam, batch 64)")
        learned = learned_solve(torch, dev)
        log(f"[bench] learned {learned}")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a sample")
        cpu = cpu_baseline(cfg, img, args.cpu_views_every)
        log(f"[bench] cpu baseline {cpu}")

    value = M / (ms_step * 1e-3) / 1e6
    out = {
        "metric": "Mrays/s fwd+adj at 256\u00b3 cone (%HBM roofline); time-to-1e-3 learned vs CGLS",
        "value": round(value, 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: seeded random-ellipsoid volume",
        "config": {"workload": cfg["name"], "volume": [256, 256, 256], "views": 360, "detector": [384, 512],
                   "sod": 1000.0, "sdd": 1500.0, "rays": M, "nnz": nnz, "adjoint": args.adjoint,
                   "intersections_per_s": round(2 * nnz / (ms_step * 1e-3), 1),
                   "crossing_parameter_dtype": "f64", "parallelism": "single GPU", "launch": tuning},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "learned": learned,
        "batched": batched,
        "attenuated": attenuated,
        "workloads_2d": w2d,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
