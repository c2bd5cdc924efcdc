"""Benchmark: POT solves/s at eps = 1e-2 on one MI355X.

A step is one whole solve through the C ABI (pot_solve): setup
("Approximating POT"), the ASPOT loop (three fused statistics passes per
iteration with the on-device decisions), the FP64 rounding onto U(r, c, s)
and the objective.  Inputs are resident in HBM before the timed region.

Default workload: one instance, n = m = 4096, 3-D points in 8 Gaussian
clusters (sigma 0.05) with 10 % uniform outliers, squared-Euclidean cost
normalised to max 1 and stored dense in FP32, uniform masses with totals
1.0 / 1.0, s = 0.9, eps = 1e-2, cold start.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _build_if_missing():
    from paper_2601_17196_amd import pot
    if not os.path.exists(pot.lib_path()):
        import __graft_entry__
        __graft_entry__.build()


def run_solve(pot, d, eps, algo, kind, **kw):
    if kind == "points":
        return pot.solve(d["r"], d["c"], d["s"], eps, x=d["x"], y=d["y"], cost_scale=d["cost_scale"],
                         cmax=1.0, algo=algo, **kw)
    return pot.solve(d["r"], d["c"], d["s"], eps, C=d["C"], kind=d["kind"], ldc=d["ldc"], cmax=1.0,
                     algo=algo, **kw)


def time_solves(pot, d, eps, algo, kind, steps, warmup, workspace):
    import torch
    for _ in range(warmup):
        run_solve(pot, d, eps, algo, kind, workspace=workspace, want_factors=False)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    outs = []
    for _ in range(steps):
        outs.append(run_solve(pot, d, eps, algo, kind, workspace=workspace, want_factors=False))
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    return outs, wall, ev_ms


def cpu_baseline(inst, iters_full, eps, budget_iters):
    """The FP64 oracle (as it stands) timed on the host cores on a bounded
    sample: `budget_iters` ASPOT iterations of the same instance, scaled to
    solves/s with the full solve's iteration count."""
    import numpy as np

    from oracle import potref
    C = inst.C32.astype(np.float64)
    gam, tol, M, rt, ct_ = potref.setup(inst.r, inst.c, inst.s, eps, cmax=1.0)
    t0 = time.perf_counter()
    potref.aspot(C, gam, tol, rt, ct_, inst.s, M, max_iter=budget_iters)
    dt = time.perf_counter() - t0
    per_iter = dt / budget_iters
    return {
        "value": 1.0 / (per_iter * iters_full),
        "unit": "solves/s",
        "cores": potref.threads(),
        "kind": "oracle",
        "sample": (f"{budget_iters} ASPOT iterations of the same n=m={inst.n} instance "
                   f"({dt:.1f} s, {per_iter * 1e3:.1f} ms/iteration), scaled by the full solve's "
                   f"{iters_full} iterations"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--algo", default="aspot", choices=["aspot", "sinkhorn"])
    ap.add_argument("--kind", default="f32", choices=["f32", "bf16", "points"])
    ap.add_argument("--cpu-iters", type=int, default=16)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the solver has no multi-GPU path in this build "
              "(see DESIGN.md for how it would shard)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    _build_if_missing()
    from paper_2601_17196_amd import instances as I
    from paper_2601_17196_amd import pot

    dev = torch.device("cuda:0")
    eps = 1e-2
    log(f"generating workload n=m={args.n}")
    inst = I.c2(0, n=args.n)
    d = pot.to_device_instance(inst, dev, kind=args.kind)
    algo = pot.ASPOT if args.algo == "aspot" else pot.SINKHORN
    first = run_solve(pot, d, eps, algo, args.kind)
    # workspace sized once, reused by every timed solve
    prob = pot.make_problem(d["r"], d["c"], d["s"], C=d.get("C"), x=d.get("x"), y=d.get("y"),
                            kind=d.get("kind"), ldc=d.get("ldc"), cost_scale=d.get("cost_scale", 0.0),
                            cmax=1.0)
    ws = torch.empty(pot.workspace_bytes(prob, pot.make_options(eps, algo=algo)) + 256, dtype=torch.uint8,
                     device=dev)
    log(f"first solve: status {first.status} iters {first.result['iters']} cost {first.result['cost']:.9e}")
    outs, wall, ev_ms = time_solves(pot, d, eps, algo, args.kind, args.steps, args.warmup, ws)
    iters = outs[-1].result["iters"]
    ms_per_step = ev_ms / args.steps
    value = args.steps / (ev_ms / 1e3)
    log(f"timed {args.steps} solves: {ev_ms:.2f} ms (events), {wall * 1e3:.2f} ms (wall); "
        f"{value:.3f} solves/s, {iters} iterations, {ms_per_step / max(iters, 1) * 1e3:.2f} us/iteration")

    # roofline of the dominant kernel: the fused statistics pass at the
    # converged duals, timed with HIP events around each dispatch
    o = first
    kw = dict(u0=o.u, v0=o.v, w0=o.w)
    if args.kind == "points":
        pass_ms, fin_ms = pot.time_pass(d["r"], d["c"], d["s"], eps, reps=50, x=d["x"], y=d["y"],
                                        cost_scale=d["cost_scale"], cmax=1.0, **kw)
    else:
        pass_ms, fin_ms = pot.time_pass(d["r"], d["c"], d["s"], eps, reps=50, C=d["C"], kind=d["kind"],
                                        ldc=d["ldc"], cmax=1.0, **kw)
    n = m = args.n
    elem_bytes = {"f32": 4, "bf16": 2, "points": 0}[args.kind]
    if args.kind == "points":
        # ALU-bound: algorithmic work = n*m exponentials per pass
        achieved = n * m / (pass_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": None, "unit": "Texp/s", "frac": None,
                "traffic": None}
    else:
        alg_bytes = n * m * elem_bytes
        achieved = alg_bytes / (pass_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None}
    log(f"tile kernel: {pass_ms * 1e3:.2f} us/launch -> {achieved:.1f} {roof['unit']}; "
        f"finalising kernel {fin_ms * 1e3:.2f} us")

    extra = {"iters": iters, "us_per_iteration": ms_per_step / max(iters, 1) * 1e3,
             "tile_kernel_us": pass_ms * 1e3, "fin_kernel_us": fin_ms * 1e3,
             "cost": outs[-1].result["cost"], "E": outs[-1].result["E"]}
    if not args.no_extra:
        for name, kind2, algo2 in [("sinkhorn_f32", "f32", pot.SINKHORN), ("aspot_points", "points", pot.ASPOT),
                                   ("aspot_bf16", "bf16", pot.ASPOT)]:
            if kind2 == args.kind and algo2 == algo:
                continue
            d2 = d if kind2 == args.kind else pot.to_device_instance(inst, dev, kind=kind2)
            o2, w2, ev2 = time_solves(pot, d2, eps, algo2, kind2, 3, 1, None)
            extra[name] = {"solves_per_s": 3 / (ev2 / 1e3), "iters": o2[-1].result["iters"],
                           "cost": o2[-1].result["cost"]}
            log(f"{name}: {extra[name]}")
            del d2
            torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        log(f"cpu baseline: {args.cpu_iters} oracle iterations")
        cpu = cpu_baseline(inst, iters, eps, args.cpu_iters)
        log(f"cpu baseline: {cpu}")

    line = {
        "metric": "POT solves/s at eps=1e-2 (ASPOT, cold start)",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 state/exponent + f32 exp" if args.kind != "bf16" else "bf16 cost + f32 exp/f64 sums",
        "data": "synthetic",
        "config": {"workload": f"single POT instance n=m={n}, 3-D 8 clusters + 10% outliers, "
                               f"{args.kind} cost, uniform masses 1/1, s=0.9, eps=1e-2, {args.algo} cold",
                   "n": n, "m": m, "algo": args.algo, "cost": args.kind},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
