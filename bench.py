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
COPY_BYTES = 256 << 20          # the plain copy of the counter-scale probe (bytes read, and written)
PMC_SUMMARY = os.path.join(ROOT, "profiles", "stats_pass_c2_4096_f32_traffic.json")


def measured_traffic():
    """HBM bytes per launch of the tile kernel from the committed counter
    summary, or None when it is missing or was taken on other kernel sources."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    from paper_2601_17196_amd import profile_summary as PS
    s = json.load(open(PMC_SUMMARY))
    if s.get("kernel_source_hash") != PS.kernel_source_hash():
        return None
    return s.get("traffic_bytes")


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


def time_solves(pot, d, eps, algo, kind, steps, warmup, workspace, **kw):
    import torch
    for _ in range(warmup):
        run_solve(pot, d, eps, algo, kind, workspace=workspace, want_factors=False, **kw)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    outs = []
    for _ in range(steps):
        outs.append(run_solve(pot, d, eps, algo, kind, workspace=workspace, want_factors=False, **kw))
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    return outs, wall, ev_ms


def _batch_probs(pot, insts, dev):
    probs = []
    for inst in insts:
        d = pot.to_device_instance(inst, dev, kind="f32", pad_ldc=True)
        probs.append(dict(r=d["r"], c=d["c"], s=d["s"], C=d["C"], kind=d["kind"], ldc=d["ldc"], cmax=1.0))
    return probs


def _timed(fn, reps):
    import torch
    fn()                                   # warm-up (first call also autotunes the batched launch)
    torch.cuda.synchronize()
    best, out = None, None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        out = fn()
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1)
        best = t if best is None else min(best, t)
    return best, out


def bench_batched(pot, I, dev, eps, reps, plain_sample):
    """The uneven batch (512 instances, n, m log-uniform in [64, 1024]):
    pot_solve_batched against sequential pot_solve calls on a sample."""
    import numpy as np
    import torch
    insts = I.c4_batch(512)
    probs = _batch_probs(pot, insts, dev)
    ws = torch.empty(pot.workspace_bytes_batched(probs) + 512, dtype=torch.uint8, device=dev)
    t, (st, res, _) = _timed(lambda: pot.solve_batched(probs, eps, workspace=ws, want_duals=False), reps)
    its = np.array([r["iters"] for r in res])
    ok = all(r["status"] == 0 for r in res)
    sample = list(range(0, len(insts), len(insts) // plain_sample))[:plain_sample]

    def plain():
        for j in sample:
            pot.solve(probs[j]["r"], probs[j]["c"], probs[j]["s"], eps, C=probs[j]["C"], cmax=1.0, want_factors=False)
    tp, _ = _timed(plain, 1)
    out = {"instances": len(insts), "solves_per_s": len(insts) / (t / 1e3), "ms": t, "all_ok": ok,
           "iters_median": float(np.median(its)), "iters_max": int(its.max()),
           "plain_solves_per_s": len(sample) / (tp / 1e3), "plain_sample": len(sample)}
    del ws, probs
    torch.cuda.empty_cache()
    return out


def bench_warm(pot, I, dev, eps, reps, plain_sample):
    """The learned warm start on the n = m = 256 mixture batch (1024
    instances): inference + warm-started batched ASPOT against cold batched
    ASPOT and sequential plain solves (sample)."""
    import numpy as np
    import torch
    insts = I.c5_batch(1024)
    probs = _batch_probs(pot, insts, dev)
    pts = [dict(x=torch.from_numpy(np.ascontiguousarray(i.x, dtype=np.float32)).to(dev),
                y=torch.from_numpy(np.ascontiguousarray(i.y, dtype=np.float32)).to(dev),
                r=p["r"], c=p["c"], cost_scale=i.cost_scale) for i, p in zip(insts, probs)]
    ws = torch.empty(pot.workspace_bytes_batched(probs) + 512, dtype=torch.uint8, device=dev)
    blob = pot.warm_blob(device=dev)

    def warm():
        preds = pot.warm_predict(pts, eps, blob)
        return pot.solve_batched(probs, eps, u0=[p[0] for p in preds], v0=[p[1] for p in preds],
                                 w0=[0.0] * len(preds), warm_check=True, workspace=ws, want_duals=False)
    tc, (stc, resc, _) = _timed(lambda: pot.solve_batched(probs, eps, workspace=ws, want_duals=False), reps)
    tw, (stw, resw, _) = _timed(warm, reps)
    ti, _ = _timed(lambda: pot.warm_predict(pts, eps, blob), reps)
    sample = list(range(0, len(insts), len(insts) // plain_sample))[:plain_sample]

    def plain():
        for j in sample:
            pot.solve(probs[j]["r"], probs[j]["c"], probs[j]["s"], eps, C=probs[j]["C"], cmax=1.0, want_factors=False)
    tp, _ = _timed(plain, 1)
    itc = np.array([r["iters"] for r in resc])
    itw = np.array([r["iters"] for r in resw])
    out = {"instances": len(insts),
           "warm_batched_solves_per_s": len(insts) / (tw / 1e3),
           "cold_batched_solves_per_s": len(insts) / (tc / 1e3),
           "plain_solves_per_s": len(sample) / (tp / 1e3), "plain_sample": len(sample),
           "inference_ms": ti, "warm_kept": int(sum(r["used_warm"] for r in resw)),
           "iters_median_warm": float(np.median(itw)), "iters_median_cold": float(np.median(itc)),
           "iters_total_warm": int(itw.sum()), "iters_total_cold": int(itc.sum()),
           "max_cost_gap_warm_vs_cold": float(max(abs(a["cost"] - b["cost"]) for a, b in zip(resw, resc))),
           "all_ok": all(r["status"] == 0 for r in resw) and all(r["status"] == 0 for r in resc)}
    del ws, probs, pts
    torch.cuda.empty_cache()
    return out


def cpu_baseline(inst, iters_full, eps, budget_iters, one_core_iters=2):
    """The FP64 oracle (as it stands) timed on the host cores on a bounded
    sample: `budget_iters` ASPOT iterations of the same instance, scaled to
    solves/s with the full solve's iteration count; then `one_core_iters`
    iterations on one thread."""
    import numpy as np

    from oracle import potref
    C = inst.C32.astype(np.float64)
    gam, tol, M, rt, ct_ = potref.setup(inst.r, inst.c, inst.s, eps, cmax=1.0)
    cores = potref.threads()
    t0 = time.perf_counter()
    potref.aspot(C, gam, tol, rt, ct_, inst.s, M, max_iter=budget_iters)
    dt = time.perf_counter() - t0
    per_iter = dt / budget_iters
    potref.set_threads(1)
    t0 = time.perf_counter()
    potref.aspot(C, gam, tol, rt, ct_, inst.s, M, max_iter=one_core_iters)
    dt1 = time.perf_counter() - t0
    potref.set_threads(cores)
    per_iter1 = dt1 / one_core_iters
    return {
        "value": 1.0 / (per_iter * iters_full),
        "unit": "solves/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{budget_iters} ASPOT iterations of the same n=m={inst.n} instance "
                   f"({dt:.1f} s, {per_iter * 1e3:.1f} ms/iteration), scaled by the full solve's "
                   f"{iters_full} iterations; on 1 core {one_core_iters} iterations "
                   f"({per_iter1 * 1e3:.0f} ms/iteration)"),
        "value_1core": 1.0 / (per_iter1 * iters_full),
    }


def bench_shard(pot, I, dev, eps):
    """The statistics pass on one GPU's share of the 20000^2 instance split by
    rows over 8 GPUs: rows 0..2499 of its cost against all 20000 columns
    (FP32, the same normalisation), solved as an instance of its own (source
    masses rescaled to total 1, s = 0.7) to get representative duals, then
    the pass timed at them."""
    import numpy as np
    import torch
    inst = I.c3(0, dense=False)
    ns, m = inst.n // 8, inst.m
    x = torch.from_numpy(inst.x[:ns].astype(np.float64)).to(dev)
    y = torch.from_numpy(inst.y.astype(np.float64)).to(dev)
    D = torch.zeros((ns, m), dtype=torch.float64, device=dev)
    for k in range(x.shape[1]):
        diff = x[:, k:k + 1] - y[None, :, k]
        D += diff * diff
    C = (D * inst.cost_scale).to(torch.float32)
    del D
    r = torch.full((ns,), 1.0 / ns, dtype=torch.float64, device=dev)
    c = torch.from_numpy(inst.c).to(dev)
    o = pot.solve(r, c, 0.7, eps, C=C, cmax=1.0, want_factors=False)
    ms = pot.time_pass(r, c, 0.7, eps, reps=20, C=C, cmax=1.0, u0=o.u, v0=o.v, w0=o.w)[0]
    gbs = ns * m * 4 / (ms * 1e-3) / 1e9
    nx, ny = (m + 255) // 256, (ns + 127) // 128
    return {"n": ns, "m": m, "iters": o.result["iters"], "tile_kernel_us": ms * 1e3, "GB_per_s": gbs,
            "frac_hbm": gbs / HBM_PEAK_GBS, "column_partials_bytes": ny * m * 8,
            "allreduce_bytes_per_pass": (m + 3) * 8}


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
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--plain-sample", type=int, default=32)
    ap.add_argument("--pmc-probe", action="store_true",
                    help="profiling workload only: a 256 MiB device copy (the counters' scale), then one "
                         "solve and 20 timed statistics passes of the default workload; prints no JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the solver has no multi-GPU path (batches would shard by "
              "instance, one instance by rows of C with one all-reduce of m + 3 values per pass)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    _build_if_missing()
    from paper_2601_17196_amd import instances as I
    from paper_2601_17196_amd import pot

    dev = torch.device("cuda:0")
    eps = 1e-2
    if args.pmc_probe:
        a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
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
    if args.pmc_probe:
        kw = dict(u0=first.u, v0=first.v, w0=first.w)
        if args.kind == "points":
            pot.time_pass(d["r"], d["c"], d["s"], eps, reps=20, x=d["x"], y=d["y"], cost_scale=d["cost_scale"],
                          cmax=1.0, **kw)
        else:
            pot.time_pass(d["r"], d["c"], d["s"], eps, reps=20, C=d["C"], kind=d["kind"], ldc=d["ldc"], cmax=1.0, **kw)
        torch.cuda.synchronize()
        log("pmc probe done")
        return
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
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic() if args.kind == "f32" and n == 4096 else None}
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
        # the solver variants against the canonical readings (same instance)
        if args.kind == "f32" and algo == pot.ASPOT:
            for name, kw in [("aspot_step_rule1", dict(step_rule=1)), ("aspot_block_rule1", dict(block_rule=1))]:
                probe = run_solve(pot, d, eps, pot.ASPOT, "f32", raise_on_error=False, want_factors=False, **kw)
                if probe.status != pot.OK:
                    # e.g. the proof-form step, whose first move from the cold start can take
                    # every term of B(z) below the FP64 range of the sums
                    extra[name] = {"status": pot.status_string(probe.status), "iters": probe.result["iters"]}
                else:
                    o2, w2, ev2 = time_solves(pot, d, eps, pot.ASPOT, "f32", 3, 1, None, **kw)
                    rr = o2[-1].result
                    extra[name] = {"solves_per_s": 3 / (ev2 / 1e3), "iters": rr["iters"], "cost": rr["cost"],
                                   "cost_minus_canonical": rr["cost"] - outs[-1].result["cost"]}
                log(f"{name}: {extra[name]}")
        log("shard: rows 0..2499 of the 20000^2 instance (one GPU of 8)")
        extra["c3_shard_2500x20000"] = bench_shard(pot, I, dev, eps)
        log(f"shard: {extra['c3_shard_2500x20000']}")
        torch.cuda.empty_cache()
        # the tuned rule of Algorithm 3 (Theorem 2) on the same instance; its
        # cost is compared with the ASPOT cost (within eps of the optimum)
        if args.kind == "f32":
            for p in (2.0, 3.0):
                name = f"sinkhorn_tuned_p{int(p)}"
                o2, w2, ev2 = time_solves(pot, d, eps, pot.SINKHORN, "f32", 3, 1, None, gamma_rule=1, p=p)
                rr = o2[-1].result
                extra[name] = {"solves_per_s": 3 / (ev2 / 1e3), "iters": rr["iters"], "cost": rr["cost"],
                               "gamma": rr["gamma"], "tol": rr["tol"],
                               "cost_minus_aspot": rr["cost"] - outs[-1].result["cost"] if algo == pot.ASPOT else None}
                log(f"{name}: {extra[name]}")

    if not args.no_batched:
        log("batched: 512 uneven instances")
        extra["batched_uneven_512"] = bench_batched(pot, I, dev, eps, 3, args.plain_sample)
        log(f"batched: {extra['batched_uneven_512']}")
        from paper_2601_17196_amd import warmstart as W
        if os.path.exists(W.WEIGHTS):
            log("warm start: 1024 instances n = m = 256")
            extra["warm_batched_1024x256"] = bench_warm(pot, I, dev, eps, 2, args.plain_sample)
            log(f"warm start: {extra['warm_batched_1024x256']}")

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
