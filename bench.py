"""Benchmark: POT solves/s at eps = 1e-2 on one MI355X, warm-started and
batched ASPOT against cold batched and plain ASPOT.

A step is one batch of 1024 POT instances (n = m = 256, 2-D Gaussian
mixtures with 2-5 components, Dirichlet(0.5) masses with totals in
[0.8, 1.2], s uniform in [0.5, 0.9] x the smaller mass, squared-Euclidean
cost normalised to max 1, stored dense in FP32, eps = 1e-2): the warm-start
network's inference kernels predict every instance's duals, then one
persistent launch of pot_solve_batched runs, for all 1024 instances, the
setup of Algorithm 2, the warm-start check (the prediction is kept only if
it lowers phi), the ASPOT loop and the FP64 rounding onto U(r, c, s).  value =
1024 x steps / elapsed time of the timed steps (HIP events), inputs resident
in HBM.  Beside it, in `extra`: the same batch cold (batched), plain cold
pot_solve calls one after another (a sample), the 512-instance uneven batch,
the single 4096^2 instance (streamed FP32 / BF16 cost, recomputed points
cost), the 20000^2 instance's HBM roofline (FP32 and BF16) and the other
solver options.

Rooflines.  The headline's dominant kernel is the persistent batched kernel:
its work is n m exponentials per statistics pass (three passes per ASPOT
iteration), bound by the vector ALU (each 256-column C5 row costs about 13.75
VALU instructions per element, the exponential at a quarter rate, which
gives the peak BATCHED_PEAK_GELEM below at 256 CUs x 64 lanes x 2.4 GHz).
The single-instance tile kernel streams C and is bound by HBM (8 TB/s).
Kernel times come from HIP events recorded around each launch on the stream
it runs on (medians of >= 10 launches after 3 warm-ups); the committed
rocprofv3 summaries under profiles/ give the same kernels' durations.

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
# Vector-ALU ceilings in G elements/s: 256 CUs x 64 lanes x 2.4 GHz =
# 3.93e13 lane-instructions/s, divided by the issue cost of one element of the
# statistics pass in the compiled inner loops (the exponential counts 4: it
# issues at a quarter rate).  Batched 256-column rows: 13.75 VALU incl. the
# exponential (440 per 32-element step of the compiled sweep) -> 16.75; tile
# kernel, points cost (d = 3): 12.44 -> 15.44.
ALU_LANE_OPS = 256 * 64 * 2.4e9
BATCHED_PEAK_GELEM = ALU_LANE_OPS / 16.75 / 1e9
POINTS_PEAK_GELEM = ALU_LANE_OPS / 15.44 / 1e9
COPY_BYTES = 256 << 20          # the plain copy of the counter-scale probe (bytes read, and written)
PROFILES = os.path.join(ROOT, "profiles")


def measured_traffic(name):
    """HBM bytes per launch of a kernel from a committed counter summary, or
    None when it is missing or was taken on other kernel sources."""
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None
    from paper_2601_17196_amd import profile_summary as PS
    s = json.load(open(path))
    if s.get("kernel_source_hash") != PS.kernel_source_hash(s.get("kernel_sources")):
        return None
    return s.get("traffic_bytes")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _build_if_missing():
    from paper_2601_17196_amd import pot
    if not os.path.exists(pot.lib_path()):
        import __graft_entry__
        __graft_entry__.build()


def _median(xs):
    xs = sorted(xs)
    k = len(xs)
    return xs[k // 2] if k % 2 else 0.5 * (xs[k // 2 - 1] + xs[k // 2])


def _event_ms(fn):
    """(ms of fn's GPU work on the current stream, fn's return value)."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    out = fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), out


def _batch_probs(pot, insts, dev):
    probs = []
    for inst in insts:
        d = pot.to_device_instance(inst, dev, kind="f32", pad_ldc=True)
        probs.append(dict(r=d["r"], c=d["c"], s=d["s"], C=d["C"], kind=d["kind"], ldc=d["ldc"], cmax=1.0))
    return probs


def _work_elems(insts, res):
    """Statistics-pass elements of a batched ASPOT run: three passes over
    n x m per iteration."""
    return sum(3 * r["iters"] * i.n * i.m for i, r in zip(insts, res))


def headline(pot, I, dev, eps, steps, warmup, plain_sample, cold_reps):
    """C5: warm-started batched ASPOT (the metric), cold batched, plain."""
    import numpy as np
    import torch
    insts = I.c5_batch(1024)
    probs = _batch_probs(pot, insts, dev)
    pts = [dict(x=torch.from_numpy(np.ascontiguousarray(i.x, dtype=np.float32)).to(dev),
                y=torch.from_numpy(np.ascontiguousarray(i.y, dtype=np.float32)).to(dev),
                r=p["r"], c=p["c"], cost_scale=i.cost_scale) for i, p in zip(insts, probs)]
    ws = torch.empty(pot.workspace_bytes_batched(probs) + 512, dtype=torch.uint8, device=dev)
    wws = torch.empty(pot.load().pot_warm_workspace_bytes(len(pts)) + 512, dtype=torch.uint8, device=dev)
    blob = pot.warm_blob(device=dev)
    t_inf, t_bat, last = [], [], {}

    def step():
        # inference, then the batched solve, each bracketed by events on the stream it runs on
        ti, preds = _event_ms(lambda: pot.warm_predict(pts, eps, blob, workspace=wws))
        tb, out = _event_ms(lambda: pot.solve_batched(
            probs, eps, u0=[p[0] for p in preds], v0=[p[1] for p in preds], w0=[0.0] * len(preds),
            warm_check=True, workspace=ws, want_duals=False))
        t_inf.append(ti)
        t_bat.append(tb)
        last["res"] = out[1]
        last["st"] = out[0]

    for _ in range(warmup):
        step()
    t_inf.clear()
    t_bat.clear()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    resw = last["res"]
    log(f"warm+batched: {steps} steps in {ms:.1f} ms (wall {wall * 1e3:.1f}); batched launch median "
        f"{_median(t_bat):.1f} ms, inference median {_median(t_inf):.2f} ms")
    # cold batched (the same launch without warm starts) and plain sequential solves
    tc = []
    for k in range(cold_reps + 1):
        t, out = _event_ms(lambda: pot.solve_batched(probs, eps, workspace=ws, want_duals=False))
        if k > 0:
            tc.append(t)
    resc = out[1]
    sample = list(range(0, len(insts), max(1, len(insts) // max(plain_sample, 1))))[:plain_sample]
    tp = None
    if sample:
        pot.solve(probs[0]["r"], probs[0]["c"], probs[0]["s"], eps, C=probs[0]["C"], cmax=1.0, want_factors=False)

        def plain():
            for j in sample:
                pot.solve(probs[j]["r"], probs[j]["c"], probs[j]["s"], eps, C=probs[j]["C"], cmax=1.0,
                          want_factors=False)
        tp, _ = _event_ms(plain)
    itw = np.array([r["iters"] for r in resw])
    itc = np.array([r["iters"] for r in resc])
    elems = _work_elems(insts, resw)
    med_b = _median(t_bat)
    achieved = elems / (med_b * 1e-3) / 1e9
    roof = {"bound": "alu", "achieved": round(achieved, 1), "peak": round(BATCHED_PEAK_GELEM, 1),
            "unit": "Gelem/s", "frac": round(achieved / BATCHED_PEAK_GELEM, 4),
            "traffic": measured_traffic("batched_c5_1024x256_traffic.json")}
    info = {
        "instances": len(insts),
        "warm_batched_solves_per_s": len(insts) * steps / (ms / 1e3),
        "cold_batched_solves_per_s": len(insts) / (_median(tc) / 1e3),
        "plain_solves_per_s": len(sample) / (tp / 1e3) if tp else None, "plain_sample": len(sample),
        "batched_launch_ms_median": med_b, "inference_ms_median": _median(t_inf),
        "cold_batched_launch_ms_median": _median(tc),
        "warm_kept": int(sum(r["used_warm"] for r in resw)),
        "iters_median_warm": float(np.median(itw)), "iters_median_cold": float(np.median(itc)),
        "iters_max_warm": int(itw.max()), "iters_max_cold": int(itc.max()),
        "iters_total_warm": int(itw.sum()), "iters_total_cold": int(itc.sum()),
        "statistics_elements_per_launch": elems,
        "all_ok": last["st"] == 0 and all(r["status"] == 0 for r in resw) and all(r["status"] == 0 for r in resc),
        "max_E_over_tol": float(max(r["E"] / r["tol"] for r in resw)),
    }
    del ws, probs, pts
    torch.cuda.empty_cache()
    return ms / steps, info, roof, insts, itc


def cpu_baseline(insts, iters_cold, eps, per_inst_iters=150, sample=6):
    """The FP64 oracle (as it stands) on the host cores, on a bounded sample
    of the headline workload: `per_inst_iters` ASPOT iterations on each of
    `sample` instances of the batch (all n = m = 256), whose per-iteration
    time, times the batch's total cold iteration count, gives the oracle's
    solves/s for the batch."""
    import numpy as np

    from oracle import potref
    cores = potref.threads()
    tot_t, tot_it = 0.0, 0
    for inst in insts[:sample]:
        C = inst.C32.astype(np.float64)
        gam, tol, M, rt, ct_ = potref.setup(inst.r, inst.c, inst.s, eps, cmax=1.0)
        t0 = time.perf_counter()
        _, _, _, it, _, _, _ = potref.aspot(C, gam, tol, rt, ct_, inst.s, M, max_iter=per_inst_iters)
        tot_t += time.perf_counter() - t0
        tot_it += it
    per_iter = tot_t / tot_it
    total = float(np.sum(iters_cold))
    return {"value": len(insts) / (per_iter * total), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": (f"{tot_it} ASPOT iterations over the first {sample} instances of the batch (n = m = 256, "
                       f"{tot_t:.1f} s, {per_iter * 1e3:.2f} ms/iteration), scaled by the batch's "
                       f"{int(total)} cold iterations")}


def tile_roofline(pot, d, eps, u0, v0, w0, nbytes, reps, kind="f32", traffic=None, points=False, elems=None):
    """Median tile-kernel time (HIP events around each launch, 3 warm-ups)
    of the statistics pass at the given duals, and its roofline."""
    kw = dict(u0=u0, v0=v0, w0=w0)
    if points:
        ms, fin = pot.time_pass(d["r"], d["c"], d["s"], eps, reps=reps, x=d["x"], y=d["y"],
                                cost_scale=d["cost_scale"], cmax=1.0, **kw)
        ach = elems / (ms * 1e-3) / 1e9
        return ms, fin, {"bound": "alu", "achieved": round(ach, 1), "peak": round(POINTS_PEAK_GELEM, 1),
                         "unit": "Gelem/s", "frac": round(ach / POINTS_PEAK_GELEM, 4), "traffic": None}
    ms, fin = pot.time_pass(d["r"], d["c"], d["s"], eps, reps=reps, C=d["C"], kind=d["kind"], ldc=d["ldc"],
                            cmax=d.get("cmax_given", 1.0), **kw)
    ach = nbytes / (ms * 1e-3) / 1e9
    return ms, fin, {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic}


def time_solves(pot, fn, steps, warmup=1):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ms, outs = _event_ms(lambda: [fn() for _ in range(steps)])
    return steps / (ms / 1e3), outs[-1]


def bench_c2(pot, I, dev, eps, reps):
    """The single 4096^2 instance (3-D clusters + outliers, s = 0.9): plain
    cold solves with the streamed FP32 / BF16 cost and the recomputed points
    cost, the solver options, and the tile kernel's roofline."""
    import torch
    inst = I.c2(0, n=4096)
    out = {}
    for kind in ("f32", "bf16", "points"):
        d = pot.to_device_instance(inst, dev, kind=kind)
        if kind == "points":
            fn = lambda: pot.solve(d["r"], d["c"], d["s"], eps, x=d["x"], y=d["y"], cost_scale=d["cost_scale"],
                                   cmax=1.0, want_factors=False)
        else:
            fn = lambda: pot.solve(d["r"], d["c"], d["s"], eps, C=d["C"], kind=d["kind"], ldc=d["ldc"], cmax=1.0,
                                   want_factors=False)
        sps, o = time_solves(pot, fn, 10 if kind == "f32" else 3)
        nb = inst.n * inst.m * {"f32": 4, "bf16": 2, "points": 0}[kind]
        ms, fin, roof = tile_roofline(pot, d, eps, o.u, o.v, o.w, nb, reps, kind=kind, points=kind == "points",
                                      elems=inst.n * inst.m,
                                      traffic=measured_traffic("stats_pass_c2_4096_f32_traffic.json")
                                      if kind == "f32" else None)
        out[f"aspot_{kind}"] = {"solves_per_s": sps, "iters": o.result["iters"], "cost": o.result["cost"],
                                "us_per_iteration": 1e6 / sps / max(o.result["iters"], 1),
                                "tile_kernel_us": ms * 1e3, "fin_kernel_us": fin * 1e3, "roofline": roof}
        log(f"c2 {kind}: {out[f'aspot_{kind}']}")
        if kind == "f32":
            f32 = d
            base_cost = o.result["cost"]
        else:
            del d
    d = f32
    sps, o = time_solves(pot, lambda: pot.solve(d["r"], d["c"], d["s"], eps, C=d["C"], cmax=1.0, algo=pot.SINKHORN,
                                               want_factors=False), 5)
    out["sinkhorn_f32"] = {"solves_per_s": sps, "iters": o.result["iters"], "cost": o.result["cost"]}
    sps, o = time_solves(pot, lambda: pot.solve(d["r"], d["c"], d["s"], eps, C=d["C"], cmax=1.0, algo=pot.SINKHORN,
                                               gamma_rule=1, p=2.0, want_factors=False), 5)
    out["sinkhorn_tuned_p2"] = {"solves_per_s": sps, "iters": o.result["iters"], "cost": o.result["cost"],
                                "gamma": o.result["gamma"], "cost_minus_aspot": o.result["cost"] - base_cost}
    for name, kw in (("aspot_step_rule1", dict(step_rule=1)), ("aspot_block_rule1", dict(block_rule=1))):
        sps, o = time_solves(pot, lambda: pot.solve(d["r"], d["c"], d["s"], eps, C=d["C"], cmax=1.0,
                                                   want_factors=False, **kw), 2)
        out[name] = {"solves_per_s": sps, "iters": o.result["iters"], "cost_minus_canonical": o.result["cost"] - base_cost}
    log(f"c2 options: { {k: out[k] for k in ('sinkhorn_f32', 'sinkhorn_tuned_p2', 'aspot_step_rule1', 'aspot_block_rule1')} }")
    del d, f32
    torch.cuda.empty_cache()
    return out


def _device_cost(inst, dtype, dev):
    import numpy as np
    import torch
    x = torch.from_numpy(inst.x.astype(np.float64)).to(dev)
    y = torch.from_numpy(inst.y.astype(np.float64)).to(dev)
    C = torch.empty((inst.n, inst.m), dtype=torch.float32 if dtype == "f32" else torch.bfloat16, device=dev)
    for i0 in range(0, inst.n, 2048):
        xb = x[i0:i0 + 2048]
        D = torch.zeros((xb.shape[0], inst.m), dtype=torch.float64, device=dev)
        for k in range(x.shape[1]):
            diff = xb[:, k:k + 1] - y[None, :, k]
            D += diff * diff
        C[i0:i0 + 2048] = (D * inst.cost_scale).to(C.dtype)
    return C if dtype == "f32" else C.view(torch.int16)


def bench_c3(pot, I, dev, eps, reps):
    """The 20000^2 instance: one solve per cost type for its converged duals,
    then the tile kernel timed there (HBM roofline: n m x bytes per element
    per launch), and the solve time."""
    import torch
    inst = I.c3(0, dense=False)
    r = torch.from_numpy(inst.r).to(dev)
    c = torch.from_numpy(inst.c).to(dev)
    out = {}
    for kind in ("f32", "bf16"):
        C = _device_cost(inst, kind, dev)
        k = pot.COST_F32 if kind == "f32" else pot.COST_BF16
        fn = lambda: pot.solve(r, c, inst.s, eps, C=C, kind=k, ldc=inst.m, cmax=0.0, want_factors=False)
        sps, o = time_solves(pot, fn, 2)
        d = {"r": r, "c": c, "s": inst.s, "C": C, "kind": k, "ldc": inst.m, "cmax_given": o.result["cmax"]}
        nb = inst.n * inst.m * (4 if kind == "f32" else 2)
        ms, fin, roof = tile_roofline(pot, d, eps, o.u, o.v, o.w, nb, reps, kind=kind,
                                      traffic=measured_traffic(f"stats_pass_c3_20000_{kind}_traffic.json"))
        out[kind] = {"solves_per_s": sps, "iters": o.result["iters"], "tile_kernel_us": ms * 1e3,
                     "fin_kernel_us": fin * 1e3, "roofline": roof}
        log(f"c3 {kind}: {out[kind]}")
        del C, d
        torch.cuda.empty_cache()
    return out


def bench_c4(pot, I, dev, eps, reps, plain_sample):
    """The uneven batch (512 instances, n, m log-uniform in [64, 1024])."""
    import numpy as np
    import torch
    insts = I.c4_batch(512)
    probs = _batch_probs(pot, insts, dev)
    ws = torch.empty(pot.workspace_bytes_batched(probs) + 512, dtype=torch.uint8, device=dev)
    ts = []
    for k in range(reps + 1):
        t, (st, res, _) = _event_ms(lambda: pot.solve_batched(probs, eps, workspace=ws, want_duals=False))
        if k > 0:
            ts.append(t)
    its = np.array([r["iters"] for r in res])
    sample = list(range(0, len(insts), len(insts) // plain_sample))[:plain_sample]

    def plain():
        for j in sample:
            pot.solve(probs[j]["r"], probs[j]["c"], probs[j]["s"], eps, C=probs[j]["C"], cmax=1.0, want_factors=False)
    tp, _ = _event_ms(plain)
    t = _median(ts)
    ach = _work_elems(insts, res) / (t * 1e-3) / 1e9
    out = {"instances": len(insts), "solves_per_s": len(insts) / (t / 1e3), "ms_median": t,
           "all_ok": all(r["status"] == 0 for r in res), "iters_median": float(np.median(its)),
           "iters_max": int(its.max()), "plain_solves_per_s": len(sample) / (tp / 1e3), "plain_sample": len(sample),
           "roofline": {"bound": "alu", "achieved": round(ach, 1), "peak": round(BATCHED_PEAK_GELEM, 1),
                        "unit": "Gelem/s", "frac": round(ach / BATCHED_PEAK_GELEM, 4), "traffic": None}}
    del ws, probs
    torch.cuda.empty_cache()
    return out


def bench_shard(pot, I, dev, eps, reps):
    """The statistics pass on one GPU's share of the 20000^2 instance split by
    rows over 8 GPUs: rows 0..2499 against all 20000 columns (FP32), solved as
    an instance of its own (source masses rescaled to total 1, s = 0.7) to get
    representative duals, then the pass timed at them."""
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
    ms = pot.time_pass(r, c, 0.7, eps, reps=reps, C=C, cmax=1.0, u0=o.u, v0=o.v, w0=o.w)[0]
    gbs = ns * m * 4 / (ms * 1e-3) / 1e9
    nx, ny = (m + 255) // 256, (ns + 127) // 128
    return {"n": ns, "m": m, "iters": o.result["iters"], "tile_kernel_us": ms * 1e3, "GB_per_s": gbs,
            "frac_hbm": gbs / HBM_PEAK_GBS, "column_partials_bytes": ny * m * 8,
            "allreduce_bytes_per_pass": (m + 3) * 8}


def bench_register(pot, dev, eps, n=4096):
    """Rigid registration through POT (Section 4): X = n 3-D points in four
    Gaussian blobs, Y = half of them moved by a rigid map; alpha = 0.4,
    gamma0 = 4.4e-3 annealed by 0.83 per registration.  Warm starts from the
    previous registration's duals against cold starts: registrations,
    iterations and time."""
    import numpy as np
    import torch
    g = np.random.default_rng(3)
    centres = np.array([[0.0, 0.0, 0.0], [0.5, 0.2, 0.1], [1.0, 0.5, 0.0], [1.4, 1.0, 0.3]])
    X = (centres[g.integers(0, 4, n)] + 0.08 * g.standard_normal((n, 3))).astype(np.float32)
    idx = g.permutation(n)[: n // 2]
    a = np.array([0.2, 1.0, 0.4]) / np.linalg.norm([0.2, 1.0, 0.4])
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    R0 = np.eye(3) + np.sin(0.5) * K + (1 - np.cos(0.5)) * K @ K
    t0 = np.array([0.3, -0.2, 0.15])
    Y = ((X[idx].astype(np.float64) - t0) @ R0).astype(np.float32)
    x, y = torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev)
    m = len(Y)
    r = torch.full((n,), 1.0 / n, dtype=torch.float64, device=dev)
    c = torch.full((m,), 1.0 / m, dtype=torch.float64, device=dev)
    s = 0.4 * m / n
    out = {"n": n, "m": m, "s": s}
    for warm in (True, False):
        pot.register(x, y, r, c, s, eps=eps, max_steps=2, warm=warm)            # warm-up
        ms, o = _event_ms(lambda: pot.register(x, y, r, c, s, eps=eps, max_steps=60, warm=warm))
        err = float(np.max(np.abs((Y.astype(np.float64) @ o.R.T + o.t) - X[idx])))
        out["warm" if warm else "cold"] = {"registrations": o.steps, "iters_total": o.total_iters,
                                           "iters_per_registration": [int(k) for k in o.iters], "ms": ms,
                                           "solves_per_s": o.steps / (ms / 1e3), "alignment_error": err}
    out["iteration_ratio_warm_over_cold"] = out["warm"]["iters_total"] / max(out["cold"]["iters_total"], 1)
    return out


def bench_tracking(pot, I, dev, eps, count=1024, reps=3):
    """Warm starts from a previous solve on the C5 batch shape: every
    instance's clouds move by a small rigid step (target rotated by 1 degree
    about its centroid and shifted by 0.005, as in one step of tracking or
    registration), and the moved batch is solved batched from the previous
    solution's duals (warm, with the phi check) and from zero (cold)."""
    import numpy as np
    import torch
    insts = I.c5_batch(count)
    probs = _batch_probs(pot, insts, dev)
    ws = torch.empty(pot.workspace_bytes_batched(probs) + 512, dtype=torch.uint8, device=dev)
    st0, res0, duals = pot.solve_batched(probs, eps, workspace=ws, want_uv=True)
    th = np.deg2rad(1.0)
    Rz = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    moved = []
    for i in insts:
        y = i.y.astype(np.float64)
        mu = y.mean(0)
        y2 = ((y - mu) @ Rz.T + mu + 0.005).astype(np.float32)
        x = i.x.astype(np.float64)
        D = ((x[:, None, :] - y2.astype(np.float64)[None, :, :]) ** 2).sum(-1) * i.cost_scale
        moved.append(np.ascontiguousarray(D.astype(np.float32)))
    probs2 = []
    for p, C in zip(probs, moved):
        q = dict(p)
        q["C"] = torch.from_numpy(C).to(dev)
        q["ldc"] = C.shape[1]
        q["cmax"] = 0.0
        probs2.append(q)
    u0 = [d[2] for d in duals]
    v0 = [d[3] for d in duals]
    w0 = [r["w"] for r in res0]
    run_w = lambda: pot.solve_batched(probs2, eps, u0=u0, v0=v0, w0=w0, warm_check=True, workspace=ws,
                                      want_duals=False)
    run_c = lambda: pot.solve_batched(probs2, eps, workspace=ws, want_duals=False)
    out = {}
    for name, fn in (("warm", run_w), ("cold", run_c)):
        fn()
        ts = []
        for _ in range(reps):
            t, (st, res, _) = _event_ms(fn)
            ts.append(t)
        its = np.array([r["iters"] for r in res])
        out[name] = {"solves_per_s": count / (_median(ts) / 1e3), "ms_median": _median(ts),
                     "iters_total": int(its.sum()), "iters_median": float(np.median(its)), "iters_max": int(its.max()),
                     "all_ok": st == 0, "warm_kept": int(sum(r["used_warm"] for r in res))}
    out["speedup_warm_over_cold"] = out["warm"]["solves_per_s"] / out["cold"]["solves_per_s"]
    del ws, probs, probs2
    torch.cuda.empty_cache()
    return out


BF16_MFMA_PEAK_TFLOPS = 2500.0


def bench_shared(pot, dev, eps, n=4096, B=256):
    """Shared-cost batch (pot_solve_shared): B members with their own
    Dirichlet marginals and s on one n x n cost (2-D uniform points), gamma =
    max C / 60; members/s, and the matrix-core product's roofline (2 x rows x
    depth x 2 batch flops per launch against the dense BF16 peak)."""
    import numpy as np
    import torch
    from paper_2601_17196_amd import instances as I
    inst = I.uniform_pair(n, n, 2, 77)
    C = torch.from_numpy(inst.C32).to(dev)
    cmax = float(inst.C32.max())
    gamma = cmax / 60.0
    g = np.random.default_rng(5)
    mem = []
    for _ in range(B):
        r = g.dirichlet(np.ones(n)) * g.uniform(0.8, 1.2)
        c = g.dirichlet(np.ones(n)) * g.uniform(0.8, 1.2)
        mem.append(dict(r=torch.from_numpy(r).to(dev), c=torch.from_numpy(c).to(dev),
                        s=float(g.uniform(0.5, 0.9) * min(r.sum(), c.sum()))))
    ws = torch.empty(pot.workspace_bytes_shared(C, B) + 512, dtype=torch.uint8, device=dev)
    pot.solve_shared(C, mem, eps, gamma, cmax=cmax, workspace=ws, want_duals=False)        # warm-up
    ms, (st, res, _) = _event_ms(lambda: pot.solve_shared(C, mem, eps, gamma, cmax=cmax, workspace=ws,
                                                          want_duals=False))
    its = [r["iters"] for r in res]
    gms, (rows, cols, depth) = pot.time_shared_gemm(C, B, gamma, cmax, reps=20)
    flops = 2.0 * rows * cols * depth
    ach = flops / (gms * 1e-3) / 1e12
    return {"n": n, "members": B, "gamma": gamma, "status": st, "members_per_s": B / (ms / 1e3), "ms": ms,
            "iters_max": int(max(its)), "iters_median": float(np.median(its)), "gemm_us": gms * 1e3,
            "gemm_shape": [rows, cols, depth],
            "roofline": {"bound": "mfma", "achieved": round(ach, 1), "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(ach / BF16_MFMA_PEAK_TFLOPS, 4),
                         "traffic": measured_traffic(f"shared_gemm_{n}x{B}_traffic.json")},
            "gemm_hbm_GB_per_s": (rows * depth * 2 + cols * depth * 2 + cols * rows * 4) / (gms * 1e-3) / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--reps", type=int, default=20, help="timed launches per kernel-time median (after 3 warm-ups)")
    ap.add_argument("--plain-sample", type=int, default=32)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--pmc-probe", choices=["none", "c5", "c3f32", "c3bf16", "c2", "shared"], default="none",
                    help="profiling workload only: a 256 MiB device copy (the counters' scale), then the named "
                         "workload's kernel once or a few times; prints no JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the solver has no multi-GPU path (batches would shard by "
              "instance, one instance by rows of C with one all-reduce of m + 3 values per pass)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    _build_if_missing()
    from paper_2601_17196_amd import instances as I
    from paper_2601_17196_amd import pot

    dev = torch.device("cuda:0")
    eps = 1e-2
    if args.pmc_probe != "none":
        a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        if args.pmc_probe == "c5":
            headline(pot, I, dev, eps, 1, 0, 0, 1)
        elif args.pmc_probe == "shared":
            log(f"shared: {bench_shared(pot, dev, eps)}")
        elif args.pmc_probe == "c2":
            inst = I.c2(0, n=4096)
            d = pot.to_device_instance(inst, dev, kind="f32")
            o = pot.solve(d["r"], d["c"], d["s"], eps, C=d["C"], cmax=1.0)
            pot.time_pass(d["r"], d["c"], d["s"], eps, reps=10, C=d["C"], cmax=1.0, u0=o.u, v0=o.v, w0=o.w)
        else:
            kind = args.pmc_probe[2:]
            inst = I.c3(0, dense=False)
            r = torch.from_numpy(inst.r).to(dev)
            c = torch.from_numpy(inst.c).to(dev)
            C = _device_cost(inst, kind, dev)
            k = pot.COST_F32 if kind == "f32" else pot.COST_BF16
            o = pot.solve(r, c, inst.s, eps, C=C, kind=k, ldc=inst.m, cmax=0.0)
            pot.time_pass(r, c, inst.s, eps, reps=10, C=C, kind=k, ldc=inst.m, cmax=o.result["cmax"], u0=o.u,
                          v0=o.v, w0=o.w)
        torch.cuda.synchronize()
        log("pmc probe done")
        return

    log("headline: 1024 instances n = m = 256, learned warm start + batched ASPOT")
    ms_step, info, roof, insts, itc = headline(pot, I, dev, eps, args.steps, args.warmup, args.plain_sample, 3)
    value = info["instances"] / (ms_step / 1e3)
    log(f"headline: {value:.1f} solves/s; {info}")
    log(f"batched kernel roofline: {roof}")
    extra = {"c5_warm_cold_plain": info}
    if not args.no_extra:
        log("tracking: the C5 batch moved by a small rigid step, warm from the previous solve vs cold")
        extra["c5_tracking_warm_batched"] = bench_tracking(pot, I, dev, eps)
        log(f"tracking: {extra['c5_tracking_warm_batched']}")
        log("c4: 512 uneven instances")
        extra["c4_batched_uneven_512"] = bench_c4(pot, I, dev, eps, 3, args.plain_sample)
        log(f"c4: {extra['c4_batched_uneven_512']}")
        log("c2: single 4096^2 instance")
        extra["c2_single_4096"] = bench_c2(pot, I, dev, eps, args.reps)
        log("c3: 20000^2 instance, HBM roofline")
        extra["c3_single_20000"] = bench_c3(pot, I, dev, eps, args.reps)
        log("registration: 4096 / 2048 points, warm vs cold")
        extra["registration_4096x2048"] = bench_register(pot, dev, eps)
        log(f"registration: {extra['registration_4096x2048']}")
        log("shared cost: 256 members on one 4096^2 cost")
        extra["shared_cost_4096_x256"] = bench_shared(pot, dev, eps)
        log(f"shared: {extra['shared_cost_4096_x256']}")
        log("shard: rows 0..2499 of the 20000^2 instance (one GPU of 8)")
        extra["c3_shard_2500x20000"] = bench_shard(pot, I, dev, eps, args.reps)
        log(f"shard: {extra['c3_shard_2500x20000']}")
    cpu = None
    if not args.no_cpu:
        log("cpu baseline: the oracle on a sample of the batch")
        cpu = cpu_baseline(insts, itc, eps)
        log(f"cpu baseline: {cpu}")

    line = {
        "metric": "POT solves/s at eps=1e-2 (ASPOT, learned warm start + batched)",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 cost, f64 state/exponent, f32 exp, f64 sums",
        "data": "synthetic",
        "config": {"workload": "1024 POT instances n=m=256, 2-D Gaussian mixtures (2-5 components), Dir(0.5) masses "
                               "with totals in [0.8,1.2], s=U[0.5,0.9]*min mass, f32 cost, eps=1e-2; learned warm "
                               "start (BF16 MFMA inference) + one persistent batched ASPOT launch",
                   "instances": 1024, "n": 256, "m": 256, "algo": "aspot", "cost": "f32"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
