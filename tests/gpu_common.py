"""Shared helpers of the GPU tests: run the HIP path through the C ABI and the
FP64 oracle on exactly the same inputs."""
import numpy as np

from paper_2601_17196_amd import instances as I


def oracle_cost_matrix(inst, kind):
    """The FP64 cost the oracle must use so that both sides see the same C:
    the stored FP32 values, the stored BF16 values, or the points-defined FP64
    cost."""
    if kind == "f32":
        return inst.C32.astype(np.float64)
    if kind == "bf16":
        return I.bf16_bits_to_f64(I.to_bf16_bits(inst.C32))
    if kind == "points":
        return inst.C64
    raise ValueError(kind)


def gpu_solve(inst, kind="f32", algo="aspot", dev="cuda:0", trace_cap=0, pad_ldc=False,
              want_plan=False, cmax=None, **kw):
    import torch

    from paper_2601_17196_amd import pot
    d = pot.to_device_instance(inst, dev, kind=kind, pad_ldc=pad_ldc)
    a = pot.ASPOT if algo == "aspot" else pot.SINKHORN
    if kind == "points":
        out = pot.solve(d["r"], d["c"], d["s"], inst.eps, x=d["x"], y=d["y"], cost_scale=d["cost_scale"],
                        cmax=1.0 if cmax is None else cmax, algo=a, trace_cap=trace_cap,
                        want_plan=want_plan, raise_on_error=False, **kw)
    else:
        out = pot.solve(d["r"], d["c"], d["s"], inst.eps, C=d["C"], kind=d["kind"], ldc=d["ldc"],
                        cmax=1.0 if cmax is None else cmax, algo=a, trace_cap=trace_cap,
                        want_plan=want_plan, raise_on_error=False, **kw)
    torch.cuda.synchronize()
    return out


def feasible(X, r, c, s, rtol=1e-12):
    X = np.asarray(X)
    tol = rtol * max(1.0, float(np.max(r)), float(np.max(c)))
    return (bool(np.all(X >= 0.0)) and bool(np.all(X.sum(1) <= r + tol))
            and bool(np.all(X.sum(0) <= c + tol)) and abs(float(X.sum()) - s) <= 1e-11 * max(1.0, s))


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)
