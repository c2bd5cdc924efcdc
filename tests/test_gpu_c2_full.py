"""The benchmark's own workload at full size (n = m = 4096, 3-D clustered
points with outliers, FP32 cost, uniform masses 1.0 / 1.0, s = 0.9,
eps = 1e-2, cold ASPOT) in the launch configuration bench.py times (default
tile geometry, graph-replayed loop), checked through the FP64 oracle at the
same size on quantities it computes in one pass:

* E(z) of the GPU's output point recomputed by the oracle equals the GPU's
  E and is within the threshold.  E sums |R_i + e^u_i - r~_i| terms that
  cancel almost exactly near convergence, so the bar is absolute, from the
  arithmetic: each FP32 term carries at most a few units of 2^-24 relative
  error (split exponential, sums of 4 FP32 terms before FP64), so
  |dE| <= 8 2^-24 (T + sum R + sum Q) with every sum about s;
* the oracle's FP64 rounding applied to the GPU's duals gives the same
  rounding factors (alpha, beta to 1e-9) and cost (1e-9 relative);
* the dense FP64 plan written by the GPU is exactly feasible and its
  <C, X> is the reported cost;
* the whole Definition 1 check of tests/gpu_common.py, with the optimum
  bounded by weak duality from the GPU's duals (no LP at this size).
"""
import numpy as np
import pytest

from oracle import potref as O
from paper_2601_17196_amd import instances as I
from tests.gpu_common import check_definition1, feasible, rel

pytestmark = pytest.mark.gpu


def test_c2_full_size_through_the_oracle():
    import torch

    from paper_2601_17196_amd import pot
    inst = I.c2(0, n=4096)
    print(f"c2 full size: n = m = {inst.n}", flush=True)
    d = pot.to_device_instance(inst, "cuda:0", kind="f32")
    out = pot.solve(d["r"], d["c"], d["s"], inst.eps, C=d["C"], kind=d["kind"], ldc=d["ldc"], cmax=1.0,
                    want_plan=True)
    torch.cuda.synchronize()
    res = out.result
    assert out.status == 0 and res["E"] <= res["tol"]
    C = inst.C32.astype(np.float64)
    gam, tol, M, rt, ct_ = O.setup(inst.r, inst.c, inst.s, inst.eps, cmax=1.0)
    assert rel(res["gamma"], gam) <= 1e-15 and rel(res["tol"], tol) <= 1e-15
    u, v, w = out.u.cpu().numpy(), out.v.cpu().numpy(), out.w
    E = O.error(C, gam, rt, ct_, inst.s, u, v, w)
    print(f"E gpu {res['E']:.9e} oracle {E:.9e}", flush=True)
    assert abs(res["E"] - E) <= 8 * 2.0 ** -24 * 3 * inst.s
    assert E <= tol
    f, g = out.f.cpu().numpy(), out.g.cpu().numpy()
    rd = O.round_plan(C, gam, f, g, inst.r, inst.c, inst.s)
    assert np.max(np.abs(out.alpha.cpu().numpy() - rd["alpha"])) <= 1e-9
    assert np.max(np.abs(out.beta.cpu().numpy() - rd["beta"])) <= 1e-9
    assert rel(res["cost"], rd["cost"]) <= 1e-9
    X = out.plan.cpu().numpy()
    assert feasible(X, inst.r, inst.c, inst.s)
    assert rel(float(np.sum(C * X)), res["cost"]) <= 1e-12
    info = check_definition1(inst, "f32", "aspot", out, lp_key=None)
    print(f"c2 Definition 1: {info}", flush=True)
