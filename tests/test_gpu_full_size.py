"""The full-size single instance (n = m = 20000, 2-D shifted mixtures,
s = 0.7, eps = 1e-2 and 5e-3) through pot_solve, FP32 and BF16 costs, in the
launch configuration the benchmark times, judged through the FP64 oracle:

  * E of Section 3.1 recomputed by the oracle at the GPU's output point (on
    the cost values the GPU saw) equals the GPU's E and is within the
    threshold, to the bound of tests/gpu_common.e_bar;
  * the oracle's FP64 rounding of the GPU's X~ = exp(f + g - C / gamma)
    reproduces the GPU's factors alpha, beta (1e-9) and cost (1e-9);
  * the GPU's factored plan, evaluated entry by entry by the oracle, is in
    U(r, c, s), and its cost on the exact FP64 cost (from the points) is
    within eps of the optimum: a weak-duality lower bound built from the
    GPU's duals (tests/lp_pot.dual_lower_bound) certifies cost - OPT <= eps
    with no LP solve at this size.  For the BF16 cost the plan is priced on
    the exact cost, so the bound covers the BF16 rounding of C as well."""
import numpy as np
import pytest

from oracle import potref as O
from paper_2601_17196_amd import instances as I
from tests.gpu_common import check_dual_certificate, e_bar, rel

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _device_cost(inst, dtype):
    """C = cost_scale |x_i - y_j|^2 in FP64 on the device (the generator's
    formula, coordinate by coordinate), stored as FP32 or BF16 bits."""
    import torch
    x = torch.from_numpy(inst.x.astype(np.float64)).cuda()
    y = torch.from_numpy(inst.y.astype(np.float64)).cuda()
    C = torch.empty((inst.n, inst.m), dtype=torch.float32 if dtype == "f32" else torch.bfloat16, device="cuda")
    for i0 in range(0, inst.n, 2048):
        xb = x[i0:i0 + 2048]
        D = torch.zeros((xb.shape[0], inst.m), dtype=torch.float64, device="cuda")
        for k in range(x.shape[1]):
            diff = xb[:, k:k + 1] - y[None, :, k]
            D += diff * diff
        C[i0:i0 + 2048] = (D * inst.cost_scale).to(C.dtype)
    return C if dtype == "f32" else C.view(torch.int16)


def _exact_cost(inst):
    """The exact FP64 cost from the points (the generator's formula)."""
    X = inst.x.astype(np.float64)
    Y = inst.y.astype(np.float64)
    C = np.empty((inst.n, inst.m))
    for i0 in range(0, inst.n, 2048):
        D = np.zeros((min(inst.n, i0 + 2048) - i0, inst.m))
        for k in range(X.shape[1]):
            diff = X[i0:i0 + 2048, k:k + 1] - Y[None, :, k]
            D += diff * diff
        C[i0:i0 + 2048] = D * inst.cost_scale
    return C


@pytest.mark.parametrize("kind", ["f32", "bf16"])
@pytest.mark.parametrize("eps", [1e-2, 5e-3])
def test_full_size_instance(eps, kind):
    import torch

    from paper_2601_17196_amd import pot
    inst = I.c3(0, eps=eps, dense=False)
    print(f"full size: n = m = {inst.n}, eps = {eps}, {kind}", flush=True)
    r = torch.from_numpy(inst.r).cuda()
    c = torch.from_numpy(inst.c).cuda()
    Cd = _device_cost(inst, kind)
    if kind == "f32":
        out = pot.solve(r, c, inst.s, inst.eps, C=Cd, cmax=0.0)
    else:
        out = pot.solve(r, c, inst.s, inst.eps, C=Cd, kind=pot.COST_BF16, ldc=inst.m, cmax=0.0)
    torch.cuda.synchronize()
    res = out.result
    print(f"{kind}: status {out.status} iters {res['iters']} cost {res['cost']:.9e} E {res['E']:.3e}", flush=True)
    assert out.status == 0 and res["E"] <= res["tol"]
    assert abs(res["mass"] - inst.s) <= 1e-11
    # the cost values the GPU saw, in FP64
    Cp = Cd.cpu().numpy()
    Cp = Cp.astype(np.float64) if kind == "f32" else I.bf16_bits_to_f64(Cp.view(np.uint16))
    del Cd
    torch.cuda.empty_cache()
    Ce = _exact_cost(inst)
    if kind == "f32":
        # the device cost is the generator's FP64 arithmetic rounded to FP32
        assert np.array_equal(Cp, Ce.astype(np.float32).astype(np.float64))
    cmax = float(Cp.max())
    assert res["cmax"] == cmax
    gam, tol, M, rt, ct_ = O.setup(inst.r, inst.c, inst.s, inst.eps, cmax=cmax)
    assert rel(res["gamma"], gam) <= 1e-15 and rel(res["tol"], tol) <= 1e-15
    u, v, w = out.u.cpu().numpy(), out.v.cpu().numpy(), res["w"]
    E = O.error(Cp, gam, rt, ct_, inst.s, u, v, w)
    amax = 1.4426950408889634 * (np.max(np.abs(u + w)) + np.max(np.abs(v)))
    bar = e_bar(kind, inst.s, gamma=gam, cmax=cmax, amax=amax)
    print(f"E gpu {res['E']:.9e} oracle {E:.9e} (bar {bar:.2e})", flush=True)
    assert abs(res["E"] - E) <= bar
    assert E <= tol + bar
    f, g = out.f.cpu().numpy(), out.g.cpu().numpy()
    rd = O.round_plan(Cp, gam, f, g, inst.r, inst.c, inst.s)
    al, be = out.alpha.cpu().numpy(), out.beta.cpu().numpy()
    assert np.max(np.abs(al - rd["alpha"])) <= 1e-9
    assert np.max(np.abs(be - rd["beta"])) <= 1e-9
    assert rel(res["cost"], rd["cost"]) <= 1e-9
    pe = O.plan_eval(Cp, gam, f, g, al, be, res["kappa"], res["lambda_"], out.pp.cpu().numpy(),
                     out.qq.cpu().numpy(), Ce=Ce)
    assert pe["min"] >= 0.0
    assert np.all(pe["rows"] <= inst.r * (1 + 1e-12)) and np.all(pe["cols"] <= inst.c * (1 + 1e-12))
    assert abs(pe["mass"] - inst.s) <= 1e-11 * inst.s
    assert res["viol_row"] <= 1e-12 and res["viol_col"] <= 1e-12 and res["viol_mass"] <= 1e-11
    lb, gap = check_dual_certificate(Ce, inst, "aspot", res, v, pe["cost"])
    print(f"exact cost {pe['cost']:.9e}, dual lower bound {lb:.9e}, gap {gap:.3e} <= eps {inst.eps}", flush=True)
