"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars (FP32 path and points path): with the oracle's decisions replayed, the
rounded plan's cost within 1e-6 relative of the oracle run on the same cost
values, phi within 1e-8 of max |phi| and E within 5e-8 of the mass scale at every
iteration; running free, the same bars whenever every decision agrees, else
(a near tie of two scores decided the other way on FP32 sums) both plans are
eps-approximations.  The plan is always exactly feasible.  BF16 path: within
eps of the FP64 oracle on the exact cost.
"""
import numpy as np
import pytest

from oracle import potref as O
from paper_2601_17196_amd import instances as I
from tests.gpu_common import feasible, gpu_solve, oracle_cost_matrix, rel

pytestmark = pytest.mark.gpu

COST_RTOL = 1e-6


def _cases():
    return {
        "c1": lambda: I.c1(0),
        "u300x257": lambda: I.uniform_pair(300, 257, 2, 5, mass_r=1.0, mass_c=1.3, s_frac=0.7),
        "u70x1000": lambda: I.uniform_pair(70, 1000, 3, 6, mass_r=0.9, mass_c=1.1, s_frac=0.6),
        "u513x130dir05": lambda: I.uniform_pair(513, 130, 2, 7, mass_r=1.2, mass_c=0.8, s_frac=0.9,
                                                dirichlet=0.5),
        "balanced64": lambda: I.uniform_pair(64, 64, 2, 8, mass_r=1.0, mass_c=1.0, s_frac=1.0),
    }


CASES = _cases()


def _oracle(inst, kind, algo, **kw):
    C = oracle_cost_matrix(inst, kind)
    return O.solve(C, inst.r, inst.c, inst.s, inst.eps, algo=algo, cmax=1.0, trace=True, dense=True,
                   **kw)


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("algo", ["aspot", "sinkhorn"])
def test_free_running_parity_f32(name, algo):
    """Both sides decide freely.  Where every decision agrees, the results agree
    to 1e-6; a decision taken on a near tie of two FP64 scores may go the other
    way on FP32 sums, and then both runs are valid: each plan must be an
    eps-approximation, and the forced-decision test covers the arithmetic."""
    inst = CASES[name]()
    print(f"case {name} {algo} n={inst.n} m={inst.m}", flush=True)
    ref = _oracle(inst, "f32", algo)
    out = gpu_solve(inst, "f32", algo, trace_cap=ref.iters + 8, want_plan=True)
    res = out.result
    assert out.status == 0
    X = out.plan.cpu().numpy()
    assert feasible(X, inst.r, inst.c, inst.s)
    assert rel(float(np.sum(oracle_cost_matrix(inst, "f32") * X)), res["cost"]) <= 1e-12
    same = res["iters"] == ref.iters
    if algo == "aspot" and same:
        ti = out.trace_i.cpu().numpy().reshape(-1, 3)[:ref.iters]
        dec = np.stack([ref.trace.bhat, ref.trace.pick, ref.trace.bchk], axis=1)
        bad = np.nonzero(np.any(ti != dec, axis=1))[0]
        same = len(bad) == 0
        if not same:
            print(f"decisions differ first at iteration {bad[0]} of {ref.iters}")
    if not same:
        assert res["E"] <= res["tol"]
        assert abs(res["cost"] - ref.rounded["cost"]) <= inst.eps
        return
    assert rel(res["cost"], ref.rounded["cost"]) <= COST_RTOL
    assert rel(res["E"], ref.E) <= 1e-4
    f = out.f.cpu().numpy()
    g = out.g.cpu().numpy()
    # Sinkhorn on the extended instance is invariant under (f + k, g - k) with
    # the dummy duals moved the other way: only f - k and g + k are defined,
    # and rounding moves the iterates along k.  ASPOT's w term fixes k.
    k = float(np.mean(f - ref.f)) if algo == "sinkhorn" else 0.0
    assert np.max(np.abs(f - k - ref.f)) <= 1e-6 * max(1.0, np.max(np.abs(ref.f)))
    assert np.max(np.abs(g + k - ref.g)) <= 1e-6 * max(1.0, np.max(np.abs(ref.g)))
    Xo = ref.rounded["X"]
    assert np.max(np.abs(X - Xo)) <= 1e-6 * np.max(Xo)


@pytest.mark.parametrize("name", sorted(CASES))
def test_forced_decision_trajectory(name):
    """Replay the oracle's decisions; the per-iteration E and phi agree."""
    import torch
    inst = CASES[name]()
    ref = _oracle(inst, "f32", "aspot")
    tr = ref.trace
    force = np.stack([tr.bhat, tr.pick, tr.bchk], axis=1).astype(np.int32).ravel()
    ft = torch.from_numpy(force).cuda()
    out = gpu_solve(inst, "f32", "aspot", trace_cap=ref.iters + 4, force=ft)
    assert out.status == 0 and out.result["iters"] == ref.iters
    td = out.trace_d.cpu().numpy().reshape(-1, 4)[:ref.iters]
    # E sums |R_i + e^{u_i} - r~_i|, differences of nearly equal numbers: its
    # error is bounded on the scale of the masses, not relative to E itself
    mass_scale = inst.r.sum() + inst.c.sum() + inst.s
    assert np.max(np.abs(td[:, 0] - tr.E)) <= 5e-8 * mass_scale
    # phi may cross 0 along the trajectory: compare on the scale of max |phi|
    phi_scale = max(1.0, float(np.max(np.abs(tr.phichk))))
    assert np.max(np.abs(td[:, 1] - tr.phichk)) <= 1e-8 * phi_scale
    assert np.max(np.abs(td[:, 2] - tr.phihat)) <= 1e-8 * phi_scale
    assert np.max(np.abs(td[:, 3] - tr.theta)) <= 1e-15
    assert rel(out.result["cost"], ref.rounded["cost"]) <= COST_RTOL


@pytest.mark.parametrize("algo", ["aspot", "sinkhorn"])
@pytest.mark.parametrize("name,d", [("pts2", 2), ("pts3", 3)])
def test_points_path_parity(algo, name, d):
    inst = I.uniform_pair(333, 271, d, 11 + d, mass_r=1.0, mass_c=1.2, s_frac=0.75)
    ref = _oracle(inst, "points", algo)
    out = gpu_solve(inst, "points", algo, trace_cap=ref.iters + 8, want_plan=True)
    assert out.status == 0
    assert out.result["iters"] == ref.iters
    assert rel(out.result["cost"], ref.rounded["cost"]) <= COST_RTOL
    assert feasible(out.plan.cpu().numpy(), inst.r, inst.c, inst.s)


def test_points_path_computed_scale():
    """cost_scale <= 0: the library computes 1 / max |x - y|^2 on the device."""
    import torch

    from paper_2601_17196_amd import pot
    inst = I.uniform_pair(200, 150, 3, 21)
    d = pot.to_device_instance(inst, "cuda:0", kind="points")
    out = pot.solve(d["r"], d["c"], d["s"], inst.eps, x=d["x"], y=d["y"], cost_scale=0.0, cmax=0.0)
    torch.cuda.synchronize()
    assert rel(out.result["cost_scale"], inst.cost_scale) <= 1e-15
    ref = _oracle(inst, "points", "aspot")
    assert rel(out.result["cost"], ref.rounded["cost"]) <= COST_RTOL


@pytest.mark.parametrize("algo", ["aspot", "sinkhorn"])
def test_bf16_path_within_eps(algo):
    inst = I.uniform_pair(400, 384, 2, 31, mass_r=1.0, mass_c=1.1, s_frac=0.8)
    out = gpu_solve(inst, "bf16", algo, want_plan=True)
    assert out.status == 0
    X = out.plan.cpu().numpy()
    assert feasible(X, inst.r, inst.c, inst.s)
    # against the FP64 oracle on the exact cost: within eps (Definition 1 budget)
    ref = _oracle(inst, "points", algo)
    true_cost = float(np.sum(inst.C64 * X))
    assert abs(true_cost - ref.rounded["cost"]) <= inst.eps
    # against the oracle on the same BF16 values: the FP32 exponent costs ~1e-4
    refb = _oracle(inst, "bf16", algo)
    assert abs(out.result["cost"] - refb.rounded["cost"]) <= 1e-3 * inst.eps


@pytest.mark.parametrize("tile_rows", [16, 64, 128, 256])
def test_tile_shapes_agree(tile_rows):
    inst = CASES["u300x257"]()
    ref = _oracle(inst, "f32", "aspot")
    out = gpu_solve(inst, "f32", "aspot", tile_rows=tile_rows)
    assert out.result["iters"] == ref.iters
    assert rel(out.result["cost"], ref.rounded["cost"]) <= COST_RTOL


def test_strided_and_unaligned_ldc():
    """A padded leading dimension (vector loads) and an odd one (scalar loads)."""
    import torch

    from paper_2601_17196_amd import pot
    inst = CASES["u300x257"]()
    ref = _oracle(inst, "f32", "aspot")
    out = gpu_solve(inst, "f32", "aspot", pad_ldc=True)
    assert rel(out.result["cost"], ref.rounded["cost"]) <= COST_RTOL
    n, m = inst.C32.shape
    buf = np.zeros((n, m + 3), dtype=np.float32)
    buf[:, :m] = inst.C32
    t = torch.from_numpy(buf).cuda()
    d = pot.to_device_instance(inst, "cuda:0", kind="f32")
    o2 = pot.solve(d["r"], d["c"], d["s"], inst.eps, C=t, ldc=m + 3, cmax=1.0)
    torch.cuda.synchronize()
    assert rel(o2.result["cost"], ref.rounded["cost"]) <= COST_RTOL


def test_deterministic_bitwise():
    inst = CASES["u513x130dir05"]()
    a = gpu_solve(inst, "f32", "aspot")
    b = gpu_solve(inst, "f32", "aspot")
    assert a.result["cost"] == b.result["cost"]
    assert np.array_equal(a.f.cpu().numpy(), b.f.cpu().numpy())
    assert np.array_equal(a.g.cpu().numpy(), b.g.cpu().numpy())


def test_computed_cmax_matches_given():
    inst = CASES["u300x257"]()
    a = gpu_solve(inst, "f32", "aspot", cmax=0.0)
    b = gpu_solve(inst, "f32", "aspot", cmax=float(inst.C32.max()))
    assert a.result["cmax"] == float(inst.C32.max())
    assert a.result["cost"] == b.result["cost"]


@pytest.mark.parametrize("name", ["u300x257", "u513x130dir05", "c1"])
@pytest.mark.parametrize("variant", [dict(step_rule=1), dict(block_rule=1)])
def test_solver_variants_parity(name, variant):
    """The proof-form step (step_rule = 1) and the cyclic block rule
    (block_rule = 1) against the oracle run with the same option: the same
    bars as the canonical rules, and with the cyclic rule the GPU's recorded
    blocks follow the cycle exactly."""
    inst = CASES[name]()
    print(f"variant {variant} case {name}", flush=True)
    ref = _oracle(inst, "f32", "aspot", **variant)
    out = gpu_solve(inst, "f32", "aspot", trace_cap=ref.iters + 8, want_plan=True, **variant)
    res = out.result
    assert out.status == 0 and res["E"] <= res["tol"]
    assert feasible(out.plan.cpu().numpy(), inst.r, inst.c, inst.s)
    ti = out.trace_i.cpu().numpy().reshape(-1, 3)[:res["iters"]]
    if variant.get("block_rule") == 1:
        t = np.arange(res["iters"])
        assert np.array_equal(ti[:, 0], (2 * t) % 3)
        assert np.array_equal(ti[:-1, 2], (2 * t[:-1] + 1) % 3)
    if res["iters"] == ref.iters:
        assert rel(res["cost"], ref.rounded["cost"]) <= COST_RTOL
    else:
        assert abs(res["cost"] - ref.rounded["cost"]) <= inst.eps
