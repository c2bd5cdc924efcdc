"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars (FP32 path and points path): with the oracle's decisions replayed, the
duals u, v, w, the log-scalings f, g and the dense rounded plan agree with the
oracle's element by element to 1e-6 (relative to the largest entry), the cost
to 1e-6 relative, phi to 1e-8 of max |phi| and E to 5e-8 of the mass scale at
every iteration.  Running free, every plan passes the Definition 1 check of
tests/gpu_common.py (E recomputed by the oracle at the GPU's output point,
the oracle's rounding of the GPU's duals, exact feasibility of the factored
plan evaluated entry by entry, and 0 <= cost - LP* <= eps against the exact
LP); where every decision also agrees with the oracle's, the results agree
to 1e-6 element by element as above.  BF16 path: the same Definition 1 check
on the exact (points-defined) cost, within eps.
"""
import numpy as np
import pytest

from oracle import potref as O
from paper_2601_17196_amd import instances as I
from tests.gpu_common import check_definition1, feasible, gpu_solve, oracle_cost_matrix, rel, tally

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


def _compare_elementwise(inst, algo, out, ref, X):
    """u, v, w (ASPOT), f, g and the dense plan against the oracle's, 1e-6
    relative to the largest entry.  Feasible Sinkhorn on the extended
    instance is invariant under (f + k, g - k) with the dummy duals moved the
    other way: only f - k and g + k are defined, so its f and g are compared
    modulo k (the plan is gauge-free)."""
    f = out.f.cpu().numpy()
    g = out.g.cpu().numpy()
    k = float(np.mean(f - ref.f)) if algo == "sinkhorn" else 0.0
    assert np.max(np.abs(f - k - ref.f)) <= 1e-6 * max(1.0, np.max(np.abs(ref.f)))
    assert np.max(np.abs(g + k - ref.g)) <= 1e-6 * max(1.0, np.max(np.abs(ref.g)))
    if algo == "aspot":
        u = out.u.cpu().numpy()
        v = out.v.cpu().numpy()
        assert np.max(np.abs(u - ref.u)) <= 1e-6 * max(1.0, np.max(np.abs(ref.u)))
        assert np.max(np.abs(v - ref.v)) <= 1e-6 * max(1.0, np.max(np.abs(ref.v)))
        assert abs(out.result["w"] - ref.w) <= 1e-6 * max(1.0, abs(ref.w))
    Xo = ref.rounded["X"]
    assert np.max(np.abs(X - Xo)) <= 1e-6 * np.max(Xo)


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("algo", ["aspot", "sinkhorn"])
def test_free_running_parity_f32(name, algo):
    """Both sides decide freely.  Every plan passes the Definition 1 check;
    where every decision agrees, the results also agree to 1e-6 element by
    element.  A decision taken on a near tie of two FP64 scores may go the
    other way on FP32 sums; the forced-decision test covers the arithmetic
    of such a case."""
    inst = CASES[name]()
    print(f"case {name} {algo} n={inst.n} m={inst.m}", flush=True)
    ref = _oracle(inst, "f32", algo)
    out = gpu_solve(inst, "f32", algo, trace_cap=ref.iters + 8, want_plan=True)
    res = out.result
    assert out.status == 0
    X = out.plan.cpu().numpy()
    assert feasible(X, inst.r, inst.c, inst.s)
    assert rel(float(np.sum(oracle_cost_matrix(inst, "f32") * X)), res["cost"]) <= 1e-12
    info = check_definition1(inst, "f32", algo, out, lp_key=f"{name}:f32")
    print(f"  Definition 1: {info}", flush=True)
    same = res["iters"] == ref.iters
    if algo == "aspot" and same:
        ti = out.trace_i.cpu().numpy().reshape(-1, 3)[:ref.iters]
        dec = np.stack([ref.trace.bhat, ref.trace.pick, ref.trace.bchk], axis=1)
        bad = np.nonzero(np.any(ti != dec, axis=1))[0]
        same = len(bad) == 0
        if not same:
            print(f"decisions differ first at iteration {bad[0]} of {ref.iters}")
    if not same:
        tally("def1", f"{name}/{algo} ({res['iters']} vs {ref.iters} iterations)")
        return
    tally("strict", f"{name}/{algo}")
    assert rel(res["cost"], ref.rounded["cost"]) <= COST_RTOL
    assert rel(res["E"], ref.E) <= 1e-4
    _compare_elementwise(inst, algo, out, ref, X)


VARIANTS = {"canonical": {}, "step_rule1": dict(step_rule=1), "block_rule1": dict(block_rule=1)}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_forced_decision_trajectory(name, variant):
    """Replay the oracle's decisions (block choice, argmin, stop): the
    per-iteration E and phi agree, and so do the final duals, scalings and
    dense plan, element by element."""
    import torch
    inst = CASES[name]()
    kw = VARIANTS[variant]
    print(f"forced {name} {variant}", flush=True)
    ref = _oracle(inst, "f32", "aspot", **kw)
    tr = ref.trace
    force = np.stack([tr.bhat, tr.pick, tr.bchk], axis=1).astype(np.int32).ravel()
    ft = torch.from_numpy(force).cuda()
    out = gpu_solve(inst, "f32", "aspot", trace_cap=ref.iters + 4, force=ft, want_plan=True, **kw)
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
    _compare_elementwise(inst, "aspot", out, ref, out.plan.cpu().numpy())


@pytest.mark.parametrize("name", sorted(CASES))
def test_sinkhorn_fixed_iterations_elementwise(name):
    """Feasible Sinkhorn has no decision but its stop: with the iteration
    count fixed on both sides (max_iter = the oracle's free-running count, a
    threshold nothing reaches), the scalings and the dense rounded plan agree
    element by element to 1e-6."""
    inst = CASES[name]()
    free = _oracle(inst, "f32", "sinkhorn")
    K = free.iters
    ref = _oracle(inst, "f32", "sinkhorn", tol=1e-300, max_iter=K)
    assert ref.iters == K
    out = gpu_solve(inst, "f32", "sinkhorn", want_plan=True, tol=1e-300, max_iter=K)
    from paper_2601_17196_amd import pot
    assert out.status == pot.ERR_NO_CONVERGENCE and out.result["iters"] == K
    assert rel(out.result["cost"], ref.rounded["cost"]) <= COST_RTOL
    _compare_elementwise(inst, "sinkhorn", out, ref, out.plan.cpu().numpy())


@pytest.mark.parametrize("algo", ["aspot", "sinkhorn"])
@pytest.mark.parametrize("name,d", [("pts2", 2), ("pts3", 3)])
def test_points_path_parity(algo, name, d):
    inst = I.uniform_pair(333, 271, d, 11 + d, mass_r=1.0, mass_c=1.2, s_frac=0.75)
    ref = _oracle(inst, "points", algo)
    out = gpu_solve(inst, "points", algo, trace_cap=ref.iters + 8, want_plan=True)
    assert out.status == 0
    assert feasible(out.plan.cpu().numpy(), inst.r, inst.c, inst.s)
    check_definition1(inst, "points", algo, out, lp_key=f"{name}:points")
    assert out.result["iters"] == ref.iters
    tally("strict", f"{name}/{algo}/points")
    assert rel(out.result["cost"], ref.rounded["cost"]) <= COST_RTOL
    _compare_elementwise(inst, algo, out, ref, out.plan.cpu().numpy())


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
    # Definition 1 on the exact cost (the FP64 points-defined C): E recomputed
    # on the BF16 values the GPU saw, feasibility, and cost - LP* <= eps
    info = check_definition1(inst, "bf16", algo, out, lp_key="u400x384:exact", C_exact=inst.C64)
    print(f"bf16 {algo}: {info}", flush=True)
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
    check_definition1(inst, "f32", "aspot", out, lp_key=f"{name}:f32")
    if res["iters"] == ref.iters:
        tally("strict", f"{name}/{'+'.join(variant)}")
        assert rel(res["cost"], ref.rounded["cost"]) <= COST_RTOL
    else:
        tally("def1", f"{name}/{'+'.join(variant)} ({res['iters']} vs {ref.iters} iterations)")
