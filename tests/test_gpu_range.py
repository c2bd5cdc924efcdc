"""ASPOT where the statistics leave the FP64 range, against the FP64 oracle.

On tightly clustered points (n = m = 512) the proof-form step (step_rule = 1:
the momentum step of Algorithm 2 with the step size of the convergence proof,
1/gamma times the printed one) moves w from the cold start to about -4600 in
its first iteration, so every term of B(z) at the next point is far below
2^-1074.  The oracle computes in the log domain.  The HIP path carries each
tile's partial sums with the tile's binary shift and combines them as mantissa
and exponent, so log T and the decisions stay exact; it must follow the oracle
decision by decision and converge to the same plan.
"""
import numpy as np
import pytest

from oracle import potref as O
from paper_2601_17196_amd import instances as I
from tests.gpu_common import (check_definition1, check_definition1_batched, feasible, gpu_solve,
                              oracle_cost_matrix, rel, tally)

pytestmark = pytest.mark.gpu

N_TRACE = 40


def _inst():
    return I.tight_clusters(512, 0)


@pytest.mark.parametrize("kind", ["f32", "points"])
def test_first_iterations_follow_the_oracle(kind):
    inst = _inst()
    print(f"range: tight clusters n=512, {kind}, step_rule=1, 40 iterations", flush=True)
    C = oracle_cost_matrix(inst, kind)
    gam, tol, M, rt, ct_ = O.setup(inst.r, inst.c, inst.s, inst.eps, cmax=1.0)
    u, v, w, k, E, st, tr = O.aspot(C, gam, tol, rt, ct_, inst.s, M, max_iter=N_TRACE, step_rule=1,
                                    trace=True, trace_ztil=True)
    assert k == N_TRACE and st == 2
    # the case is what it claims: after the first step every term of B is
    # below e^(w + max u + max v) < 2^-1074
    zt = tr.ztil[1]
    assert zt[-1] + zt[:512].max() + zt[512:-1].max() < -1100.0
    out = gpu_solve(inst, kind, "aspot", trace_cap=N_TRACE + 8, step_rule=1, max_iter=N_TRACE)
    from paper_2601_17196_amd import pot
    assert out.status == pot.ERR_NO_CONVERGENCE, pot.last_error()
    res = out.result
    assert res["iters"] == N_TRACE
    ti = out.trace_i.cpu().numpy().reshape(-1, 3)[:N_TRACE]
    td = out.trace_d.cpu().numpy().reshape(-1, 4)[:N_TRACE]
    assert np.array_equal(ti[:, 0], tr.bhat)
    assert np.array_equal(ti[:, 1], tr.pick)
    assert np.array_equal(ti[:-1, 2], tr.bchk[:-1])
    # E, phi-check, phi-hat and theta of every iteration
    assert np.max(np.abs(td[:, 0] - tr.E) / np.abs(tr.E)) <= 1e-6
    assert np.max(np.abs(td[:, 1] - tr.phichk) / np.abs(tr.phichk)) <= 1e-6
    assert np.max(np.abs(td[:, 2] - tr.phihat) / np.abs(tr.phihat)) <= 1e-6
    assert np.max(np.abs(td[:, 3] - tr.theta)) <= 1e-15
    # the output point z^t
    assert abs(out.w - w) <= 1e-6 * max(1.0, abs(w))
    assert np.max(np.abs(out.u.cpu().numpy() - u)) <= 1e-6 * max(1.0, np.max(np.abs(u)))
    assert np.max(np.abs(out.v.cpu().numpy() - v)) <= 1e-6 * max(1.0, np.max(np.abs(v)))


def test_solve_converges_like_the_oracle():
    inst = _inst()
    print("range: tight clusters n=512, step_rule=1, full solve", flush=True)
    C = oracle_cost_matrix(inst, "f32")
    ref = O.solve(C, inst.r, inst.c, inst.s, inst.eps, algo="aspot", cmax=1.0, step_rule=1)
    assert ref.status == 0
    out = gpu_solve(inst, "f32", "aspot", want_plan=True, step_rule=1)
    res = out.result
    assert out.status == 0 and res["E"] <= res["tol"]
    assert feasible(out.plan.cpu().numpy(), inst.r, inst.c, inst.s)
    print(f"iterations gpu {res['iters']} oracle {ref.iters}; cost gpu {res['cost']:.9e} "
          f"oracle {ref.rounded['cost']:.9e}", flush=True)
    check_definition1(inst, "f32", "aspot", out, lp_key="tight512:f32")
    if res["iters"] == ref.iters:
        tally("strict", "range-tight512")
        assert rel(res["cost"], ref.rounded["cost"]) <= 1e-6
    else:
        tally("def1", f"range-tight512 ({res['iters']} vs {ref.iters} iterations)")


def _batched(inst, **kw):
    import torch

    from paper_2601_17196_amd import pot
    d = pot.to_device_instance(inst, "cuda:0", kind="f32")
    prob = dict(r=d["r"], c=d["c"], s=d["s"], C=d["C"], kind=d["kind"], ldc=d["ldc"], cmax=1.0)
    st, res, fg = pot.solve_batched([prob], inst.eps, algo=pot.ASPOT, step_rule=1, want_uv=True, **kw)
    torch.cuda.synchronize()
    return st, res[0], fg[0]


def test_batched_lone_member_follows_the_single_solve():
    """pot_solve_batched with the instance in one workgroup (member_elems =
    n m) carries the same range: it converges with the single solve."""
    inst = _inst()
    print("range: batched, one member", flush=True)
    st, r, fguv = _batched(inst, member_elems=512 * 512)
    one = gpu_solve(inst, "f32", "aspot", step_rule=1).result
    assert st == 0 and r["status"] == 0
    print(f"iterations batched {r['iters']} single {one['iters']}", flush=True)
    check_definition1_batched(inst, "f32", "aspot", r, *fguv, lp_key="tight512:f32")
    if r["iters"] == one["iters"]:
        assert rel(r["cost"], one["cost"]) <= 1e-6


def test_batched_group_reports_the_range_limit():
    """Split over a group of members (row shares), the batched path keeps
    plain FP64 sums: it reports the unrepresentable statistics instead of
    continuing."""
    from paper_2601_17196_amd import pot
    inst = _inst()
    print("range: batched, group of members", flush=True)
    st, r, _ = _batched(inst, member_elems=1 << 15)
    assert r["status"] == pot.ERR_NUMERIC
