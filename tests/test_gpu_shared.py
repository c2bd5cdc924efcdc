"""Shared-cost batches (pot_solve_shared): feasible Sinkhorn of Algorithm 3 in
the exponential domain for many members on one cost, the products on the
matrix cores, against the FP64 oracle, through the C ABI.

The GPU's kernel K~ is rounded to BF16 once, so its fixed point is that of
the effective cost C' = -gamma ln K~_bf16 (within gamma 2^-8 of C).  The
oracle runs the same algorithm (log domain, FP64) on C' with the same gamma
and threshold, then rounds with the true cost, as the library does.  Bars:
where the iteration counts agree, the rounded cost and the scalings (f, g
modulo the extended instance's gauge, absolute, i.e. relative in the
scalings) to t x 2 (2^-16 + d 2^-24) after t iterations: each product K~ b
takes the scaling as the sum of two BF16 numbers (relative error <= 2^-16)
and accumulates d terms in FP32 (<= d 2^-24), in each of the two half
iterations;
always, for every member: the stopping error of Algorithm 3 recomputed by the
oracle at the GPU's extended scalings (on C') within the threshold (bound:
the products carry about 2^-16 relative error from the split scalings and
FP32 accumulation), the oracle's rounding of the GPU's scalings giving the
GPU's cost (1e-9), and the rounded plan exactly feasible.  (The gap to the
LP optimum is printed, not bounded: gamma here is the caller's, at least
max C / 80 for the kernel to be representable, and the entropic bias at such
gamma is about eps on these sizes, so Definition 1's eps is the caller's to
choose through gamma.)
"""
import numpy as np
import pytest

from oracle import potref as O
from paper_2601_17196_amd import instances as I
from tests.gpu_common import lp_optimum, rel, tally

pytestmark = pytest.mark.gpu


def _members(n, m, B, seed):
    g = np.random.default_rng(seed)
    out = []
    for k in range(B):
        a = float(g.uniform(0.5, 2.0))
        r = g.dirichlet(np.full(n, a)) * g.uniform(0.8, 1.2)
        c = g.dirichlet(np.full(m, a)) * g.uniform(0.8, 1.2)
        s = float(g.uniform(0.5, 0.9) * min(r.sum(), c.sum()))
        out.append((r, c, s))
    return out


def _effective_cost(C32, gamma):
    K = np.exp(-C32.astype(np.float64) / gamma).astype(np.float32)
    Kb = I.bf16_bits_to_f64(I.to_bf16_bits(K))
    with np.errstate(divide="ignore"):
        return -gamma * np.log(Kb)


def _run(C32, mem, eps, gamma, **kw):
    import torch

    from paper_2601_17196_amd import pot
    Cd = torch.from_numpy(C32).cuda()
    dm = [dict(r=torch.from_numpy(r).cuda(), c=torch.from_numpy(c).cuda(), s=s) for r, c, s in mem]
    st, res, fg = pot.solve_shared(Cd, dm, eps, gamma, cmax=float(C32.max()), **kw)
    torch.cuda.synchronize()
    return st, res, fg


@pytest.mark.parametrize("n,m,B", [(200, 150, 40), (97, 301, 7)])
def test_shared_cost_members_match_the_oracle(n, m, B):
    inst = I.uniform_pair(n, m, 2, 61 + n)
    C32 = inst.C32
    gamma = float(C32.max()) / 60.0
    eps = 1e-2
    mem = _members(n, m, B, n + m)
    st, res, fg = _run(C32, mem, eps, gamma)
    print(f"shared: {B} members {n} x {m}, gamma {gamma:.4f}; iterations {[r['iters'] for r in res]}", flush=True)
    assert st == 0
    Ceff = _effective_cost(C32, gamma)
    Ct = C32.astype(np.float64)
    for k, ((r, c, s), rr, (f, g)) in enumerate(zip(mem, res, fg)):
        assert rr["status"] == 0 and rr["E"] <= rr["tol"]
        gam, tol, M, rt, ct_ = O.setup(r, c, s, eps, cmax=float(C32.max()), gamma=gamma)
        assert abs(rr["gamma"] - gamma) <= 1e-15 * gamma and abs(rr["tol"] - tol) <= 1e-15 * tol
        f, g = f.cpu().numpy(), g.cpu().numpy()
        A = 8.0 * float(C32.max()) / eps
        # the stopping error at the GPU's extended scalings, on the effective cost
        E = O.sk_error(Ceff, gamma, rt, ct_, s, A, np.append(f, rr["ext_a"]), np.append(g, rr["ext_b"]))
        Mext = rt.sum() + ct_.sum() - s
        bar = 4 * 2.0 ** -16 * 2 * Mext
        assert abs(E - rr["E"]) <= bar and E <= tol + bar, (k, E, rr["E"], tol)
        # the oracle's rounding of the GPU's scalings (true cost): the GPU's cost
        rd = O.round_plan(Ct, gamma, f, g, r, c, s, dense=k < 2)
        assert rel(rr["cost"], rd["cost"]) <= 1e-9, (k, rr["cost"], rd["cost"])
        assert abs(rr["mass"] - s) <= 1e-11 * max(1.0, s)
        # the oracle's run of Algorithm 3 on the effective cost
        a, b, it, Eo, sto, _ = O.sinkhorn(Ceff, gamma, tol, rt, ct_, s, A)
        ro = O.round_plan(Ct, gamma, a[:-1], b[:-1], r, c, s)
        if it == rr["iters"]:
            tally("strict", f"shared {n}x{m} member {k}")
            dbar = max(it, 1) * 2 * (2.0 ** -16 + (max(n, m) + 1) * 2.0 ** -24)
            assert rel(rr["cost"], ro["cost"]) <= dbar, (k, rr["cost"], ro["cost"], dbar)
            kk = float(np.mean(f - a[:-1]))
            assert np.max(np.abs(f - kk - a[:-1])) <= dbar, k
            assert np.max(np.abs(g + kk - b[:-1])) <= dbar, k
        else:
            tally("def1", f"shared {n}x{m} member {k} ({rr['iters']} vs {it} iterations)")
        if k < 2:
            X = rd["X"]
            assert np.all(X >= 0) and np.all(X.sum(1) <= r * (1 + 1e-12)) and np.all(X.sum(0) <= c * (1 + 1e-12))
            assert abs(X.sum() - s) <= 1e-11 * max(1.0, s)
            lp = lp_optimum(f"shared{n}x{m}:{k}", Ct, r, c, s)
            print(f"  member {k}: cost - LP* = {float(np.sum(Ct * X)) - lp:.3e} at gamma = max C / 60", flush=True)


def test_shared_cost_invalid_member_and_limits():
    from paper_2601_17196_amd import pot
    inst = I.uniform_pair(60, 50, 2, 5)
    C32 = inst.C32
    mem = _members(60, 50, 3, 9)
    r, c, s = mem[1]
    mem[1] = (r, c, 3.0 * max(r.sum(), c.sum()))            # s above the masses
    st, res, fg = _run(C32, mem, 1e-2, float(C32.max()) / 30.0)
    assert st == pot.ERR_INVALID_ARG and res[1]["status"] == pot.ERR_INVALID_ARG
    assert res[0]["status"] == 0 and res[2]["status"] == 0
    # a gamma for which the exponential-domain kernel would underflow
    st, res, _ = _run(C32, _members(60, 50, 2, 3), 1e-2, float(C32.max()) / 200.0)
    assert st == pot.ERR_UNSUPPORTED and "80" in pot.last_error()
