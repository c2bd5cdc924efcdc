"""pot_solve with POT_FLAG_ASYNC (everything enqueued, every decision on the
device, the result block written to device memory) and the warm-start check
of pot_solve, through the C ABI.

* An asynchronous solve gives the synchronous one's result exactly (the
  same kernels in the same order).
* Captured whole in a caller's HIP graph (torch.cuda.graph) and replayed
  several times, with the program's own work between the replays, every
  replay reproduces the eager solve and passes the Definition 1 check
  through the oracle (E at its duals, exact feasibility, cost - LP* <= eps),
  also with |C|_max computed on the device inside the graph.
* An invalid problem is reported in the device result, with no output
  written.
* warm_check = 1: a warm start at the oracle's optimum is kept (one or two
  iterations); a start worse than zero, or one whose statistics overflow, is
  replaced by the zero start and the solve equals the cold one.
"""
import numpy as np
import pytest

from oracle import potref as O
from paper_2601_17196_amd import instances as I
from tests.gpu_common import check_definition1, gpu_solve, rel

pytestmark = pytest.mark.gpu


def _dev(inst, kind="f32"):
    from paper_2601_17196_amd import pot
    return pot.to_device_instance(inst, "cuda:0", kind=kind)


def _same(a, b):
    for k in ("status", "iters", "cost", "E", "mass", "kappa", "lambda_", "w", "gamma", "tol", "viol_row",
              "viol_col", "viol_mass"):
        assert a[k] == b[k], (k, a[k], b[k])


@pytest.mark.parametrize("algo", ["aspot", "sinkhorn"])
def test_async_equals_sync(algo):
    import torch

    from paper_2601_17196_amd import pot
    inst = I.uniform_pair(300, 257, 2, 5, mass_r=1.0, mass_c=1.3, s_frac=0.7)
    d = _dev(inst)
    a = pot.ASPOT if algo == "aspot" else pot.SINKHORN
    sync = pot.solve(d["r"], d["c"], d["s"], inst.eps, C=d["C"], cmax=1.0, algo=a, want_plan=True, max_iter=3000)
    asy = pot.solve(d["r"], d["c"], d["s"], inst.eps, C=d["C"], cmax=1.0, algo=a, want_plan=True, max_iter=3000,
                    async_=True)
    torch.cuda.synchronize()
    ra = pot.result_from_device(asy.result_dev)
    _same(ra, sync.result)
    assert torch.equal(asy.plan, sync.plan) and torch.equal(asy.f, sync.f) and torch.equal(asy.g, sync.g)


@pytest.mark.parametrize("cmax", [1.0, 0.0])
def test_async_solve_captured_in_caller_graph(cmax):
    """The whole solve captured in the caller's graph and replayed 4 times."""
    import torch

    from paper_2601_17196_amd import pot
    inst = I.c1(0)
    d = _dev(inst)
    print(f"graph capture of an asynchronous solve, cmax {cmax}", flush=True)
    eager = pot.solve(d["r"], d["c"], d["s"], inst.eps, C=d["C"], cmax=cmax, want_plan=True, max_iter=1000)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):       # warm-up outside the capture (first-launch setup of the kernels)
        pot.solve(d["r"], d["c"], d["s"], inst.eps, C=d["C"], cmax=cmax, want_plan=True, max_iter=1000,
                  async_=True)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cap = pot.solve(d["r"], d["c"], d["s"], inst.eps, C=d["C"], cmax=cmax, want_plan=True, max_iter=1000,
                        async_=True)
    assert cap.status == pot.OK
    ref = O.solve(inst.C32.astype(np.float64), inst.r, inst.c, inst.s, inst.eps, algo="aspot", cmax=1.0)
    for rep in range(4):
        cap.result_dev.zero_()
        cap.plan.zero_()
        junk = torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")   # eager work
        g.replay()
        torch.cuda.synchronize()
        r = pot.result_from_device(cap.result_dev)
        _same(r, eager.result)
        assert torch.equal(cap.plan, eager.plan)
        cap.result = r
        cap.w = r["w"]
        info = check_definition1(inst, "f32", "aspot", cap, lp_key="c1:f32")
        print(f"replay {rep}: iters {r['iters']} (oracle {ref.iters}) cost {r['cost']:.12e} "
              f"gap to LP {info['gap']:.3e}", flush=True)
        del junk


def test_async_invalid_problem_reported_on_device():
    """An invalid mass (found by the setup kernel) is reported in the device
    result; the caller's output buffers keep their contents.  Host-side
    checks (here max_iter) still return at once."""
    import ctypes as ct

    import torch

    from paper_2601_17196_amd import pot
    lib = pot.load()
    inst = I.uniform_pair(40, 50, 2, 9)
    d = _dev(inst)
    for case in ("negative mass", "s above the masses"):
        r = d["r"].clone()
        s = inst.s
        if case == "negative mass":
            r[3] = -1.0
        else:
            s = 2.0 * max(inst.r.sum(), inst.c.sum())
        prob = pot.make_problem(r, d["c"], s, C=d["C"], cmax=1.0)
        opts = pot.make_options(inst.eps, max_iter=50, flags=pot.FLAG_ASYNC | pot.FLAG_WANT_PLAN)
        nb = pot.workspace_bytes(prob, opts)
        ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
        base = (ws.data_ptr() + 255) & ~255
        f = torch.full((inst.n,), 7.0, dtype=torch.float64, device="cuda")
        g = torch.full((inst.m,), 7.0, dtype=torch.float64, device="cuda")
        plan = torch.full((inst.n, inst.m), 7.0, dtype=torch.float64, device="cuda")
        alpha = torch.full((inst.n,), 7.0, dtype=torch.float64, device="cuda")
        out = pot.Outputs()
        out.plan, out.f, out.g, out.alpha = plan.data_ptr(), f.data_ptr(), g.data_ptr(), alpha.data_ptr()
        resd = torch.zeros(ct.sizeof(pot.Result), dtype=torch.uint8, device="cuda")
        st = lib.pot_solve(ct.byref(prob), ct.byref(opts), ct.c_void_p(base), ct.c_size_t(nb),
                           ct.cast(ct.c_void_p(resd.data_ptr()), ct.POINTER(pot.Result)), ct.byref(out),
                           ct.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == pot.OK                      # nothing was checked on the host
        torch.cuda.synchronize()
        assert pot.result_from_device(resd)["status"] == pot.ERR_INVALID_ARG, case
        for t in (f, g, plan, alpha):
            assert bool(torch.all(t == 7.0)), case
    out2 = pot.solve(d["r"], d["c"], inst.s, inst.eps, C=d["C"], cmax=1.0, max_iter=0, async_=True,
                     raise_on_error=False)
    assert out2.status == pot.ERR_INVALID_ARG


def test_warm_check_keeps_a_good_start_and_drops_a_bad_one():
    import torch

    from paper_2601_17196_amd import pot
    inst = I.c1(0)
    C = inst.C32.astype(np.float64)
    gam, tol, M, rt, ct_ = O.setup(inst.r, inst.c, inst.s, inst.eps, cmax=1.0)
    u, v, w, it, E, st, _ = O.aspot(C, gam, 1e-9, rt, ct_, inst.s, M)
    cold = gpu_solve(inst, "f32", "aspot")
    good = gpu_solve(inst, "f32", "aspot", u0=torch.from_numpy(u).cuda(), v0=torch.from_numpy(v).cuda(), w0=w,
                     warm_check=1)
    assert good.status == 0 and good.result["used_warm"] == 1 and good.result["iters"] <= 2
    check_definition1(inst, "f32", "aspot", good, lp_key="c1:f32")
    n, m = C.shape
    for level in (3.0, 50.0):             # phi above phi(0); statistics beyond the FP64 range
        bad = gpu_solve(inst, "f32", "aspot", u0=torch.full((n,), level, dtype=torch.float64, device="cuda"),
                        v0=torch.full((m,), level, dtype=torch.float64, device="cuda"), warm_check=1)
        assert bad.status == 0 and bad.result["used_warm"] == 0, (level, bad.status, bad.result)
        assert bad.result["iters"] == cold.result["iters"]
        assert rel(bad.result["cost"], cold.result["cost"]) <= 1e-12
