"""pot_solve_batched (one persistent launch for many instances) against the
FP64 oracle, through the C ABI.

Every instance passes the Definition 1 check of tests/gpu_common.py
(check_definition1_batched: E recomputed by the oracle at the GPU's output
point, the oracle's rounding of the GPU's duals reproducing the GPU's cost,
factors and mass, and on selected instances 0 <= cost - LP* <= eps against
the exact LP).  Where the oracle and the GPU take the same number of
iterations, the rounded cost also agrees to 1e-6 relative and the ASPOT
log-scalings to 1e-6 element by element.
"""
import numpy as np
import pytest

from oracle import potref as O
from paper_2601_17196_amd import instances as I
from tests.gpu_common import check_definition1_batched, oracle_cost_matrix, rel, tally

pytestmark = pytest.mark.gpu

SIZES = [(37, 300), (300, 37), (64, 64), (129, 257), (5, 9), (200, 180), (1, 50), (512, 40), (1024, 96),
         (700, 650)]


def _insts(sizes, seed0=300, d=3):
    out = []
    for k, (n, m) in enumerate(sizes):
        g = np.random.default_rng(seed0 + k)
        out.append(I.uniform_pair(n, m, d, seed0 + k, mass_r=float(g.uniform(0.8, 1.2)),
                                  mass_c=float(g.uniform(0.8, 1.2)), s_frac=float(g.uniform(0.5, 0.9))))
    return out


def _dev(insts, kind="f32"):
    from paper_2601_17196_amd import pot
    probs = []
    for inst in insts:
        d = pot.to_device_instance(inst, "cuda:0", kind=kind)
        probs.append(dict(r=d["r"], c=d["c"], s=d["s"], C=d["C"], kind=d["kind"], ldc=d["ldc"], cmax=1.0))
    return probs


def _solve(insts, algo="aspot", kind="f32", **kw):
    import torch

    from paper_2601_17196_amd import pot
    a = pot.ASPOT if algo == "aspot" else pot.SINKHORN
    print(f"batched {algo} {kind}: {len(insts)} instances {kw}", flush=True)
    kw.setdefault("want_uv", True)
    st, res, fg = pot.solve_batched(_dev(insts, kind), insts[0].eps, algo=a, **kw)
    torch.cuda.synchronize()
    return st, res, fg


def _check(inst, res, algo, kind="f32", fguv=None, lp=False, label="batched"):
    """Definition 1 (always, with the exact LP where lp), and 1e-6 parity
    where the iteration counts agree."""
    ref = O.solve(oracle_cost_matrix(inst, kind), inst.r, inst.c, inst.s, inst.eps, algo=algo, cmax=1.0)
    assert res["status"] == 0, res
    assert abs(res["mass"] - inst.s) <= 1e-11 * max(1.0, inst.s)
    assert res["E"] <= res["tol"]
    if fguv is not None:
        f, g, u, v = fguv
        check_definition1_batched(inst, kind, algo, res, f, g, u, v,
                                  lp_key=f"{inst.name}:{kind}" if lp else None)
    if res["iters"] == ref.iters:
        tally("strict", f"{label}:{inst.name}/{algo}")
        assert rel(res["cost"], ref.rounded["cost"]) <= 1e-6, (inst.name, res["cost"], ref.rounded["cost"])
        if fguv is not None and algo == "aspot":
            fe = fguv[0].cpu().numpy()
            assert np.max(np.abs(fe - ref.f)) <= 1e-6 * max(1.0, np.max(np.abs(ref.f)))
    else:
        assert fguv is not None, "a differing run needs the duals for the Definition 1 check"
        tally("def1", f"{label}:{inst.name}/{algo} ({res['iters']} vs {ref.iters} iterations)")
    return ref


@pytest.mark.parametrize("algo", ["aspot", "sinkhorn"])
def test_batched_uneven_matches_oracle(algo):
    insts = _insts(SIZES)
    st, res, fg = _solve(insts, algo)
    assert st == 0
    same = 0
    for inst, r, fguv in zip(insts, res, fg):
        ref = _check(inst, r, algo, fguv=fguv, lp=True)
        same += r["iters"] == ref.iters
    assert same >= len(insts) // 2      # most runs take every decision the same way


def test_batched_bitwise_reproducible():
    """The same batch solved twice gives the same bits: iteration counts,
    costs and log-scalings (every sum is taken in a fixed order, and no
    workgroup reads shared memory that another may still be writing).
    Instances with more rows and columns than threads step several per
    thread, which is where a missed barrier would show."""
    insts = _insts(SIZES, seed0=500)
    st1, res1, fg1 = _solve(insts, "aspot")
    st2, res2, fg2 = _solve(insts, "aspot")
    assert st1 == 0 and st2 == 0
    for inst, a, b, x, y in zip(insts, res1, res2, fg1, fg2):
        assert a["iters"] == b["iters"], inst.name
        assert a["cost"] == b["cost"], inst.name
        for u, v in zip(x, y):
            assert np.array_equal(u.cpu().numpy(), v.cpu().numpy()), inst.name


def test_batched_padded_rows_masked():
    """Rows with a stride beyond m (aligned, so the sweep reads whole 16-byte
    groups and a lane past the row's end reads the stride's padding): the
    padding is filled with NaN and the results are bit for bit those of the
    unpadded rows, for FP32 and BF16."""
    import torch

    from paper_2601_17196_amd import pot
    insts = _insts([(70, 180), (33, 252), (129, 100), (40, 8)], seed0=900)
    for kind in ("f32", "bf16"):
        plain = _dev(insts, kind)
        padded = []
        for inst, pr in zip(insts, plain):
            m = inst.m
            ld = (m + 7) // 8 * 8 + 8
            host = inst.C32 if kind == "f32" else I.to_bf16_bits(inst.C32).view(np.int16)
            buf = np.empty((inst.n, ld), dtype=host.dtype)
            if kind == "f32":
                buf[:] = np.nan
            else:
                buf[:] = np.int16(0x7FC0)              # a BF16 NaN
            buf[:, :m] = host
            t = torch.from_numpy(buf).cuda()
            q = dict(pr)
            q["C"] = t
            q["ldc"] = ld
            padded.append(q)
        print(f"batched padded rows ({kind})", flush=True)
        st1, res1, fg1 = pot.solve_batched(plain, insts[0].eps, want_uv=True)
        st2, res2, fg2 = pot.solve_batched(padded, insts[0].eps, want_uv=True)
        torch.cuda.synchronize()
        assert st1 == 0 and st2 == 0
        for inst, a, b, x, y in zip(insts, res1, res2, fg1, fg2):
            assert a["iters"] == b["iters"] and a["cost"] == b["cost"], (kind, inst.name)
            for u, v in zip(x, y):
                assert np.array_equal(u.cpu().numpy(), v.cpu().numpy()), (kind, inst.name)


@pytest.mark.parametrize("algo", ["aspot", "sinkhorn"])
def test_batched_groups_split_rows(algo):
    """member_elems = 4096 splits every instance above 4096 entries over up to
    8 workgroups that exchange column partials; the results match the oracle
    and the unsplit run."""
    insts = _insts(SIZES[-4:], seed0=400)
    st1, res1, fg1 = _solve(insts, algo, member_elems=4096)
    st2, res2, _ = _solve(insts, algo, member_elems=1 << 22)
    assert st1 == 0 and st2 == 0
    for inst, a, b, fguv in zip(insts, res1, res2, fg1):
        _check(inst, a, algo, fguv=fguv, label="split")
        # the split changes which rows share an FP32 accumulation batch: the
        # two runs agree to the FP32 path's bar, not bitwise
        if a["iters"] == b["iters"]:
            assert rel(a["cost"], b["cost"]) <= 1e-6


def test_batched_bf16_within_eps():
    insts = _insts(SIZES[:6], seed0=500)
    st, res, fg = _solve(insts, "aspot", kind="bf16")
    assert st == 0
    for inst, r, (f, g, u, v) in zip(insts, res, fg):
        assert r["status"] == 0
        # Definition 1 on the exact (points-defined) cost
        check_definition1_batched(inst, "bf16", "aspot", r, f, g, u, v, lp_key=f"{inst.name}:exact",
                                  C_exact=inst.C64)
        ref = O.solve(inst.C64, inst.r, inst.c, inst.s, inst.eps, algo="aspot", cmax=1.0)
        assert abs(r["cost"] - ref.rounded["cost"]) <= inst.eps
        assert abs(r["mass"] - inst.s) <= 1e-11


def test_batched_warm_start_at_optimum_and_fallback():
    """Warm starts at the oracle's converged duals finish in one or two
    iterations; a poor warm start (phi above phi(0)) is dropped for a cold
    start and still reaches eps."""
    import torch
    insts = _insts([(90, 70), (60, 120), (100, 100)], seed0=600)
    u0, v0, w0 = [], [], []
    for k, inst in enumerate(insts):
        C = inst.C32.astype(np.float64)
        gam, tol, M, rt, ct_ = O.setup(inst.r, inst.c, inst.s, inst.eps, cmax=1.0)
        if k < 2:
            u, v, w, _, _, _, _ = O.aspot(C, gam, 1e-9, rt, ct_, inst.s, M)
        else:
            u, v, w = np.full(inst.n, 3.0), np.full(inst.m, 3.0), 0.0   # B(z0) ~ e^6 B(0)
        u0.append(torch.from_numpy(u).cuda())
        v0.append(torch.from_numpy(v).cuda())
        w0.append(float(w))
    st, res, fg = _solve(insts, "aspot", u0=u0, v0=v0, w0=w0, warm_check=True)
    assert st == 0
    for k, (inst, r) in enumerate(zip(insts, res)):
        assert r["status"] == 0
        assert abs(r["mass"] - inst.s) <= 1e-11
        if k < 2:
            assert r["used_warm"] == 1 and r["iters"] <= 2
            check_definition1_batched(inst, "f32", "aspot", r, *fg[k], lp_key=f"{inst.name}:f32")
        else:
            assert r["used_warm"] == 0
            _check(inst, r, "aspot", fguv=fg[k], label="fallback")


def test_batched_invalid_instance_reported_others_solved():
    from paper_2601_17196_amd import pot
    insts = _insts([(40, 50), (30, 20), (60, 61)], seed0=700)
    insts[1].s = 2.0 * max(insts[1].r.sum(), insts[1].c.sum())     # s above the masses
    st, res, fg = _solve(insts, "aspot")
    assert st == pot.ERR_INVALID_ARG
    assert res[1]["status"] == pot.ERR_INVALID_ARG
    for k in (0, 2):
        _check(insts[k], res[k], "aspot", fguv=fg[k], label="invalid-neighbour")


def test_batched_rejects_unsupported():
    import torch

    from paper_2601_17196_amd import pot
    insts = _insts([(40, 50), (30, 20)], seed0=800)
    big = I.uniform_pair(1100, 20, 2, 801)
    with pytest.raises(pot.PotError):
        pot.solve_batched(_dev([big]), big.eps)
    probs = _dev(insts)
    probs[1]["C"] = I.to_bf16_bits(insts[1].C32)
    probs[1]["C"] = torch.from_numpy(probs[1]["C"].view(np.int16)).cuda()
    probs[1]["kind"] = pot.COST_BF16
    probs[1]["ldc"] = insts[1].m
    st, _, _ = pot.solve_batched(probs, insts[0].eps)
    assert st == pot.ERR_UNSUPPORTED
    assert "same cost kind" in pot.last_error()
    # a row stride of 2^31 bytes or more is rejected before anything is read
    probs = _dev(insts)
    probs[0]["ldc"] = 1 << 29
    st, _, _ = pot.solve_batched(probs, insts[0].eps)
    assert st == pot.ERR_INVALID_ARG
    assert "row stride" in pot.last_error()


def test_batched_max_iter_still_feasible():
    from paper_2601_17196_amd import pot
    insts = _insts([(40, 50), (300, 200)], seed0=900)
    st, res, _ = _solve(insts, "aspot", max_iter=3)
    assert st == pot.ERR_NO_CONVERGENCE
    for inst, r in zip(insts, res):
        assert r["status"] == pot.ERR_NO_CONVERGENCE and r["iters"] == 3
        assert abs(r["mass"] - inst.s) <= 1e-11
        ref = O.solve(inst.C32.astype(np.float64), inst.r, inst.c, inst.s, inst.eps, algo="aspot", cmax=1.0,
                      max_iter=3)
        assert rel(r["cost"], ref.rounded["cost"]) <= 1e-6


def test_batched_uneven_batch_full_size():
    """The 512-instance uneven batch (n, m log-uniform in [64, 1024]) in the
    launch configuration the benchmark times: every instance passes the
    Definition 1 check through the oracle (E recomputed at its duals, the
    oracle's rounding reproducing its cost and factors, and cost - OPT <= eps
    certified by a weak-duality bound from its duals); the exact LP optimum
    is also checked on the four smallest instances and on the one nearest
    256 x 256."""
    insts = I.c4_batch(512)
    st, res, fg = _solve(insts, "aspot")
    assert st == 0
    by_size = sorted(range(len(insts)), key=lambda k: insts[k].n * insts[k].m)
    mid = min(range(len(insts)), key=lambda k: abs(insts[k].n * insts[k].m - 256 * 256))
    with_lp = set(by_size[:4]) | {mid}
    worst = 0.0
    gaps = []
    for k, (inst, r) in enumerate(zip(insts, res)):
        assert r["status"] == 0 and r["E"] <= r["tol"]
        info = check_definition1_batched(inst, "f32", "aspot", r, *fg[k],
                                         lp_key=f"{inst.name}:f32" if k in with_lp else None, dual=True)
        worst = max(worst, abs(info["E_oracle"] - info["E_gpu"]))
        gaps.append(info["gap"])
    print(f"c4: 512 instances through the oracle, largest |E_gpu - E_oracle| {worst:.3e}, "
          f"cost - lower bound: median {np.median(gaps):.2e} max {np.max(gaps):.2e}", flush=True)


def test_batched_tracking_warm_start():
    """Warm starts from a previous solve (the tracking use of the benchmark):
    four instances of the 256 x 256 mixture batch are solved cold, every
    target cloud is moved by a small rigid step (1 degree about its centroid,
    shift 0.005, the cost renormalised to max 1), and the moved instances are solved from
    the first solve's duals with the phi check.  Every warm start is kept,
    every moved instance passes Definition 1 (E recomputed by the oracle at
    the GPU's output point, the oracle's rounding of the GPU's duals, and
    cost - LB <= eps for the weak-duality bound from the GPU's duals), and the
    warm solves take fewer iterations in total than the cold ones."""
    base = I.c5_batch(4)
    st0, res0, fg0 = _solve(base, "aspot")
    assert st0 == 0
    th = np.deg2rad(1.0)
    Rz = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    moved = []
    for inst in base:
        y = inst.y.astype(np.float64)
        mu = y.mean(0)
        y2 = ((y - mu) @ Rz.T + mu + 0.005).astype(np.float32).astype(np.float64)
        D = ((inst.x.astype(np.float64)[:, None, :] - y2[None, :, :]) ** 2).sum(-1)
        C = D / D.max()
        mv = I.Instance(x=inst.x, y=y2.astype(np.float32), r=inst.r, c=inst.c, s=inst.s, cost_scale=1.0 / D.max(),
                        C64=C, C32=np.ascontiguousarray(C.astype(np.float32)), eps=inst.eps,
                        name=inst.name + " moved")
        moved.append(mv)
    u0 = [fg[2] for fg in fg0]
    v0 = [fg[3] for fg in fg0]
    w0 = [r["w"] for r in res0]
    stw, resw, fgw = _solve(moved, "aspot", u0=u0, v0=v0, w0=w0, warm_check=True)
    stc, resc, _ = _solve(moved, "aspot")
    assert stw == 0 and stc == 0
    for inst, r, fg in zip(moved, resw, fgw):
        assert r["used_warm"] == 1, (inst.name, r)
        check_definition1_batched(inst, "f32", "aspot", r, *fg, dual=True)
    itw = sum(r["iters"] for r in resw)
    itc = sum(r["iters"] for r in resc)
    print(f"tracking: warm {itw} vs cold {itc} iterations", flush=True)
    assert itw < itc
