"""Warm-start inference kernels (pot_warm_predict) against the FP32
reference of the same arithmetic, and warm-started batched solves."""
import os

import numpy as np
import pytest

from oracle import potref as O
from paper_2601_17196_amd import instances as I
from paper_2601_17196_amd import warmstart as W
from tests.test_warmstart_host import _random_weights

pytestmark = pytest.mark.gpu


def _dev_points(inst):
    import torch
    return dict(x=torch.from_numpy(np.ascontiguousarray(inst.x, dtype=np.float32)).cuda(),
                y=torch.from_numpy(np.ascontiguousarray(inst.y, dtype=np.float32)).cuda(),
                r=torch.from_numpy(inst.r).cuda(), c=torch.from_numpy(inst.c).cuda(),
                cost_scale=inst.cost_scale)


@pytest.mark.parametrize("n,m", [(1, 1), (5, 70), (64, 64), (65, 130), (256, 256), (1000, 37)])
def test_inference_matches_reference(n, m):
    import torch

    from paper_2601_17196_amd import pot
    inst = I.uniform_pair(n, m, 2, 100 + n + m, mass_r=1.0, mass_c=1.1, s_frac=0.5)
    inst.r[0] = 0.0                                  # a zero mass: the clipped feature
    arr = _random_weights(n + m)
    blob = pot.warm_blob(arr)
    gamma = 1e-3
    d = _dev_points(inst)
    d["gamma"] = gamma
    print(f"warm inference n={n} m={m}", flush=True)
    (u0, v0), = pot.warm_predict([d], 1e-2, blob)
    torch.cuda.synchronize()
    fs = W.features_np(inst.x, inst.y, inst.r, inst.cost_scale)
    ft = W.features_np(inst.y, inst.x, inst.c, inst.cost_scale)
    ps, pt = W.reference_predict(arr, fs, ft)
    scale = max(1.0, float(np.max(np.abs(ps))), float(np.max(np.abs(pt))))
    assert np.max(np.abs(u0.cpu().numpy() * gamma - ps)) <= 2e-4 * scale
    assert np.max(np.abs(v0.cpu().numpy() * gamma - pt)) <= 2e-4 * scale


def test_inference_batch_equals_single():
    import torch

    from paper_2601_17196_amd import pot
    insts = [I.c5(k) for k in range(3)]
    arr = _random_weights(9)
    blob = pot.warm_blob(arr)
    ds = [_dev_points(i) for i in insts]
    outs = pot.warm_predict(ds, 1e-2, blob)
    one = pot.warm_predict(ds[1:2], 1e-2, blob)
    torch.cuda.synchronize()
    assert torch.equal(outs[1][0], one[0][0]) and torch.equal(outs[1][1], one[0][1])


@pytest.mark.skipif(not os.path.exists(W.WEIGHTS), reason="trained warm-start weights not present")
def test_warm_started_batch_reaches_eps():
    """Validation instances of the n = m = 256 mixture family: predictions of
    the trained network, then ASPOT in one batched launch with the phi check.
    Every instance reaches E <= eps~ with a feasible rounding; the costs agree
    with cold starts within eps, and two of them with the oracle."""
    import torch

    from paper_2601_17196_amd import pot
    insts = [I.c5(k) for k in range(20000, 20064)]
    blob = pot.warm_blob()
    preds = pot.warm_predict([_dev_points(i) for i in insts], 1e-2, blob)
    probs = []
    for inst in insts:
        d = pot.to_device_instance(inst, "cuda:0", kind="f32", pad_ldc=True)
        probs.append(dict(r=d["r"], c=d["c"], s=d["s"], C=d["C"], kind=d["kind"], ldc=d["ldc"], cmax=1.0))
    st_w, res_w, _ = pot.solve_batched(probs, 1e-2, u0=[p[0] for p in preds], v0=[p[1] for p in preds],
                                       w0=[0.0] * len(preds), warm_check=True)
    st_c, res_c, _ = pot.solve_batched(probs, 1e-2)
    torch.cuda.synchronize()
    bad = [(k, r["status"], r["iters"], r["used_warm"]) for k, r in enumerate(res_w) if r["status"] != 0]
    assert st_w == 0 and st_c == 0, bad
    it_w = np.array([r["iters"] for r in res_w])
    it_c = np.array([r["iters"] for r in res_c])
    used = sum(r["used_warm"] for r in res_w)
    print(f"warm kept on {used}/{len(insts)}; iterations median warm {np.median(it_w)} cold {np.median(it_c)}; "
          f"total warm {it_w.sum()} cold {it_c.sum()}")
    for inst, rw, rc in zip(insts, res_w, res_c):
        assert rw["E"] <= rw["tol"]
        assert abs(rw["mass"] - inst.s) <= 1e-11
        assert abs(rw["cost"] - rc["cost"]) <= inst.eps
    for k in (0, 1):
        ref = O.solve(insts[k].C32.astype(np.float64), insts[k].r, insts[k].c, insts[k].s, insts[k].eps,
                      algo="aspot", cmax=1.0)
        assert abs(res_w[k]["cost"] - ref.rounded["cost"]) <= insts[k].eps
