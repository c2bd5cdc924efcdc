"""Rigid registration through POT (pot_register: Section 4 and its appendix)
against the FP64 oracle, through the C ABI.

Workload: a 3-D cloud X of 400 points (four Gaussian blobs along a bent
line) and Y = half of it (200 points) moved away by a known rigid map;
uniform masses, s = 0.4 min(n, m) / max(n, m), gamma0 = 4.4e-3 annealed by
0.83 per registration, eps = 1e-2.

* Every inner solve is checked against the oracle on exactly the inputs the
  GPU saw (the moved cloud and the warm start recorded by the library):
  the same iteration count and cost to 1e-6, or, after a near tie decided
  the other way, E recomputed at the GPU's duals within the threshold and
  the oracle's rounding of those duals giving the GPU's cost (1e-9).
* The map update of every registration (device moments of the rounded plan,
  host rotation) equals the oracle's SVD Procrustes on the oracle's rounding
  of the GPU's duals, composed onto the previous map (1e-9).
* The loop recovers the map: every point of the moved copy lands on its
  original to within 1e-2 of the cloud's extent.
* Warm starts from the previous registration's duals take fewer iterations
  in total than cold starts.
"""
import numpy as np
import pytest

from oracle import potref as O
from oracle import register as G
from tests.gpu_common import e_bar, rel, tally

pytestmark = pytest.mark.gpu


def _rot(axis, ang):
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K


def _clouds(n=400, seed=3):
    g = np.random.default_rng(seed)
    centres = np.array([[0.0, 0.0, 0.0], [0.5, 0.2, 0.1], [1.0, 0.5, 0.0], [1.4, 1.0, 0.3]])
    X = centres[g.integers(0, 4, n)] + 0.08 * g.standard_normal((n, 3))
    X = X.astype(np.float32)
    idx = g.permutation(n)[: n // 2]
    R0, t0 = _rot([0.2, 1.0, 0.4], 0.5), np.array([0.3, -0.2, 0.15])
    # Y with R0 y + t0 = X[idx]
    Y = ((X[idx].astype(np.float64) - t0) @ R0).astype(np.float32)
    return X, Y, idx


def _run(X, Y, warm, history=True):
    import torch

    from paper_2601_17196_amd import pot
    n, m = len(X), len(Y)
    x = torch.from_numpy(X).cuda()
    y = torch.from_numpy(Y).cuda()
    r = torch.full((n,), 1.0 / n, dtype=torch.float64, device="cuda")
    c = torch.full((m,), 1.0 / m, dtype=torch.float64, device="cuda")
    s = 0.4 * min(n, m) / max(n, m)
    out = pot.register(x, y, r, c, s, eps=1e-2, gamma0=4.4e-3, anneal=0.83, tol=1e-5, max_steps=40, warm=warm,
                       history=history)
    torch.cuda.synchronize()
    return out, s


def test_registration_aligns_and_every_step_matches_the_oracle():
    X, Y, idx = _clouds()
    n, m = len(X), len(Y)
    out, s = _run(X, Y, warm=True)
    print(f"registration: {out.steps} steps, iterations {list(out.iters)}", flush=True)
    assert out.status == 0
    moved = G.apply(out.R, out.t, Y.astype(np.float64))
    err = np.max(np.abs(moved - X[idx]))
    extent = np.max(X.max(0) - X.min(0))
    print(f"alignment error {err:.3e} (extent {extent:.2f})", flush=True)
    assert err <= 1e-2 * extent
    r = np.full(n, 1.0 / n)
    c = np.full(m, 1.0 / m)
    Xd = X.astype(np.float64)
    yh = out.y_hist.cpu().numpy().astype(np.float64)
    dh = out.dual_hist.cpu().numpy()
    # the cost scale the library fixed at the initial pose
    scale = 1.0 / G.sqeuclid(Xd, Y.astype(np.float64)).max()
    Rprev, tprev = np.eye(3), np.zeros(3)
    for k in range(out.steps):
        gam = out.gammas[k]
        C = scale * G.sqeuclid(Xd, yh[k])
        z0 = None
        if k > 0:
            sc = out.gammas[k - 1] / gam
            z0 = (dh[k - 1, :n] * sc, dh[k - 1, n:n + m] * sc, dh[k - 1, n + m] * sc)
        ref = O.solve(C, r, c, s, 1e-2, algo="aspot", cmax=float(C.max()), gamma=gam, z0=z0)
        u, v, w = dh[k, :n], dh[k, n:n + m], dh[k, n + m]
        g0, tol, M, rt, ct_ = O.setup(r, c, s, 1e-2, cmax=float(C.max()), gamma=gam)
        if out.iters[k] == ref.iters:
            tally("strict", f"register step {k}")
            assert rel(out.costs[k], ref.rounded["cost"]) <= 1e-6, (k, out.costs[k], ref.rounded["cost"])
        else:
            tally("def1", f"register step {k} ({out.iters[k]} vs {ref.iters} iterations)")
            E = O.error(C, gam, rt, ct_, s, u, v, w)
            amax = 1.4426950408889634 * (np.max(np.abs(u + w)) + np.max(np.abs(v)))
            assert E <= tol + e_bar("points", s, gamma=gam, amax=amax), (k, E, tol)
        # the oracle's rounding of the GPU's duals: the GPU's cost, and the map update
        rd = O.round_plan(C, gam, u + w, v, r, c, s, dense=True)
        assert rel(out.costs[k], rd["cost"]) <= 1e-9, (k, out.costs[k], rd["cost"])
        dR, dt = G.procrustes(Xd, yh[k], rd["X"])
        Rk, tk = dR @ Rprev, dR @ tprev + dt
        assert np.max(np.abs(Rk - out.Rt[k, :9].reshape(3, 3))) <= 1e-9, k
        assert np.max(np.abs(tk - out.Rt[k, 9:])) <= 1e-9, k
        Rprev, tprev = out.Rt[k, :9].reshape(3, 3), out.Rt[k, 9:]


def test_warm_starts_save_iterations():
    X, Y, idx = _clouds(seed=5)
    warm, _ = _run(X, Y, warm=True, history=False)
    cold, _ = _run(X, Y, warm=False, history=False)
    print(f"iterations warm {warm.total_iters} over {warm.steps} registrations, cold {cold.total_iters} over "
          f"{cold.steps}", flush=True)
    assert warm.status == 0 and cold.status == 0
    assert warm.total_iters < cold.total_iters
    moved = G.apply(warm.R, warm.t, Y.astype(np.float64))
    assert np.max(np.abs(moved - X[idx])) <= 1e-2 * np.max(X.max(0) - X.min(0))


def test_registration_rejects_bad_options():
    import torch

    from paper_2601_17196_amd import pot
    X, Y, _ = _clouds(n=40)
    x, y = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    r = torch.full((40,), 1 / 40, dtype=torch.float64, device="cuda")
    c = torch.full((20,), 1 / 20, dtype=torch.float64, device="cuda")
    for kw in (dict(anneal=1.5), dict(gamma0=0.0), dict(max_steps=0), dict(tol=0.0)):
        with pytest.raises(pot.PotError):
            pot.register(x, y, r, c, 0.2, **kw)
