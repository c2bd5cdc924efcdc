"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check is an exact LP
optimum, an independent solver, a textbook routine, a closed form, or an
identity stated in the paper's proofs.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize
from scipy.special import logsumexp

from paper_2601_17196_amd import instances as I
from tests.lp_pot import assignment_brute_force, dual_lower_bound, extended_ot_lp, in_polytope, pot_lp


def _tiny(n, m, seed, mass_r=1.0, mass_c=1.2, s_frac=0.8, dirichlet=1.0, d=2):
    inst = I.uniform_pair(n, m, d, seed, mass_r=mass_r, mass_c=mass_c, s_frac=s_frac,
                          dirichlet=dirichlet)
    return inst.C64, inst.r, inst.c, inst.s


# ---------------------------------------------------------------------------
# The exact LP and the reduction to extended OT (appendix, LP form and
# "Reduction to Extended OT"): the two LPs agree, which pins the helper.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(6))
def test_lp_helpers_agree(seed):
    n, m = 3 + seed % 4, 2 + (seed * 5) % 6
    C, r, c, s = _tiny(n, m, seed)
    v1, X = pot_lp(C, r, c, s)
    v2 = extended_ot_lp(C, r, c, s)
    assert abs(v1 - v2) <= 1e-9
    assert in_polytope(X, r, c, s, rtol=1e-8)


# The weak-duality bound used to certify Definition 1 where no LP can be
# solved: exact at the LP's own optimal duals, never above the optimum for any
# duals, the same whether C comes whole or by rows, and within eps of the
# rounded plan's cost at the entropic duals of a converged ASPOT solve.
@pytest.mark.parametrize("seed", range(6))
def test_dual_lower_bound(oracle, seed):
    n, m = 3 + seed % 5, 4 + (seed * 3) % 5
    C, r, c, s = _tiny(n, m, seed)
    v, X, (al, be, lam) = pot_lp(C, r, c, s, duals=True)
    assert abs(dual_lower_bound(C, r, c, s, be, lam) - v) <= 1e-9
    rng = np.random.default_rng(seed)
    for _ in range(5):
        b = rng.normal(0.0, 0.5, m)
        la = float(rng.normal(0.0, 0.5))
        lb = dual_lower_bound(C, r, c, s, b, la)
        assert lb <= v + 1e-12
        assert lb == dual_lower_bound(lambda i0, i1: C[i0:i1], r, c, s, b, la, chunk=2)
    sol = oracle.solve(C, r, c, s, 1e-2, algo="aspot", cmax=float(C.max()))
    lb = dual_lower_bound(C, r, c, s, sol.gamma * sol.v, sol.gamma * sol.w)
    assert lb <= v + 1e-12
    assert sol.rounded["cost"] - lb <= 1e-2


# ---------------------------------------------------------------------------
# Definition 1: the rounded plan is an eps-approximation of POT(r, c, s).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("algo", ["aspot", "sinkhorn"])
@pytest.mark.parametrize("seed", range(8))
def test_eps_approximation_vs_exact_lp(oracle, algo, seed):
    rng = np.random.default_rng(seed)
    n, m = int(rng.integers(2, 9)), int(rng.integers(2, 9))
    mass_r = float(rng.uniform(0.6, 1.4))
    mass_c = float(rng.uniform(0.6, 1.4))
    C, r, c, s = _tiny(n, m, 10 + seed, mass_r=mass_r, mass_c=mass_c,
                       s_frac=float(rng.uniform(0.3, 0.95)))
    lp, _ = pot_lp(C, r, c, s)
    for eps in (1e-2, 2e-3):
        try:
            sol = oracle.solve(C, r, c, s, eps, algo=algo, cmax=float(C.max()), dense=True,
                               max_iter=200000)
        except ValueError:
            # eps~ capped to 0 (s equal to a mass above 1): rejected by design
            continue
        assert sol.status == 0
        X = sol.rounded["X"]
        assert in_polytope(X, r, c, s)
        val = float(np.sum(C * X))
        assert val >= lp - 1e-9
        assert val - lp <= eps, (val, lp, eps)


def test_eps_approximation_dirichlet_half(oracle):
    """Sparse-ish Dirichlet(0.5) masses (many near-zero entries)."""
    for seed in range(4):
        C, r, c, s = _tiny(7, 5, 40 + seed, mass_r=0.9, mass_c=1.1, s_frac=0.7, dirichlet=0.5)
        lp, _ = pot_lp(C, r, c, s)
        for algo in ("aspot", "sinkhorn"):
            sol = oracle.solve(C, r, c, s, 1e-2, algo=algo, cmax=float(C.max()), dense=True)
            X = sol.rounded["X"]
            assert in_polytope(X, r, c, s)
            assert 0.0 <= float(np.sum(C * X)) - lp + 1e-9 <= 1e-2


# ---------------------------------------------------------------------------
# The entropic problem solved by an independent primal method.  The dual of
# Section 2.1 is the Lagrange dual of
#   min_{X, p, q >= 0} sum X (C/gamma + log X - 1) + sum p (log p - 1) + sum q (log q - 1)
#   s.t. X 1 + p = r~, X^T 1 + q = c~, 1^T X 1 = s,
# with p = e^u, q = e^v and X = B(z).  SLSQP on this primal (no use of phi)
# must find the plan ASPOT converges to, and strong duality ties the values.
# ---------------------------------------------------------------------------
def _primal_value(C, gamma, X, p, q):
    def h(x):
        x = np.asarray(x)
        return float(np.sum(np.where(x > 0, x * (np.log(np.where(x > 0, x, 1.0)) - 1.0), 0.0)))
    return float(np.sum(C * X)) / gamma + h(X) + h(p) + h(q)


def _slsqp_primal(C, gamma, rt, ct_, s):
    n, m = C.shape
    nv = n * m + n + m

    def f(x):
        X = x[:n * m]
        return float(np.sum(C.ravel() * X) / gamma + np.sum(x * (np.log(x) - 1.0)))

    def grad(x):
        g = np.log(x)
        g[:n * m] += C.ravel() / gamma
        return g

    cons = []
    for i in range(n):
        a = np.zeros(nv)
        a[i * m:(i + 1) * m] = 1.0
        a[n * m + i] = 1.0
        cons.append({"type": "eq", "fun": (lambda x, a=a, b=rt[i]: a @ x - b), "jac": (lambda x, a=a: a)})
    for j in range(m):
        a = np.zeros(nv)
        a[j:n * m:m] = 1.0
        a[n * m + n + j] = 1.0
        cons.append({"type": "eq", "fun": (lambda x, a=a, b=ct_[j]: a @ x - b), "jac": (lambda x, a=a: a)})
    a = np.zeros(nv)
    a[:n * m] = 1.0
    cons.append({"type": "eq", "fun": (lambda x, a=a: a @ x - s), "jac": (lambda x, a=a: a)})
    x0 = np.full(nv, 0.5 * s / (n * m))
    x0[n * m:n * m + n] = np.maximum(rt - s / n, 1e-3) * 0.5 + 1e-3
    x0[n * m + n:] = np.maximum(ct_ - s / m, 1e-3) * 0.5 + 1e-3
    res = minimize(f, x0, jac=grad, constraints=cons, bounds=[(1e-12, None)] * nv,
                   method="SLSQP", options={"ftol": 1e-15, "maxiter": 2000})
    return res.x[:n * m].reshape(n, m), res.x[n * m:n * m + n], res.x[n * m + n:], res


@pytest.mark.parametrize("seed,n,m,gamma", [(0, 3, 2, 0.2), (1, 2, 3, 0.1), (2, 3, 3, 0.15)])
def test_entropic_optimum_vs_independent_primal(oracle, seed, n, m, gamma):
    C, r, c, s = _tiny(n, m, 70 + seed, mass_r=1.0, mass_c=1.1, s_frac=0.7)
    _, tol, M, rt, ct_ = oracle.setup(r, c, s, 1e-2, cmax=float(C.max()), gamma=gamma)
    u, v, w, it, E, st, _ = oracle.aspot(C, gamma, 1e-13, rt, ct_, s, M, max_iter=200000)
    assert st == 0
    B = np.exp(u[:, None] + v[None, :] + w - C / gamma)
    Xp, pp, qq, res = _slsqp_primal(C, gamma, rt, ct_, s)
    assert res.success, res.message
    assert np.max(np.abs(B - Xp)) <= 2e-6
    assert np.max(np.abs(np.exp(u) - pp)) <= 2e-6
    assert np.max(np.abs(np.exp(v) - qq)) <= 2e-6
    # strong duality: primal value at (B, e^u, e^v) equals -phi(z*)
    ph = oracle.phi(C, gamma, rt, ct_, s, u, v, w)
    pv = _primal_value(C, gamma, B, np.exp(u), np.exp(v))
    assert abs(pv + ph) <= 1e-9 * max(1.0, abs(ph))


# ---------------------------------------------------------------------------
# Algorithm 1: each block step is the exact minimiser of phi over that block
# (zero partial derivatives by central differences of phi's definition), and
# the decrease of phi equals the block's score (proof of Theorem 3).
# ---------------------------------------------------------------------------
def _rand_point(rng, n, m, scale=1.0):
    return rng.normal(0, scale, n) - 2.0, rng.normal(0, scale, m) - 2.0, float(rng.normal(0, 0.5))


@pytest.mark.parametrize("block", [0, 1, 2])
def test_greenkhorn_block_is_exact_minimiser(oracle, block):
    rng = np.random.default_rng(block)
    C, r, c, s = _tiny(4, 3, 90 + block)
    gamma = 0.3
    _, _, _, rt, ct_ = oracle.setup(r, c, s, 1e-2, cmax=float(C.max()), gamma=gamma)
    u, v, w = _rand_point(rng, 4, 3)
    u1, v1, w1, b, _ = oracle.greenkhorn(C, gamma, rt, ct_, s, u, v, w, block=block)
    assert b == block
    h = 1e-5

    def ph(uu, vv, ww):
        return oracle.phi(C, gamma, rt, ct_, s, uu, vv, ww)

    if block == 0:
        for i in range(4):
            e = np.zeros(4)
            e[i] = h
            d = (ph(u1 + e, v1, w1) - ph(u1 - e, v1, w1)) / (2 * h)
            assert abs(d) <= 1e-8
    elif block == 1:
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            d = (ph(u1, v1 + e, w1) - ph(u1, v1 - e, w1)) / (2 * h)
            assert abs(d) <= 1e-8
    else:
        d = (ph(u1, v1, w1 + h) - ph(u1, v1, w1 - h)) / (2 * h)
        assert abs(d) <= 1e-8
    # only the chosen block moved
    assert np.array_equal(u1, u) or block == 0
    assert np.array_equal(v1, v) or block == 1
    assert w1 == w or block == 2


@pytest.mark.parametrize("seed", range(5))
def test_greenkhorn_decrease_equals_score(oracle, seed):
    rng = np.random.default_rng(100 + seed)
    n, m = int(rng.integers(2, 12)), int(rng.integers(2, 12))
    C, r, c, s = _tiny(n, m, 100 + seed)
    gamma = float(rng.uniform(0.01, 0.5))
    _, _, _, rt, ct_ = oracle.setup(r, c, s, 1e-2, cmax=float(C.max()), gamma=gamma)
    u, v, w = _rand_point(rng, n, m)
    ph0 = oracle.phi(C, gamma, rt, ct_, s, u, v, w)
    for block in range(3):
        u1, v1, w1, _, sc = oracle.greenkhorn(C, gamma, rt, ct_, s, u, v, w, block=block)
        ph1 = oracle.phi(C, gamma, rt, ct_, s, u1, v1, w1)
        assert abs((ph0 - ph1) - sc[block]) <= 1e-10 * max(1.0, abs(ph0))
    # greedy picks the largest score, ties u < v < w
    _, _, _, b, sc = oracle.greenkhorn(C, gamma, rt, ct_, s, u, v, w, block=-1)
    assert b == int(np.argmax(sc))


# ---------------------------------------------------------------------------
# Algorithm 2 loop: invariants from the proofs of Lemma 1, Lemma 2, Theorem 3.
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c1_aspot_trace(oracle):
    inst = I.c1(0)
    C = inst.C32.astype(np.float64)
    gamma, tol, M, rt, ct_ = oracle.setup(inst.r, inst.c, inst.s, inst.eps, cmax=1.0)
    out = oracle.aspot(C, gamma, tol, rt, ct_, inst.s, M, max_iter=20000, trace=True)
    return inst, C, gamma, tol, M, rt, ct_, out


def test_aspot_monotone_chain(c1_aspot_trace):
    *_, out = c1_aspot_trace
    tr = out[6]
    k = out[3]
    assert out[5] == 0 and k > 10
    rel = 1e-12
    for t in range(k):
        sc = rel * max(1.0, abs(tr.phigrave[t]))
        assert tr.phihat[t] <= tr.phigrave[t] + sc      # phi(z-grave) >= phi(z-hat)
        assert tr.phiz[t] <= tr.phihat[t] + sc          # phi(z-hat) >= phi(z^t)
        assert tr.phiz[t] <= tr.phichk[t] + sc          # argmin keeps the smaller value
        if t + 1 < k:
            assert tr.phinext[t] <= tr.phiz[t] + sc     # phi(z^t) >= phi(z-check^{t+1})
            assert tr.phichk[t + 1] == tr.phinext[t]


def test_aspot_theta_recursion(c1_aspot_trace):
    *_, out = c1_aspot_trace
    th = out[6].theta
    assert th[0] == 1.0
    for t in range(len(th) - 1):
        assert abs(th[t + 1] / th[t] - math.sqrt(1.0 - th[t + 1])) <= 1e-13  # Lemma 2 proof
        assert th[t] <= 2.0 / (t + 2) + 1e-15                                  # theta_t <= 2/(t+2)


def test_aspot_descent_lemma(c1_aspot_trace):
    """phi(z-grave) <= phi(zbar) + theta (z~'-z~)^T grad + L/2 theta^2 |z~'-z~|^2
    with L = 3 M / gamma (Lemma 1 and its proof), which checks that z-grave is
    the printed combination of zbar and the two z~ iterates."""
    inst, C, gamma, tol, M, rt, ct_, out = c1_aspot_trace
    tr = out[6]
    L = 3.0 * M / gamma
    for t in range(out[3]):
        rhs = tr.phibar[t] + tr.gdot[t] + 0.5 * L * tr.theta[t] ** 2 * tr.step2[t]
        assert tr.phigrave[t] <= rhs + 1e-12 * max(1.0, abs(rhs))


def _fd_grad(oracle, C, gamma, rt, ct_, s, u, v, w, h=1e-6):
    """Central-difference gradient of phi (from its definition)."""
    def ph(uu, vv, ww):
        return oracle.phi(C, gamma, rt, ct_, s, uu, vv, ww)
    gu = np.empty_like(u)
    gv = np.empty_like(v)
    for i in range(len(u)):
        e = np.zeros_like(u)
        e[i] = h
        gu[i] = (ph(u + e, v, w) - ph(u - e, v, w)) / (2 * h)
    for j in range(len(v)):
        e = np.zeros_like(v)
        e[j] = h
        gv[j] = (ph(u, v + e, w) - ph(u, v - e, w)) / (2 * h)
    gw = (ph(u, v, w + h) - ph(u, v, w - h)) / (2 * h)
    return gu, gv, gw


@pytest.mark.parametrize("step_rule", [0, 1])
def test_aspot_first_iterations_special_case(oracle, step_rule):
    """With theta_0 = 1 and z~^0 = z-check^0 = 0, zbar^0 = 0 and z-grave^0 =
    z~^1 is a plain gradient step from 0 of length gamma/(3M) (printed rule)
    or 1/(3M) (mirror rule).  The gradient here comes from central
    differences of phi, the block step from the pinned Greenkhorn step;
    zbar^1 = (1 - theta_1) z-check^1 + theta_1 z~^1 with theta_1 = (sqrt5 - 1)/2."""
    C, r, c, s = _tiny(6, 5, 77, mass_r=1.0, mass_c=1.2, s_frac=0.8)
    gamma = 0.05
    _, tol, M, rt, ct_ = oracle.setup(r, c, s, 1e-2, cmax=float(C.max()), gamma=gamma)
    *_, tr = oracle.aspot(C, gamma, 1e-300, rt, ct_, s, M, max_iter=3, step_rule=step_rule,
                          trace=True)
    n, m = C.shape
    z0 = (np.zeros(n), np.zeros(m), 0.0)
    eta = (gamma if step_rule == 0 else 1.0) / (3.0 * M)
    gu, gv, gw = _fd_grad(oracle, C, gamma, rt, ct_, s, *z0)
    ug, vg, wg = -eta * gu, -eta * gv, -eta * gw
    tol_phi = 1e-7
    assert abs(tr.phibar[0] - oracle.phi(C, gamma, rt, ct_, s, *z0)) <= 1e-12
    assert abs(tr.phigrave[0] - oracle.phi(C, gamma, rt, ct_, s, ug, vg, wg)) <= tol_phi
    uh, vh, wh, bh, _ = oracle.greenkhorn(C, gamma, rt, ct_, s, ug, vg, wg)
    assert bh == tr.bhat[0]
    assert abs(tr.phihat[0] - oracle.phi(C, gamma, rt, ct_, s, uh, vh, wh)) <= tol_phi
    z = (uh, vh, wh) if tr.pick[0] == 1 else z0
    uc, vc, wc, bc, _ = oracle.greenkhorn(C, gamma, rt, ct_, s, *z)
    assert bc == tr.bchk[0]
    th1 = (math.sqrt(5.0) - 1.0) / 2.0
    assert abs(tr.theta[1] - th1) <= 1e-15
    ub = (1 - th1) * uc + th1 * ug
    vb = (1 - th1) * vc + th1 * vg
    wb = (1 - th1) * wc + th1 * wg
    assert abs(tr.phibar[1] - oracle.phi(C, gamma, rt, ct_, s, ub, vb, wb)) <= tol_phi


def test_aspot_stop_rule_and_bound(c1_aspot_trace):
    """E(z^t) > eps~ before the last iteration and <= eps~ at it; the count is
    within the Theorem 3 bound t <= 1 + (12 sqrt(14 n L) R / eps')^(2/3)."""
    inst, C, gamma, tol, M, rt, ct_, out = c1_aspot_trace
    tr = out[6]
    k = out[3]
    assert np.all(tr.E[:-1] > tol) and tr.E[-1] <= tol
    n = inst.n
    L = 3.0 * M / gamma
    mx = max(inst.r.sum(), inst.c.sum())
    R = 1.0 * mx / (gamma * (mx - inst.s)) - math.log(min(inst.r.min(), inst.c.min()))
    bound = 1.0 + (12.0 * math.sqrt(14.0 * n * L) * R / tol) ** (2.0 / 3.0)
    assert k <= bound


def test_aspot_final_point_error_matches_definition(oracle, c1_aspot_trace):
    inst, C, gamma, tol, M, rt, ct_, out = c1_aspot_trace
    u, v, w = out[0], out[1], out[2]
    lR, lQ, lT = oracle.stats(C, gamma, u, v, w)
    # E computed here from scipy's logsumexp on the dense exponent matrix
    X = u[:, None] + v[None, :] + w - C / gamma
    R = np.exp(logsumexp(X, axis=1))
    Q = np.exp(logsumexp(X, axis=0))
    T = np.exp(logsumexp(X))
    E = abs(T - inst.s) + np.abs(R + np.exp(u) - rt).sum() + np.abs(Q + np.exp(v) - ct_).sum()
    assert abs(E - out[4]) <= 1e-12
    assert np.allclose(lR, np.log(R), rtol=0, atol=1e-12)
    assert np.allclose(lQ, np.log(Q), rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# ASPOT and extended Sinkhorn target the same entropic plan: with A/gamma
# large the corner entry is 0 and the extended OT is POT with slack entropy
# (appendix, "Reduction to Extended OT").  Map: u_i = a_i + b_{m+1},
# v_j = a_{n+1} + b_j, w = -(a_{n+1} + b_{m+1}).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(3))
def test_aspot_and_extended_sinkhorn_same_fixed_point(oracle, seed):
    C, r, c, s = _tiny(9, 7, 200 + seed, mass_r=1.0, mass_c=1.3, s_frac=0.75)
    gamma = 0.05
    _, _, M, rt, ct_ = oracle.setup(r, c, s, 1e-2, cmax=float(C.max()), gamma=gamma)
    u, v, w, it1, E1, st1, _ = oracle.aspot(C, gamma, 1e-12, rt, ct_, s, M, max_iter=500000)
    a, b, it2, E2, st2, _ = oracle.sinkhorn(C, gamma, 1e-12, rt, ct_, s, A=8.0 / 1e-2,
                                            max_iter=500000)
    assert st1 == 0 and st2 == 0
    Xa = np.exp(u[:, None] + v[None, :] + w - C / gamma)
    Xs = np.exp(a[:-1, None] + b[None, :-1] - C / gamma)
    assert np.max(np.abs(Xa - Xs)) <= 1e-9
    assert np.max(np.abs(np.exp(u) - np.exp(a[:-1] + b[-1]))) <= 1e-9
    assert np.max(np.abs(np.exp(v) - np.exp(a[-1] + b[:-1]))) <= 1e-9


# ---------------------------------------------------------------------------
# Balanced special case |r|_1 = |c|_1 = s = 1: the dummy masses vanish and
# Algorithm 3 is textbook log-domain Sinkhorn on (C, r~, c~); the rounding is
# the rounding of Altschuler, Weed and Rigollet (2017, Algorithm 2); uniform
# masses give an assignment problem solvable by brute force.
# ---------------------------------------------------------------------------
def _textbook_log_sinkhorn(C, gamma, a_marg, b_marg, iters):
    f = np.zeros(C.shape[0])
    g = np.zeros(C.shape[1])
    K = -C / gamma
    for _ in range(iters):
        f = np.log(a_marg) - logsumexp(K + g[None, :], axis=1)
        g = np.log(b_marg) - logsumexp(K + f[:, None], axis=0)
    return f, g


def _altschuler_round(F, r, c):
    F = F.copy()
    x = np.minimum(r / F.sum(1), 1.0)
    F = x[:, None] * F
    y = np.minimum(c / F.sum(0), 1.0)
    F = F * y[None, :]
    er = r - F.sum(1)
    ec = c - F.sum(0)
    return F + np.outer(er, ec) / np.abs(er).sum()


@pytest.mark.parametrize("seed", range(3))
def test_balanced_sinkhorn_is_textbook(oracle, seed):
    C, r, c, s = _tiny(6, 6, 300 + seed, mass_r=1.0, mass_c=1.0, s_frac=1.0)
    r = r / r.sum()
    c = c / c.sum()
    s = min(r.sum(), c.sum())
    gamma = 0.05
    _, _, _, rt, ct_ = oracle.setup(r, c, s, 1e-2, cmax=float(C.max()), gamma=gamma)
    a, b, it, err, st, _ = oracle.sinkhorn(C, gamma, 1e-13, rt, ct_, s, A=800.0, max_iter=100000)
    assert st == 0
    # dummy masses are 0 up to rounding of the smoothed sums: no dummy flow
    assert np.exp(a[-1]) <= 1e-14 and np.exp(b[-1]) <= 1e-14
    f, g = _textbook_log_sinkhorn(C, gamma, rt, ct_, 4 * it)
    # potentials agree up to the gauge (a + k, b - k); the plans agree
    Xo = np.exp(a[:-1, None] + b[None, :-1] - C / gamma)
    Xt = np.exp(f[:, None] + g[None, :] - C / gamma)
    assert np.max(np.abs(Xo - Xt)) <= 1e-12
    d = a[:-1] - f
    assert np.ptp(d) <= 1e-9


@pytest.mark.parametrize("seed", range(4))
def test_balanced_rounding_is_altschuler(oracle, seed):
    rng = np.random.default_rng(400 + seed)
    n = 7
    r = rng.dirichlet(np.ones(n))
    c = rng.dirichlet(np.ones(n))
    F = rng.uniform(0, 1, (n, n)) * rng.uniform(0, 2) / n
    X = oracle.round_dense(F, r, c, 1.0)
    Y = _altschuler_round(F, r, c)
    assert np.max(np.abs(X - Y)) <= 1e-14


@pytest.mark.parametrize("n", [3, 4, 5, 6])
def test_balanced_uniform_assignment(oracle, n):
    inst = I.uniform_pair(n, n, 2, 500 + n)
    C = inst.C64
    r = np.full(n, 1.0 / n)
    c = np.full(n, 1.0 / n)
    s = min(r.sum(), c.sum())   # 1 up to rounding of the sum of n copies of 1/n
    opt = assignment_brute_force(C)
    lp, _ = pot_lp(C, r, c, s)
    assert abs(opt - lp) <= 1e-9
    for algo in ("aspot", "sinkhorn"):
        sol = oracle.solve(C, r, c, s, 1e-2, algo=algo, cmax=float(C.max()), dense=True)
        X = sol.rounded["X"]
        assert in_polytope(X, r, c, s)
        assert 0.0 <= float(np.sum(C * X)) - opt + 1e-12 <= 1e-2


# ---------------------------------------------------------------------------
# Setup of Algorithm 2: the cap on eps~ is exactly the point where the
# smoothed mass |c~|_1 falls to s (so the extended marginal |c~|_1 - s >= 0).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,m", [(10, 10), (10, 13), (17, 6)])
def test_setup_cap_keeps_extension_nonnegative(oracle, n, m):
    r = np.full(n, 1.0 / n)
    c = np.full(m, 1.3 / m)   # |c|_1 = 1.3
    s = 1.0 - 1e-6         # cap 8 (1.3 - s)/0.3 ~ 8 binds only when eps/8 exceeds it
    for eps in (1e-2, 10.0, 100.0):
        gamma, tol, M, rt, ct_ = oracle.setup(r, c, s, eps, cmax=1.0)
        cap = 8.0 * (c.sum() - s) / (c.sum() - 1.0)
        assert tol == pytest.approx(min(eps / 8.0, cap), rel=1e-15)
        assert ct_.sum() - s >= -1e-15
        if eps / 8.0 > cap:
            assert abs(ct_.sum() - s) <= 1e-14
        assert rt.sum() - s >= -1e-15
        assert gamma == pytest.approx(eps / (4 * math.log(max(n, m))), rel=1e-15)
        assert M == pytest.approx(r.sum() + c.sum() - s, rel=1e-15)


def test_setup_rejects_bad_arguments(oracle):
    r = np.full(4, 0.25)
    c = np.full(4, 0.25)
    with pytest.raises(ValueError):
        oracle.setup(r, c, 1.5, 1e-2)          # s > min mass
    with pytest.raises(ValueError):
        oracle.setup(r, c, 0.5, -1.0)          # eps <= 0
    with pytest.raises(ValueError):
        oracle.setup(-r, c, 0.5, 1e-2)         # negative mass
    with pytest.raises(ValueError):
        oracle.setup(np.ones(1), np.ones(1), 0.5, 1e-2)   # ln 1 = 0 without a user gamma
    r2 = np.full(4, 0.5)                       # |r|_1 = 2 = s: eps~ capped to 0
    with pytest.raises(ValueError):
        oracle.setup(r2, r2, 2.0, 1e-2)


# ---------------------------------------------------------------------------
# Closed forms.
# ---------------------------------------------------------------------------
def test_single_point(oracle):
    C = np.array([[0.37]])
    r = np.array([0.9])
    c = np.array([1.4])
    sol = oracle.solve(C, r, c, 0.6, 1e-2, algo="aspot", cmax=1.0, gamma=1e-2, dense=True)
    assert sol.rounded["X"][0, 0] == pytest.approx(0.6, rel=1e-14)
    assert sol.rounded["cost"] == pytest.approx(0.37 * 0.6, rel=1e-14)


@pytest.mark.parametrize("algo", ["aspot", "sinkhorn"])
def test_constant_cost(oracle, algo):
    n, m, kap = 6, 9, 0.42
    C = np.full((n, m), kap)
    rng = np.random.default_rng(7)
    r = rng.dirichlet(np.ones(n)) * 0.9
    c = rng.dirichlet(np.ones(m)) * 1.1
    s = 0.5
    sol = oracle.solve(C, r, c, s, 1e-2, algo=algo, cmax=kap, dense=True)
    assert in_polytope(sol.rounded["X"], r, c, s)
    assert sol.rounded["cost"] == pytest.approx(kap * s, rel=1e-13)


@pytest.mark.parametrize("algo", ["aspot", "sinkhorn"])
def test_identical_clouds_zero_optimum(oracle, algo):
    inst = I.uniform_pair(8, 8, 2, 600)
    C, _ = I.sqeuclid_cost(inst.x, inst.x)
    r = np.full(8, 1.0 / 8)
    s = 0.8
    sol = oracle.solve(C, r, r, s, 1e-2, algo=algo, cmax=1.0, dense=True)
    assert in_polytope(sol.rounded["X"], r, r, s)
    assert 0.0 <= sol.rounded["cost"] <= 1e-2


# ---------------------------------------------------------------------------
# Rounding onto U(r, c, s): feasible for any nonnegative input, the identity
# on feasible plans.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(20))
def test_rounding_feasible_any_input(oracle, seed):
    rng = np.random.default_rng(800 + seed)
    n, m = int(rng.integers(1, 12)), int(rng.integers(1, 12))
    r = rng.dirichlet(np.ones(n)) * rng.uniform(0.3, 2.0)
    c = rng.dirichlet(np.ones(m)) * rng.uniform(0.3, 2.0)
    if seed % 3 == 0:
        r[rng.integers(0, n)] = 0.0
    s = rng.uniform(0.05, 1.0) * min(r.sum(), c.sum())
    X = rng.exponential(1.0, (n, m)) * rng.choice([1e-3, 1.0, 50.0])
    X[rng.uniform(size=(n, m)) < 0.3] = 0.0
    if seed % 4 == 0:
        X[:] = 0.0
        X[0, 0] = 1e-300
    Xb = oracle.round_dense(X, r, c, s)
    assert in_polytope(Xb, r, c, s)


@pytest.mark.parametrize("seed", range(5))
def test_rounding_identity_on_feasible(oracle, seed):
    rng = np.random.default_rng(900 + seed)
    n, m = 5, 7
    r = rng.dirichlet(np.ones(n))
    c = rng.dirichlet(np.ones(m)) * 1.5
    s = 0.6
    _, X = pot_lp(rng.uniform(0, 1, (n, m)), r, c, s)
    X = np.maximum(X, 0)
    X *= s / X.sum()
    Xb = oracle.round_dense(X, r, c, s)
    assert np.max(np.abs(Xb - X)) <= 1e-15


def test_cost_compensated_sum(oracle):
    C = np.ones((3, 4))
    X = np.full((3, 4), 0.1)
    X[0, 0] = 1e16
    X[0, 1] = -1e16
    assert oracle.cost(C, X) == pytest.approx(1.0, rel=1e-12)


# ---------------------------------------------------------------------------
# tuned rule of Algorithm 3 (Theorem 2): gamma = (2 eps / (49 H_min))^(1/p),
# eps' = H_min gamma^p, H_min = min(H(r), H(c))
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("p", [1.0, 2.0, 3.0, 4.5])
def test_tuned_rule_uniform_marginals(oracle, p):
    """Uniform marginals have H = ln n (a closed form, not the code's sum):
    H_min = ln 8 for n = 8 against m = 16; gamma^p 49 H_min / 2 = eps, and
    eps' = 2 eps / 49 whatever p."""
    eps = 1e-2
    g, tol, h = oracle.tuned(np.full(8, 1 / 8), np.full(16, 1 / 16), eps, p)
    assert abs(h - math.log(8)) <= 1e-14
    assert abs(g ** p * 49 * math.log(8) / 2 - eps) <= 1e-13 * eps
    assert abs(tol - 2 * eps / 49) <= 1e-13 * eps


def test_tuned_rule_entropy_conventions(oracle):
    """0 ln 0 = 0: r = (1/2, 1/2, 0) has H = ln 2; the masses enter as given
    (not normalised): n equal masses a give H = -n a ln a; the smaller
    entropy of the two sides is taken."""
    _, _, h = oracle.tuned(np.array([0.5, 0.5, 0.0]), np.full(5, 0.2), 1e-2, 1)
    assert abs(h - math.log(2)) <= 1e-15
    a = 0.3
    _, _, h = oracle.tuned(np.full(4, a), np.full(50, 0.02), 1e-2, 2)
    assert abs(h - (-4 * a * math.log(a))) <= 1e-14
    _, _, h2 = oracle.tuned(np.full(50, 0.02), np.full(4, a), 1e-2, 2)
    assert h2 == h


def test_tuned_rule_rejects(oracle):
    with pytest.raises(ValueError):
        oracle.tuned(np.array([1.0]), np.full(3, 1 / 3), 1e-2, 1)      # H(r) = 0
    with pytest.raises(ValueError):
        oracle.tuned(np.full(3, 1 / 3), np.full(3, 1 / 3), 1e-2, 0.5)  # p < 1
    with pytest.raises(ValueError):
        oracle.solve(np.ones((3, 3)), np.full(3, 1 / 3), np.full(3, 1 / 3), 0.5, 1e-2, algo="aspot",
                     gamma_rule=1, p=2)


@pytest.mark.parametrize("seed", [1, 2])
def test_tuned_sinkhorn_vs_exact_lp(oracle, seed):
    """The tuned Sinkhorn (smoothing and extension as the default feasible
    Sinkhorn, only gamma and the threshold change) returns a feasible plan,
    stops at E <= eps'; for p = 1, 2 it is within eps of the exact LP.
    Larger p needs far fewer iterations (the trend the paper reports)."""
    n, m = (6, 7) if seed == 1 else (8, 8)
    inst = I.uniform_pair(n, m, 2, seed, mass_r=1.0, mass_c=1.2, s_frac=0.8)
    lp = pot_lp(inst.C64, inst.r, inst.c, inst.s)[0]
    iters = []
    for p in (1, 2, 3):
        sol = oracle.solve(inst.C64, inst.r, inst.c, inst.s, inst.eps, algo="sinkhorn", gamma_rule=1, p=p,
                           cmax=1.0, dense=True)
        g, tol, _ = oracle.tuned(inst.r, inst.c, inst.eps, p)
        assert sol.gamma == g and sol.tol == tol and sol.status == 0 and sol.E <= tol
        assert in_polytope(sol.rounded["X"], inst.r, inst.c, inst.s)
        assert sol.rounded["cost"] >= lp - 1e-12
        if p <= 2:
            assert sol.rounded["cost"] - lp <= inst.eps
        iters.append(sol.iters)
    assert iters[0] > iters[1] > iters[2]


# ---------------------------------------------------------------------------
# solver variants (readings 5 and 6): the proof-form step and the cyclic block
# rule also end in eps-approximations; the cyclic rule takes u, v, w in turn
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("variant", [dict(step_rule=1), dict(block_rule=1)])
@pytest.mark.parametrize("seed", range(4))
def test_aspot_variants_vs_exact_lp(oracle, variant, seed):
    rng = np.random.default_rng(100 + seed)
    n, m = int(rng.integers(2, 9)), int(rng.integers(2, 9))
    C, r, c, s = _tiny(n, m, 50 + seed, mass_r=float(rng.uniform(0.6, 1.4)), mass_c=float(rng.uniform(0.6, 1.4)),
                       s_frac=float(rng.uniform(0.3, 0.95)))
    lp, _ = pot_lp(C, r, c, s)
    try:
        sol = oracle.solve(C, r, c, s, 1e-2, algo="aspot", cmax=float(C.max()), dense=True, max_iter=400000,
                           trace=True, **variant)
    except ValueError:
        return                               # eps~ capped to 0: rejected by design
    assert sol.status == 0
    X = sol.rounded["X"]
    assert in_polytope(X, r, c, s)
    val = float(np.sum(C * X))
    assert lp - 1e-9 <= val <= lp + 1e-2
    if variant.get("block_rule") == 1:
        # one counter over both Greenkhorn steps of an iteration: z-hat takes
        # block 2t mod 3, z-check block 2t + 1 mod 3
        it = sol.iters
        bh = np.asarray(sol.trace.bhat[:it])
        bc = np.asarray(sol.trace.bchk[:it - 1])
        assert np.array_equal(bh, (2 * np.arange(it)) % 3)
        assert np.array_equal(bc, (2 * np.arange(it - 1) + 1) % 3)


# ---------------------------------------------------------------------------
# Checks of another solver's output point.  The Sinkhorn stopping error of
# Algorithm 3 at extended scalings (a, b) relates to E(z) of Section 3.1 at
# the ASPOT point of the same plan (appendix, "Reduction to Extended OT"):
# with u_i = a_i + b_{m+1}, v_j = a_{n+1} + b_j, w = -(a_{n+1} + b_{m+1}),
# the real rows and columns of the extended error are E's row and column
# terms, and the dummy row (column) compares sum_j e^{v_j} (sum_i e^{u_i})
# plus the corner entry with |c~|_1 - s (|r~|_1 - s); E's |T - s| term has
# no counterpart.  potref_error and potref_sk_error are separate code.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(4))
def test_sk_error_relates_to_aspot_error(oracle, seed):
    C, r, c, s = _tiny(7, 9, 900 + seed, mass_r=1.1, mass_c=0.9, s_frac=0.7)
    gamma, A = 0.07, 3.0
    _, _, _, rt, ct_ = oracle.setup(r, c, s, 1e-2, cmax=float(C.max()), gamma=gamma)
    g = np.random.default_rng(seed)
    a = g.normal(-1.0, 0.6, 8)
    b = g.normal(-1.5, 0.6, 10)
    u, v, w = a[:-1] + b[-1], a[-1] + b[:-1], -(a[-1] + b[-1])
    E = oracle.error(C, gamma, rt, ct_, s, u, v, w)
    _, _, lT = oracle.stats(C, gamma, u, v, w)
    corner = math.exp(a[-1] + b[-1] - A / gamma)
    dummy = (abs(np.exp(v).sum() + corner - (ct_.sum() - s)) +
             abs(np.exp(u).sum() + corner - (rt.sum() - s)))
    expect = E - abs(math.exp(lT) - s) + dummy
    assert abs(oracle.sk_error(C, gamma, rt, ct_, s, A, a, b) - expect) <= 1e-12 * max(1.0, expect)


def test_sk_error_zero_columns_after_column_update(oracle):
    """At the scalings Algorithm 3 returns, the columns were just fitted: the
    error is the row part alone, and it is the error the loop reported."""
    C, r, c, s = _tiny(8, 6, 950, mass_r=1.0, mass_c=1.2, s_frac=0.8)
    gamma = 0.05
    _, _, _, rt, ct_ = oracle.setup(r, c, s, 1e-2, cmax=float(C.max()), gamma=gamma)
    a, b, it, err, st, _ = oracle.sinkhorn(C, gamma, 1e-6, rt, ct_, s, 8.0 / 1e-2, max_iter=10000)
    assert st == 0
    e = oracle.sk_error(C, gamma, rt, ct_, s, 8.0 / 1e-2, a, b)
    assert abs(e - err) <= 1e-13
    # column marginals exact: moving only the columns' target changes nothing
    Ce = np.zeros((9, 7))
    Ce[:8, :6] = C
    Ce[8, 6] = 8.0 / 1e-2
    X = np.exp(a[:, None] + b[None, :] - Ce / gamma)
    chat = np.concatenate([ct_, [rt.sum() - s]])
    assert np.max(np.abs(X.sum(0) - chat)) <= 1e-14


# A factored plan evaluated entry by entry agrees with the dense rounding of
# the same scalings (potref_round, which forms and rounds the dense matrix):
# row and column sums, mass and cost; priced on another cost, the cost is
# the dense plan's inner product with that cost.
@pytest.mark.parametrize("seed", range(4))
def test_plan_eval_matches_dense_rounding(oracle, seed):
    C, r, c, s = _tiny(11, 8, 970 + seed, mass_r=1.0, mass_c=1.3, s_frac=0.6 + 0.1 * seed)
    gamma = 0.04
    g = np.random.default_rng(seed)
    f = g.normal(-2.0, 0.5, 11)
    gg = g.normal(-2.0, 0.5, 8)
    rd = oracle.round_plan(C, gamma, f, gg, r, c, s, dense=True)
    X = rd["X"]
    Cb = I.bf16_bits_to_f64(I.to_bf16_bits(C.astype(np.float32)))
    pe = oracle.plan_eval(C, gamma, f, gg, rd["alpha"], rd["beta"], rd["kappa"], rd["lam"], rd["pp"],
                          rd["qq"], Ce=Cb)
    assert np.max(np.abs(pe["rows"] - X.sum(1))) <= 1e-15
    assert np.max(np.abs(pe["cols"] - X.sum(0))) <= 1e-15
    assert abs(pe["mass"] - s) <= 1e-14
    assert abs(pe["min"] - X.min()) <= 1e-16
    assert abs(pe["cost"] - float(np.sum(Cb * X))) <= 1e-14
    pe2 = oracle.plan_eval(C, gamma, f, gg, rd["alpha"], rd["beta"], rd["kappa"], rd["lam"], rd["pp"], rd["qq"])
    assert abs(pe2["cost"] - rd["cost"]) <= 1e-14


# ---------------------------------------------------------------------------
# Registration (Section 4 and the appendix's POT formulation): the weighted
# Procrustes step recovers a known rigid map exactly from a matching plan,
# returns a proper rotation even where the unconstrained optimum is a
# reflection, and no other rotation does better on the stated objective.
# ---------------------------------------------------------------------------
def _rot(axis, ang):
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K


def _objective(X, Y, P, R, t):
    from oracle import register as G
    return float(np.sum(P * G.sqeuclid(X, G.apply(R, t, Y))))


@pytest.mark.parametrize("seed", range(4))
def test_procrustes_recovers_a_known_map(seed):
    from oracle import register as G
    g = np.random.default_rng(seed)
    Y = g.normal(size=(40, 3))
    R0 = _rot(g.normal(size=3), g.uniform(0.1, 3.0))
    t0 = g.normal(size=3)
    X = G.apply(R0, t0, Y)
    P = np.diag(g.uniform(0.5, 1.5, 40))          # point i matched to point i, uneven weights
    R, t = G.procrustes(X, Y, P)
    assert np.max(np.abs(R - R0)) <= 1e-12 and np.max(np.abs(t - t0)) <= 1e-12


def test_procrustes_proper_rotation_and_optimal():
    from oracle import register as G
    g = np.random.default_rng(7)
    Y = g.normal(size=(30, 3))
    X = Y * np.array([1.0, 1.0, -1.0])             # a mirror image: the best orthogonal map is a reflection
    P = g.uniform(0.0, 1.0, (30, 30)) * 0.01 + np.eye(30)
    R, t = G.procrustes(X, Y, P)
    assert abs(np.linalg.det(R) - 1.0) <= 1e-12 and np.max(np.abs(R @ R.T - np.eye(3))) <= 1e-12
    best = _objective(X, Y, P, R, t)
    for k in range(200):                           # random proper rotations with their best translations
        Rr = _rot(g.normal(size=3), g.uniform(0, np.pi))
        ux, uy, _, _ = G.plan_moments(X, Y, P)
        assert best <= _objective(X, Y, P, Rr, ux - Rr @ uy) + 1e-12
    # the increment composed onto a pose is the pose that aligns the original cloud
    R1, t1 = _rot([1, 2, 3], 0.4), np.array([0.1, -0.2, 0.3])
    dR, dt = G.procrustes(X, G.apply(R1, t1, Y), P)
    Rd, td = G.procrustes(X, Y, P)
    assert np.max(np.abs(dR @ R1 - Rd)) <= 1e-10 and np.max(np.abs(dR @ t1 + dt - td)) <= 1e-10


def test_registration_loop_aligns_a_partial_copy(oracle):
    """A cloud and a misaligned copy of half of it: the loop recovers the
    map (the copy's points land on their originals) and the transport cost
    falls to about the entropic floor."""
    from oracle import register as G
    g = np.random.default_rng(11)
    X = g.normal(0.0, 0.3, size=(60, 3)) + g.choice([-0.6, 0.6], size=(60, 1)) * np.array([1.0, 0.0, 0.0])
    R0, t0 = _rot([0.3, 1.0, 0.2], 0.35), np.array([0.15, -0.1, 0.05])
    Y = G.apply(R0.T, -R0.T @ t0, X[:30]).astype(np.float32).astype(np.float64)   # X[:30] = R0 y + t0
    r = np.full(60, 1.0 / 60)
    c = np.full(30, 1.0 / 30)
    s = 0.4 * 30 / 60
    R, t, steps = G.register(X, Y, r, c, s, max_steps=40)
    err = np.max(np.abs(G.apply(R, t, Y) - X[:30]))
    assert err <= 0.02, err
    assert steps[-1].cost <= 0.05 * steps[0].cost
