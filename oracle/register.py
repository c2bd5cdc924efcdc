"""FP64 CPU oracle of rigid point-cloud registration through POT.

TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this module.  The solver library
never calls it and shares no code with it.

What it computes (Truong et al., "Accelerated Sinkhorn Algorithms for Partial
Optimal Transport", Section 4 "Point Cloud Registration" and the appendix on
its POT formulation): clouds X (n points, fixed) and Y (m points, moved by a
rigid map F(y) = R y + t), uniform masses, transported mass
s = alpha min(n, m) / max(n, m); each registration solves POT between X and
F(Y) with the squared-Euclidean cost (ASPOT, the entropic parameter annealed
by a constant factor per registration), then recovers the rigid map from the
rounded plan by the weighted-barycentre alignment of the appendix.

Readings (where the text is ambiguous):
  * the appendix writes the SVD of X^T pi Y = U S V^T and R = V D U^T; for
    the objective it states, sum pi_ij |x_i - (R y_j + t)|^2, the minimiser
    over SO(3) is R = U D V^T with D = diag(1, 1, det(U V^T)) (the printed
    form is its transpose); the objective decides;
  * the plan of registration k is computed on the current pose F_k(Y); the
    alignment of F_k(Y) to X under that plan gives an increment (dR, dt),
    and F_{k+1} = (dR R_k, dR t_k + dt), the same map as aligning the
    original Y (rotations form a group);
  * gamma is "4.4^-3" in the text, read as 4.4e-3 with the cost normalised
    to max 1 at the initial pose (the scale is then kept fixed), annealed by
    0.83 per registration down to the default gamma of Algorithm 2 at eps;
  * the stopping threshold 1e-5 is read as the relative change of the
    transport cost <C, X> between consecutive registrations;
  * each ASPOT solve is warm-started from the previous registration's duals,
    rescaled to the new gamma (the potentials gamma u, gamma v, gamma w in
    cost units are kept).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import potref


def plan_moments(X, Y, P):
    """Weighted barycentres and centred cross-covariance of a plan P (n x m)
    between rows X (n x 3) and columns Y (m x 3): u_x = sum_i (P 1)_i x_i / |P|,
    u_y = sum_j (P^T 1)_j y_j / |P|, H = sum_ij P_ij (x_i - u_x)(y_j - u_y)^T."""
    P = np.asarray(P, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    tot = P.sum()
    ux = (P.sum(1) @ X) / tot
    uy = (P.sum(0) @ Y) / tot
    Xc = X - ux
    Yc = Y - uy
    H = Xc.T @ P @ Yc
    return ux, uy, H, tot


def procrustes(X, Y, P):
    """The rigid map (R, t) minimising sum_ij P_ij |x_i - (R y_j + t)|^2 over
    R in SO(3), t in R^3 (appendix: weighted barycentres, SVD of the centred
    cross-covariance, determinant correction, t = u_x - R u_y)."""
    ux, uy, H, _ = plan_moments(X, Y, P)
    U, S, Vt = np.linalg.svd(H)
    D = np.diag([1.0, 1.0, np.sign(np.linalg.det(U @ Vt)) or 1.0])
    R = U @ D @ Vt
    t = ux - R @ uy
    return R, t


def sqeuclid(X, Y):
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    D = np.zeros((X.shape[0], Y.shape[0]))
    for k in range(X.shape[1]):
        diff = X[:, k:k + 1] - Y[None, :, k]
        D += diff * diff
    return D


def apply(R, t, Y):
    """F(Y) = R y + t for every row, in FP64."""
    return np.asarray(Y, dtype=np.float64) @ np.asarray(R).T + np.asarray(t)


@dataclasses.dataclass
class RegistrationStep:
    gamma: float
    iters: int
    cost: float          # <C_k, Xbar_k> with C_k the scaled cost at the pose of this registration
    R: np.ndarray        # pose after this registration
    t: np.ndarray
    duals: tuple         # (u, v, w) of the solve


def register(X, Y, r, c, s, eps=1e-2, gamma0=4.4e-3, anneal=0.83, max_steps=60, tol=1e-5, cost_scale=None,
             warm=True, R0=None, t0=None):
    """The registration loop: per registration, POT between X and F_k(Y)
    (ASPOT, gamma_k = max(gamma0 anneal^k, eps / (4 ln max(n, m))), warm
    start from the previous duals in cost units), Procrustes on the rounded
    plan, composition of the maps; stop when the transport cost changes by
    less than tol relative.  Y is passed through FP32 after each map (the
    precision in which the clouds are stored).  Returns (R, t, steps)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    n, m = X.shape[0], Y.shape[0]
    R = np.eye(3) if R0 is None else np.asarray(R0, dtype=np.float64)
    t = np.zeros(3) if t0 is None else np.asarray(t0, dtype=np.float64)
    if cost_scale is None:
        cost_scale = 1.0 / sqeuclid(X, apply(R, t, Y).astype(np.float32)).max()
    gfloor = eps / (4.0 * np.log(max(n, m)))
    steps = []
    prev = None
    for k in range(max_steps):
        Yk = apply(R, t, Y).astype(np.float32).astype(np.float64)
        C = cost_scale * sqeuclid(X, Yk)
        gam = max(gamma0 * anneal ** k, gfloor)
        z0 = None
        if warm and prev is not None:
            sc = prev.gamma / gam
            z0 = (prev.duals[0] * sc, prev.duals[1] * sc, prev.duals[2] * sc)
        sol = potref.solve(C, r, c, s, eps, algo="aspot", cmax=float(C.max()), gamma=gam, z0=z0, dense=True)
        P = sol.rounded["X"]
        dR, dt = procrustes(X, Yk, P)
        R = dR @ R
        t = dR @ t + dt
        step = RegistrationStep(gamma=gam, iters=sol.iters, cost=sol.rounded["cost"], R=R.copy(), t=t.copy(),
                                duals=(sol.u, sol.v, sol.w))
        steps.append(step)
        if prev is not None and abs(step.cost - prev.cost) <= tol * abs(prev.cost):
            break
        prev = step
    return R, t, steps
