"""Exact LP solutions of tiny POT instances (test helper, independent of the oracle).

Two formulations from the paper's appendix "Reformulating POT as Extended OT":
  * the slack LP: x = (vec X, p, q) >= 0 with X 1 + p = r, X^T 1 + q = c,
    1^T X 1 = s, minimising <C, X>;
  * the extended OT LP on the (n+1) x (m+1) instance with the dummy row and
    column (cost 0) and corner cost A > max C, marginals (r, |c|_1 - s) and
    (c, |r|_1 - s); its optimum equals the POT optimum.
Both are solved with scipy's HiGHS.
"""
import itertools

import numpy as np
import scipy.sparse as sp
from scipy.optimize import linprog


def pot_lp(C, r, c, s, duals=False):
    """Optimum of the slack LP and an optimal plan (and, with duals=True, the
    optimal dual (alpha, beta, lam) of its equality constraints).  The
    constraint matrix is sparse (three nonzeros per plan entry), so instances
    of a few hundred points per side solve in seconds."""
    C = np.asarray(C, dtype=np.float64)
    n, m = C.shape
    nm = n * m
    ii = np.repeat(np.arange(n), m)
    jj = np.tile(np.arange(m), n)
    k = np.arange(nm)
    rows = np.concatenate([ii, n + jj, np.full(nm, n + m), np.arange(n), n + np.arange(m)])
    cols = np.concatenate([k, k, k, nm + np.arange(n), nm + n + np.arange(m)])
    A = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n + m + 1, nm + n + m))
    b = np.concatenate([r, c, [s]])
    d = np.concatenate([C.ravel(), np.zeros(n + m)])
    res = linprog(d, A_eq=A, b_eq=b, bounds=(0, None), method="highs")
    assert res.status == 0, res.message
    if duals:
        y = res.eqlin.marginals
        return float(res.fun), res.x[:nm].reshape(n, m), (y[:n], y[n:n + m], float(y[n + m]))
    return float(res.fun), res.x[:nm].reshape(n, m)


def dual_lower_bound(C, r, c, s, beta, lam, chunk=1024):
    """A lower bound on the POT optimum from any column duals beta (m) and
    mass dual lam, by weak duality for the slack LP.  Its dual is
        max r.alpha + c.beta + s lam
        s.t. alpha_i + beta_j + lam <= C_ij, alpha <= 0, beta <= 0
    (one constraint per plan entry and per slack).  With beta' = min(beta, 0)
    and alpha_i = min(0, min_j (C_ij - beta'_j - lam)) the point is feasible;
    then beta''_j = min(0, min_i (C_ij - alpha_i - lam)) keeps it feasible
    and can only raise the value, which is <= OPT.  C: an n x m array, or a
    function rows(i0, i1) returning rows i0..i1-1 in FP64 (for sizes whose
    dense FP64 cost is better not kept).  Entropic duals map to LP duals by
    beta = gamma v, lam = gamma w (X_ij = exp(u_i + v_j + w - C_ij / gamma),
    slack p_i = e^{u_i})."""
    r = np.asarray(r, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    n, m = len(r), len(c)
    rows = C if callable(C) else (lambda i0, i1: np.asarray(C[i0:i1], dtype=np.float64))
    b1 = np.minimum(np.asarray(beta, dtype=np.float64), 0.0)
    alpha = np.empty(n)
    for i0 in range(0, n, chunk):
        blk = rows(i0, min(n, i0 + chunk))
        alpha[i0:i0 + blk.shape[0]] = np.minimum(0.0, np.min(blk - b1[None, :], axis=1) - lam)
    b2 = np.zeros(m)
    for i0 in range(0, n, chunk):
        blk = rows(i0, min(n, i0 + chunk))
        b2 = np.minimum(b2, np.min(blk - alpha[i0:i0 + blk.shape[0], None], axis=0) - lam)
    return float(np.dot(r, alpha) + np.dot(c, b2) + s * lam)


def extended_ot_lp(C, r, c, s, A_corner=None):
    C = np.asarray(C, dtype=np.float64)
    n, m = C.shape
    if A_corner is None:
        A_corner = 2.0 * max(C.max(), 1e-3) + 1.0
    Ce = np.zeros((n + 1, m + 1))
    Ce[:n, :m] = C
    Ce[n, m] = A_corner
    re = np.concatenate([r, [c.sum() - s]])
    ce = np.concatenate([c, [r.sum() - s]])
    N, M = n + 1, m + 1
    Aeq = np.zeros((N + M, N * M))
    for i in range(N):
        Aeq[i, i * M:(i + 1) * M] = 1.0
    for j in range(M):
        Aeq[N + j, j::M] = 1.0
    res = linprog(Ce.ravel(), A_eq=Aeq, b_eq=np.concatenate([re, ce]), bounds=(0, None),
                  method="highs")
    assert res.status == 0, res.message
    return float(res.fun)


def assignment_brute_force(C):
    """Balanced OT with uniform masses 1/n on an n x n cost: by Birkhoff's
    theorem the optimum is attained at a permutation matrix / n."""
    C = np.asarray(C)
    n = C.shape[0]
    best = min(sum(C[i, p[i]] for i in range(n)) for p in itertools.permutations(range(n)))
    return best / n


def in_polytope(X, r, c, s, rtol=1e-12):
    X = np.asarray(X)
    scale = max(1.0, float(np.max(r)), float(np.max(c)), s)
    tol = rtol * scale
    ok_nonneg = bool(np.all(X >= -tol))
    ok_rows = bool(np.all(X.sum(1) <= r + tol))
    ok_cols = bool(np.all(X.sum(0) <= c + tol))
    ok_mass = abs(X.sum() - s) <= rtol * max(1.0, s) * 10
    return ok_nonneg and ok_rows and ok_cols and ok_mass
