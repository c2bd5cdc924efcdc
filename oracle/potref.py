"""ctypes binding of the FP64 oracle library ``libpotref.so`` (built from potref.c).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each function follows the passage of the paper named in its docstring; the
arithmetic itself lives in potref.c.
"""
from __future__ import annotations

import ctypes as ct
import dataclasses
import os
import subprocess

import numpy as np

__all__ = [
    "build_oracle",
    "load",
    "setup",
    "tuned",
    "stats",
    "phi",
    "error",
    "greenkhorn",
    "aspot",
    "sinkhorn",
    "round_plan",
    "round_dense",
    "cost",
    "solve",
    "threads",
    "sk_error",
    "plan_eval",
    "set_threads",
    "AspotTrace",
    "OracleSolution",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "potref.c")
_LIB = os.path.join(_HERE, "libpotref.so")
_lib = None

_D = ct.POINTER(ct.c_double)
_I = ct.POINTER(ct.c_int)


def build_oracle(force: bool = True) -> str:
    """Compile potref.c with gcc (FP64, OpenMP) into oracle/libpotref.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _AspotOpts(ct.Structure):
    _fields_ = [
        ("max_iter", ct.c_int), ("block_rule", ct.c_int), ("step_rule", ct.c_int),
        ("trace_cap", ct.c_int),
        ("tr_bhat", _I), ("tr_pick", _I), ("tr_bchk", _I),
        ("tr_E", _D), ("tr_theta", _D), ("tr_phibar", _D), ("tr_phigrave", _D),
        ("tr_phihat", _D), ("tr_phichk", _D), ("tr_phiz", _D), ("tr_phinext", _D),
        ("tr_gdot", _D), ("tr_step2", _D), ("tr_ztil", _D),
    ]


def load():
    """Load libpotref.so, building it first if it is missing or stale.
    POTREF_LIB names another build of potref.c (the mutation test plants
    mistakes in a copy of the source to check that the pins catch them)."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("POTREF_LIB")
    if not path:
        path = _LIB
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_oracle(force=True)
    lib = ct.CDLL(path)
    lib.potref_setup.argtypes = [ct.c_int, ct.c_int, _D, _D, ct.c_double, ct.c_double,
                                 ct.c_double, ct.c_double, ct.c_double, _D, _D, _D]
    lib.potref_setup.restype = ct.c_int
    lib.potref_tuned.argtypes = [ct.c_int, ct.c_int, _D, _D, ct.c_double, ct.c_double, _D]
    lib.potref_tuned.restype = ct.c_int
    lib.potref_stats.argtypes = [ct.c_int, ct.c_int, _D, ct.c_long, ct.c_double, _D, _D,
                                 ct.c_double, _D, _D, _D]
    lib.potref_stats.restype = None
    lib.potref_phi.argtypes = [ct.c_int, ct.c_int, _D, ct.c_long, ct.c_double, _D, _D,
                               ct.c_double, _D, _D, ct.c_double]
    lib.potref_phi.restype = ct.c_double
    lib.potref_error.argtypes = lib.potref_phi.argtypes
    lib.potref_error.restype = ct.c_double
    lib.potref_greenkhorn.argtypes = [ct.c_int, ct.c_int, _D, ct.c_long, ct.c_double, _D, _D,
                                      ct.c_double, _D, _D, _D, ct.c_int, _D]
    lib.potref_greenkhorn.restype = ct.c_int
    lib.potref_aspot.argtypes = [ct.c_int, ct.c_int, _D, ct.c_long, ct.c_double, ct.c_double,
                                 _D, _D, ct.c_double, ct.c_double, _D, _D, ct.c_double,
                                 ct.POINTER(_AspotOpts), _D, _D, _D, _I, _D]
    lib.potref_aspot.restype = ct.c_int
    lib.potref_sinkhorn.argtypes = [ct.c_int, ct.c_int, _D, ct.c_long, ct.c_double, ct.c_double,
                                    _D, _D, ct.c_double, ct.c_double, ct.c_int, _D, _D, _I, _D, _D]
    lib.potref_sinkhorn.restype = ct.c_int
    lib.potref_round.argtypes = [ct.c_int, ct.c_int, _D, ct.c_long, ct.c_double, _D, _D, _D, _D,
                                 ct.c_double, _D, _D, _D, _D, _D, _D]
    lib.potref_round.restype = ct.c_int
    lib.potref_round_dense.argtypes = [ct.c_int, ct.c_int, _D, _D, _D, ct.c_double, _D]
    lib.potref_round_dense.restype = ct.c_int
    lib.potref_cost.argtypes = [ct.c_int, ct.c_int, _D, ct.c_long, _D]
    lib.potref_cost.restype = ct.c_double
    lib.potref_sk_error.argtypes = [ct.c_int, ct.c_int, _D, ct.c_long, ct.c_double, _D, _D, ct.c_double,
                                    ct.c_double, _D, _D]
    lib.potref_sk_error.restype = ct.c_double
    lib.potref_plan_eval.argtypes = [ct.c_int, ct.c_int, _D, ct.c_long, _D, ct.c_long, ct.c_double, _D, _D,
                                     _D, _D, ct.c_double, ct.c_double, _D, _D, _D, _D, _D]
    lib.potref_plan_eval.restype = ct.c_int
    lib.potref_threads.argtypes = []
    lib.potref_threads.restype = ct.c_int
    lib.potref_set_threads.argtypes = [ct.c_int]
    lib.potref_set_threads.restype = None
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(_D)


def _pi(a):
    return None if a is None else a.ctypes.data_as(_I)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def threads() -> int:
    return int(load().potref_threads())


def set_threads(t: int) -> None:
    """OpenMP threads of later oracle calls."""
    load().potref_set_threads(int(t))


def setup(r, c, s, eps, cmax=1.0, gamma=0.0, tol=0.0):
    """Algorithm 2, "Approximating POT".  Returns (gamma, tol, M, r~, c~)."""
    lib = load()
    r = _f64(r)
    c = _f64(c)
    rt = np.empty_like(r)
    cc = np.empty_like(c)
    out = np.empty(3)
    st = lib.potref_setup(len(r), len(c), _p(r), _p(c), float(s), float(eps), float(cmax),
                          float(gamma), float(tol), _p(rt), _p(cc), _p(out))
    if st != 0:
        raise ValueError("invalid POT setup arguments")
    return float(out[0]), float(out[1]), float(out[2]), rt, cc


def tuned(r, c, eps, p):
    """Tuned rule of Algorithm 3 (Theorem 2): returns (gamma, eps', H_min)."""
    lib = load()
    r = _f64(r)
    c = _f64(c)
    out = np.empty(3)
    st = lib.potref_tuned(len(r), len(c), _p(r), _p(c), float(eps), float(p), _p(out))
    if st != 0:
        raise ValueError("tuned rule needs p >= 1, valid masses and min(H(r), H(c)) > 0")
    return float(out[0]), float(out[1]), float(out[2])


def stats(C, gamma, u, v, w):
    """log row sums, log column sums and log total of B(z) (Section 2.1)."""
    lib = load()
    C = _f64(C)
    n, m = C.shape
    lR = np.empty(n)
    lQ = np.empty(m)
    lT = np.empty(1)
    lib.potref_stats(n, m, _p(C), m, float(gamma), _p(_f64(u)), _p(_f64(v)), float(w),
                     _p(lR), _p(lQ), _p(lT))
    return lR, lQ, float(lT[0])


def phi(C, gamma, rt, ct_, s, u, v, w):
    """The dual objective phi(z) of Section 2.1, from its definition."""
    lib = load()
    C = _f64(C)
    n, m = C.shape
    return float(lib.potref_phi(n, m, _p(C), m, float(gamma), _p(_f64(rt)), _p(_f64(ct_)),
                                float(s), _p(_f64(u)), _p(_f64(v)), float(w)))


def error(C, gamma, rt, ct_, s, u, v, w):
    """E(z) of Section 3.1 with p~ = e^u, q~ = e^v."""
    lib = load()
    C = _f64(C)
    n, m = C.shape
    return float(lib.potref_error(n, m, _p(C), m, float(gamma), _p(_f64(rt)), _p(_f64(ct_)),
                                  float(s), _p(_f64(u)), _p(_f64(v)), float(w)))


def greenkhorn(C, gamma, rt, ct_, s, u, v, w, block=-1):
    """Algorithm 1 on a copy of z.  Returns (u', v', w', block, scores)."""
    lib = load()
    C = _f64(C)
    n, m = C.shape
    u = _f64(u).copy()
    v = _f64(v).copy()
    ww = np.array([float(w)])
    sc = np.empty(3)
    b = lib.potref_greenkhorn(n, m, _p(C), m, float(gamma), _p(_f64(rt)), _p(_f64(ct_)),
                              float(s), _p(u), _p(v), _p(ww), int(block), _p(sc))
    return u, v, float(ww[0]), int(b), sc


@dataclasses.dataclass
class AspotTrace:
    bhat: np.ndarray
    pick: np.ndarray
    bchk: np.ndarray
    E: np.ndarray
    theta: np.ndarray
    phibar: np.ndarray
    phigrave: np.ndarray
    phihat: np.ndarray
    phichk: np.ndarray
    phiz: np.ndarray
    phinext: np.ndarray
    gdot: np.ndarray
    step2: np.ndarray
    ztil: np.ndarray | None


def aspot(C, gamma, tol, rt, ct_, s, M, max_iter=100000, block_rule=0, step_rule=0,
          z0=None, trace=False, trace_ztil=False):
    """ASPOT (Algorithm 2).  Returns (u, v, w, iters, E, status, trace)."""
    lib = load()
    C = _f64(C)
    n, m = C.shape
    u = np.empty(n)
    v = np.empty(m)
    w = np.empty(1)
    it = np.zeros(1, dtype=np.int32)
    E = np.empty(1)
    o = _AspotOpts()
    o.max_iter = int(max_iter)
    o.block_rule = int(block_rule)
    o.step_rule = int(step_rule)
    tr = None
    keep = []
    if trace:
        cap = int(max_iter)
        ints = [np.full(cap, -9, dtype=np.int32) for _ in range(3)]
        dbls = [np.full(cap, np.nan) for _ in range(10)]
        zt = np.zeros((cap, n + m + 1)) if trace_ztil else None
        keep += ints + dbls + [zt]
        o.trace_cap = cap
        o.tr_bhat, o.tr_pick, o.tr_bchk = (_pi(a) for a in ints)
        (o.tr_E, o.tr_theta, o.tr_phibar, o.tr_phigrave, o.tr_phihat, o.tr_phichk,
         o.tr_phiz, o.tr_phinext, o.tr_gdot, o.tr_step2) = (_p(a) for a in dbls)
        o.tr_ztil = _p(zt)
    u0 = v0 = None
    w0 = 0.0
    if z0 is not None:
        u0 = _f64(z0[0])
        v0 = _f64(z0[1])
        w0 = float(z0[2])
    st = lib.potref_aspot(n, m, _p(C), m, float(gamma), float(tol), _p(_f64(rt)), _p(_f64(ct_)),
                          float(s), float(M), _p(u0), _p(v0), w0, ct.byref(o),
                          _p(u), _p(v), _p(w), _pi(it), _p(E))
    k = int(it[0])
    if trace:
        ints, dbls = keep[:3], keep[3:13]
        tr = AspotTrace(*(a[:k] for a in ints), *(a[:k] for a in dbls),
                        ztil=(keep[13][:k] if trace_ztil else None))
    return u, v, float(w[0]), k, float(E[0]), int(st), tr


def sinkhorn(C, gamma, tol, rt, ct_, s, A, max_iter=100000, trace=False):
    """Feasible Sinkhorn on the extended instance (Algorithm 3 loop).
    Returns (a (n+1), b (m+1), iters, err, status, err_trace)."""
    lib = load()
    C = _f64(C)
    n, m = C.shape
    a = np.empty(n + 1)
    b = np.empty(m + 1)
    it = np.zeros(1, dtype=np.int32)
    err = np.empty(1)
    tr = np.full(int(max_iter), np.nan) if trace else None
    st = lib.potref_sinkhorn(n, m, _p(C), m, float(gamma), float(tol), _p(_f64(rt)),
                             _p(_f64(ct_)), float(s), float(A), int(max_iter), _p(a), _p(b),
                             _pi(it), _p(err), _p(tr))
    k = int(it[0])
    return a, b, k, float(err[0]), int(st), (tr[:k] if trace else None)


def round_plan(C, gamma, f, g, r, c, s, dense=False):
    """Rounding of X~_ij = exp(f_i + g_j - C_ij/gamma) onto U(r, c, s).
    Returns dict(alpha, beta, pp, qq, kappa, lam, T2, cost, mass, X)."""
    lib = load()
    C = _f64(C)
    n, m = C.shape
    alpha = np.empty(n)
    beta = np.empty(m)
    pp = np.empty(n)
    qq = np.empty(m)
    out = np.empty(5)
    X = np.empty((n, m)) if dense else None
    lib.potref_round(n, m, _p(C), m, float(gamma), _p(_f64(f)), _p(_f64(g)), _p(_f64(r)),
                     _p(_f64(c)), float(s), _p(alpha), _p(beta), _p(pp), _p(qq), _p(out), _p(X))
    return dict(alpha=alpha, beta=beta, pp=pp, qq=qq, kappa=float(out[0]), lam=float(out[1]),
                T2=float(out[2]), cost=float(out[3]), mass=float(out[4]), X=X)


def round_dense(X, r, c, s):
    """The same rounding applied to an arbitrary nonnegative matrix."""
    lib = load()
    X = _f64(X)
    n, m = X.shape
    out = np.empty_like(X)
    lib.potref_round_dense(n, m, _p(X), _p(_f64(r)), _p(_f64(c)), float(s), _p(out))
    return out


def cost(C, X):
    lib = load()
    C = _f64(C)
    X = _f64(X)
    n, m = C.shape
    return float(lib.potref_cost(n, m, _p(C), m, _p(X)))


def sk_error(C, gamma, rt, ct_, s, A, a, b):
    """Stopping error of feasible Sinkhorn (Algorithm 3) at the extended
    log-scalings a (n + 1), b (m + 1), every entry summed directly."""
    lib = load()
    C = _f64(C)
    n, m = C.shape
    a = _f64(a)
    b = _f64(b)
    assert a.shape == (n + 1,) and b.shape == (m + 1,)
    return float(lib.potref_sk_error(n, m, _p(C), C.strides[0] // 8, float(gamma), _p(_f64(rt)), _p(_f64(ct_)),
                                     float(s), float(A), _p(a), _p(b)))


def plan_eval(Cp, gamma, f, g, alpha, beta, kappa, lam, pp, qq, Ce=None):
    """A factored plan kappa diag(alpha) X~ diag(beta) + lam p' q'^T,
    X~_ij = exp(f_i + g_j - Cp_ij / gamma), evaluated entry by entry.
    Returns dict(rows, cols, cost (priced with Ce, default Cp), mass, min)."""
    lib = load()
    Cp = _f64(Cp)
    Ce = Cp if Ce is None else _f64(Ce)
    n, m = Cp.shape
    assert Ce.shape == (n, m)
    rows = np.empty(n)
    cols = np.empty(m)
    out = np.empty(3)
    lib.potref_plan_eval(n, m, _p(Cp), Cp.strides[0] // 8, _p(Ce), Ce.strides[0] // 8, float(gamma),
                         _p(_f64(f)), _p(_f64(g)), _p(_f64(alpha)), _p(_f64(beta)), float(kappa), float(lam),
                         _p(_f64(pp)), _p(_f64(qq)), _p(rows), _p(cols), _p(out))
    return dict(rows=rows, cols=cols, cost=float(out[0]), mass=float(out[1]), min=float(out[2]))


def tuned_tol(r, c, gamma, p):
    """eps' = H_min gamma^p of the tuned rule at a given gamma."""
    _, _, h = tuned(r, c, 1.0, p)
    return h * gamma ** p


@dataclasses.dataclass
class OracleSolution:
    algo: str
    gamma: float
    tol: float
    iters: int
    E: float
    status: int
    u: np.ndarray          # ASPOT: u; Sinkhorn: a[:n]
    v: np.ndarray          # ASPOT: v; Sinkhorn: b[:m]
    w: float               # ASPOT: w; Sinkhorn: 0
    f: np.ndarray          # row log-scaling of the plan: X~_ij = exp(f_i + g_j - C_ij/gamma)
    g: np.ndarray
    rounded: dict
    trace: object = None


def solve(C, r, c, s, eps, algo="aspot", cmax=None, gamma=0.0, tol=0.0, max_iter=100000,
          block_rule=0, step_rule=0, trace=False, A=None, z0=None, dense=False, gamma_rule=0, p=1.0):
    """Setup, solve and round: Algorithm 2 (algo="aspot") or Algorithm 3 with
    the default gamma and stopping rule (algo="sinkhorn"); gamma_rule=1 takes
    Algorithm 3's tuned gamma and threshold (Theorem 2) where gamma and tol
    are not given."""
    C = _f64(C)
    if cmax is None:
        cmax = float(C.max())
    if gamma_rule == 1:
        if algo != "sinkhorn":
            raise ValueError("the tuned rule is Algorithm 3's (Sinkhorn)")
        tg, tt, _ = tuned(r, c, eps, p)
        if not gamma > 0.0:
            gamma = tg
        if not tol > 0.0:
            tol = tt if gamma == tg else tuned_tol(r, c, gamma, p)
    gam, tl, M, rt, cc = setup(r, c, s, eps, cmax=cmax, gamma=gamma, tol=tol)
    if algo == "aspot":
        u, v, w, it, E, st, tr = aspot(C, gam, tl, rt, cc, s, M, max_iter=max_iter,
                                       block_rule=block_rule, step_rule=step_rule,
                                       z0=z0, trace=trace)
        f = u + w
        g = v
    elif algo == "sinkhorn":
        if A is None:
            A = 8.0 * cmax / eps
        a, b, it, E, st, tr = sinkhorn(C, gam, tl, rt, cc, s, A, max_iter=max_iter, trace=trace)
        u, v, w = a[:-1], b[:-1], 0.0
        f, g = a[:-1], b[:-1]
    else:
        raise ValueError(algo)
    rd = round_plan(C, gam, f, g, r, c, s, dense=dense)
    return OracleSolution(algo=algo, gamma=gam, tol=tl, iters=it, E=E, status=st, u=u, v=v, w=w,
                          f=f, g=g, rounded=rd, trace=tr)
