"""Python binding of libpot.so (argument marshalling only).

Every step of a solve runs in the HIP library; this module only builds the
C structs of include/pot.h from torch tensors (which provide device memory
and streams) and reads the results back.  It raises if the library is not
built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import dataclasses
import os

import numpy as np

__all__ = [
    "load", "lib_path", "ASPOT", "SINKHORN", "COST_F32", "COST_BF16", "COST_POINTS",
    "FLAG_WANT_PLAN", "FLAG_NO_ROUND", "Problem", "Options", "Result", "Outputs",
    "solve", "solve_batched", "workspace_bytes", "status_string", "last_error", "SolveOutput",
    "PotError", "time_pass", "result_from_device", "FLAG_ASYNC", "register", "rigid_align", "solve_shared", "time_shared_gemm", "workspace_bytes_shared",
]

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(HERE, "libpot.so")

ASPOT, SINKHORN = 0, 1
COST_F32, COST_BF16, COST_POINTS = 0, 1, 3
FLAG_WANT_PLAN, FLAG_NO_ROUND, FLAG_NO_GRAPH, FLAG_ASYNC = 1, 2, 4, 8

OK, ERR_INVALID_ARG, ERR_NO_CONVERGENCE, ERR_NUMERIC, ERR_DEVICE, ERR_WORKSPACE, ERR_UNSUPPORTED = range(7)
NOALLOC_SCRATCH_BYTES = 32 << 20   # POT_NOALLOC_SCRATCH_BYTES


class PotError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libpot status {status}: {msg}")
        self.status = status


class Problem(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("m", ct.c_int32), ("d", ct.c_int32), ("kind", ct.c_int32),
                ("C", ct.c_void_p), ("ldc", ct.c_int64), ("x", ct.c_void_p), ("y", ct.c_void_p),
                ("cost_scale", ct.c_double), ("cmax", ct.c_double), ("r", ct.c_void_p),
                ("c", ct.c_void_p), ("s", ct.c_double)]


class Options(ct.Structure):
    _fields_ = [("algo", ct.c_int32), ("max_iter", ct.c_int32), ("eps", ct.c_double),
                ("gamma", ct.c_double), ("tol", ct.c_double), ("A", ct.c_double),
                ("block_rule", ct.c_int32), ("step_rule", ct.c_int32), ("check_every", ct.c_int32),
                ("flags", ct.c_uint32), ("u0", ct.c_void_p), ("v0", ct.c_void_p), ("w0", ct.c_double),
                ("force", ct.c_void_p), ("force_len", ct.c_int32), ("trace_i", ct.c_void_p),
                ("trace_d", ct.c_void_p), ("trace_cap", ct.c_int32), ("tile_rows", ct.c_int32),
                ("member_elems", ct.c_int32), ("gamma_rule", ct.c_int32), ("p", ct.c_double),
                ("warm_check", ct.c_int32), ("reserved0", ct.c_int32)]


class BatchOutputs(ct.Structure):
    _fields_ = [("f", ct.c_void_p), ("g", ct.c_void_p), ("u", ct.c_void_p), ("v", ct.c_void_p)]


class WarmInstance(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("m", ct.c_int32), ("x", ct.c_void_p), ("y", ct.c_void_p),
                ("r", ct.c_void_p), ("c", ct.c_void_p), ("cost_scale", ct.c_double), ("gamma", ct.c_double),
                ("u0", ct.c_void_p), ("v0", ct.c_void_p)]


class Warm(ct.Structure):
    _fields_ = [("u0", ct.c_void_p), ("v0", ct.c_void_p), ("w0", ct.c_void_p), ("check", ct.c_int32)]


class Result(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("iters", ct.c_int32), ("algo", ct.c_int32),
                ("used_warm", ct.c_int32), ("cost", ct.c_double), ("E", ct.c_double),
                ("gamma", ct.c_double), ("tol", ct.c_double), ("phi", ct.c_double),
                ("mass", ct.c_double), ("kappa", ct.c_double), ("lambda_", ct.c_double),
                ("T2", ct.c_double), ("cost_scale", ct.c_double), ("cmax", ct.c_double), ("w", ct.c_double),
                ("viol_row", ct.c_double), ("viol_col", ct.c_double), ("viol_mass", ct.c_double),
                ("ext_a", ct.c_double), ("ext_b", ct.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Outputs(ct.Structure):
    _fields_ = [("plan", ct.c_void_p), ("f", ct.c_void_p), ("g", ct.c_void_p), ("u", ct.c_void_p),
                ("v", ct.c_void_p), ("alpha", ct.c_void_p), ("beta", ct.c_void_p),
                ("pp", ct.c_void_p), ("qq", ct.c_void_p), ("w", ct.POINTER(ct.c_double)),
                ("moments", ct.c_void_p)]


class SharedCost(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("m", ct.c_int32), ("kind", ct.c_int32), ("pad", ct.c_int32),
                ("C", ct.c_void_p), ("ldc", ct.c_int64), ("cmax", ct.c_double)]


class SharedMember(ct.Structure):
    _fields_ = [("r", ct.c_void_p), ("c", ct.c_void_p), ("s", ct.c_double), ("f", ct.c_void_p), ("g", ct.c_void_p)]


class RegProblem(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("m", ct.c_int32), ("x", ct.c_void_p), ("y", ct.c_void_p),
                ("r", ct.c_void_p), ("c", ct.c_void_p), ("s", ct.c_double), ("cost_scale", ct.c_double)]


class RegOptions(ct.Structure):
    _fields_ = [("eps", ct.c_double), ("gamma0", ct.c_double), ("anneal", ct.c_double),
                ("gamma_min", ct.c_double), ("tol", ct.c_double), ("max_steps", ct.c_int32),
                ("warm", ct.c_int32), ("max_iter", ct.c_int32), ("algo", ct.c_int32),
                ("R0", ct.c_double * 9), ("t0", ct.c_double * 3)]


class RegResult(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("steps", ct.c_int32), ("total_iters", ct.c_int32), ("pad", ct.c_int32),
                ("R", ct.c_double * 9), ("t", ct.c_double * 3), ("cost", ct.c_double)]


class RegHistory(ct.Structure):
    _fields_ = [("iters", ct.c_void_p), ("cost", ct.c_void_p), ("gamma", ct.c_void_p), ("E", ct.c_void_p),
                ("Rt", ct.c_void_p), ("y_hist", ct.c_void_p), ("dual_hist", ct.c_void_p)]


_lib = None


def lib_path() -> str:
    return _LIB


def load():
    """Load libpot.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("POT_LIB") or _LIB   # POT_LIB: another build of the same sources
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ct.CDLL(path)
    lib.pot_workspace_bytes.argtypes = [ct.POINTER(Problem), ct.POINTER(Options)]
    lib.pot_workspace_bytes.restype = ct.c_size_t
    lib.pot_workspace_bytes_batched.argtypes = [ct.c_int32, ct.POINTER(Problem), ct.POINTER(Options)]
    lib.pot_workspace_bytes_batched.restype = ct.c_size_t
    lib.pot_solve.argtypes = [ct.POINTER(Problem), ct.POINTER(Options), ct.c_void_p, ct.c_size_t,
                              ct.POINTER(Result), ct.POINTER(Outputs), ct.c_void_p]
    lib.pot_solve.restype = ct.c_int
    lib.pot_solve_batched.argtypes = [ct.c_int32, ct.POINTER(Problem), ct.POINTER(Options), ct.POINTER(Warm),
                                      ct.c_void_p, ct.c_size_t, ct.POINTER(Result), ct.POINTER(BatchOutputs),
                                      ct.c_void_p]
    lib.pot_solve_batched.restype = ct.c_int
    lib.pot_warm_workspace_bytes.argtypes = [ct.c_int32]
    lib.pot_warm_workspace_bytes.restype = ct.c_size_t
    lib.pot_warm_predict.argtypes = [ct.c_int32, ct.POINTER(WarmInstance), ct.c_double, ct.c_void_p, ct.c_void_p,
                                     ct.c_size_t, ct.c_void_p]
    lib.pot_warm_predict.restype = ct.c_int
    lib.pot_solve_noalloc.argtypes = [ct.POINTER(Problem), ct.POINTER(Options), ct.POINTER(Result),
                                      ct.POINTER(Outputs), ct.c_void_p]
    lib.pot_solve_noalloc.restype = ct.c_int
    lib.pot_workspace_bytes_shared.argtypes = [ct.POINTER(SharedCost), ct.c_int32]
    lib.pot_workspace_bytes_shared.restype = ct.c_size_t
    lib.pot_solve_shared.argtypes = [ct.POINTER(SharedCost), ct.c_int32, ct.POINTER(SharedMember), ct.POINTER(Options),
                                     ct.c_void_p, ct.c_size_t, ct.POINTER(Result), ct.c_void_p]
    lib.pot_solve_shared.restype = ct.c_int
    lib.pot_time_shared_gemm.argtypes = [ct.POINTER(SharedCost), ct.c_int32, ct.c_double, ct.c_void_p, ct.c_size_t,
                                         ct.c_int32, ct.POINTER(ct.c_double), ct.c_void_p]
    lib.pot_time_shared_gemm.restype = ct.c_int
    lib.pot_register_workspace_bytes.argtypes = [ct.POINTER(RegProblem)]
    lib.pot_register_workspace_bytes.restype = ct.c_size_t
    lib.pot_register.argtypes = [ct.POINTER(RegProblem), ct.POINTER(RegOptions), ct.c_void_p, ct.c_size_t,
                                 ct.POINTER(RegResult), ct.POINTER(RegHistory), ct.c_void_p, ct.c_void_p]
    lib.pot_register.restype = ct.c_int
    lib.pot_rigid_align.argtypes = [ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)]
    lib.pot_rigid_align.restype = None
    lib.pot_time_pass.argtypes = [ct.POINTER(Problem), ct.POINTER(Options), ct.c_void_p, ct.c_size_t,
                                  ct.c_int32, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double), ct.c_void_p]
    lib.pot_time_pass.restype = ct.c_int
    lib.pot_status_string.argtypes = [ct.c_int]
    lib.pot_status_string.restype = ct.c_char_p
    lib.pot_last_error.argtypes = []
    lib.pot_last_error.restype = ct.c_char_p
    lib.pot_version.argtypes = []
    lib.pot_version.restype = ct.c_char_p
    _lib = lib
    return lib


def status_string(st: int) -> str:
    return load().pot_status_string(int(st)).decode()


def last_error() -> str:
    return load().pot_last_error().decode()


def _ptr(t):
    return None if t is None else ct.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ct.c_void_p(stream.cuda_stream)


def make_problem(r, c, s, C=None, x=None, y=None, kind=None, ldc=None, cost_scale=0.0, cmax=0.0):
    """Build a Problem from device tensors.  C: (n, ldc) float32 or
    uint16/bfloat16 bit patterns (row-major, the first m columns used);
    x, y: (n, d), (m, d) float32 points."""
    import torch
    n, m = int(r.shape[0]), int(c.shape[0])
    p = Problem()
    p.n, p.m = n, m
    p.r, p.c = _ptr(r), _ptr(c)
    p.s = float(s)
    p.cost_scale = float(cost_scale)
    p.cmax = float(cmax)
    if C is not None:
        if kind is None:
            kind = COST_F32 if C.dtype == torch.float32 else COST_BF16
        p.kind = kind
        p.C = _ptr(C)
        p.ldc = int(ldc if ldc is not None else C.stride(0))
        p.d = 0
    else:
        p.kind = COST_POINTS
        p.x, p.y = _ptr(x), _ptr(y)
        p.d = int(x.shape[1])
    return p


def make_options(eps, algo=ASPOT, max_iter=100000, gamma=0.0, tol=0.0, A=0.0, block_rule=0,
                 step_rule=0, check_every=0, flags=0, u0=None, v0=None, w0=0.0, force=None,
                 trace_i=None, trace_d=None, trace_cap=0, tile_rows=0, member_elems=0, gamma_rule=0, p=1.0,
                 warm_check=0):
    o = Options()
    o.algo = int(algo)
    o.max_iter = int(max_iter)
    o.eps = float(eps)
    o.gamma = float(gamma)
    o.tol = float(tol)
    o.A = float(A)
    o.block_rule = int(block_rule)
    o.step_rule = int(step_rule)
    o.check_every = int(check_every)
    o.flags = int(flags)
    o.u0, o.v0 = _ptr(u0), _ptr(v0)
    o.w0 = float(w0)
    o.force = _ptr(force)
    o.force_len = 0 if force is None else int(force.numel() // 3)
    o.trace_i, o.trace_d = _ptr(trace_i), _ptr(trace_d)
    o.trace_cap = int(trace_cap)
    o.tile_rows = int(tile_rows)
    o.member_elems = int(member_elems)
    o.gamma_rule = int(gamma_rule)
    o.p = float(p)
    o.warm_check = int(warm_check)
    o.reserved0 = 0
    return o


def workspace_bytes(prob: Problem, opts: Options) -> int:
    return int(load().pot_workspace_bytes(ct.byref(prob), ct.byref(opts)))


@dataclasses.dataclass
class SolveOutput:
    status: int
    result: dict
    f: object = None
    g: object = None
    u: object = None
    v: object = None
    w: float = 0.0
    alpha: object = None
    beta: object = None
    pp: object = None
    qq: object = None
    plan: object = None
    trace_i: object = None
    trace_d: object = None
    result_dev: object = None     # asynchronous solve: device bytes of the pot_result
    workspace: object = None      # the workspace tensor (kept alive with the output)


def result_from_device(t) -> dict:
    """The pot_result an asynchronous solve wrote to device memory (a uint8
    tensor of sizeof(pot_result) bytes), as a dict."""
    raw = bytes(t.cpu().numpy().tobytes())
    return Result.from_buffer_copy(raw).as_dict()


def solve(r, c, s, eps, C=None, x=None, y=None, kind=None, ldc=None, cost_scale=0.0, cmax=0.0,
          algo=ASPOT, want_plan=False, want_factors=True, workspace=None, stream=None,
          raise_on_error=True, trace_cap=0, async_=False, **opt_kw):
    """Solve one POT instance through pot_solve.  Tensors must be on the GPU.

    async_=True sets POT_FLAG_ASYNC: the call only enqueues, the result block
    is written to a device tensor (SolveOutput.result_dev, read it with
    result_from_device after the stream has reached it) and result is {}."""
    import torch
    lib = load()
    dev = r.device
    prob = make_problem(r, c, s, C=C, x=x, y=y, kind=kind, ldc=ldc, cost_scale=cost_scale, cmax=cmax)
    tr_i = tr_d = None
    if trace_cap > 0:
        tr_i = torch.full((trace_cap * 3,), -9, dtype=torch.int32, device=dev)
        tr_d = torch.full((trace_cap * 4,), float("nan"), dtype=torch.float64, device=dev)
    flags = (FLAG_WANT_PLAN if want_plan else 0) | (FLAG_ASYNC if async_ else 0) | int(opt_kw.pop("flags", 0))
    opts = make_options(eps, algo=algo, flags=flags, trace_i=tr_i, trace_d=tr_d, trace_cap=trace_cap,
                        **opt_kw)
    nbytes = workspace_bytes(prob, opts)
    if nbytes == 0:
        raise PotError(ERR_INVALID_ARG, "invalid sizes")
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    base = workspace.data_ptr()
    aligned = (base + 255) & ~255
    avail = workspace.numel() - (aligned - base)
    n, m = prob.n, prob.m
    f64 = dict(dtype=torch.float64, device=dev)
    out = Outputs()
    so = SolveOutput(status=-1, result={})
    so.f, so.g = torch.empty(n, **f64), torch.empty(m, **f64)
    so.u, so.v = torch.empty(n, **f64), torch.empty(m, **f64)
    if want_factors:
        so.alpha, so.pp = torch.empty(n, **f64), torch.empty(n, **f64)
        so.beta, so.qq = torch.empty(m, **f64), torch.empty(m, **f64)
    if want_plan:
        so.plan = torch.empty((n, m), **f64)
    wbox = ct.c_double(0.0)
    out.plan = _ptr(so.plan)
    out.f, out.g, out.u, out.v = _ptr(so.f), _ptr(so.g), _ptr(so.u), _ptr(so.v)
    out.alpha, out.beta, out.pp, out.qq = _ptr(so.alpha), _ptr(so.beta), _ptr(so.pp), _ptr(so.qq)
    so.trace_i, so.trace_d = tr_i, tr_d
    so.workspace = workspace
    if flags & FLAG_ASYNC:
        so.result_dev = torch.zeros(ct.sizeof(Result), dtype=torch.uint8, device=dev)
        st = lib.pot_solve(ct.byref(prob), ct.byref(opts), ct.c_void_p(aligned), ct.c_size_t(avail),
                           ct.cast(ct.c_void_p(so.result_dev.data_ptr()), ct.POINTER(Result)), ct.byref(out),
                           _stream_ptr(stream))
        so.status = int(st)
        if raise_on_error and st != OK:
            raise PotError(st, last_error())
        return so
    out.w = ct.pointer(wbox)
    res = Result()
    st = lib.pot_solve(ct.byref(prob), ct.byref(opts), ct.c_void_p(aligned), ct.c_size_t(avail),
                       ct.byref(res), ct.byref(out), _stream_ptr(stream))
    so.status = int(st)
    so.result = res.as_dict()
    so.w = wbox.value
    if raise_on_error and st not in (OK, ERR_NO_CONVERGENCE):
        raise PotError(st, last_error())
    return so


def solve_shared(C, members, eps, gamma, tol=0.0, A=0.0, max_iter=100000, kind=None, ldc=None, cmax=0.0,
                 want_duals=True, flags=0, stream=None, workspace=None, raise_on_error=False):
    """Feasible Sinkhorn for many members on one shared cost
    (pot_solve_shared).  C: (n, ldc) float32 or BF16 bit patterns on the GPU;
    members: list of dicts with r, c (device float64) and s.  Returns
    (status, list of result dicts, list of (f, g) or None)."""
    import torch
    lib = load()
    n, m = int(members[0]["r"].shape[0]), int(members[0]["c"].shape[0])
    B = len(members)
    cost = _shared_cost(C, cmax, kind, ldc)
    mem = (SharedMember * B)()
    outs = []
    dev = C.device
    for k, d in enumerate(members):
        mem[k].r, mem[k].c, mem[k].s = _ptr(d["r"]), _ptr(d["c"]), float(d["s"])
        if want_duals:
            f = torch.empty(n, dtype=torch.float64, device=dev)
            g = torch.empty(m, dtype=torch.float64, device=dev)
            mem[k].f, mem[k].g = _ptr(f), _ptr(g)
            outs.append((f, g))
    opts = make_options(eps, algo=SINKHORN, gamma=gamma, tol=tol, A=A, max_iter=max_iter, flags=flags)
    nbytes = int(lib.pot_workspace_bytes_shared(ct.byref(cost), B))
    if nbytes == 0:
        raise PotError(ERR_INVALID_ARG, "invalid sizes")
    if workspace is None or workspace.numel() < nbytes + 256:
        workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    aligned = (workspace.data_ptr() + 255) & ~255
    res = (Result * B)()
    st = lib.pot_solve_shared(ct.byref(cost), B, mem, ct.byref(opts), ct.c_void_p(aligned),
                              ct.c_size_t(workspace.numel() - (aligned - workspace.data_ptr())), res,
                              _stream_ptr(stream))
    if raise_on_error and st not in (OK, ERR_NO_CONVERGENCE):
        raise PotError(st, last_error())
    return int(st), [res[k].as_dict() for k in range(B)], (outs if want_duals else None)


def _shared_cost(C, cmax=0.0, kind=None, ldc=None):
    import torch
    cost = SharedCost()
    cost.n, cost.m = int(C.shape[0]), int(C.shape[1])
    cost.kind = (COST_F32 if C.dtype == torch.float32 else COST_BF16) if kind is None else int(kind)
    cost.C = _ptr(C)
    cost.ldc = int(ldc if ldc is not None else C.stride(0))
    cost.cmax = float(cmax)
    return cost


def workspace_bytes_shared(C, batch, kind=None, ldc=None) -> int:
    return int(load().pot_workspace_bytes_shared(ct.byref(_shared_cost(C, 0.0, kind, ldc)), int(batch)))


def time_shared_gemm(C, batch, gamma, cmax, reps=20, stream=None):
    """Median time (ms) of the shared-cost product K~ x scalings for
    `batch` members (pot_time_shared_gemm) and the padded sizes
    (rows, cols, depth)."""
    import torch
    lib = load()
    cost = _shared_cost(C, cmax)
    nbytes = int(lib.pot_workspace_bytes_shared(ct.byref(cost), int(batch)))
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=C.device)
    aligned = (ws.data_ptr() + 255) & ~255
    ms = ct.c_double(0.0)
    st = lib.pot_time_shared_gemm(ct.byref(cost), int(batch), float(gamma), ct.c_void_p(aligned), ct.c_size_t(nbytes),
                                  int(reps), ct.byref(ms), _stream_ptr(stream))
    if st != OK:
        raise PotError(st, last_error())
    up = lambda x, k: (x + k - 1) // k * k
    return ms.value, (up(cost.n + 1, 64), 2 * up(int(batch), 64), up(cost.m + 1, 64))


def rigid_align(H):
    """The rotation in SO(3) maximising tr(R^T H) (pot_rigid_align, host)."""
    Hc = (ct.c_double * 9)(*[float(v) for v in np.asarray(H, dtype=np.float64).ravel()])
    Rc = (ct.c_double * 9)()
    load().pot_rigid_align(Hc, Rc)
    return np.array(list(Rc)).reshape(3, 3)


@dataclasses.dataclass
class RegisterOutput:
    status: int
    R: np.ndarray
    t: np.ndarray
    steps: int
    total_iters: int
    cost: float
    iters: np.ndarray
    costs: np.ndarray
    gammas: np.ndarray
    E: np.ndarray
    Rt: np.ndarray
    y_out: object = None
    y_hist: object = None
    dual_hist: object = None


def register(x, y, r, c, s, eps=1e-2, gamma0=4.4e-3, anneal=0.83, gamma_min=0.0, tol=1e-5, max_steps=60,
             warm=True, max_iter=0, algo=ASPOT, cost_scale=0.0, R0=None, t0=None, history=False, stream=None,
             raise_on_error=True):
    """Rigid registration of the cloud y (m x 3) onto x (n x 3) through POT
    (pot_register).  Tensors on the GPU: x, y float32, r, c float64."""
    import torch
    lib = load()
    dev = x.device
    n, m = int(x.shape[0]), int(y.shape[0])
    prob = RegProblem()
    prob.n, prob.m = n, m
    prob.x, prob.y, prob.r, prob.c = _ptr(x), _ptr(y), _ptr(r), _ptr(c)
    prob.s = float(s)
    prob.cost_scale = float(cost_scale)
    o = RegOptions()
    o.eps, o.gamma0, o.anneal, o.gamma_min, o.tol = float(eps), float(gamma0), float(anneal), float(gamma_min), float(tol)
    o.max_steps, o.warm, o.max_iter, o.algo = int(max_steps), int(bool(warm)), int(max_iter), int(algo)
    R0 = np.eye(3) if R0 is None else np.asarray(R0, dtype=np.float64)
    t0 = np.zeros(3) if t0 is None else np.asarray(t0, dtype=np.float64)
    for k in range(9):
        o.R0[k] = float(R0.ravel()[k])
    for k in range(3):
        o.t0[k] = float(t0[k])
    nbytes = int(lib.pot_register_workspace_bytes(ct.byref(prob)))
    if nbytes == 0:
        raise PotError(ERR_INVALID_ARG, "invalid sizes")
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    aligned = (ws.data_ptr() + 255) & ~255
    iters = np.zeros(max_steps, dtype=np.int32)
    costs, gammas, Es = np.zeros(max_steps), np.zeros(max_steps), np.zeros(max_steps)
    Rt = np.zeros((max_steps, 12))
    h = RegHistory()
    h.iters, h.cost, h.gamma, h.E, h.Rt = (a.ctypes.data for a in (iters, costs, gammas, Es, Rt))
    yh = dh = None
    if history:
        yh = torch.zeros((max_steps, m, 3), dtype=torch.float32, device=dev)
        dh = torch.zeros((max_steps, n + m + 1), dtype=torch.float64, device=dev)
        h.y_hist, h.dual_hist = yh.data_ptr(), dh.data_ptr()
    y_out = torch.empty((m, 3), dtype=torch.float32, device=dev)
    res = RegResult()
    st = lib.pot_register(ct.byref(prob), ct.byref(o), ct.c_void_p(aligned), ct.c_size_t(nbytes), ct.byref(res),
                          ct.byref(h), ct.c_void_p(y_out.data_ptr()), _stream_ptr(stream))
    if raise_on_error and st not in (OK, ERR_NO_CONVERGENCE):
        raise PotError(st, last_error())
    k = int(res.steps)
    return RegisterOutput(status=int(st), R=np.array(list(res.R)).reshape(3, 3), t=np.array(list(res.t)), steps=k,
                          total_iters=int(res.total_iters), cost=float(res.cost), iters=iters[:k], costs=costs[:k],
                          gammas=gammas[:k], E=Es[:k], Rt=Rt[:k], y_out=y_out,
                          y_hist=None if yh is None else yh[:k], dual_hist=None if dh is None else dh[:k])


def batch_problems(problems):
    """ctypes array of Problem for a list of dicts with keys r, c, s, C (device
    tensors; optional ldc, kind, cmax)."""
    probs = (Problem * len(problems))()
    for k, pr in enumerate(problems):
        probs[k] = make_problem(pr["r"], pr["c"], pr["s"], C=pr["C"], kind=pr.get("kind"), ldc=pr.get("ldc"),
                                cmax=pr.get("cmax", 0.0))
    return probs


def workspace_bytes_batched(problems, opts=None) -> int:
    probs = problems if isinstance(problems, ct.Array) else batch_problems(problems)
    return int(load().pot_workspace_bytes_batched(len(probs), probs, ct.byref(opts) if opts else None))


def solve_batched(problems, eps, algo=ASPOT, u0=None, v0=None, w0=None, warm_check=True, want_duals=True,
                  want_uv=False, stream=None, workspace=None, raise_on_error=False, **opt_kw):
    """Solve a list of instances through pot_solve_batched (one persistent
    launch).  problems: list of dicts with keys r, c, s, C (device tensors;
    optional ldc, kind, cmax).  u0 / v0: optional lists of device FP64
    tensors (entries may be None), w0: optional list of floats.
    Returns (status, list of result dicts, list of (f, g) tensors or None);
    with want_uv the third item holds (f, g, u, v) tuples."""
    import torch
    lib = load()
    B = len(problems)
    probs = batch_problems(problems)
    opts = make_options(eps, algo=algo, **opt_kw)
    nbytes = int(lib.pot_workspace_bytes_batched(B, probs, ct.byref(opts)))
    if nbytes == 0:
        raise PotError(ERR_INVALID_ARG, "invalid batch sizes")
    dev = problems[0]["r"].device
    if workspace is None or workspace.numel() < nbytes + 256:
        workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    base = workspace.data_ptr()
    aligned = (base + 255) & ~255
    avail = workspace.numel() - (aligned - base)
    keep = []
    outs = None
    bo = None
    if want_duals or want_uv:
        f64 = dict(dtype=torch.float64, device=dev)
        fs = [torch.empty(p["r"].shape[0], **f64) for p in problems]
        gs = [torch.empty(p["c"].shape[0], **f64) for p in problems]
        bo = BatchOutputs()

        def arr(ts):
            a = (ct.c_void_p * B)(*[t.data_ptr() for t in ts])
            keep.append(a)
            return ct.cast(a, ct.c_void_p)
        bo.f, bo.g = arr(fs), arr(gs)
        outs = list(zip(fs, gs))
        if want_uv:
            us = [torch.empty(p["r"].shape[0], **f64) for p in problems]
            vs = [torch.empty(p["c"].shape[0], **f64) for p in problems]
            bo.u, bo.v = arr(us), arr(vs)
            outs = list(zip(fs, gs, us, vs))
    warm = None
    if u0 is not None or v0 is not None:
        warm = Warm()
        if u0 is not None:
            ua = (ct.c_void_p * B)(*[_ptr(t) for t in u0])
            keep.append(ua)
            warm.u0 = ct.cast(ua, ct.c_void_p)
        if v0 is not None:
            va = (ct.c_void_p * B)(*[_ptr(t) for t in v0])
            keep.append(va)
            warm.v0 = ct.cast(va, ct.c_void_p)
        if w0 is not None:
            wa = (ct.c_double * B)(*[float(x) for x in w0])
            keep.append(wa)
            warm.w0 = ct.cast(wa, ct.c_void_p)
        warm.check = 1 if warm_check else 0
    res = (Result * B)()
    st = lib.pot_solve_batched(B, probs, ct.byref(opts), ct.byref(warm) if warm is not None else None,
                               ct.c_void_p(aligned), ct.c_size_t(avail), res,
                               ct.byref(bo) if bo is not None else None, _stream_ptr(stream))
    if raise_on_error and st not in (OK, ERR_NO_CONVERGENCE):
        raise PotError(st, last_error())
    return int(st), [res[k].as_dict() for k in range(B)], outs


def warm_blob(arrays=None, device="cuda"):
    """Device weight blob of the warm-start network (uint8 tensor); arrays:
    dict of FP32/FP64 numpy weights (default: the trained weights shipped
    with the package)."""
    import torch

    from . import warmstart as W
    arr = arrays if arrays is not None else W.load_arrays()
    return torch.from_numpy(W.pack_blob(arr)).to(device)


def warm_predict(instances, eps, blob, stream=None, workspace=None):
    """Warm starts (u0, v0) for a list of dicts with keys x, y (n x 2 and
    m x 2 float32), r, c (float64), cost_scale and optional gamma (device
    tensors).  Runs the inference kernels; returns a list of (u0, v0)."""
    import torch
    lib = load()
    B = len(instances)
    arr = (WarmInstance * B)()
    outs = []
    dev = instances[0]["r"].device
    for k, d in enumerate(instances):
        n, m = int(d["x"].shape[0]), int(d["y"].shape[0])
        u0 = torch.empty(n, dtype=torch.float64, device=dev)
        v0 = torch.empty(m, dtype=torch.float64, device=dev)
        w = arr[k]
        w.n, w.m = n, m
        w.x, w.y, w.r, w.c = _ptr(d["x"]), _ptr(d["y"]), _ptr(d["r"]), _ptr(d["c"])
        w.cost_scale = float(d["cost_scale"])
        w.gamma = float(d.get("gamma", 0.0))
        w.u0, w.v0 = _ptr(u0), _ptr(v0)
        outs.append((u0, v0))
    nbytes = int(lib.pot_warm_workspace_bytes(B))
    if workspace is None or workspace.numel() < nbytes + 256:
        workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    base = workspace.data_ptr()
    aligned = (base + 255) & ~255
    st = lib.pot_warm_predict(B, arr, float(eps), ct.c_void_p(blob.data_ptr()), ct.c_void_p(aligned),
                              ct.c_size_t(workspace.numel() - (aligned - base)), _stream_ptr(stream))
    if st != OK:
        raise PotError(st, last_error())
    return outs


def to_device_instance(inst, device="cuda", kind="f32", pad_ldc=False):
    """Host Instance (paper_2601_17196_amd.instances) -> dict of device tensors."""
    import torch
    from . import instances as I
    d = {"r": torch.from_numpy(inst.r).to(device), "c": torch.from_numpy(inst.c).to(device), "s": inst.s}
    if kind == "points":
        d["x"] = torch.from_numpy(inst.x).to(device)
        d["y"] = torch.from_numpy(inst.y).to(device)
        d["cost_scale"] = inst.cost_scale
        d["cmax"] = 1.0
        return d
    if kind == "f32":
        host = inst.C32
    elif kind == "bf16":
        host = I.to_bf16_bits(inst.C32).view(np.int16)
    else:
        raise ValueError(kind)
    n, m = host.shape
    if pad_ldc:
        ld = (m + 3) // 4 * 4 + 4
        buf = np.zeros((n, ld), dtype=host.dtype)
        buf[:, :m] = host
        host = buf
    t = torch.from_numpy(np.ascontiguousarray(host)).to(device)
    d["C"] = t[:, :m] if pad_ldc else t
    d["ldc"] = t.stride(0)
    d["kind"] = COST_F32 if kind == "f32" else COST_BF16
    d["cmax"] = 0.0
    return d


def time_pass(r, c, s, eps, reps=50, C=None, x=None, y=None, kind=None, ldc=None, cost_scale=0.0,
              cmax=1.0, u0=None, v0=None, w0=0.0, stream=None, tile_rows=0):
    """Median kernel times (ms) of the statistics pass at (u0, v0, w0) over
    `reps` launches after 3 untimed ones, from HIP events recorded around each
    dispatch (pot_time_pass): returns (tile kernel, finalising kernel)."""
    import torch
    lib = load()
    prob = make_problem(r, c, s, C=C, x=x, y=y, kind=kind, ldc=ldc, cost_scale=cost_scale, cmax=cmax)
    opts = make_options(eps, u0=u0, v0=v0, w0=w0, tile_rows=tile_rows)
    nbytes = workspace_bytes(prob, opts)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=r.device)
    aligned = (ws.data_ptr() + 255) & ~255
    ms = ct.c_double(0.0)
    ms2 = ct.c_double(0.0)
    st = lib.pot_time_pass(ct.byref(prob), ct.byref(opts), ct.c_void_p(aligned), ct.c_size_t(nbytes),
                           int(reps), ct.byref(ms), ct.byref(ms2), _stream_ptr(stream))
    if st != OK:
        raise PotError(st, last_error())
    return ms.value, ms2.value
