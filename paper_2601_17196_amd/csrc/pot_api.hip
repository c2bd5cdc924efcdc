// pot_api.hip -- host side of libpot: argument checks, workspace layout, the
// solve driver and the C ABI declared in include/pot.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pot_internal.h"

namespace pot {

hipError_t launch_setup(const SetupArgs& S, hipStream_t st);
hipError_t launch_stats(const PassArgs& A, hipStream_t st);
hipError_t launch_round(const PassArgs& A, hipStream_t st);
hipError_t launch_cost_max(int kind, const void* C, int64_t ldc, const float* x, const float* y, int n,
                           int m, int d, unsigned long long* out, hipStream_t st);
hipError_t launch_finish(const PassArgs& A, int algo, double* f, double* g, double* u, double* v,
                         hipStream_t st);
hipError_t launch_copy_out(const PassArgs& A, double* alpha, double* beta, double* pp, double* qq,
                           hipStream_t st);

hipError_t launch_stats_timed(const PassArgs& A, hipStream_t st, hipEvent_t e0, hipEvent_t e1, hipEvent_t e2,
                              hipEvent_t e3);

static thread_local std::string g_last_error;

static pot_status fail(pot_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Tile geometry of one problem.
struct Geometry {
    int br, bc, nx, ny;
};

static int vec_width(int kind) { return kind == POT_COST_BF16 ? 8 : 4; }

static Geometry geometry(const pot_problem* p, const pot_options* o) {
    Geometry g;
    g.bc = 64 * vec_width(p->kind);
    int br = (o && o->tile_rows > 0) ? o->tile_rows : 0;
    if (br == 0) {
        // default: rows per tile so that the grid has a few WGs per CU
        const int64_t elems = (int64_t)p->n * p->m;
        br = elems >= (int64_t)8192 * 8192 ? 128 : 64;
    }
    br = std::max(4, std::min(br, 256));
    g.br = br;
    g.nx = (p->m + g.bc - 1) / g.bc;
    g.ny = (p->n + g.br - 1) / g.br;
    return g;
}

// Workspace layout; returns total bytes and fills ws if base != nullptr.
static size_t layout(const pot_problem* p, const Geometry& g, char* base, Ws* ws) {
    const int64_t n = p->n, m = p->m;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return base ? (void*)(base + o) : nullptr;
    };
    Ws w{};
    w.ctl = (Ctl*)take(sizeof(Ctl));
    w.rowcnt = (int32_t*)take(sizeof(int32_t) * (size_t)g.ny);
    w.colcnt = (int32_t*)take(sizeof(int32_t) * (size_t)g.nx);
    w.glob = (int32_t*)take(sizeof(int32_t) * 4);
    w.tshift = (int32_t*)take(sizeof(int32_t) * (size_t)g.nx * g.ny);
    w.rowpart = take(std::max<size_t>(4 * (size_t)g.nx * n, 8 * 3 * (size_t)g.nx * n));
    w.colpart = take(8 * (size_t)g.ny * m);
    w.rowscal = (double*)take(8 * (size_t)std::max(g.ny, (p->n + 63) / 64) * kScal);
    w.colscal = (double*)take(8 * (size_t)std::max(g.nx, (p->m + 63) / 64) * kScal);
    double** rv[] = {&w.rt, &w.lrt, &w.uchk0, &w.uchk1, &w.util0, &w.util1,
                     &w.ubar, &w.ugrave, &w.uz, &w.du, &w.alpha, &w.pp};
    for (double** q : rv) *q = (double*)take(8 * (size_t)n);
    double** cv[] = {&w.ct, &w.lct, &w.vchk0, &w.vchk1, &w.vtil0, &w.vtil1,
                     &w.vbar, &w.vgrave, &w.vz, &w.dv, &w.beta, &w.qq};
    for (double** q : cv) *q = (double*)take(8 * (size_t)m);
    take(16);   // cost max scratch (last 16 bytes region)
    if (ws) *ws = w;
    return off;
}

static unsigned long long* maxbuf(char* base, size_t total) {
    return (unsigned long long*)(base + total - 256);
}

static pot_status check_problem(const pot_problem* p, const pot_options* o) {
    if (!p || !o) return fail(POT_ERR_INVALID_ARG, "null problem or options");
    if (p->n < 1 || p->m < 1) return fail(POT_ERR_INVALID_ARG, "n and m must be >= 1");
    if (p->kind != POT_COST_F32 && p->kind != POT_COST_BF16 && p->kind != POT_COST_SQEUCLID_POINTS)
        return fail(POT_ERR_INVALID_ARG, "unknown cost kind");
    if (p->kind == POT_COST_SQEUCLID_POINTS) {
        if (!p->x || !p->y) return fail(POT_ERR_INVALID_ARG, "points kind needs x and y");
        if (p->d != 2 && p->d != 3) return fail(POT_ERR_UNSUPPORTED, "points kind supports d = 2 or 3");
        if (!std::isfinite(p->cost_scale)) return fail(POT_ERR_INVALID_ARG, "cost_scale not finite");
    } else {
        if (!p->C) return fail(POT_ERR_INVALID_ARG, "dense kind needs C");
        if (p->ldc < p->m) return fail(POT_ERR_INVALID_ARG, "ldc < m");
    }
    if (!p->r || !p->c) return fail(POT_ERR_INVALID_ARG, "r and c are required");
    if (!(p->s > 0.0) || !std::isfinite(p->s)) return fail(POT_ERR_INVALID_ARG, "s must be finite and > 0");
    if (!std::isfinite(p->cmax)) return fail(POT_ERR_INVALID_ARG, "cmax not finite");
    if (!(o->eps > 0.0) || !std::isfinite(o->eps)) return fail(POT_ERR_INVALID_ARG, "eps must be finite and > 0");
    if (!std::isfinite(o->gamma) || !std::isfinite(o->tol) || !std::isfinite(o->A))
        return fail(POT_ERR_INVALID_ARG, "gamma, tol and A must be finite");
    if (o->gamma <= 0.0 && std::max(p->n, p->m) < 2)
        return fail(POT_ERR_INVALID_ARG, "default gamma needs max(n, m) >= 2 (ln 1 = 0)");
    if (o->algo != POT_ASPOT && o->algo != POT_SINKHORN) return fail(POT_ERR_INVALID_ARG, "unknown algo");
    if (o->block_rule < 0 || o->block_rule > 1) return fail(POT_ERR_INVALID_ARG, "block_rule");
    if (o->step_rule < 0 || o->step_rule > 1) return fail(POT_ERR_INVALID_ARG, "step_rule");
    if (o->force_len < 0 || (o->force_len > 0 && !o->force)) return fail(POT_ERR_INVALID_ARG, "force");
    if (o->trace_cap < 0) return fail(POT_ERR_INVALID_ARG, "trace_cap");
    if (o->tile_rows < 0 || o->tile_rows > 256) return fail(POT_ERR_INVALID_ARG, "tile_rows in [0, 256]");
    if (!std::isfinite(o->w0)) return fail(POT_ERR_INVALID_ARG, "w0 not finite");
    return POT_OK;
}

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(POT_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// pinned slots for convergence polling (host memory, allocated once per thread)
struct PollSlots {
    int32_t* flag = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
};
static thread_local PollSlots g_poll;

static pot_status ensure_poll() {
    if (!g_poll.flag) {
        HIPCHK(hipHostMalloc((void**)&g_poll.flag, 2 * sizeof(int32_t), hipHostMallocDefault));
        HIPCHK(hipEventCreateWithFlags(&g_poll.ev[0], hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&g_poll.ev[1], hipEventDisableTiming));
    }
    return POT_OK;
}

// The iteration loop as a HIP graph: one chunk of `chunk` iterations (every
// launch of a phase has the same arguments: the kernels read the iteration
// state from the control block) is captured once on a private stream and
// replayed on the caller's stream.  Executables are cached per thread by the
// bytes of their launch arguments.
struct GraphEntry {
    std::string key;
    hipGraphExec_t exec = nullptr;
};
static thread_local GraphEntry g_graphs[8];
static thread_local int g_graph_next = 0;
static thread_local hipStream_t g_capture_stream = nullptr;

static void enqueue_iterations(PassArgs A, int algo, int iters, hipStream_t st, hipError_t* err) {
    for (int it = 0; it < iters && *err == hipSuccess; ++it) {
        if (algo == POT_ASPOT) {
            for (int ph : {PH_BAR, PH_GRAVE, PH_Z}) {
                A.phase = ph;
                *err = launch_stats(A, st);
                if (*err != hipSuccess) return;
            }
        } else {
            A.phase = PH_SK_ROW;
            *err = launch_stats(A, st);
            if (*err != hipSuccess) return;
            A.phase = PH_SK_COL;
            *err = launch_stats(A, st);
        }
    }
}

static hipError_t chunk_graph(const PassArgs& A, int algo, int chunk, hipGraphExec_t* out) {
    std::string key((const char*)&A, sizeof(A));
    key.append((const char*)&algo, sizeof(algo));
    key.append((const char*)&chunk, sizeof(chunk));
    for (auto& g : g_graphs)
        if (g.exec && g.key == key) {
            *out = g.exec;
            return hipSuccess;
        }
    hipError_t e;
    if (!g_capture_stream) {
        e = hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    e = hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    enqueue_iterations(A, algo, chunk, g_capture_stream, &le);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(g_capture_stream, &graph);
    if (le != hipSuccess) e = le;
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return e;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    GraphEntry& slot = g_graphs[g_graph_next];
    g_graph_next = (g_graph_next + 1) % 8;
    if (slot.exec) (void)hipGraphExecDestroy(slot.exec);
    slot.exec = exec;
    slot.key = key;
    *out = exec;
    return hipSuccess;
}

static pot_status solve_one(const pot_problem* p, const pot_options* o, void* wsp, size_t ws_bytes,
                            pot_result* res, const pot_outputs* out, hipStream_t st) {
    pot_status cs = check_problem(p, o);
    if (cs != POT_OK) return cs;
    if (!res) return fail(POT_ERR_INVALID_ARG, "res is required");
    const Geometry g = geometry(p, o);
    const size_t need = layout(p, g, nullptr, nullptr);
    if (!wsp || ws_bytes < need) return fail(POT_ERR_WORKSPACE, "workspace too small");
    if (((uintptr_t)wsp) & 255) return fail(POT_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    char* base = (char*)wsp;
    Ws w;
    layout(p, g, base, &w);
    pot_status ps = ensure_poll();
    if (ps != POT_OK) return ps;

    // --- cost scale and |C|_max (B10): one pass when not given
    double cost_scale = 1.0, cmax = p->cmax;
    if (p->kind == POT_COST_SQEUCLID_POINTS) {
        cost_scale = p->cost_scale;
        if (cost_scale <= 0.0 || cmax <= 0.0) {
            unsigned long long* mb = maxbuf(base, need);
            HIPCHK(hipMemsetAsync(mb, 0, 16, st));
            HIPCHK(launch_cost_max(p->kind, nullptr, 0, p->x, p->y, p->n, p->m, p->d, mb, st));
            unsigned long long h[2];
            HIPCHK(hipMemcpyAsync(h, mb, 16, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            double mx;
            std::memcpy(&mx, &h[0], 8);
            if (h[1] != 0) return fail(POT_ERR_INVALID_ARG, "non-finite point coordinates");
            if (!(mx > 0.0)) return fail(POT_ERR_INVALID_ARG, "all points coincide (max cost 0)");
            if (cost_scale <= 0.0) cost_scale = 1.0 / mx;
            if (cmax <= 0.0) cmax = cost_scale * mx;
        }
    } else if (cmax <= 0.0) {
        unsigned long long* mb = maxbuf(base, need);
        HIPCHK(hipMemsetAsync(mb, 0, 16, st));
        HIPCHK(launch_cost_max(p->kind, p->C, p->ldc, nullptr, nullptr, p->n, p->m, 0, mb, st));
        unsigned long long h[2];
        HIPCHK(hipMemcpyAsync(h, mb, 16, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (h[1] != 0) return fail(POT_ERR_INVALID_ARG, "cost has negative or non-finite entries");
        std::memcpy(&cmax, &h[0], 8);
        if (!(cmax > 0.0)) return fail(POT_ERR_INVALID_ARG, "cost is identically 0 (|C|_max = 0)");
    }

    // every exponent log2(e) C_ij / gamma must stay below 2^29 (the kernels
    // split exponents into an int32 part and a fraction)
    {
        const int N = std::max(p->n, p->m);
        const double gam = o->gamma > 0.0 ? o->gamma : o->eps / (4.0 * std::log((double)N));
        if (!(1.4426950408889634 * cmax / gam < 536870912.0))
            return fail(POT_ERR_INVALID_ARG, "|C|_max / gamma too large (exponents beyond 2^29)");
    }

    // --- setup (Algorithm 2, "Approximating POT") and validation of r, c, s
    SetupArgs S;
    S.n = p->n; S.m = p->m; S.algo = o->algo; S.nx = g.nx; S.ny = g.ny;
    S.s = p->s; S.eps = o->eps; S.gamma_user = o->gamma; S.tol_user = o->tol; S.A_user = o->A;
    S.cmax = cmax; S.cost_scale = cost_scale; S.w0 = o->w0;
    S.r = p->r; S.c = p->c; S.ws = w;
    HIPCHK(launch_setup(S, st));
    int32_t valid = 0;
    HIPCHK(hipMemcpyAsync(&valid, &w.ctl->valid, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (valid != 0) {
        static const char* why[] = {"", "r or c has a negative or non-finite entry",
                                    "s must satisfy 0 < s <= min(|r|_1, |c|_1)", "gamma is not positive",
                                    "eps~ capped to 0 (s equals a mass above 1) and no tol given",
                                    "a smoothed marginal is not positive"};
        return fail(POT_ERR_INVALID_ARG, why[valid < 6 ? valid : 0]);
    }

    PassArgs A;
    std::memset(&A, 0, sizeof(A));
    A.C = p->C; A.ldc = p->ldc; A.x = p->x; A.y = p->y; A.r = p->r; A.c = p->c;
    A.n = p->n; A.m = p->m; A.d = p->d; A.kind = p->kind;
    A.br = g.br; A.bc = g.bc; A.nx = g.nx; A.ny = g.ny;
    A.nrb = (p->n + 63) / 64; A.ncb = (p->m + 63) / 64;
    A.max_iter = o->max_iter > 0 ? o->max_iter : 100000;
    A.block_rule = o->block_rule; A.step_rule = o->step_rule;
    A.u0 = o->u0; A.v0 = o->v0; A.w0 = o->w0;
    A.force = o->force; A.force_len = o->force_len;
    A.trace_i = o->trace_i; A.trace_d = o->trace_d; A.trace_cap = o->trace_cap;
    A.ws = w;

    // --- the iteration loop, enqueued in chunks; the host polls the done
    // flag of the previous chunk while the next one runs.
    const int chunk = o->check_every > 0 ? o->check_every : 16;
    if (o->algo == POT_ASPOT) {
        A.phase = PH_INIT;
        HIPCHK(launch_stats(A, st));
    }
    int enq = 0, k = 0;
    bool done = false;
    hipGraphExec_t gexec = nullptr;
    if (!(o->flags & POT_FLAG_NO_GRAPH) && A.max_iter >= chunk) HIPCHK(chunk_graph(A, o->algo, chunk, &gexec));
    while (!done && enq < A.max_iter) {
        const int todo = std::min(chunk, A.max_iter - enq);
        if (gexec && todo == chunk) {
            HIPCHK(hipGraphLaunch(gexec, st));
        } else {
            hipError_t le = hipSuccess;
            enqueue_iterations(A, o->algo, todo, st, &le);
            HIPCHK(le);
        }
        enq += todo;
        const int slot = k & 1;
        HIPCHK(hipMemcpyAsync(&g_poll.flag[slot], &w.ctl->done, 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord(g_poll.ev[slot], st));
        if (k > 0) {
            HIPCHK(hipEventSynchronize(g_poll.ev[slot ^ 1]));
            done = g_poll.flag[slot ^ 1] != 0;
        }
        ++k;
    }
    if (o->algo == POT_SINKHORN) {
        // the row pass that checks the last iterate (and stops at max_iter)
        A.phase = PH_SK_ROW;
        HIPCHK(launch_stats(A, st));
    }

    // --- form primal and round onto U(r, c, s) in FP64
    HIPCHK(launch_finish(A, o->algo, out ? out->f : nullptr, out ? out->g : nullptr,
                         out ? out->u : nullptr, out ? out->v : nullptr, st));
    Ctl hc;
    HIPCHK(hipMemcpyAsync(&hc, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const bool round = !(o->flags & POT_FLAG_NO_ROUND) && hc.status != POT_ERR_NUMERIC && hc.done;
    if (round) {
        for (int ph : {PH_R1, PH_R2, PH_R3}) {
            A.phase = ph;
            HIPCHK(launch_round(A, st));
        }
        if ((o->flags & POT_FLAG_WANT_PLAN) && out && out->plan) {
            A.phase = PH_R4;
            A.plan = out->plan;
            HIPCHK(launch_round(A, st));
        }
        if (out) HIPCHK(launch_copy_out(A, out->alpha, out->beta, out->pp, out->qq, st));
        HIPCHK(hipMemcpyAsync(&hc, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    if (!hc.done) return fail(POT_ERR_DEVICE, "solver loop ended without a decision");

    std::memset(res, 0, sizeof(*res));
    res->status = hc.status;
    res->iters = hc.iters;
    res->algo = o->algo;
    res->used_warm = (o->u0 || o->v0) ? 1 : 0;
    res->cost = hc.cost;
    res->E = hc.E;
    res->gamma = hc.gamma;
    res->tol = hc.tol;
    res->phi = hc.phichk;
    res->mass = hc.mass;
    res->kappa = hc.kappa;
    res->lambda = hc.lambda;
    res->T2 = hc.T2;
    res->cost_scale = cost_scale;
    res->cmax = cmax;
    if (out && out->w) *out->w = o->algo == POT_ASPOT ? hc.wz : 0.0;
    if (hc.status == POT_ERR_NUMERIC) g_last_error = "non-finite row or column sum (overflow)";
    else if (hc.status == POT_ERR_NO_CONVERGENCE) g_last_error = "max_iter reached before E <= tol";
    else g_last_error.clear();
    return (pot_status)hc.status;
}

}  // namespace pot

using namespace pot;

extern "C" {

size_t pot_workspace_bytes(const pot_problem* prob, const pot_options* opts) {
    if (!prob || prob->n < 1 || prob->m < 1) return 0;
    pot_options dflt;
    std::memset(&dflt, 0, sizeof(dflt));
    const Geometry g = geometry(prob, opts ? opts : &dflt);
    return layout(prob, g, nullptr, nullptr);
}

pot_status pot_solve(const pot_problem* prob, const pot_options* opts, void* ws, size_t ws_bytes,
                     pot_result* res, const pot_outputs* out, void* stream) {
    try {
        return solve_one(prob, opts, ws, ws_bytes, res, out, (hipStream_t)stream);
    } catch (...) {
        return fail(POT_ERR_DEVICE, "internal error");
    }
}

size_t pot_workspace_bytes_batched(int32_t batch, const pot_problem* probs, const pot_options* opts) {
    if (batch < 1 || !probs) return 0;
    size_t mx = 0;
    for (int k = 0; k < batch; ++k) mx = std::max(mx, pot_workspace_bytes(&probs[k], opts));
    return mx;
}

pot_status pot_solve_batched(int32_t batch, const pot_problem* probs, const pot_options* opts, void* ws,
                             size_t ws_bytes, pot_result* res, double* const* f_out, double* const* g_out,
                             void* stream) {
    if (batch < 1 || !probs || !opts || !res) return fail(POT_ERR_INVALID_ARG, "batch arguments");
    pot_status first = POT_OK;
    for (int k = 0; k < batch; ++k) {
        pot_outputs o;
        std::memset(&o, 0, sizeof(o));
        o.f = f_out ? f_out[k] : nullptr;
        o.g = g_out ? g_out[k] : nullptr;
        pot_status st = pot_solve(&probs[k], opts, ws, ws_bytes, &res[k], &o, stream);
        if (st != POT_OK && first == POT_OK) first = st;
    }
    return first;
}

pot_status pot_time_pass(const pot_problem* prob, const pot_options* opts, void* ws, size_t ws_bytes,
                         int32_t reps, double* avg_ms, double* fin_ms, void* stream) {
    try {
        if (reps < 1 || !avg_ms) return fail(POT_ERR_INVALID_ARG, "reps >= 1 and avg_ms required");
        pot_status cs = check_problem(prob, opts);
        if (cs != POT_OK) return cs;
        hipStream_t st = (hipStream_t)stream;
        const Geometry g = geometry(prob, opts);
        const size_t need = layout(prob, g, nullptr, nullptr);
        if (!ws || ws_bytes < need || (((uintptr_t)ws) & 255)) return fail(POT_ERR_WORKSPACE, "workspace");
        if (prob->cmax <= 0.0 || (prob->kind == POT_COST_SQEUCLID_POINTS && prob->cost_scale <= 0.0))
            return fail(POT_ERR_INVALID_ARG, "pot_time_pass needs cmax (and cost_scale) given");
        Ws w;
        layout(prob, g, (char*)ws, &w);
        SetupArgs S;
        S.n = prob->n; S.m = prob->m; S.algo = POT_ASPOT; S.nx = g.nx; S.ny = g.ny;
        S.s = prob->s; S.eps = opts->eps; S.gamma_user = opts->gamma; S.tol_user = opts->tol;
        S.A_user = opts->A; S.cmax = prob->cmax;
        S.cost_scale = prob->kind == POT_COST_SQEUCLID_POINTS ? prob->cost_scale : 1.0;
        S.w0 = opts->w0; S.r = prob->r; S.c = prob->c; S.ws = w;
        HIPCHK(launch_setup(S, st));
        PassArgs A;
        std::memset(&A, 0, sizeof(A));
        A.C = prob->C; A.ldc = prob->ldc; A.x = prob->x; A.y = prob->y; A.r = prob->r; A.c = prob->c;
        A.n = prob->n; A.m = prob->m; A.d = prob->d; A.kind = prob->kind;
        A.br = g.br; A.bc = g.bc; A.nx = g.nx; A.ny = g.ny;
        A.nrb = (prob->n + 63) / 64; A.ncb = (prob->m + 63) / 64;
        A.max_iter = 1; A.u0 = opts->u0; A.v0 = opts->v0; A.w0 = opts->w0;
        A.ws = w;
        A.phase = PH_INIT;
        std::vector<hipEvent_t> ev(4 * (size_t)reps);
        for (auto& e : ev) HIPCHK(hipEventCreate(&e));
        for (int k = 0; k < reps; ++k)
            HIPCHK(launch_stats_timed(A, st, ev[4 * k], ev[4 * k + 1], ev[4 * k + 2], ev[4 * k + 3]));
        HIPCHK(hipStreamSynchronize(st));
        double tot = 0.0, tot2 = 0.0;
        for (int k = 0; k < reps; ++k) {
            float ms = 0.f, ms2 = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ev[4 * k], ev[4 * k + 1]));
            HIPCHK(hipEventElapsedTime(&ms2, ev[4 * k + 2], ev[4 * k + 3]));
            tot += ms;
            tot2 += ms2;
        }
        for (auto& e : ev) (void)hipEventDestroy(e);
        Ctl hc;
        HIPCHK(hipMemcpy(&hc, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
        if (hc.valid != 0) return fail(POT_ERR_INVALID_ARG, "invalid problem");
        if (hc.status != POT_OK) return fail((pot_status)hc.status, "pass reported a non-finite sum");
        *avg_ms = tot / reps;
        if (fin_ms) *fin_ms = tot2 / reps;
        return POT_OK;
    } catch (...) {
        return fail(POT_ERR_DEVICE, "internal error");
    }
}

const char* pot_status_string(pot_status st) {
    switch (st) {
    case POT_OK: return "ok";
    case POT_ERR_INVALID_ARG: return "invalid argument";
    case POT_ERR_NO_CONVERGENCE: return "no convergence within max_iter (plan still feasible)";
    case POT_ERR_NUMERIC: return "non-finite statistic";
    case POT_ERR_DEVICE: return "HIP runtime error";
    case POT_ERR_WORKSPACE: return "workspace too small or misaligned";
    case POT_ERR_UNSUPPORTED: return "unsupported option";
    default: return "unknown status";
    }
}

const char* pot_last_error(void) { return g_last_error.c_str(); }

const char* pot_version(void) { return "libpot 0.1 (gfx950)"; }

}  // extern "C"
