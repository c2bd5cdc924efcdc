// pot_api.hip -- host side of libpot: argument checks, workspace layout, the
// solve driver and the C ABI declared in include/pot.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include <unistd.h>

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
hipError_t launch_zero_words(unsigned long long* p, int n, hipStream_t st);
hipError_t launch_warm_decide(const PassArgs& A, int mode, hipStream_t st);
hipError_t launch_result(const PassArgs& A, int algo, pot_result* res, hipStream_t st);
hipError_t launch_moments(const PassArgs& A, double* mom, hipStream_t st);

hipError_t launch_stats_timed(const PassArgs& A, hipStream_t st, hipEvent_t e0, hipEvent_t e1, hipEvent_t e2,
                              hipEvent_t e3);
int batched_blocks_per_cu(int kind);
hipError_t launch_warm(const WDesc* desc_dev, int batch, const void* blob, float* ctx, hipStream_t st);
size_t warm_desc_bytes();
void warm_fill_desc(void* dst, const float* x, const float* y, const double* r, const double* c, double* u0,
                    double* v0, double cost_scale, double inv_gamma, int n, int m);
hipError_t launch_batched(const BArgs& B, int kind, int grid, hipStream_t st);

// last error of this thread: a fixed buffer (recording an error allocates nothing)
static thread_local char g_last_error[512];

static pot_status fail(pot_status st, const char* msg, const char* detail = nullptr) {
    if (detail) std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s", msg, detail);
    else std::snprintf(g_last_error, sizeof(g_last_error), "%s", msg);
    return st;
}

static void clear_error() { g_last_error[0] = '\0'; }

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
        // default: 128-row tiles when they give at least 2 workgroups per CU
        // (512 on 256 CUs), else 64; measured best on 4096 x 4096 (FP32: 128,
        // BF16: 64) and on 20000 x 20000 (128 beats 256 and 64)
        const int nx = (p->m + g.bc - 1) / g.bc;
        br = (int64_t)nx * ((p->n + 127) / 128) >= 512 ? 128 : 64;
    }
    br = std::max(4, std::min(br, 256));
    g.br = br;
    g.nx = (p->m + g.bc - 1) / g.bc;
    g.ny = (p->n + g.br - 1) / g.br;
    return g;
}

// Tile heights the tuner tries (tile_rows = -1).
static const int kTileCand[] = {64, 128, 256};

static Geometry geometry_rows(const pot_problem* p, int br) {
    pot_options o;
    std::memset(&o, 0, sizeof(o));
    o.tile_rows = br;
    return geometry(p, &o);
}

// Workspace bytes of a solve (tile_rows = -1: enough for every candidate height).
static size_t layout(const pot_problem* p, const Geometry& g, char* base, Ws* w);
static size_t workspace_bytes(const pot_problem* p, const pot_options* o) {
    size_t need = layout(p, geometry(p, o), nullptr, nullptr);
    if (o && o->tile_rows == -1)
        for (int br : kTileCand) need = std::max(need, layout(p, geometry_rows(p, br), nullptr, nullptr));
    return need;
}

// ---------------------------------------------------------------------------
// Tuning results, kept in memory and, when the environment variable
// POT_TUNE_CACHE names a file, in that file: one JSON object whose keys name
// the device architecture, the tuned launch, the cost kind and the shape
// bucket, and whose values are arrays of integers.  The file is read when a
// lookup misses in memory and rewritten (merged with what it holds, through a
// temporary file and a rename) after each new entry; a file that does not
// parse is ignored.
// ---------------------------------------------------------------------------
typedef std::map<std::string, std::vector<long long>> TuneMap;
static std::mutex g_tc_mu;
static TuneMap g_tc;

static bool tc_parse(const std::string& t, TuneMap& out) {
    size_t i = 0;
    auto ws = [&]() { while (i < t.size() && (t[i] == ' ' || t[i] == '\n' || t[i] == '\r' || t[i] == '\t')) ++i; };
    auto eat = [&](char c) { ws(); if (i < t.size() && t[i] == c) { ++i; return true; } return false; };
    if (!eat('{')) return false;
    if (eat('}')) return true;
    for (;;) {
        if (!eat('"')) return false;
        const size_t k0 = i;
        while (i < t.size() && t[i] != '"' && t[i] != '\\') ++i;
        if (i >= t.size() || t[i] != '"') return false;
        const std::string key = t.substr(k0, i - k0);
        ++i;
        if (!eat(':') || !eat('[')) return false;
        std::vector<long long> v;
        if (!eat(']')) {
            for (;;) {
                ws();
                char* end = nullptr;
                const long long x = std::strtoll(t.c_str() + i, &end, 10);
                if (end == t.c_str() + i) return false;
                i = end - t.c_str();
                v.push_back(x);
                if (eat(']')) break;
                if (!eat(',')) return false;
            }
        }
        out[key] = v;
        if (eat('}')) return true;
        if (!eat(',')) return false;
    }
}

static bool tc_read_file(const char* path, TuneMap& out) {
    std::ifstream f(path, std::ios::binary);
    if (!f) return false;
    std::string text((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
    TuneMap m;
    if (!tc_parse(text, m)) return false;
    for (auto& kv : m) out[kv.first] = kv.second;
    return true;
}

static std::string tc_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a(prop.gcnArchName);
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

static bool tc_lookup(const std::string& key, std::vector<long long>& v) {
    std::lock_guard<std::mutex> lk(g_tc_mu);
    auto it = g_tc.find(key);
    if (it == g_tc.end()) {
        const char* path = std::getenv("POT_TUNE_CACHE");
        if (!path || !*path) return false;
        tc_read_file(path, g_tc);
        it = g_tc.find(key);
        if (it == g_tc.end()) return false;
    }
    v = it->second;
    return true;
}

static void tc_store(const std::string& key, const std::vector<long long>& v) {
    std::lock_guard<std::mutex> lk(g_tc_mu);
    g_tc[key] = v;
    const char* path = std::getenv("POT_TUNE_CACHE");
    if (!path || !*path) return;
    TuneMap all;
    tc_read_file(path, all);                 // entries other processes wrote meanwhile
    for (auto& kv : g_tc) all[kv.first] = kv.second;
    const std::string tmp = std::string(path) + ".tmp." + std::to_string((long long)getpid());   // (one per process)
    {
        std::ofstream f(tmp, std::ios::binary | std::ios::trunc);
        if (!f) return;
        f << "{";
        bool first = true;
        for (auto& kv : all) {
            f << (first ? "\n" : ",\n") << "  \"" << kv.first << "\": [";
            for (size_t k = 0; k < kv.second.size(); ++k) f << (k ? ", " : "") << kv.second[k];
            f << "]";
            first = false;
        }
        f << "\n}\n";
        if (!f) {
            f.close();
            std::remove(tmp.c_str());
            return;
        }
    }
    if (std::rename(tmp.c_str(), path) != 0) std::remove(tmp.c_str());
}

// shape bucket of a dimension: the power of two nearest to it (in log scale)
static int tc_bucket(int x) {
    int b = 1;
    while ((int64_t)b * 2 <= x) b *= 2;
    return ((int64_t)x * x >= (int64_t)b * b * 2) ? 2 * b : b;
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
    if (o->gamma_rule < 0 || o->gamma_rule > 1) return fail(POT_ERR_INVALID_ARG, "gamma_rule is 0 or 1");
    if (o->gamma_rule == 1 && o->algo != POT_SINKHORN)
        return fail(POT_ERR_INVALID_ARG, "gamma_rule 1 (the tuned rule of Algorithm 3) is for algo Sinkhorn");
    if (o->gamma_rule == 1 && !(o->p >= 1.0 && std::isfinite(o->p)))
        return fail(POT_ERR_INVALID_ARG, "the tuned rule needs a finite p >= 1");
    if (o->gamma <= 0.0 && o->gamma_rule == 0 && std::max(p->n, p->m) < 2)
        return fail(POT_ERR_INVALID_ARG, "default gamma needs max(n, m) >= 2 (ln 1 = 0)");
    if (o->algo != POT_ASPOT && o->algo != POT_SINKHORN) return fail(POT_ERR_INVALID_ARG, "unknown algo");
    if (o->block_rule < 0 || o->block_rule > 1) return fail(POT_ERR_INVALID_ARG, "block_rule");
    if (o->step_rule < 0 || o->step_rule > 1) return fail(POT_ERR_INVALID_ARG, "step_rule");
    if (o->force_len < 0 || (o->force_len > 0 && !o->force)) return fail(POT_ERR_INVALID_ARG, "force");
    if (o->trace_cap < 0) return fail(POT_ERR_INVALID_ARG, "trace_cap");
    if (o->tile_rows < -1 || o->tile_rows > 256) return fail(POT_ERR_INVALID_ARG, "tile_rows in [-1, 256]");
    if (!std::isfinite(o->w0)) return fail(POT_ERR_INVALID_ARG, "w0 not finite");
    return POT_OK;
}

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(POT_ERR_DEVICE, #expr, hipGetErrorString(e_));                \
    } while (0)

// pinned slots for convergence polling (host memory, allocated once per thread)
struct PollSlots {
    int32_t* flag = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
};
static thread_local PollSlots g_poll;

static pot_status ensure_poll() {
    if (!g_poll.flag) {
        HIPCHK(hipHostMalloc((void**)&g_poll.flag, 2 * sizeof(int32_t), hipHostMallocCoherent));
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

// Median durations (ms) of the statistics pass at the start point (opts'
// u0, v0, w0) with tile geometry g, over `reps` launches after 3 untimed
// ones: the tile kernel in *avg_ms, the finalising kernel in *fin_ms (the
// host waits for the launches).  prob->cmax (and cost_scale) must be set.
static pot_status time_tile(const pot_problem* prob, const pot_options* opts, const Geometry& g, void* ws, int reps,
                            double* avg_ms, double* fin_ms, hipStream_t st) {
    Ws w;
    layout(prob, g, (char*)ws, &w);
    SetupArgs S{};
    S.n = prob->n; S.m = prob->m; S.algo = POT_ASPOT; S.nx = g.nx; S.ny = g.ny;
    S.gamma_rule = opts->gamma_rule; S.p = opts->p;
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
    // 3 untimed launches, then `reps` timed ones; the medians are reported
    for (int k = 0; k < 3; ++k) HIPCHK(launch_stats(A, st));
    std::vector<hipEvent_t> ev(4 * (size_t)reps);
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    for (int k = 0; k < reps; ++k)
        HIPCHK(launch_stats_timed(A, st, ev[4 * k], ev[4 * k + 1], ev[4 * k + 2], ev[4 * k + 3]));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<double> t1(reps), t2(reps);
    for (int k = 0; k < reps; ++k) {
        float ms = 0.f, ms2 = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ev[4 * k], ev[4 * k + 1]));
        HIPCHK(hipEventElapsedTime(&ms2, ev[4 * k + 2], ev[4 * k + 3]));
        t1[k] = ms;
        t2[k] = ms2;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    auto median = [](std::vector<double>& v) {
        std::sort(v.begin(), v.end());
        const size_t h = v.size() / 2;
        return v.size() % 2 ? v[h] : 0.5 * (v[h - 1] + v[h]);
    };
    Ctl hc;
    HIPCHK(hipMemcpy(&hc, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    if (hc.valid != 0) return fail(POT_ERR_INVALID_ARG, "invalid problem");
    if (hc.status != POT_OK) return fail((pot_status)hc.status, "pass reported a non-finite sum");
    *avg_ms = median(t1);
    if (fin_ms) *fin_ms = median(t2);
    return POT_OK;
}

// Tile height for tile_rows = -1: from the tuning results when this
// architecture, cost kind and shape bucket have been tuned; otherwise, in a
// synchronous solve, each of kTileCand is timed on the problem's start pass
// (3 launches each, in the caller's workspace, which pot_workspace_bytes
// sizes for every candidate) and the fastest is kept; an asynchronous solve
// does not time (it takes the default height).
static Geometry tuned_geometry(const pot_problem* p, const pot_options* o, void* ws, bool async, hipStream_t st) {
    const Geometry dflt = geometry(p, o);
    char key[160];
    std::snprintf(key, sizeof(key), "%s/tile/kind%d/n%d/m%d", tc_arch().c_str(), p->kind, tc_bucket(p->n),
                  tc_bucket(p->m));
    std::vector<long long> v;
    // (a recorded height is taken only if it is a candidate: the workspace is
    // sized for the candidates)
    if (tc_lookup(key, v) && v.size() == 1 && std::count(std::begin(kTileCand), std::end(kTileCand), v[0]) == 1)
        return geometry_rows(p, (int)v[0]);
    if (async) return dflt;
    pot_problem q = *p;                                   // (timing only: any scale will do)
    if (!(q.cmax > 0.0)) q.cmax = 1.0;
    if (q.kind == POT_COST_SQEUCLID_POINTS && !(q.cost_scale > 0.0)) q.cost_scale = 1.0;
    int best = dflt.br;
    double best_ms = 1e300;
    for (int br : kTileCand) {
        double ms = 0.0;
        if (time_tile(&q, o, geometry_rows(p, br), ws, 3, &ms, nullptr, st) != POT_OK) return dflt;
        if (ms < best_ms) {
            best_ms = ms;
            best = br;
        }
    }
    tc_store(key, {best});
    return geometry_rows(p, best);
}

// Largest max_iter of an asynchronous solve (every iteration is enqueued).
constexpr int kAsyncMaxIter = 1 << 20;

// One solve.  Synchronous (the default): the host polls a pinned done flag
// between chunks of iterations and fills the host pot_result.  Asynchronous
// (POT_FLAG_ASYNC, or `force_async` for the entry point without allocation):
// everything is enqueued on `st`, every decision is taken on the device and
// `res` is a device pointer.  `direct` launches every kernel from the host
// (no graph is instantiated).
static pot_status solve_one(const pot_problem* p, const pot_options* o, void* wsp, size_t ws_bytes,
                            pot_result* res, const pot_outputs* out, hipStream_t st, bool force_async = false,
                            bool direct = false) {
    pot_status cs = check_problem(p, o);
    if (cs != POT_OK) return cs;
    if (!res) return fail(POT_ERR_INVALID_ARG, "res is required");
    if (o->warm_check < 0 || o->warm_check > 1) return fail(POT_ERR_INVALID_ARG, "warm_check is 0 or 1");
    if (o->reserved0 != 0) return fail(POT_ERR_INVALID_ARG, "reserved0 must be 0");
    const bool async = force_async || (o->flags & POT_FLAG_ASYNC);
    if (async) {
        if (o->max_iter < 1 || o->max_iter > kAsyncMaxIter)
            return fail(POT_ERR_INVALID_ARG, "an asynchronous solve needs 1 <= max_iter <= 2^20 (every iteration is enqueued)");
        if (out && out->w) return fail(POT_ERR_INVALID_ARG, "out->w (host) must be NULL in an asynchronous solve");
    }
    if (out && out->moments && p->kind != POT_COST_SQEUCLID_POINTS)
        return fail(POT_ERR_INVALID_ARG, "plan moments need the points cost");
    if (!wsp || ws_bytes < workspace_bytes(p, o)) return fail(POT_ERR_WORKSPACE, "workspace too small");
    if (((uintptr_t)wsp) & 255) return fail(POT_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    const Geometry g = o->tile_rows == -1 ? tuned_geometry(p, o, wsp, async, st) : geometry(p, o);
    const size_t need = layout(p, g, nullptr, nullptr);
    char* base = (char*)wsp;
    Ws w;
    layout(p, g, base, &w);
    if (!async) {
        pot_status ps = ensure_poll();
        if (ps != POT_OK) return ps;
    }

    // --- cost scale and |C|_max: one pass when not given.  Synchronously the
    // host reads the maximum back and checks it; asynchronously the setup
    // kernel reads it on the device.
    double cost_scale = p->kind == POT_COST_SQEUCLID_POINTS ? p->cost_scale : 1.0, cmax = p->cmax;
    const bool need_max = p->kind == POT_COST_SQEUCLID_POINTS ? (cost_scale <= 0.0 || cmax <= 0.0) : cmax <= 0.0;
    const unsigned long long* maxdev = nullptr;
    if (need_max) {
        unsigned long long* mb = maxbuf(base, need);
        HIPCHK(launch_zero_words(mb, 2, st));
        if (p->kind == POT_COST_SQEUCLID_POINTS)
            HIPCHK(launch_cost_max(p->kind, nullptr, 0, p->x, p->y, p->n, p->m, p->d, mb, st));
        else
            HIPCHK(launch_cost_max(p->kind, p->C, p->ldc, nullptr, nullptr, p->n, p->m, 0, mb, st));
        if (async) {
            maxdev = mb;
        } else {
            unsigned long long h[2];
            HIPCHK(hipMemcpyAsync(h, mb, 16, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            double mx;
            std::memcpy(&mx, &h[0], 8);
            if (p->kind == POT_COST_SQEUCLID_POINTS) {
                if (h[1] != 0) return fail(POT_ERR_INVALID_ARG, "non-finite point coordinates");
                if (!(mx > 0.0)) return fail(POT_ERR_INVALID_ARG, "all points coincide (max cost 0)");
                if (cost_scale <= 0.0) cost_scale = 1.0 / mx;
                if (cmax <= 0.0) cmax = cost_scale * mx;
            } else {
                if (h[1] != 0) return fail(POT_ERR_INVALID_ARG, "cost has negative or non-finite entries");
                cmax = mx;
                if (!(cmax > 0.0)) return fail(POT_ERR_INVALID_ARG, "cost is identically 0 (|C|_max = 0)");
            }
        }
    }

    // every exponent log2(e) C_ij / gamma must stay below 2^29 (the kernels
    // split exponents into an int32 part and a fraction; the setup kernel
    // checks it again, also for the tuned rule's gamma and a device-side cmax)
    if (!maxdev && (o->gamma > 0.0 || o->gamma_rule == 0)) {
        const int N = std::max(p->n, p->m);
        const double gam = o->gamma > 0.0 ? o->gamma : o->eps / (4.0 * std::log((double)N));
        if (!(1.4426950408889634 * cmax / gam < 536870912.0))
            return fail(POT_ERR_INVALID_ARG, "|C|_max / gamma too large (exponents beyond 2^29)");
    }

    // --- setup (Algorithm 2, "Approximating POT") and validation of r, c, s
    SetupArgs S{};
    S.n = p->n; S.m = p->m; S.algo = o->algo; S.nx = g.nx; S.ny = g.ny;
    S.gamma_rule = o->gamma_rule; S.p = o->p;
    S.s = p->s; S.eps = o->eps; S.gamma_user = o->gamma; S.tol_user = o->tol; S.A_user = o->A;
    S.cmax = cmax; S.cost_scale = cost_scale; S.w0 = o->w0;
    S.r = p->r; S.c = p->c; S.maxbuf = maxdev; S.kind = p->kind;
    S.warm = (o->algo == POT_ASPOT && (o->u0 || o->v0)) ? 1 : 0;
    S.ws = w;
    HIPCHK(launch_setup(S, st));
    if (!async) {
        int32_t valid = 0;
        HIPCHK(hipMemcpyAsync(&valid, &w.ctl->valid, 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (valid != 0) {
            static const char* why[] = {"", "r or c has a negative or non-finite entry",
                                        "s must satisfy 0 < s <= min(|r|_1, |c|_1)", "gamma is not positive",
                                        "eps~ capped to 0 (s equals a mass above 1) and no tol given",
                                        "a smoothed marginal is not positive", "",
                                        "|C|_max / gamma too large (exponents beyond 2^29)",
                                        "the tuned rule needs min(H(r), H(c)) > 0",
                                        "cost has negative or non-finite entries",
                                        "cost is identically 0 (|C|_max = 0)",
                                        "non-finite point coordinates", "all points coincide (max cost 0)"};
            return fail(POT_ERR_INVALID_ARG, why[valid < 13 ? valid : 0]);
        }
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
    A.host_done = async ? nullptr : g_poll.flag;
    A.ws = w;

    // --- start point.  With warm_check the zero start is evaluated first and
    // the warm start is kept only if phi is lower there; the third start pass
    // evaluates whichever was kept.  (The pinned flag is cleared before any
    // pass that may set it.)
    if (!async) *(volatile int32_t*)g_poll.flag = 0;
    if (o->algo == POT_ASPOT) {
        if (S.warm && o->warm_check) {
            PassArgs Z = A;
            Z.u0 = nullptr;
            Z.v0 = nullptr;
            Z.w0 = 0.0;
            Z.phase = PH_INIT;
            HIPCHK(launch_stats(Z, st));
            HIPCHK(launch_warm_decide(A, 0, st));
            A.phase = PH_INIT;
            HIPCHK(launch_stats(A, st));
            HIPCHK(launch_warm_decide(A, 1, st));
        }
        A.phase = PH_INIT;
        HIPCHK(launch_stats(A, st));
    }

    // --- the iteration loop, enqueued in chunks (a captured graph of `chunk`
    // iterations, unless disabled, the caller's stream is being captured or
    // no graph may be instantiated).  Synchronously, the decider sets a pinned
    // host flag when the solve finishes, and the host reads it after the
    // previous chunk has completed while the next one runs (no copy is
    // enqueued between chunks).  Asynchronously every iteration is enqueued;
    // passes after the stop return at once.
    const int chunk = o->check_every > 0 ? o->check_every : 16;
    bool capturing = false;
    if (st) {           // (the null stream cannot be captured)
        hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
        HIPCHK(hipStreamIsCapturing(st, &cst));
        capturing = cst != hipStreamCaptureStatusNone;
    }
    if (capturing && !async) return fail(POT_ERR_INVALID_ARG, "a solve inside a stream capture needs POT_FLAG_ASYNC");
    hipGraphExec_t gexec = nullptr;
    if (!direct && !capturing && !(o->flags & POT_FLAG_NO_GRAPH) && A.max_iter >= chunk)
        HIPCHK(chunk_graph(A, o->algo, chunk, &gexec));
    int enq = 0, k = 0;
    bool done = false;
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
        if (!async) {
            const int slot = k & 1;
            HIPCHK(hipEventRecord(g_poll.ev[slot], st));
            if (k > 0) {
                HIPCHK(hipEventSynchronize(g_poll.ev[slot ^ 1]));
                done = *(volatile int32_t*)g_poll.flag != 0;
            }
        }
        ++k;
    }
    if (o->algo == POT_SINKHORN) {
        // the row pass that checks the last iterate (and stops at max_iter)
        A.phase = PH_SK_ROW;
        HIPCHK(launch_stats(A, st));
    }

    // --- form primal and round onto U(r, c, s) in FP64 (the rounding kernels
    // run only after a finished loop with representable statistics)
    HIPCHK(launch_finish(A, o->algo, out ? out->f : nullptr, out ? out->g : nullptr,
                         out ? out->u : nullptr, out ? out->v : nullptr, st));
    auto enqueue_round = [&]() -> pot_status {
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
        if (out && out->moments) {
            A.phase = PH_R5;
            HIPCHK(launch_round(A, st));
            HIPCHK(launch_moments(A, out->moments, st));
        }
        return POT_OK;
    };
    if (async) {
        if (!(o->flags & POT_FLAG_NO_ROUND)) {
            pot_status rs = enqueue_round();
            if (rs != POT_OK) return rs;
        }
        HIPCHK(launch_result(A, o->algo, res, st));
        clear_error();
        return POT_OK;
    }
    Ctl hc;
    HIPCHK(hipMemcpyAsync(&hc, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (!(o->flags & POT_FLAG_NO_ROUND) && hc.status != POT_ERR_NUMERIC && hc.done) {
        pot_status rs = enqueue_round();
        if (rs != POT_OK) return rs;
    }
    HIPCHK(launch_result(A, o->algo, nullptr, st));
    HIPCHK(hipMemcpyAsync(&hc, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (!hc.done) return fail(POT_ERR_DEVICE, "solver loop ended without a decision");

    std::memset(res, 0, sizeof(*res));
    fill_result(hc, o->algo, *res);
    if (out && out->w) *out->w = res->w;
    if (hc.status == POT_ERR_NUMERIC) fail(POT_ERR_NUMERIC, "non-finite row or column sum (overflow)");
    else if (hc.status == POT_ERR_NO_CONVERGENCE) fail(POT_ERR_NO_CONVERGENCE, "max_iter reached before E <= tol");
    else clear_error();
    return (pot_status)hc.status;
}

// ---------------------------------------------------------------------------
// the solve that allocates nothing: its workspace is a file-scope device
// array, one per GPU, reached through the address the runtime reports for it
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[POT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// Device address of this device's copy of `scratch` (looked up once per
// device, with that device current).
static pot_status scratch_ptr(void** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(POT_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(POT_ERR_DEVICE, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return POT_OK;
}

// ---------------------------------------------------------------------------
// rigid registration (Section 4 and its appendix): the outer loop around the
// single-instance solve
// ---------------------------------------------------------------------------
hipError_t launch_transform(const float* y, float* yk, int m, const RigidMap& F, hipStream_t st);
hipError_t launch_scale_duals(const double* u, const double* v, double* u0, double* v0, int n, int m, double sc,
                              hipStream_t st);
hipError_t launch_record_step(const float* yk, const double* u, const double* v, int n, int m, double w, float* yh,
                              double* dh, hipStream_t st);
void rigid_align(const double* H, double* R);

// workspace of a registration: the solve's workspace, then the moved cloud,
// the solve's outputs, the warm-start duals and the plan moments
struct RegLayout {
    size_t solve, yk, vec, total;
};

static pot_problem reg_solve_problem(const pot_reg_problem* p, const float* yk, double cost_scale) {
    pot_problem q;
    std::memset(&q, 0, sizeof(q));
    q.n = p->n;
    q.m = p->m;
    q.d = 3;
    q.kind = POT_COST_SQEUCLID_POINTS;
    q.x = p->x;
    q.y = yk;
    q.cost_scale = cost_scale;
    q.cmax = 0.0;
    q.r = p->r;
    q.c = p->c;
    q.s = p->s;
    return q;
}

static RegLayout reg_layout(const pot_reg_problem* p) {
    pot_options so;
    std::memset(&so, 0, sizeof(so));
    const pot_problem q = reg_solve_problem(p, nullptr, 1.0);
    RegLayout L;
    L.solve = layout(&q, geometry(&q, &so), nullptr, nullptr);
    L.yk = L.solve;
    L.vec = L.yk + align256(sizeof(float) * 3 * (size_t)p->m);
    // f, u, alpha, pp, u0 (n each); g, v, beta, qq, v0 (m each); moments (16)
    L.total = L.vec + 5 * align256(8 * (size_t)p->n) + 5 * align256(8 * (size_t)p->m) + 256;
    return L;
}

static pot_status check_reg(const pot_reg_problem* p, const pot_reg_options* o) {
    if (!p || !o) return fail(POT_ERR_INVALID_ARG, "null problem or options");
    if (p->n < 2 || p->m < 2) return fail(POT_ERR_INVALID_ARG, "registration needs n, m >= 2");
    if (!p->x || !p->y || !p->r || !p->c) return fail(POT_ERR_INVALID_ARG, "x, y, r and c are required");
    if (!(p->s > 0.0) || !std::isfinite(p->s)) return fail(POT_ERR_INVALID_ARG, "s must be finite and > 0");
    if (!std::isfinite(p->cost_scale)) return fail(POT_ERR_INVALID_ARG, "cost_scale not finite");
    if (!(o->eps > 0.0) || !std::isfinite(o->eps)) return fail(POT_ERR_INVALID_ARG, "eps must be finite and > 0");
    if (!(o->gamma0 > 0.0) || !std::isfinite(o->gamma0)) return fail(POT_ERR_INVALID_ARG, "gamma0 must be > 0");
    if (!(o->anneal > 0.0 && o->anneal <= 1.0)) return fail(POT_ERR_INVALID_ARG, "anneal must lie in (0, 1]");
    if (!std::isfinite(o->gamma_min)) return fail(POT_ERR_INVALID_ARG, "gamma_min not finite");
    if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return fail(POT_ERR_INVALID_ARG, "tol must be > 0");
    if (o->max_steps < 1) return fail(POT_ERR_INVALID_ARG, "max_steps >= 1");
    if (o->algo != POT_ASPOT && o->algo != POT_SINKHORN) return fail(POT_ERR_INVALID_ARG, "unknown algo");
    if (o->warm < 0 || o->warm > 1) return fail(POT_ERR_INVALID_ARG, "warm is 0 or 1");
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(o->R0[k])) return fail(POT_ERR_INVALID_ARG, "R0 not finite");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(o->t0[k])) return fail(POT_ERR_INVALID_ARG, "t0 not finite");
    return POT_OK;
}

static pot_status register_rigid(const pot_reg_problem* p, const pot_reg_options* o, void* wsp, size_t ws_bytes,
                                 pot_reg_result* res, const pot_reg_history* hist, float* y_out, hipStream_t st) {
    pot_status cs = check_reg(p, o);
    if (cs != POT_OK) return cs;
    if (!res) return fail(POT_ERR_INVALID_ARG, "res is required");
    const RegLayout L = reg_layout(p);
    if (!wsp || ws_bytes < L.total) return fail(POT_ERR_WORKSPACE, "workspace too small");
    if (((uintptr_t)wsp) & 255) return fail(POT_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    const int n = p->n, m = p->m;
    char* base = (char*)wsp;
    float* yk = (float*)(base + L.yk);
    size_t off = L.vec;
    auto vecn = [&](size_t len) {
        double* q = (double*)(base + off);
        off += align256(8 * len);
        return q;
    };
    double *f = vecn(n), *u = vecn(n), *alpha = vecn(n), *pp = vecn(n), *u0 = vecn(n);
    double *g = vecn(m), *v = vecn(m), *beta = vecn(m), *qq = vecn(m), *v0 = vecn(m);
    double* mom = (double*)(base + off);

    RigidMap F;
    std::memcpy(F.R, o->R0, sizeof(F.R));
    std::memcpy(F.t, o->t0, sizeof(F.t));
    // the cost scale: fixed over the run (1 / max |x - F0(y)|^2 unless given)
    double scale = p->cost_scale;
    if (!(scale > 0.0)) {
        HIPCHK(launch_transform(p->y, yk, m, F, st));
        unsigned long long* mb = (unsigned long long*)mom;
        HIPCHK(launch_zero_words(mb, 2, st));
        HIPCHK(launch_cost_max(POT_COST_SQEUCLID_POINTS, nullptr, 0, p->x, yk, n, m, 3, mb, st));
        unsigned long long h[2];
        HIPCHK(hipMemcpyAsync(h, mb, 16, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        double mx;
        std::memcpy(&mx, &h[0], 8);
        if (h[1] != 0) return fail(POT_ERR_INVALID_ARG, "non-finite point coordinates");
        if (!(mx > 0.0)) return fail(POT_ERR_INVALID_ARG, "all points coincide (max cost 0)");
        scale = 1.0 / mx;
    }
    const double gfloor = o->gamma_min > 0.0 ? o->gamma_min : o->eps / (4.0 * std::log((double)std::max(n, m)));
    std::memset(res, 0, sizeof(*res));
    res->status = POT_OK;
    double prev_cost = 0.0, prev_gamma = 0.0, prev_w = 0.0;
    int steps = 0;
    for (int k = 0; k < o->max_steps; ++k) {
        HIPCHK(launch_transform(p->y, yk, m, F, st));
        const double gam = std::max(o->gamma0 * std::pow(o->anneal, (double)k), gfloor);
        pot_options so;
        std::memset(&so, 0, sizeof(so));
        so.algo = o->algo;
        so.eps = o->eps;
        so.gamma = gam;
        so.max_iter = o->max_iter;
        const bool warm = o->warm && k > 0 && o->algo == POT_ASPOT;
        if (warm) {
            const double sc = prev_gamma / gam;
            HIPCHK(launch_scale_duals(u, v, u0, v0, n, m, sc, st));
            so.u0 = u0;
            so.v0 = v0;
            so.w0 = prev_w * sc;
        }
        const pot_problem q = reg_solve_problem(p, yk, scale);
        pot_outputs out;
        std::memset(&out, 0, sizeof(out));
        out.f = f; out.g = g; out.u = u; out.v = v;
        out.alpha = alpha; out.beta = beta; out.pp = pp; out.qq = qq;
        out.moments = mom;
        pot_result r;
        pot_status s = solve_one(&q, &so, base, L.solve, &r, &out, st);
        if (s != POT_OK && s != POT_ERR_NO_CONVERGENCE) {
            res->status = s;
            res->steps = steps;
            return s;
        }
        if (r.status == POT_ERR_NO_CONVERGENCE) res->status = POT_ERR_NO_CONVERGENCE;
        double M[16];
        HIPCHK(hipMemcpyAsync(M, mom, sizeof(M), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        // the map aligning F_k(Y) to X under the plan: barycentres, centred
        // cross-covariance H = M - mass u_x u_y^T, rotation, translation
        const double mass = M[15];
        if (!(mass > 0.0) || !std::isfinite(mass)) return fail(POT_ERR_NUMERIC, "plan of zero mass");
        double ux[3], uy[3], H[9], dR[9], dt[3];
        for (int a = 0; a < 3; ++a) {
            ux[a] = M[9 + a] / mass;
            uy[a] = M[12 + a] / mass;
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) H[3 * a + b] = M[3 * a + b] - mass * ux[a] * uy[b];
        rigid_align(H, dR);
        for (int a = 0; a < 3; ++a) dt[a] = ux[a] - (dR[3 * a] * uy[0] + dR[3 * a + 1] * uy[1] + dR[3 * a + 2] * uy[2]);
        RigidMap G;
        for (int a = 0; a < 3; ++a) {
            for (int b = 0; b < 3; ++b)
                G.R[3 * a + b] = dR[3 * a] * F.R[b] + dR[3 * a + 1] * F.R[3 + b] + dR[3 * a + 2] * F.R[6 + b];
            G.t[a] = dR[3 * a] * F.t[0] + dR[3 * a + 1] * F.t[1] + dR[3 * a + 2] * F.t[2] + dt[a];
        }
        F = G;
        if (hist) {
            if (hist->iters) hist->iters[k] = r.iters;
            if (hist->cost) hist->cost[k] = r.cost;
            if (hist->gamma) hist->gamma[k] = gam;
            if (hist->E) hist->E[k] = r.E;
            if (hist->Rt) {
                std::memcpy(hist->Rt + 12 * k, F.R, sizeof(F.R));
                std::memcpy(hist->Rt + 12 * k + 9, F.t, sizeof(F.t));
            }
            if (hist->y_hist || hist->dual_hist)
                HIPCHK(launch_record_step(yk, u, v, n, m, r.w, hist->y_hist ? hist->y_hist + (size_t)3 * m * k : nullptr,
                                          hist->dual_hist ? hist->dual_hist + (size_t)(n + m + 1) * k : nullptr, st));
        }
        res->total_iters += r.iters;
        steps = k + 1;
        res->cost = r.cost;
        prev_gamma = gam;
        prev_w = r.w;
        const bool stop = k > 0 && std::fabs(r.cost - prev_cost) <= o->tol * std::fabs(prev_cost);
        prev_cost = r.cost;
        if (stop) break;
    }
    res->steps = steps;
    std::memcpy(res->R, F.R, sizeof(F.R));
    std::memcpy(res->t, F.t, sizeof(F.t));
    if (y_out) HIPCHK(launch_transform(p->y, y_out, m, F, st));
    HIPCHK(hipStreamSynchronize(st));
    clear_error();
    return (pot_status)res->status;
}

// ---------------------------------------------------------------------------
// shared-cost batches: exponential-domain feasible Sinkhorn for many members
// on one cost, products on the matrix cores (pot_shared.hip)
// ---------------------------------------------------------------------------
hipError_t launch_shared_build(int kind, const void* C, int64_t ldc, int n, int m, int Np, int Mp, double inv_gamma,
                               double corner, uint16_t* K, uint16_t* KT, hipStream_t st);
hipError_t launch_shared_gemm(const uint16_t* A, const uint16_t* Bop, float* Out, int rows, int cols, int depth,
                              const int32_t* ndone, int B, hipStream_t st);
hipError_t launch_shared_update(const float* prod, const float* mass, const float* cur, float* next, uint16_t* op,
                                int len, int ld, int B, const int32_t* done, double* err_part, hipStream_t st);
hipError_t launch_shared_decide(const SharedCtl& S, const double* err_part, int nblk, int B, int t, int max_iter,
                                hipStream_t st);
hipError_t launch_shared_gather(const Ws& w, int n, int m, int Np, int Mp, int b, int B, float* rhat, float* chat,
                                double* tol, const SharedCtl& S, hipStream_t st);
hipError_t launch_shared_init(float* bsc, uint16_t* bop, int m, int Mp, int B, const SharedCtl& S, hipStream_t st);
hipError_t launch_shared_load_duals(const Ws& w, const float* abuf, const float* bsc, int n, int m, int Np, int Mp,
                                    int Bp, int b, const SharedCtl& S, double* fo, double* go, hipStream_t st);

static int round_up(int x, int k) { return (x + k - 1) / k * k; }

// workspace of a shared-cost batch
struct SharedLayout {
    int Np, Mp, Bp, nblk;
    size_t solve, K, KT, abuf, bsc, aop, bop, P, Q, rhat, chat, errp, done, iters, status, outpar, E, tol, ndone,
        res, total;
};

static SharedLayout shared_layout(const pot_shared_cost* cost, int batch) {
    SharedLayout L;
    L.Np = round_up(cost->n + 1, 64);
    L.Mp = round_up(cost->m + 1, 64);
    L.Bp = round_up(batch, 64);
    L.nblk = (L.Np + 255) / 256;
    pot_problem q;
    std::memset(&q, 0, sizeof(q));
    q.n = cost->n;
    q.m = cost->m;
    q.kind = cost->kind;
    q.ldc = cost->ldc;
    pot_options so;
    std::memset(&so, 0, sizeof(so));
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    L.solve = take(layout(&q, geometry(&q, &so), nullptr, nullptr));
    const size_t NM = (size_t)L.Np * L.Mp;
    L.K = take(2 * NM);
    L.KT = take(2 * NM);
    L.abuf = take(4 * 2 * (size_t)L.Bp * L.Np);
    L.bsc = take(4 * (size_t)L.Bp * L.Mp);
    L.aop = take(2 * 2 * (size_t)L.Bp * L.Np);
    L.bop = take(2 * 2 * (size_t)L.Bp * L.Mp);
    L.P = take(4 * 2 * (size_t)L.Bp * L.Np);
    L.Q = take(4 * 2 * (size_t)L.Bp * L.Mp);
    L.rhat = take(4 * (size_t)L.Bp * L.Np);
    L.chat = take(4 * (size_t)L.Bp * L.Mp);
    L.errp = take(8 * (size_t)L.Bp * L.nblk);
    L.done = take(4 * (size_t)L.Bp);
    L.iters = take(4 * (size_t)L.Bp);
    L.status = take(4 * (size_t)L.Bp);
    L.outpar = take(4 * (size_t)L.Bp);
    L.E = take(8 * (size_t)L.Bp);
    L.tol = take(8 * (size_t)L.Bp);
    L.ndone = take(4);
    L.res = take(sizeof(pot_result) * (size_t)batch);
    L.total = off;
    return L;
}

static pot_status solve_shared(const pot_shared_cost* cost, int batch, const pot_shared_member* mem,
                               const pot_options* o, void* wsp, size_t ws_bytes, pot_result* res, hipStream_t st) {
    if (!cost || !mem || !o || !res || batch < 1) return fail(POT_ERR_INVALID_ARG, "cost, members, opts, res and batch >= 1 are required");
    if (cost->n < 1 || cost->m < 1) return fail(POT_ERR_INVALID_ARG, "n and m must be >= 1");
    if (cost->kind != POT_COST_F32 && cost->kind != POT_COST_BF16)
        return fail(POT_ERR_UNSUPPORTED, "the shared cost is dense FP32 or BF16");
    if (!cost->C || cost->ldc < cost->m) return fail(POT_ERR_INVALID_ARG, "C with ldc >= m is required");
    if (!std::isfinite(cost->cmax)) return fail(POT_ERR_INVALID_ARG, "cmax not finite");
    if (o->algo != POT_SINKHORN) return fail(POT_ERR_UNSUPPORTED, "shared-cost batches run feasible Sinkhorn (algo POT_SINKHORN)");
    if (!(o->gamma > 0.0) || !std::isfinite(o->gamma)) return fail(POT_ERR_INVALID_ARG, "a shared gamma > 0 is required");
    if (!(o->eps > 0.0) || !std::isfinite(o->eps)) return fail(POT_ERR_INVALID_ARG, "eps must be finite and > 0");
    if (!std::isfinite(o->tol) || !std::isfinite(o->A)) return fail(POT_ERR_INVALID_ARG, "tol and A must be finite");
    for (int b = 0; b < batch; ++b)
        if (!mem[b].r || !mem[b].c) return fail(POT_ERR_INVALID_ARG, "every member needs r and c");
    const SharedLayout L = shared_layout(cost, batch);
    if (!wsp || ws_bytes < L.total) return fail(POT_ERR_WORKSPACE, "workspace too small");
    if (((uintptr_t)wsp) & 255) return fail(POT_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    pot_status ps = ensure_poll();
    if (ps != POT_OK) return ps;
    char* base = (char*)wsp;
    const int n = cost->n, m = cost->m, Np = L.Np, Mp = L.Mp, Bp = L.Bp, B = batch;

    // |C|_max (one pass when not given) and the representability of K~
    double cmax = cost->cmax;
    if (!(cmax > 0.0)) {
        unsigned long long* mb = (unsigned long long*)(base + L.errp);
        HIPCHK(launch_zero_words(mb, 2, st));
        HIPCHK(launch_cost_max(cost->kind, cost->C, cost->ldc, nullptr, nullptr, n, m, 0, mb, st));
        unsigned long long h[2];
        HIPCHK(hipMemcpyAsync(h, mb, 16, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (h[1] != 0) return fail(POT_ERR_INVALID_ARG, "cost has negative or non-finite entries");
        std::memcpy(&cmax, &h[0], 8);
        if (!(cmax > 0.0)) return fail(POT_ERR_INVALID_ARG, "cost is identically 0 (|C|_max = 0)");
    }
    const double gamma = o->gamma;
    if (cmax / gamma > 80.0)
        return fail(POT_ERR_UNSUPPORTED, "max C / gamma > 80: the exponential-domain kernel would underflow "
                                         "(use pot_solve_batched, which works in the log domain)");
    const double A = o->A > 0.0 ? o->A : 8.0 * cmax / o->eps;

    uint16_t* K = (uint16_t*)(base + L.K);
    uint16_t* KT = (uint16_t*)(base + L.KT);
    float* abuf = (float*)(base + L.abuf);
    float* bsc = (float*)(base + L.bsc);
    uint16_t* aop = (uint16_t*)(base + L.aop);
    uint16_t* bop = (uint16_t*)(base + L.bop);
    float* P = (float*)(base + L.P);
    float* Q = (float*)(base + L.Q);
    float* rhat = (float*)(base + L.rhat);
    float* chat = (float*)(base + L.chat);
    double* errp = (double*)(base + L.errp);
    SharedCtl S;
    S.done = (int32_t*)(base + L.done);
    S.iters = (int32_t*)(base + L.iters);
    S.status = (int32_t*)(base + L.status);
    S.out_par = (int32_t*)(base + L.outpar);
    S.E = (double*)(base + L.E);
    S.tol = (const double*)(base + L.tol);
    S.ndone = (int32_t*)(base + L.ndone);
    S.host_done = g_poll.flag;
    pot_result* resd = (pot_result*)(base + L.res);

    // the operands of padded members and rows stay zero: clear the BF16
    // operands and scalings once (kernels, not memset nodes)
    HIPCHK(launch_zero_words((unsigned long long*)aop, (int)(2 * 2 * (size_t)Bp * Np / 8), st));
    HIPCHK(launch_zero_words((unsigned long long*)bop, (int)(2 * 2 * (size_t)Bp * Mp / 8), st));
    HIPCHK(launch_zero_words((unsigned long long*)abuf, (int)(4 * 2 * (size_t)Bp * Np / 8), st));
    HIPCHK(launch_shared_build(cost->kind, cost->C, cost->ldc, n, m, Np, Mp, 1.0 / gamma, std::exp(-A / gamma), K, KT, st));
    *(volatile int32_t*)g_poll.flag = 0;
    HIPCHK(launch_shared_init(bsc, bop, m, Mp, B, S, st));

    // the single-instance workspace: each member's setup (smoothing, extension, threshold)
    pot_problem q;
    std::memset(&q, 0, sizeof(q));
    q.n = n; q.m = m; q.kind = cost->kind; q.C = cost->C; q.ldc = cost->ldc;
    pot_options so;
    std::memset(&so, 0, sizeof(so));
    const Geometry g = geometry(&q, &so);
    Ws w;
    layout(&q, g, base + L.solve, &w);
    auto setup_member = [&](int b) -> hipError_t {
        SetupArgs Sa{};
        Sa.n = n; Sa.m = m; Sa.algo = POT_SINKHORN; Sa.nx = g.nx; Sa.ny = g.ny;
        Sa.gamma_rule = 0; Sa.p = 1.0;
        Sa.s = mem[b].s; Sa.eps = o->eps; Sa.gamma_user = gamma; Sa.tol_user = o->tol; Sa.A_user = A;
        Sa.cmax = cmax; Sa.cost_scale = 1.0; Sa.w0 = 0.0;
        Sa.r = mem[b].r; Sa.c = mem[b].c; Sa.maxbuf = nullptr; Sa.kind = cost->kind; Sa.warm = 0;
        Sa.ws = w;
        return launch_setup(Sa, st);
    };
    for (int b = 0; b < B; ++b) {
        HIPCHK(setup_member(b));
        HIPCHK(launch_shared_gather(w, n, m, Np, Mp, b, B, rhat, chat, (double*)S.tol, S, st));
    }

    // the loop: per iteration two products on the matrix cores, the scaling
    // updates and the per-member decision; the host reads the pinned flag
    // after the previous chunk has completed
    const int max_iter = o->max_iter > 0 ? o->max_iter : 100000;
    const int chunk = o->check_every > 0 ? o->check_every : 16;
    bool done = false;
    int t = 0, k = 0;
    while (!done && t <= max_iter) {
        for (int c = 0; c < chunk && t <= max_iter; ++c, ++t) {
            float* acur = abuf + (size_t)(t & 1) * Bp * Np;
            float* anext = abuf + (size_t)((t + 1) & 1) * Bp * Np;
            HIPCHK(launch_shared_gemm(K, bop, P, Np, 2 * Bp, Mp, S.ndone, B, st));
            HIPCHK(launch_shared_update(P, rhat, acur, anext, aop, n + 1, Np, B, S.done, errp, st));
            HIPCHK(launch_shared_decide(S, errp, L.nblk, B, t, max_iter, st));
            HIPCHK(launch_shared_gemm(KT, aop, Q, Mp, 2 * Bp, Np, S.ndone, B, st));
            HIPCHK(launch_shared_update(Q, chat, bsc, bsc, bop, m + 1, Mp, B, S.done, nullptr, st));
        }
        const int slot = k & 1;
        HIPCHK(hipEventRecord(g_poll.ev[slot], st));
        if (k > 0) {
            HIPCHK(hipEventSynchronize(g_poll.ev[slot ^ 1]));
            done = *(volatile int32_t*)g_poll.flag != 0;
        }
        ++k;
    }

    // per member: its setup again, its output scalings as log-scalings, the
    // FP64 rounding onto U(r_b, c_b, s_b) and its result block
    PassArgs Ar;
    std::memset(&Ar, 0, sizeof(Ar));
    Ar.C = cost->C; Ar.ldc = cost->ldc; Ar.n = n; Ar.m = m; Ar.kind = cost->kind;
    Ar.br = g.br; Ar.bc = g.bc; Ar.nx = g.nx; Ar.ny = g.ny;
    Ar.nrb = (n + 63) / 64; Ar.ncb = (m + 63) / 64;
    Ar.ws = w;
    for (int b = 0; b < B; ++b) {
        HIPCHK(setup_member(b));
        HIPCHK(launch_shared_load_duals(w, abuf, bsc, n, m, Np, Mp, Bp, b, S, mem[b].f, mem[b].g, st));
        Ar.r = mem[b].r;
        Ar.c = mem[b].c;
        if (!(o->flags & POT_FLAG_NO_ROUND))
            for (int ph : {PH_R1, PH_R2, PH_R3}) {
                Ar.phase = ph;
                HIPCHK(launch_round(Ar, st));
            }
        HIPCHK(launch_result(Ar, POT_SINKHORN, resd + b, st));
    }
    HIPCHK(hipMemcpyAsync(res, resd, sizeof(pot_result) * (size_t)B, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    pot_status first = POT_OK;
    for (int b = 0; b < B; ++b)
        if (res[b].status != POT_OK && first == POT_OK) first = (pot_status)res[b].status;
    if (first != POT_OK) fail(first, "a member of the shared-cost batch did not finish with POT_OK (see res[].status)");
    else clear_error();
    return first;
}

}  // namespace pot

using namespace pot;

// ---------------------------------------------------------------------------
// batched solver
// ---------------------------------------------------------------------------
// Smallest share of cost entries per group member the autotuner tries; the
// workspace is sized for the groups it gives.
constexpr int64_t kMemberMin = 1 << 15;
static const int64_t kMemberCand[] = {1 << 15, 1 << 16, 1 << 17, 1 << 18};

// members of an instance's group: rows split so that each member sweeps at
// most `share` entries (and at least 16 rows)
static int group_size(int n, int m, int64_t share) {
    int64_t g = ((int64_t)n * m + share - 1) / share;
    g = std::min<int64_t>(g, kBMaxGroup);
    g = std::min<int64_t>(g, std::max(1, n / 16));
    return (int)std::max<int64_t>(1, g);
}

// workspace of a batch: [queue][descriptors][slots][results][instance regions]
struct BatchLayout {
    int64_t desc, slot, res, inst;
    std::vector<int64_t> off;
};

static int64_t al256(int64_t x) { return (x + 255) & ~(int64_t)255; }

static size_t batch_layout(int batch, const pot_problem* probs, BatchLayout* L) {
    int64_t nslot = 0;
    for (int k = 0; k < batch; ++k) nslot += group_size(probs[k].n, probs[k].m, kMemberMin);
    int64_t cur = 256;
    const int64_t desc = cur;
    cur += al256((int64_t)sizeof(BDesc) * batch);
    const int64_t slot = cur;
    cur += al256((int64_t)sizeof(BSlot) * nslot);
    const int64_t resb = cur;
    cur += al256((int64_t)sizeof(pot_result) * batch);
    const int64_t inst = cur;
    if (L) {
        L->desc = desc;
        L->slot = slot;
        L->res = resb;
        L->inst = inst;
        L->off.resize(batch);
    }
    for (int k = 0; k < batch; ++k) {
        if (L) L->off[k] = cur;
        cur += blayout(probs[k].n, probs[k].m, group_size(probs[k].n, probs[k].m, kMemberMin)).total;
    }
    return (size_t)cur;
}

static int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

// one launch of the batched kernels (captured as a graph unless disabled)
struct BGraphEntry {
    std::string key;
    hipGraphExec_t exec = nullptr;
};
static thread_local BGraphEntry g_bgraphs[4];
static thread_local int g_bgraph_next = 0;

static hipError_t run_batched(const BArgs& B, int kind, int grid, bool use_graph, hipStream_t st) {
    if (!use_graph) return launch_batched(B, kind, grid, st);
    std::string key((const char*)&B, sizeof(B));
    key.append((const char*)&kind, sizeof(kind));
    key.append((const char*)&grid, sizeof(grid));
    hipGraphExec_t exec = nullptr;
    for (auto& g : g_bgraphs)
        if (g.exec && g.key == key) exec = g.exec;
    if (!exec) {
        if (!g_capture_stream) {
            hipError_t e = hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return e;
        }
        hipError_t e = hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        hipError_t le = launch_batched(B, kind, grid, g_capture_stream);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(g_capture_stream, &graph);
        if (le != hipSuccess) e = le;
        if (e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return e;
        }
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return e;
        BGraphEntry& slot = g_bgraphs[g_bgraph_next];
        g_bgraph_next = (g_bgraph_next + 1) % 4;
        if (slot.exec) (void)hipGraphExecDestroy(slot.exec);
        slot.key = key;
        slot.exec = exec;
    }
    return hipGraphLaunch(exec, st);
}

// Autotuner of the batched launch: the group share of cost entries per
// member and the workgroups per CU, timed on the batch itself (3 iterations,
// no rounding) and kept with the tuning results per batch shape.
struct BTune {
    int64_t share;
    int per_cu;
};

static pot_status solve_batched(int32_t batch, const pot_problem* probs, const pot_options* o, const pot_warm* warm,
                                void* wsp, size_t ws_bytes, pot_result* res, const pot_batch_outputs* out,
                                hipStream_t st) {
    if (batch < 1 || !probs || !o || !res) return fail(POT_ERR_INVALID_ARG, "batch, probs, opts and res are required");
    if (!(o->eps > 0.0) || !std::isfinite(o->eps)) return fail(POT_ERR_INVALID_ARG, "eps must be positive");
    if (o->algo != POT_ASPOT && o->algo != POT_SINKHORN) return fail(POT_ERR_INVALID_ARG, "algo");
    if (o->block_rule < 0 || o->block_rule > 1 || o->step_rule < 0 || o->step_rule > 1)
        return fail(POT_ERR_INVALID_ARG, "block_rule and step_rule are 0 or 1");
    if (o->member_elems < 0) return fail(POT_ERR_INVALID_ARG, "member_elems >= 0");
    if (o->gamma_rule < 0 || o->gamma_rule > 1) return fail(POT_ERR_INVALID_ARG, "gamma_rule is 0 or 1");
    if (o->gamma_rule == 1 && (o->algo != POT_SINKHORN || !(o->p >= 1.0 && std::isfinite(o->p))))
        return fail(POT_ERR_INVALID_ARG, "the tuned rule needs algo Sinkhorn and a finite p >= 1");
    if (o->force || o->trace_i || o->trace_d) return fail(POT_ERR_UNSUPPORTED, "force and trace are single-solve options");
    const int kind = probs[0].kind;
    if (kind != POT_COST_F32 && kind != POT_COST_BF16)
        return fail(POT_ERR_UNSUPPORTED, "pot_solve_batched takes dense FP32 or BF16 costs");
    int64_t total = 0, largest = 0;
    for (int k = 0; k < batch; ++k) {
        const pot_problem& p = probs[k];
        if (p.kind != kind) return fail(POT_ERR_UNSUPPORTED, "every instance of a batch has the same cost kind");
        if (p.n < 1 || p.m < 1 || p.n > kBMax || p.m > kBMax)
            return fail(POT_ERR_INVALID_ARG, "batched instances need 1 <= n, m <= 1024");
        if (!p.C || !p.r || !p.c) return fail(POT_ERR_INVALID_ARG, "C, r and c are required");
        if (p.ldc < p.m) return fail(POT_ERR_INVALID_ARG, "ldc < m");
        if (p.ldc * (kind == POT_COST_BF16 ? 2 : 4) >= ((int64_t)1 << 31))
            return fail(POT_ERR_INVALID_ARG, "batched instances need a row stride below 2^31 bytes");
        if (!(p.s > 0.0) || !std::isfinite(p.s)) return fail(POT_ERR_INVALID_ARG, "s must be positive");
        if (!std::isfinite(p.cmax)) return fail(POT_ERR_INVALID_ARG, "cmax must be finite");
        total += (int64_t)p.n * p.m;
        largest = std::max<int64_t>(largest, (int64_t)p.n * p.m);
    }
    BatchLayout L;
    const size_t need = batch_layout(batch, probs, &L);
    if (!wsp || ws_bytes < need) return fail(POT_ERR_WORKSPACE, "workspace too small");
    if (((uintptr_t)wsp) & 255) return fail(POT_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    char* base = (char*)wsp;
    const int cus = device_cus();
    const int max_per_cu = std::max(1, batched_blocks_per_cu(kind));
    if (cus <= 0) return fail(POT_ERR_DEVICE, "device query failed");

    // descriptors; queue order: largest instance first, and among instances
    // of one size the larger transported mass s first (the batch time is set
    // by its slowest solve, so the likely long ones should start early; on
    // Gaussian-mixture batches of one size the iteration count grows with s:
    // the rank correlation of s and the count is about 0.6 there)
    std::vector<int> order(batch);
    for (int k = 0; k < batch; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const int64_t ea = (int64_t)probs[a].n * probs[a].m, eb = (int64_t)probs[b].n * probs[b].m;
        if (ea != eb) return ea > eb;
        return probs[a].s > probs[b].s;
    });
    auto build = [&](int64_t share, std::vector<BDesc>& desc, std::vector<BSlot>& slots) {
        desc.assign(batch, BDesc{});
        slots.clear();
        for (int k = 0; k < batch; ++k) {
            const pot_problem& p = probs[k];
            BDesc& d = desc[k];
            d.C = p.C;
            d.ldc = p.ldc;
            d.r = p.r;
            d.c = p.c;
            d.u0 = warm && warm->u0 ? warm->u0[k] : nullptr;
            d.v0 = warm && warm->v0 ? warm->v0[k] : nullptr;
            d.w0 = warm && warm->w0 ? warm->w0[k] : 0.0;
            d.f_out = out && out->f ? out->f[k] : nullptr;
            d.g_out = out && out->g ? out->g[k] : nullptr;
            d.u_out = out && out->u ? out->u[k] : nullptr;
            d.v_out = out && out->v ? out->v[k] : nullptr;
            d.s = p.s;
            d.cmax = p.cmax;
            d.n = p.n;
            d.m = p.m;
            d.G = group_size(p.n, p.m, std::max(share, kMemberMin));
            const int vw = kind == POT_COST_BF16 ? 8 : 4;
            d.vec = ((p.ldc % vw) == 0 && (((uintptr_t)p.C) & 15) == 0) ? 1 : 0;
            d.off = L.off[k];
        }
        for (int k : order)
            for (int g = 0; g < desc[k].G; ++g) slots.push_back(BSlot{k, g});
    };
    BArgs B;
    std::memset(&B, 0, sizeof(B));
    B.desc = (const BDesc*)(base + L.desc);
    B.slot = (const BSlot*)(base + L.slot);
    B.batch = batch;
    B.queue = (int32_t*)base;
    B.res = (pot_result*)(base + L.res);
    B.base = base;
    B.algo = o->algo;
    B.max_iter = o->max_iter > 0 ? o->max_iter : 100000;
    B.block_rule = o->block_rule;
    B.step_rule = o->step_rule;
    B.warm_check = warm ? warm->check : 0;
    B.spin_limit = 1 << 24;
    B.do_round = (o->flags & POT_FLAG_NO_ROUND) ? 0 : 1;
    B.eps = o->eps;
    B.gamma_user = o->gamma;
    B.gamma_rule = o->gamma_rule;
    B.p = o->p;
    B.tol_user = o->tol;
    B.A_user = o->A;
    const bool use_graph = !(o->flags & POT_FLAG_NO_GRAPH);
    std::vector<BDesc> desc;
    std::vector<BSlot> slots;
    auto upload = [&](int64_t share) -> hipError_t {
        build(share, desc, slots);
        B.nslot = (int32_t)slots.size();
        hipError_t e = hipMemcpyAsync(base + L.desc, desc.data(), sizeof(BDesc) * batch, hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(base + L.slot, slots.data(), sizeof(BSlot) * slots.size(), hipMemcpyHostToDevice, st);
        return e;
    };

    BTune tune{o->member_elems > 0 ? (int64_t)o->member_elems : 0, std::min(2, max_per_cu)};
    if (tune.share == 0) {
        // tuning results keyed by architecture, CU count, cost kind, algorithm and batch shape
        char key[200];
        std::snprintf(key, sizeof(key), "%s/batched/cus%d/kind%d/algo%d/b%d/e%lld/l%lld", tc_arch().c_str(), cus,
                      kind, o->algo, batch, (long long)(total >> 16), (long long)largest);
        std::vector<long long> cached;
        const bool have = tc_lookup(key, cached) && cached.size() == 2 && cached[0] > 0 && cached[1] >= 1 &&
                          cached[1] <= max_per_cu;
        if (have) tune = BTune{(int64_t)cached[0], (int)cached[1]};
        if (!have) {
            // time each candidate on 3 iterations of the batch (no rounding, no outputs)
            hipEvent_t e0, e1;
            HIPCHK(hipEventCreate(&e0));
            HIPCHK(hipEventCreate(&e1));
            float best = 1e30f;
            BTune bt{kMemberCand[0], 1};
            BArgs T = B;
            T.max_iter = 3;
            T.do_round = 0;
            for (int64_t share : kMemberCand) {
                for (int per_cu = 1; per_cu <= std::min(2, max_per_cu); ++per_cu) {
                    HIPCHK(upload(share));
                    for (auto& d : desc) { d.f_out = d.g_out = d.u_out = d.v_out = nullptr; }
                    HIPCHK(hipMemcpyAsync(base + L.desc, desc.data(), sizeof(BDesc) * batch, hipMemcpyHostToDevice, st));
                    T.nslot = (int32_t)slots.size();
                    const int grid = std::max(1, std::min(T.nslot, cus * per_cu));
                    HIPCHK(hipEventRecord(e0, st));
                    HIPCHK(launch_batched(T, kind, grid, st));
                    HIPCHK(hipEventRecord(e1, st));
                    HIPCHK(hipEventSynchronize(e1));
                    float ms = 0.f;
                    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                    if (ms < best) { best = ms; bt = BTune{share, per_cu}; }
                }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            tune = bt;
            tc_store(key, {(long long)tune.share, (long long)tune.per_cu});
        }
    }
    HIPCHK(upload(tune.share));
    const int grid = std::max(1, std::min(B.nslot, cus * tune.per_cu));
    HIPCHK(run_batched(B, kind, grid, use_graph, st));
    HIPCHK(hipMemcpyAsync(res, base + L.res, sizeof(pot_result) * batch, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    pot_status first = POT_OK;
    for (int k = 0; k < batch; ++k)
        if (res[k].status != POT_OK && first == POT_OK) first = (pot_status)res[k].status;
    if (first != POT_OK) fail(first, "an instance of the batch did not finish with POT_OK (see res[].status)");
    return first;
}

extern "C" {

size_t pot_workspace_bytes(const pot_problem* prob, const pot_options* opts) {
    if (!prob || prob->n < 1 || prob->m < 1) return 0;
    pot_options dflt;
    std::memset(&dflt, 0, sizeof(dflt));
    return workspace_bytes(prob, opts ? opts : &dflt);
}

pot_status pot_solve(const pot_problem* prob, const pot_options* opts, void* ws, size_t ws_bytes,
                     pot_result* res, const pot_outputs* out, void* stream) {
    try {
        return solve_one(prob, opts, ws, ws_bytes, res, out, (hipStream_t)stream);
    } catch (...) {
        return fail(POT_ERR_DEVICE, "internal error");
    }
}

size_t pot_register_workspace_bytes(const pot_reg_problem* prob) {
    if (!prob || prob->n < 1 || prob->m < 1) return 0;
    return reg_layout(prob).total;
}

pot_status pot_register(const pot_reg_problem* prob, const pot_reg_options* opts, void* ws, size_t ws_bytes,
                        pot_reg_result* res, const pot_reg_history* hist, float* y_out, void* stream) {
    try {
        return register_rigid(prob, opts, ws, ws_bytes, res, hist, y_out, (hipStream_t)stream);
    } catch (...) {
        return fail(POT_ERR_DEVICE, "internal error");
    }
}

void pot_rigid_align(const double* H, double* R) { rigid_align(H, R); }

pot_status pot_time_shared_gemm(const pot_shared_cost* cost, int32_t batch, double gamma, void* ws, size_t ws_bytes,
                                int32_t reps, double* med_ms, void* stream) {
    try {
        if (!cost || batch < 1 || reps < 1 || !med_ms || !(gamma > 0.0) || !(cost->cmax > 0.0))
            return fail(POT_ERR_INVALID_ARG, "cost (with cmax), batch >= 1, gamma > 0, reps >= 1 and med_ms are required");
        if (cost->kind != POT_COST_F32 && cost->kind != POT_COST_BF16) return fail(POT_ERR_UNSUPPORTED, "dense cost");
        const SharedLayout L = shared_layout(cost, batch);
        if (!ws || ws_bytes < L.total || (((uintptr_t)ws) & 255)) return fail(POT_ERR_WORKSPACE, "workspace");
        hipStream_t st = (hipStream_t)stream;
        char* base = (char*)ws;
        uint16_t* K = (uint16_t*)(base + L.K);
        uint16_t* KT = (uint16_t*)(base + L.KT);
        uint16_t* bop = (uint16_t*)(base + L.bop);
        float* P = (float*)(base + L.P);
        int32_t* ndone = (int32_t*)(base + L.ndone);
        HIPCHK(launch_zero_words((unsigned long long*)bop, (int)(2 * 2 * (size_t)L.Bp * L.Mp / 8), st));
        HIPCHK(launch_zero_words((unsigned long long*)ndone, 1, st));
        HIPCHK(launch_shared_build(cost->kind, cost->C, cost->ldc, cost->n, cost->m, L.Np, L.Mp, 1.0 / gamma, 0.0, K, KT,
                                   st));
        for (int k = 0; k < 3; ++k) HIPCHK(launch_shared_gemm(K, bop, P, L.Np, 2 * L.Bp, L.Mp, ndone, batch, st));
        std::vector<hipEvent_t> ev(2 * (size_t)reps);
        for (auto& e : ev) HIPCHK(hipEventCreate(&e));
        for (int k = 0; k < reps; ++k) {
            HIPCHK(hipEventRecord(ev[2 * k], st));
            HIPCHK(launch_shared_gemm(K, bop, P, L.Np, 2 * L.Bp, L.Mp, ndone, batch, st));
            HIPCHK(hipEventRecord(ev[2 * k + 1], st));
        }
        HIPCHK(hipStreamSynchronize(st));
        std::vector<double> t(reps);
        for (int k = 0; k < reps; ++k) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]));
            t[k] = ms;
        }
        for (auto& e : ev) (void)hipEventDestroy(e);
        std::sort(t.begin(), t.end());
        *med_ms = reps % 2 ? t[reps / 2] : 0.5 * (t[reps / 2 - 1] + t[reps / 2]);
        return POT_OK;
    } catch (...) {
        return fail(POT_ERR_DEVICE, "internal error");
    }
}

size_t pot_workspace_bytes_shared(const pot_shared_cost* cost, int32_t batch) {
    if (!cost || cost->n < 1 || cost->m < 1 || batch < 1) return 0;
    return shared_layout(cost, batch).total;
}

pot_status pot_solve_shared(const pot_shared_cost* cost, int32_t batch, const pot_shared_member* members,
                            const pot_options* opts, void* ws, size_t ws_bytes, pot_result* res, void* stream) {
    try {
        return solve_shared(cost, batch, members, opts, ws, ws_bytes, res, (hipStream_t)stream);
    } catch (...) {
        return fail(POT_ERR_DEVICE, "internal error");
    }
}

pot_status pot_solve_noalloc(const pot_problem* prob, const pot_options* opts, pot_result* res,
                             const pot_outputs* out, void* stream) {
    try {
        if (!prob || prob->n < 1 || prob->m < 1) return fail(POT_ERR_INVALID_ARG, "n and m must be >= 1");
        if (!opts) return fail(POT_ERR_INVALID_ARG, "null options");
        const size_t need = layout(prob, geometry(prob, opts), nullptr, nullptr);
        if (need > (size_t)POT_NOALLOC_SCRATCH_BYTES)
            return fail(POT_ERR_WORKSPACE, "the problem needs more scratch than pot_solve_noalloc holds "
                                           "(POT_NOALLOC_SCRATCH_BYTES)");
        void* ptr = nullptr;
        pot_status ps = scratch_ptr(&ptr);
        if (ps != POT_OK) return ps;
        return solve_one(prob, opts, ptr, (size_t)POT_NOALLOC_SCRATCH_BYTES, res, out, (hipStream_t)stream,
                         /*force_async=*/true, /*direct=*/true);
    } catch (...) {
        return fail(POT_ERR_DEVICE, "internal error");
    }
}

size_t pot_workspace_bytes_batched(int32_t batch, const pot_problem* probs, const pot_options* opts) {
    (void)opts;
    if (batch < 1 || !probs) return 0;
    for (int k = 0; k < batch; ++k)
        if (probs[k].n < 1 || probs[k].m < 1 || probs[k].n > kBMax || probs[k].m > kBMax) return 0;
    return batch_layout(batch, probs, nullptr);
}

pot_status pot_solve_batched(int32_t batch, const pot_problem* probs, const pot_options* opts, const pot_warm* warm,
                             void* ws, size_t ws_bytes, pot_result* res, const pot_batch_outputs* out,
                             void* stream) {
    try {
        return solve_batched(batch, probs, opts, warm, ws, ws_bytes, res, out, (hipStream_t)stream);
    } catch (...) {
        return fail(POT_ERR_DEVICE, "internal error");
    }
}

pot_status pot_time_pass(const pot_problem* prob, const pot_options* opts, void* ws, size_t ws_bytes,
                         int32_t reps, double* avg_ms, double* fin_ms, void* stream) {
    try {
        if (reps < 1 || !avg_ms) return fail(POT_ERR_INVALID_ARG, "reps >= 1 and avg_ms required");
        pot_status cs = check_problem(prob, opts);
        if (cs != POT_OK) return cs;
        const Geometry g = geometry(prob, opts);
        const size_t need = layout(prob, g, nullptr, nullptr);
        if (!ws || ws_bytes < need || (((uintptr_t)ws) & 255)) return fail(POT_ERR_WORKSPACE, "workspace");
        if (prob->cmax <= 0.0 || (prob->kind == POT_COST_SQEUCLID_POINTS && prob->cost_scale <= 0.0))
            return fail(POT_ERR_INVALID_ARG, "pot_time_pass needs cmax (and cost_scale) given");
        return time_tile(prob, opts, g, ws, reps, avg_ms, fin_ms, (hipStream_t)stream);
    } catch (...) {
        return fail(POT_ERR_DEVICE, "internal error");
    }
}

size_t pot_warm_workspace_bytes(int32_t batch) {
    if (batch < 1) return 0;
    return (size_t)(al256((int64_t)warm_desc_bytes() * batch) + al256((int64_t)sizeof(float) * 256 * batch));
}

pot_status pot_warm_predict(int32_t batch, const pot_warm_instance* inst, double eps, const void* weights,
                            void* ws, size_t ws_bytes, void* stream) {
    try {
        if (batch < 1 || !inst) return fail(POT_ERR_INVALID_ARG, "batch >= 1 and inst are required");
        if (!weights || (((uintptr_t)weights) & 15)) return fail(POT_ERR_INVALID_ARG, "weights: 16-byte aligned device blob");
        const size_t need = pot_warm_workspace_bytes(batch);
        if (!ws || ws_bytes < need || (((uintptr_t)ws) & 255)) return fail(POT_ERR_WORKSPACE, "workspace");
        std::vector<char> desc(warm_desc_bytes() * batch);
        for (int k = 0; k < batch; ++k) {
            const pot_warm_instance& w = inst[k];
            if (w.n < 1 || w.m < 1) return fail(POT_ERR_INVALID_ARG, "n, m >= 1");
            if (!w.x || !w.y || !w.r || !w.c || !w.u0 || !w.v0) return fail(POT_ERR_INVALID_ARG, "null pointer");
            if (!(w.cost_scale > 0.0) || !std::isfinite(w.cost_scale)) return fail(POT_ERR_INVALID_ARG, "cost_scale > 0");
            double gam = w.gamma;
            if (!(gam > 0.0)) {
                const int N = std::max(w.n, w.m);
                if (N < 2 || !(eps > 0.0)) return fail(POT_ERR_INVALID_ARG, "gamma or eps (with max(n, m) >= 2)");
                gam = eps / (4.0 * std::log((double)N));
            }
            warm_fill_desc(desc.data() + warm_desc_bytes() * k, w.x, w.y, w.r, w.c, w.u0, w.v0, w.cost_scale,
                           1.0 / gam, w.n, w.m);
        }
        hipStream_t st = (hipStream_t)stream;
        char* base = (char*)ws;
        float* ctx = (float*)(base + al256((int64_t)warm_desc_bytes() * batch));
        HIPCHK(hipMemcpyAsync(base, desc.data(), desc.size(), hipMemcpyHostToDevice, st));
        HIPCHK(launch_warm((const WDesc*)base, batch, weights, ctx, st));
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

const char* pot_last_error(void) { return g_last_error; }

const char* pot_version(void) { return "libpot 0.1 (gfx950)"; }

}  // extern "C"
