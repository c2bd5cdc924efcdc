/*
 * pot.h -- C ABI of libpot.so, an MI355X (gfx950) solver for entropic partial
 * optimal transport (POT) with ASPOT and feasible Sinkhorn.
 *
 * Problem (Section 2.1 of Truong et al., "Accelerated Sinkhorn Algorithms for
 * Partial Optimal Transport"): given a cost C >= 0 (n x m), marginals r >= 0
 * (n), c >= 0 (m) and a mass 0 < s <= min(|r|_1, |c|_1), find a plan
 * X in U(r, c, s) = { X >= 0 : X 1 <= r, X^T 1 <= c, 1^T X 1 = s } whose cost
 * <C, X> is within eps of the optimum (Definition 1).
 *
 * Solvers:
 *   POT_ASPOT    -- Algorithm 2 (setup "Approximating POT", Nesterov coupling,
 *                   the Greenkhorn step of Algorithm 1, the argmin safeguard,
 *                   stopping on the error E(t) of Section 3.1);
 *   POT_SINKHORN -- feasible Sinkhorn: the loop of Algorithm 3 with the
 *                   default gamma and stopping rule of Algorithm 2, on the
 *                   extended (n+1) x (m+1) instance of the appendix
 *                   "Reduction to Extended OT".
 * Both end with "Form primal" and a rounding onto U(r, c, s) computed in FP64
 * with the original r, c, s:
 *   alpha_i = min(1, r_i / (X~ 1)_i);  beta_j = min(1, c_j / (diag(alpha) X~)^T 1)_j;
 *   X'' = diag(alpha) X~ diag(beta), T'' = |X''|_1;
 *   Xbar = kappa X'' + lambda p' q'^T with kappa = min(1, s/T''),
 *   lambda = max(0, s - T'') / (|p'|_1 |q'|_1), p' = r - X'' 1, q' = c - X''^T 1.
 *
 * Conventions for every entry point:
 *   - Pointers marked (device) are HIP device pointers on the current device;
 *     (host) pointers are host memory.  The caller owns every buffer; the
 *     library keeps no pointer after a call returns and never allocates or
 *     frees device memory inside a solve: all scratch lives in the caller's
 *     workspace (size from pot_workspace_bytes*).
 *   - Work is enqueued on `stream` (a hipStream_t, NULL = default stream).
 *     pot_solve synchronises the stream before returning, after which the
 *     host pot_result is filled and all device outputs are written; with
 *     POT_FLAG_ASYNC it only enqueues (see that flag).
 *   - Dense costs are row-major with leading dimension ldc >= m (elements).
 *   - Arguments are checked before any work is enqueued that writes outside
 *     the workspace.  On POT_ERR_INVALID_ARG no output is written.
 *     pot_last_error() returns a thread-local message for the last failure.
 *   - No C++ exception crosses this interface.
 */
#ifndef POT_H
#define POT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    POT_OK = 0,
    POT_ERR_INVALID_ARG = 1,     /* bad sizes, masses, eps, pointers or options */
    POT_ERR_NO_CONVERGENCE = 2,  /* max_iter reached; the rounded plan is still in U(r,c,s) */
    POT_ERR_NUMERIC = 3,         /* a statistic overflowed the FP64 range, or is not a number.
                                    Sums far below that range are carried as mantissa and
                                    exponent; pot_solve_batched does so only for an instance
                                    held by one workgroup (see member_elems): split over a
                                    group, one leaving the FP64 range is also this error */
    POT_ERR_DEVICE = 4,          /* a HIP runtime call failed */
    POT_ERR_WORKSPACE = 5,       /* workspace too small or misaligned (needs 256 B alignment) */
    POT_ERR_UNSUPPORTED = 6      /* option combination not implemented */
} pot_status;

typedef enum { POT_ASPOT = 0, POT_SINKHORN = 1 } pot_algo;

typedef enum {
    POT_COST_F32 = 0,             /* C: float,    n x m, ld = ldc (16-byte aligned rows give vector loads) */
    POT_COST_BF16 = 1,            /* C: uint16 bfloat16 bit patterns, n x m, ld = ldc */
    POT_COST_SQEUCLID_POINTS = 3  /* C_ij = cost_scale * |x_i - y_j|^2 from float points, d in {2, 3} */
} pot_cost_kind;

typedef struct {
    int32_t n, m;          /* >= 1 */
    int32_t d;             /* point dimension (points kind only): 2 or 3 */
    int32_t kind;          /* pot_cost_kind */
    const void* C;         /* (device) dense cost, or NULL for the points kind */
    int64_t ldc;           /* leading dimension of C in elements (>= m) */
    const float* x;        /* (device) n x d row-major source points (points kind) */
    const float* y;        /* (device) m x d row-major target points (points kind) */
    double cost_scale;     /* points kind: scale of |x - y|^2; <= 0 means 1 / max_ij |x_i - y_j|^2 */
    double cmax;           /* max_ij C_ij (enters eps~ = eps / (8 cmax)); <= 0 means computed
                              on the device (points kind with computed scale: 1) */
    const double* r;       /* (device) n source masses, finite, >= 0 */
    const double* c;       /* (device) m target masses, finite, >= 0 */
    double s;              /* transported mass, 0 < s <= min(|r|_1, |c|_1) */
} pot_problem;

/* flags */
#define POT_FLAG_WANT_PLAN 1u      /* write the dense FP64 plan to outputs->plan */
#define POT_FLAG_NO_ROUND 2u       /* skip the rounding passes (duals only) */
#define POT_FLAG_NO_GRAPH 4u       /* launch every kernel from the host instead of replaying a
                                      captured HIP graph of check_every iterations */
#define POT_FLAG_ASYNC 8u          /* pot_solve only enqueues its kernels on `stream` and returns:
                                      no host synchronisation, no host read of device memory and
                                      no memset node, so that the caller may capture the call in
                                      a HIP graph.  `res` is then a DEVICE pointer to a pot_result
                                      written when the stream reaches the end of the solve
                                      (validation of r, c, s, eps and the cost happens on the
                                      device and is reported there as POT_ERR_INVALID_ARG, with
                                      no other output written); out->w must be NULL.  Every one
                                      of max_iter iterations is enqueued (passes after the stop
                                      return at once), so max_iter must be given, 1 .. 2^20.
                                      Only host-side checks of sizes, pointers and options return
                                      an error from the call itself */

typedef struct {
    int32_t algo;          /* pot_algo */
    int32_t max_iter;      /* iteration cap (<= 0: 100000) */
    double eps;            /* accuracy target of Definition 1 (> 0) */
    double gamma;          /* entropic parameter; <= 0: eps / (4 ln max(n, m)) (Algorithm 2 setup) */
    double tol;            /* stopping threshold on E; <= 0: eps~ of Algorithm 2 setup */
    double A;              /* Sinkhorn corner cost of the extended cost; <= 0: 8 cmax / eps (Algorithm 3) */
    int32_t block_rule;    /* ASPOT block choice: 0 greedy by decrease score, 1 cyclic u, v, w */
    int32_t step_rule;     /* ASPOT step: 0 as printed (base zbar, gamma/(3 M theta)),
                              1 mirror form (base ztilde, 1/(3 M theta)) */
    int32_t check_every;   /* host polls convergence every k iterations (<= 0: 16) */
    uint32_t flags;        /* POT_FLAG_* */
    const double* u0;      /* (device) warm start u (n) in log-scaling units, or NULL (zero start) */
    const double* v0;      /* (device) warm start v (m), or NULL */
    double w0;             /* warm start w */
    const int32_t* force;  /* (device) replay of decisions for tests: 3 ints per ASPOT iteration
                              {block of z-hat, pick (1 = z-hat), block of z-check or -1 = stop};
                              NULL = the solver decides */
    int32_t force_len;     /* iterations covered by force */
    int32_t* trace_i;      /* (device) per-iteration decisions, 3 ints each, or NULL */
    double* trace_d;       /* (device) per-iteration values {E, phi(z-check^t), phi(z-hat^t), theta_t}, or NULL */
    int32_t trace_cap;     /* iterations the trace buffers hold */
    int32_t tile_rows;     /* rows per tile of the statistics pass, 4..256 (0: chosen from the grid
                              size; -1: tuned: 64, 128 and 256 are timed on the problem's start pass
                              the first time an architecture, cost kind and shape bucket (n and m
                              to the nearest power of two) is solved synchronously, and the fastest
                              is kept; an asynchronous solve takes a kept result or the default).
                              Tuning results are kept in memory and, when the environment variable
                              POT_TUNE_CACHE names a file, in that JSON file across processes */
    int32_t member_elems;  /* pot_solve_batched: an instance with more than this many cost entries is
                              split by rows over a group of workgroups, each sweeping at most this
                              many (0: autotuned on the batch, kept per architecture and batch shape
                              with the tuning results) */
    int32_t gamma_rule;    /* 0: gamma and tol as above.  1 (algo Sinkhorn only): the tuned rule of
                              Algorithm 3 (Theorem 2), gamma = (2 eps / (49 H_min))^(1/p) and
                              tol = H_min gamma^p with H_min = min(H(r), H(c)),
                              H(x) = -sum_i x_i ln x_i (0 ln 0 = 0), over the masses as given; a
                              positive gamma or tol above still overrides.  Needs H_min > 0 */
    double p;              /* exponent of the tuned rule, finite and >= 1 */
    int32_t warm_check;    /* pot_solve with u0 / v0: 1 keeps the warm start only if
                              phi(u0, v0, w0) < phi(0) (Section 2.1), else starts from zero
                              (two more statistics passes); 0 always keeps it */
    int32_t reserved0;     /* must be 0 */
} pot_options;

typedef struct {
    int32_t status;        /* pot_status of this solve */
    int32_t iters;         /* iterations run */
    int32_t algo;
    int32_t used_warm;     /* 1 if the warm start was kept */
    double cost;           /* <C, Xbar> in FP64 */
    double E;              /* stopping error at the output point */
    double gamma, tol;
    double phi;            /* ASPOT: phi at the last z-check */
    double mass;           /* 1^T Xbar 1 */
    double kappa, lambda, T2;   /* rounding factors (see the header comment) */
    double cost_scale, cmax;
    double w;              /* ASPOT: w at the output point (Sinkhorn: 0) */
    double viol_row;       /* sum_i max(0, (Xbar 1)_i - r_i) over the FP64 row sums of the rounded plan
                              (0 in exact arithmetic; what remains is FP64 rounding) */
    double viol_col;       /* sum_j max(0, (Xbar^T 1)_j - c_j) */
    double viol_mass;      /* |1^T Xbar 1 - s| */
    double ext_a, ext_b;   /* Sinkhorn: log-scalings a_{n+1}, b_{m+1} of the dummy row and column
                              of the extended instance at the output point (-inf for a zero
                              dummy mass); ASPOT: 0 */
} pot_result;

typedef struct {
    double* plan;          /* (device) n x m FP64 row-major, written with POT_FLAG_WANT_PLAN, or NULL */
    double* f;             /* (device) n: X~_ij = exp(f_i + g_j - C_ij / gamma), or NULL */
    double* g;             /* (device) m, or NULL */
    double* u;             /* (device) n: ASPOT u at the output point (Sinkhorn: a_1..a_n), or NULL */
    double* v;             /* (device) m: ASPOT v (Sinkhorn: b_1..b_m), or NULL */
    double* alpha;         /* (device) n rounding row factors, or NULL */
    double* beta;          /* (device) m rounding column factors, or NULL */
    double* pp;            /* (device) n: p' = r - X'' 1, or NULL */
    double* qq;            /* (device) m: q' = c - X''^T 1, or NULL */
    double* w;             /* (host) ASPOT w at the output point, or NULL */
    double* moments;       /* (device) 16 doubles, points cost only (d = 2 or 3; missing coordinates 0), or
                              NULL: M = sum_ij Xbar_ij x_i y_j^T (3 x 3 row-major), sum_i (Xbar 1)_i x_i (3),
                              sum_j (Xbar^T 1)_j y_j (3), 1^T Xbar 1 (1) of the rounded plan, in FP64 */
} pot_outputs;

/* Bytes of workspace pot_solve needs for this problem and options (0 on
 * invalid sizes).  The workspace must be 256-byte aligned device memory. */
size_t pot_workspace_bytes(const pot_problem* prob, const pot_options* opts);

/* Solve one POT instance.  res (host) receives the result; out (host struct
 * of device pointers, may be NULL) receives the optional outputs.
 * Returns res->status (or an argument/device/workspace error). */
pot_status pot_solve(const pot_problem* prob, const pot_options* opts, void* ws, size_t ws_bytes,
                     pot_result* res, const pot_outputs* out, void* stream);

/* Size of the device array that pot_solve_noalloc uses as its workspace. */
#define POT_NOALLOC_SCRATCH_BYTES (32u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): pot_solve
 * with its workspace in a device array that the library holds for each GPU
 * it runs on (POT_NOALLOC_SCRATCH_BYTES bytes, held until the process ends).
 * The caller still passes every input and output.  It behaves as pot_solve
 * with POT_FLAG_ASYNC: `res` is a DEVICE pointer to a pot_result written when
 * the stream reaches the end of the solve, max_iter must be given
 * (1 .. 2^20), out->w must be NULL, and validation of r, c, s, eps and the
 * cost happens on the device.  Every kernel is launched directly (no graph is
 * instantiated), and the call makes no allocation of any kind.  A problem
 * whose workspace (pot_workspace_bytes) exceeds the array returns
 * POT_ERR_WORKSPACE before any work is enqueued.  Every call on one GPU uses
 * that GPU's array, which keeps the last call's contents (each solve writes
 * every word it reads first): calls on one GPU must be ordered on one stream;
 * calls that overlap (other streams, other threads) race. */
pot_status pot_solve_noalloc(const pot_problem* prob, const pot_options* opts, pot_result* res,
                             const pot_outputs* out, void* stream);

/* Warm starts of a batch (pot_solve_batched). */
typedef struct {
    const double* const* u0;   /* host array of `batch` device pointers to u0 (n_k each), entries may be NULL */
    const double* const* v0;   /* host array of device pointers to v0 (m_k each), entries may be NULL */
    const double* w0;          /* host array of `batch` values of w0, or NULL (all 0) */
    int32_t check;             /* 1: keep an instance's warm start only if phi(z0) < phi(0), else start
                                  it cold (one or two more statistics passes per instance) */
} pot_warm;

/* Optional per-instance outputs of pot_solve_batched: host arrays of `batch`
 * device pointers (each array may be NULL, and so may each entry). */
typedef struct {
    double* const* f;          /* n_k: X~_ij = exp(f_i + g_j - C_ij / gamma) */
    double* const* g;          /* m_k */
    double* const* u;          /* n_k: ASPOT u at the output point (Sinkhorn: a_1..a_n) */
    double* const* v;          /* m_k: ASPOT v (Sinkhorn: b_1..b_m) */
} pot_batch_outputs;

/* Workspace for pot_solve_batched over these problems. */
size_t pot_workspace_bytes_batched(int32_t batch, const pot_problem* probs, const pot_options* opts);

/* Solve `batch` independent instances in one persistent launch (a captured
 * HIP graph of two kernels unless POT_FLAG_NO_GRAPH).  Each instance is a
 * dense POT_COST_F32 or POT_COST_BF16 cost (the same kind for the whole
 * batch) with 1 <= n, m <= 1024 and a row stride (ldc times the element
 * size) below 2^31 bytes; the algorithm, its defaults and the
 * rounding are those of pot_solve, per instance.  Workgroups take instances
 * from a device queue, largest first (ties: larger s first); an instance
 * with more than opts->member_elems cost entries is split by rows over a
 * group of up to 8 workgroups.  probs (host array) describe the instances with device
 * pointers (cmax <= 0: scanned on the device); opts apply to all (force and
 * trace must be NULL; tile_rows is ignored); warm (may be NULL) gives
 * per-instance warm starts; res (host array of batch) receives the results
 * (used_warm reports whether the warm start was kept); out (may be NULL)
 * receives duals.  Returns POT_OK if every instance is OK, else the first
 * failing status; POT_ERR_DEVICE for an instance whose group of workgroups
 * could not meet (a bounded wait expired). */
pot_status pot_solve_batched(int32_t batch, const pot_problem* probs, const pot_options* opts,
                             const pot_warm* warm, void* ws, size_t ws_bytes, pot_result* res,
                             const pot_batch_outputs* out, void* stream);

/* ---------------------------------------------------------------------------
 * Learned warm start (a network that predicts ASPOT duals from point clouds;
 * not in the paper).  Per instance of 2-D points, with mu the mean of its
 * n + m points and cost C_ij = cost_scale |x_i - y_j|^2:
 *   features  p_i = ((x_i - mu) sqrt(cost_scale), clip(log(n r_i), -30, 30), 0)
 *   encoder   h_i = relu(W2 relu(W1 p_i + b1) + b2)                   4 -> 128 -> 128
 *   context   ctx = mean of h over the side's points
 *   head      u0_i = (w4 . relu(W3a h_i + W3b ctx_other + b3) + b4) / gamma
 * and the same for the targets (y, c, m) with the sources' context.  Weights
 * are BF16 (FP32 biases), products run on the matrix cores with FP32
 * accumulation.  Weight blob (device memory, 16-byte aligned,
 * POT_WARM_WEIGHT_BYTES bytes):
 *   float    b1[128], b2[128], b3[128], w4[128], b4, zero padding to byte 2304
 *   bfloat16 W1[128][4], W2[128][128], W3a[128][128], W3b[128][128]
 *            (row-major, output x input; bit patterns, round to nearest even)
 * The predictions feed pot_solve_batched's warm starts (pot_warm, w0 = 0,
 * check = 1: the solver takes one exact w step and keeps the prediction
 * only if it lowers phi below phi(0)).
 * ------------------------------------------------------------------------- */
#define POT_WARM_WEIGHT_BYTES 101632

typedef struct {
    int32_t n, m;          /* points per side, >= 1 */
    const float* x;        /* (device) n x 2 source points */
    const float* y;        /* (device) m x 2 target points */
    const double* r;       /* (device) n source masses */
    const double* c;       /* (device) m target masses */
    double cost_scale;     /* > 0: the cost of the solve is cost_scale |x_i - y_j|^2 */
    double gamma;          /* entropic parameter of the solve; <= 0: eps / (4 ln max(n, m)) */
    double* u0;            /* (device) n: predicted u, written */
    double* v0;            /* (device) m: predicted v, written */
} pot_warm_instance;

/* Workspace of pot_warm_predict for a batch (256-byte aligned device memory). */
size_t pot_warm_workspace_bytes(int32_t batch);

/* Predict warm starts for `batch` instances (inst: host array).  Work is
 * enqueued on `stream` (two kernel launches); u0 / v0 are written when the
 * stream reaches it.  weights: device blob as above.  Writes only the
 * workspace and the outputs.  POT_ERR_INVALID_ARG on bad sizes, pointers,
 * cost_scale or alignment (nothing enqueued). */
pot_status pot_warm_predict(int32_t batch, const pot_warm_instance* inst, double eps, const void* weights,
                            void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Many POT instances on one shared cost (members b = 1..batch with their own
 * r_b, c_b, s_b): feasible Sinkhorn, the loop of Algorithm 3, in the
 * exponential domain as printed there, a_b = r^_b / (K~ b_b),
 * b_b = c^_b / (K~^T a_b), with the kernel of the extended instance
 * K~ = exp(-C~ / gamma) built once and every member's scalings multiplied by
 * it at once on the matrix cores (BF16 K~, each scaling as a sum of two BF16
 * numbers, FP32 accumulation).  The extended instance, the smoothing, the
 * stopping rule and the rounding onto U(r_b, c_b, s_b) are those of
 * pot_solve with algo POT_SINKHORN, per member; gamma is shared and must be
 * given.  K~ is representable only if max C / gamma <= 80 (larger ratios
 * return POT_ERR_UNSUPPORTED: use pot_solve_batched, which works in the log
 * domain).  Rounding K~ to BF16 changes the effective cost by at most
 * gamma 2^-8 per entry.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t n, m;          /* cost size, >= 1 */
    int32_t kind;          /* POT_COST_F32 or POT_COST_BF16 */
    int32_t pad;
    const void* C;         /* (device) n x m row-major, leading dimension ldc */
    int64_t ldc;
    double cmax;           /* max_ij C_ij; <= 0: computed on the device */
} pot_shared_cost;

typedef struct {
    const double* r;       /* (device) n masses */
    const double* c;       /* (device) m masses */
    double s;              /* transported mass */
    double* f;             /* (device) n: output log-scalings, X~_ij = exp(f_i + g_j - C_ij / gamma), or NULL */
    double* g;             /* (device) m, or NULL */
} pot_shared_member;

/* Workspace bytes of pot_solve_shared (0 on invalid sizes). */
size_t pot_workspace_bytes_shared(const pot_shared_cost* cost, int32_t batch);

/* Solve `batch` members on the shared cost.  opts: algo POT_SINKHORN,
 * gamma > 0 (shared), eps, tol (<= 0: each member's eps~), A, max_iter
 * (<= 0: 100000), flags (POT_FLAG_NO_ROUND); other fields ignored.  members
 * and res are host arrays of `batch`.  Polls a pinned host flag every
 * check_every iterations; synchronises the stream before returning.
 * Returns POT_OK if every member is OK, else the first failing status. */
pot_status pot_solve_shared(const pot_shared_cost* cost, int32_t batch, const pot_shared_member* members,
                            const pot_options* opts, void* ws, size_t ws_bytes, pot_result* res, void* stream);

/* Measurement hook: build K~ for the shared cost (cmax and gamma given) and
 * time the first product of an iteration, K~ times every member's split
 * scalings (rows x 2 batch x columns, padded to multiples of 64 and 64
 * members), 3 untimed and then `reps` times with HIP events around each
 * launch; *med_ms receives the median.  Writes only the workspace
 * (pot_workspace_bytes_shared).  Synchronises the stream. */
pot_status pot_time_shared_gemm(const pot_shared_cost* cost, int32_t batch, double gamma, void* ws, size_t ws_bytes,
                                int32_t reps, double* med_ms, void* stream);

/* ---------------------------------------------------------------------------
 * Rigid point-cloud registration through POT (Section 4, "Point Cloud
 * Registration", and its appendix).  X (n points, fixed) and Y (m points)
 * in 3-D; the map F(y) = R y + t starts at (R0, t0).  Registration k:
 *   1. F_k(Y) is formed on the device (FP64 arithmetic, FP32 storage);
 *   2. POT between X and F_k(Y) with C_ij = cost_scale |x_i - F_k(y_j)|^2
 *      (the points cost of pot_solve; |C|_max taken on the device), masses
 *      r, c, mass s, accuracy eps, and gamma_k = max(gamma0 anneal^k,
 *      gamma_min); with warm = 1 (ASPOT) the solve starts from the previous
 *      registration's duals with the potentials in cost units kept
 *      (u, v, w scaled by gamma_{k-1} / gamma_k);
 *   3. from the rounded plan Xbar, on the device, M = sum_ij Xbar_ij x_i
 *      F_k(y_j)^T, the barycentre sums and the mass; on the host the centred
 *      cross-covariance H = M - |Xbar| u_x u_y^T and the rotation dR in SO(3)
 *      maximising tr(dR^T H) (which minimises sum_ij Xbar_ij
 *      |x_i - (dR F_k(y_j) + dt)|^2 with dt = u_x - dR u_y), and
 *      F_{k+1} = (dR R_k, dR t_k + dt);
 *   4. stop when |cost_k - cost_{k-1}| <= tol cost_{k-1} (cost_k = <C_k,
 *      Xbar_k>) or after max_steps registrations.
 * The call synchronises the stream once per registration (the host takes
 * the 3 x 3 rotation).  The caller owns every buffer; the workspace comes
 * from pot_register_workspace_bytes.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t n, m;          /* points of X and of Y, >= 2 */
    const float* x;        /* (device) n x 3 row-major, the fixed cloud */
    const float* y;        /* (device) m x 3 row-major, the moving cloud */
    const double* r;       /* (device) n masses of X */
    const double* c;       /* (device) m masses of Y */
    double s;              /* transported mass, 0 < s <= min(|r|_1, |c|_1) */
    double cost_scale;     /* > 0: C = cost_scale |x - F(y)|^2 throughout; <= 0: 1 / max_ij |x_i - F0(y_j)|^2 */
} pot_reg_problem;

typedef struct {
    double eps;            /* accuracy of every POT solve (Definition 1), > 0 */
    double gamma0;         /* entropic parameter of the first registration, > 0 */
    double anneal;         /* factor per registration, in (0, 1] */
    double gamma_min;      /* floor of gamma_k; <= 0: eps / (4 ln max(n, m)) (Algorithm 2's rule) */
    double tol;            /* relative change of the transport cost that stops the loop, > 0 */
    int32_t max_steps;     /* registrations, >= 1 */
    int32_t warm;          /* 1: warm-start every ASPOT solve from the previous duals; 0: cold */
    int32_t max_iter;      /* iteration cap of each solve (<= 0: 100000) */
    int32_t algo;          /* POT_ASPOT or POT_SINKHORN (cold starts) */
    double R0[9];          /* initial rotation, row-major */
    double t0[3];          /* initial translation */
} pot_reg_options;

typedef struct {
    int32_t status;        /* POT_OK, POT_ERR_NO_CONVERGENCE if a solve hit max_iter, or the error */
    int32_t steps;         /* registrations run */
    int32_t total_iters;   /* iterations summed over the solves */
    int32_t pad;
    double R[9], t[3];     /* final map */
    double cost;           /* transport cost of the last registration */
} pot_reg_result;

/* Per-registration record (every pointer may be NULL; arrays of max_steps
 * entries): host iters, cost, gamma, E and Rt (12 per registration: R
 * row-major then t, the map after it); device y_hist (max_steps x m x 3, the
 * moved cloud each solve saw) and dual_hist (max_steps x (n + m + 1): each
 * solve's output u, v, w). */
typedef struct {
    int32_t* iters;
    double* cost;
    double* gamma;
    double* E;
    double* Rt;
    float* y_hist;
    double* dual_hist;
} pot_reg_history;

/* Workspace bytes of pot_register (0 on invalid sizes). */
size_t pot_register_workspace_bytes(const pot_reg_problem* prob);

/* Run the registration loop.  y_out (device, m x 3, may be NULL) receives
 * F(Y) under the final map.  Returns res->status, or an argument, device or
 * workspace error (then res->steps tells how many registrations ran). */
pot_status pot_register(const pot_reg_problem* prob, const pot_reg_options* opts, void* ws, size_t ws_bytes,
                        pot_reg_result* res, const pot_reg_history* hist, float* y_out, void* stream);

/* Host helper of pot_register: the rotation R in SO(3) (row-major) that
 * maximises tr(R^T H) for a 3 x 3 matrix H (row-major), i.e. the rotation
 * of the weighted Procrustes problem with centred cross-covariance
 * H = sum_ij w_ij x_i y_j^T (R y ~ x).  Computed as the leading eigenvector of
 * Horn's 4 x 4 quaternion matrix (Jacobi rotations).  No device work. */
void pot_rigid_align(const double* H, double* R);

/* Measurement hook: set up the problem (as pot_solve does) and run the
 * statistics pass (row sums, column sums and total of B at the start point
 * u0, v0, w0 of opts: the pass every ASPOT and Sinkhorn iteration runs)
 * 3 untimed times and then `reps` times on `stream`.  A pass is two kernels,
 * the tile kernel that streams C (or recomputes it from points) and the
 * finalising kernel; each timed dispatch is bracketed by HIP events recorded
 * around it.  *avg_ms (host) receives the median time of the tile kernel,
 * *fin_ms (host, may be NULL) that of the finalising kernel.  Requires prob->cmax > 0 (and cost_scale > 0 for
 * points).  Writes only the workspace.  Synchronises the stream. */
pot_status pot_time_pass(const pot_problem* prob, const pot_options* opts, void* ws, size_t ws_bytes,
                         int32_t reps, double* avg_ms, double* fin_ms, void* stream);

/* Static description of a status code. */
const char* pot_status_string(pot_status st);

/* Thread-local description of the last error on this thread ("" if none). */
const char* pot_last_error(void);

/* Library version string. */
const char* pot_version(void);

#ifdef __cplusplus
}
#endif
#endif
