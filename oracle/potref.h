/*
 * potref.h -- FP64 CPU oracle for entropic partial optimal transport (POT).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The solver
 * library never calls it, and it shares no code, header or table with the
 * HIP path.
 *
 * What it computes (Truong, Pham, Nguyen, Luong, Tran, "Accelerated Sinkhorn
 * Algorithms for Partial Optimal Transport"):
 *   - the setup "Approximating POT" of Algorithm 2 (gamma, eps~, smoothed
 *     marginals r~, c~);
 *   - the dual phi(z), z = (u, v, w), of Section 2.1 and its statistics
 *     R = B 1, Q = B^T 1, T = 1^T B 1 with B_ij = exp(u_i + v_j + w - C_ij/gamma);
 *   - the Greenkhorn block step of Algorithm 1;
 *   - the ASPOT loop of Algorithm 2 and the error E(t) of Section 3.1;
 *   - feasible Sinkhorn (Algorithm 3 with the default gamma and stopping rule
 *     of Algorithm 2) on the extended (n+1) x (m+1) instance of the appendix
 *     "Reduction to Extended OT";
 *   - a rounding onto U(r, c, s) (the paper cites ROUND-POT without printing
 *     it; the reading used is stated in potref.c).
 * Everything is FP64 and log-domain with max-stabilised log-sum-exp; the
 * exp-domain kernel K = exp(-C/gamma) underflows for the workloads here.
 *
 * All pointers are host pointers owned by the caller.  C is row-major n x m
 * with leading dimension ldc >= m.  Functions return 0 on success, 1 on an
 * invalid argument and 2 when an iteration stopped at max_iter.
 */
#ifndef POTREF_H
#define POTREF_H

#ifdef __cplusplus
extern "C" {
#endif

#define POTREF_OK 0
#define POTREF_INVALID 1
#define POTREF_NOCONV 2

/* Setup of Algorithm 2 ("Approximating POT").  out3 = {gamma, tol, M} with
 * M = |r|_1 + |c|_1 - s.  gamma_user > 0 overrides gamma = eps/(4 ln N),
 * N = max(n, m); tol_user > 0 overrides the stopping threshold eps~ (the
 * smoothing always uses the eps~ of the rule).  cmax = max_ij C_ij.
 * rt (n) and ct (m) receive the smoothed marginals. */
int potref_setup(int n, int m, const double* r, const double* c, double s,
                 double eps, double cmax, double gamma_user, double tol_user,
                 double* rt, double* ct, double* out3);

/* Tuned rule of Algorithm 3 (Theorem 2): out3 = {gamma, eps', H_min} with
 * H_min = min{H(r), H(c)}, H(x) = -sum x_i log x_i (0 log 0 = 0),
 * gamma = (2 eps / (49 H_min))^(1/p), eps' = H_min gamma^p.  Invalid unless
 * p >= 1 and H_min > 0. */
int potref_tuned(int n, int m, const double* r, const double* c, double eps, double p, double* out3);

/* Statistics of B(z) in log domain: lR (n), lQ (m), lT (1). */
void potref_stats(int n, int m, const double* C, long ldc, double gamma,
                  const double* u, const double* v, double w,
                  double* lR, double* lQ, double* lT);

/* phi(z) of Section 2.1 evaluated from its definition (one statistics pass). */
double potref_phi(int n, int m, const double* C, long ldc, double gamma,
                  const double* rt, const double* ct, double s,
                  const double* u, const double* v, double w);

/* E(z) of Section 3.1 with p~ = e^u, q~ = e^v. */
double potref_error(int n, int m, const double* C, long ldc, double gamma,
                    const double* rt, const double* ct, double s,
                    const double* u, const double* v, double w);

/* One Greenkhorn step (Algorithm 1) applied in place to z.  block < 0 picks
 * the block greedily (largest decrease score, ties u < v < w); block in
 * {0,1,2} forces u, v or w.  scores3 (may be NULL) receives the three scores
 * sum_i rho(r~_i, R_i + e^{u_i}), sum_j rho(c~_j, Q_j + e^{v_j}), rho(s, T).
 * Returns the block applied. */
int potref_greenkhorn(int n, int m, const double* C, long ldc, double gamma,
                      const double* rt, const double* ct, double s,
                      double* u, double* v, double* w, int block, double* scores3);

typedef struct {
    int max_iter;
    int block_rule;   /* 0 greedy by decrease score, 1 cyclic u, v, w */
    int step_rule;    /* 0 as printed: base zbar, step gamma/(3 M theta);
                         1 mirror form: base ztilde, step 1/(3 M theta) */
    int trace_cap;    /* length of the trace arrays below (0: no trace) */
    int* tr_bhat;     /* block of the step on z-grave */
    int* tr_pick;     /* 1 if z^t = z-hat^t, 0 if z^t = z-check^t */
    int* tr_bchk;     /* block of the step on z^t (-1 at the stopping iteration) */
    double* tr_E;        /* E(z^t) */
    double* tr_theta;    /* theta_t */
    double* tr_phibar;   /* phi(zbar^t) */
    double* tr_phigrave; /* phi(z-grave^t) */
    double* tr_phihat;   /* phi(z-hat^t) */
    double* tr_phichk;   /* phi(z-check^t) (before the iteration) */
    double* tr_phiz;     /* phi(z^t) */
    double* tr_phinext;  /* phi(z-check^{t+1}) */
    double* tr_gdot;     /* theta_t (ztilde^{t+1} - ztilde^t)^T grad phi(zbar^t) */
    double* tr_step2;    /* |ztilde^{t+1} - ztilde^t|^2 */
    double* tr_ztil;     /* optional (n+m+1) x trace_cap history of ztilde^t */
} potref_aspot_opts;

/* ASPOT (Algorithm 2, loop and form-primal point).  rt, ct are the smoothed
 * marginals, M = |r|_1 + |c|_1 - s.  u0/v0 may be NULL (zero start).
 * Returns the final z^t in (u_out, v_out, w_out), the iteration count and
 * E(z^t). */
int potref_aspot(int n, int m, const double* C, long ldc, double gamma, double tol,
                 const double* rt, const double* ct, double s, double M,
                 const double* u0, const double* v0, double w0,
                 const potref_aspot_opts* o,
                 double* u_out, double* v_out, double* w_out,
                 int* iters_out, double* E_out);

/* Feasible Sinkhorn (Algorithm 3 loop) on the extended instance built from
 * the smoothed marginals: r^ = (r~, |c~|_1 - s), c^ = (c~, |r~|_1 - s),
 * C^ = [[C, 0], [0^T, A]].  a_out (n+1), b_out (m+1) are the log-domain
 * scalings; X^_ij = exp(a_i + b_j - C^_ij/gamma).  tr_err (may be NULL)
 * receives the stopping error of each iteration. */
int potref_sinkhorn(int n, int m, const double* C, long ldc, double gamma, double tol,
                    const double* rt, const double* ct, double s, double A, int max_iter,
                    double* a_out, double* b_out, int* iters_out, double* err_out,
                    double* tr_err);

/* Rounding of X~_ij = exp(f_i + g_j - C_ij/gamma) onto U(r, c, s) with the
 * ORIGINAL r, c, s.  Outputs the factored plan
 *   Xbar = kappa * diag(alpha) X~ diag(beta) + lambda * p' q'^T
 * as alpha (n), beta (m), pp (n), qq (m) and
 * out5 = {kappa, lambda, T'', cost <C, Xbar>, mass of Xbar}.
 * X_out (may be NULL) receives the dense n x m plan (row-major, ld m). */
int potref_round(int n, int m, const double* C, long ldc, double gamma,
                 const double* f, const double* g,
                 const double* r, const double* c, double s,
                 double* alpha, double* beta, double* pp, double* qq,
                 double* out5, double* X_out);

/* The same rounding applied to an arbitrary nonnegative dense n x m matrix. */
int potref_round_dense(int n, int m, const double* X, const double* r,
                       const double* c, double s, double* X_out);

/* <C, X> with compensated (Neumaier) summation. */
double potref_cost(int n, int m, const double* C, long ldc, const double* X);

/* Stopping error of feasible Sinkhorn (Algorithm 3) at extended
 * log-scalings a (n+1) and b (m+1): |X^ 1 - r^|_1 + |X^T 1 - c^|_1 over the
 * extended instance built from the smoothed marginals rt, ct and s, with
 * corner cost A.  Every entry is summed directly. */
double potref_sk_error(int n, int m, const double* C, long ldc, double gamma,
                       const double* rt, const double* ct, double s, double A,
                       const double* a, const double* b);

/* A factored plan Xbar = kappa diag(alpha) X~ diag(beta) + lambda p' q'^T,
 * X~_ij = exp(f_i + g_j - Cp_ij / gamma), evaluated entry by entry: row
 * sums (rows_out, n), column sums (cols_out, m) and
 * out3 = {<Ce, Xbar>, 1^T Xbar 1, min_ij Xbar_ij}. */
int potref_plan_eval(int n, int m, const double* Cp, long ldp, const double* Ce, long lde,
                     double gamma, const double* f, const double* g,
                     const double* alpha, const double* beta, double kappa, double lambda,
                     const double* pp, const double* qq,
                     double* rows_out, double* cols_out, double* out3);

/* Number of OpenMP threads the oracle uses. */
int potref_threads(void);

/* Sets the OpenMP thread count of later calls (t > 0). */
void potref_set_threads(int t);

#ifdef __cplusplus
}
#endif
#endif
