/*
 * potref.c -- FP64 CPU oracle for entropic partial optimal transport.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the solver library.  Shares
 * no code with the HIP path.
 *
 * Plain and slow on purpose: every statistic is recomputed from its
 * definition with a max-stabilised log-sum-exp, phi is evaluated by its
 * definition wherever the algorithm compares values of phi, and there is no
 * fusion or blocking beyond OpenMP over rows (or column ranges).
 *
 * Notation (Section 2.1): z = (u, v, w), B_ij(z) = exp(u_i + v_j + w - C_ij/gamma),
 * phi(z) = |B(z)|_1 + sum_i e^{u_i} + sum_j e^{v_j} - <u, r> - <v, c> - w s,
 * rho(a, b) = b - a + a log(a / b).
 */
#include "potref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int potref_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void potref_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* log(e^a + e^b) */
static double logaddexp(double a, double b) {
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    double hi = a > b ? a : b, lo = a > b ? b : a;
    return hi + log1p(exp(lo - hi));
}

/* rho(a, b) = b - a + a log(a/b) with b given by its logarithm lb.
   Written as a h(d) with d = b/a - 1 and h(d) = d - log(1 + d), which is the
   same quantity without the cancellation of b - a against a log(a/b) when
   b is close to a; for |d| < 1/2 h is summed from its Taylor series
   h(d) = sum_{k>=2} (-1)^k d^k / k. */
static double rho_log(double a, double lb) {
    if (a == 0.0) return exp(lb);
    double d = expm1(lb - log(a));
    double h;
    if (fabs(d) < 0.5) {
        double term = d * d, sum = 0.0;
        for (int k = 2; k < 80; ++k) {
            double add = ((k & 1) ? -term : term) / k;
            sum += add;
            if (fabs(add) <= 1e-18 * fabs(sum)) break;
            term *= d;
        }
        h = sum;
    } else {
        h = d - log1p(d);
    }
    return a * h;
}

static double sum_vec(int k, const double* x) {
    double s = 0.0, comp = 0.0;
    for (int i = 0; i < k; ++i) {          /* Neumaier */
        double t = s + x[i];
        if (fabs(s) >= fabs(x[i])) comp += (s - t) + x[i];
        else comp += (x[i] - t) + s;
        s = t;
    }
    return s + comp;
}

static double dot_vec(int k, const double* x, const double* y) {
    double s = 0.0, comp = 0.0;
    for (int i = 0; i < k; ++i) {
        double p = x[i] * y[i];
        double t = s + p;
        if (fabs(s) >= fabs(p)) comp += (s - t) + p;
        else comp += (p - t) + s;
        s = t;
    }
    return s + comp;
}

static double sum_exp(int k, const double* x) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += exp(x[i]);
    return s;
}

/* ---------------------------------------------------------------------- */
/* Setup: Algorithm 2, "Approximating POT".                                */
/* ---------------------------------------------------------------------- */
int potref_setup(int n, int m, const double* r, const double* c, double s,
                 double eps, double cmax, double gamma_user, double tol_user,
                 double* rt, double* ct, double* out3) {
    if (n < 1 || m < 1 || !(eps > 0.0) || !(cmax > 0.0) || !(s > 0.0)) return POTREF_INVALID;
    double nr = 0.0, nc = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!(r[i] >= 0.0) || !isfinite(r[i])) return POTREF_INVALID;
        nr += r[i];
    }
    for (int j = 0; j < m; ++j) {
        if (!(c[j] >= 0.0) || !isfinite(c[j])) return POTREF_INVALID;
        nc += c[j];
    }
    if (s > nr || s > nc) return POTREF_INVALID;

    /* gamma = eps / (4 log n); the paper has n = m, we take N = max(n, m)
       and the natural logarithm. */
    int N = n > m ? n : m;
    double gamma;
    if (gamma_user > 0.0) gamma = gamma_user;
    else {
        if (N < 2) return POTREF_INVALID;
        gamma = eps / (4.0 * log((double)N));
    }
    /* eps~ = eps / (8 |C|_max), capped when a marginal has mass above 1. */
    double et = eps / (8.0 * cmax);
    if (nr > 1.0) {
        double cap = 8.0 * (nr - s) / (nr - 1.0);
        if (cap < et) et = cap;
    }
    if (nc > 1.0) {
        double cap = 8.0 * (nc - s) / (nc - 1.0);
        if (cap < et) et = cap;
    }
    double tol = tol_user > 0.0 ? tol_user : et;
    if (!(tol > 0.0)) return POTREF_INVALID;
    /* Smoothing: r~ = (1 - eps~/8) r + eps~/(8 n) 1 (and 1/m for c). */
    for (int i = 0; i < n; ++i) {
        rt[i] = (1.0 - et / 8.0) * r[i] + et / (8.0 * n);
        if (!(rt[i] > 0.0)) return POTREF_INVALID;
    }
    for (int j = 0; j < m; ++j) {
        ct[j] = (1.0 - et / 8.0) * c[j] + et / (8.0 * m);
        if (!(ct[j] > 0.0)) return POTREF_INVALID;
    }
    out3[0] = gamma;
    out3[1] = tol;
    out3[2] = nr + nc - s;
    return POTREF_OK;
}

/* Tuned rule of Algorithm 3 (statement of Theorem 2): with the Shannon
   entropy H(x) = -sum_i x_i log x_i of each marginal as given (terms with
   x_i = 0 contribute 0), H_min = min{H(r), H(c)}, gamma = (2 eps /
   (49 H_min))^(1/p) and the stopping threshold eps' = H_min gamma^p.
   out3 = {gamma, eps', H_min}. */
int potref_tuned(int n, int m, const double* r, const double* c, double eps, double p, double* out3) {
    if (n < 1 || m < 1 || !(eps > 0.0) || !(p >= 1.0) || !isfinite(p)) return POTREF_INVALID;
    double hr = 0.0, hc = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!(r[i] >= 0.0) || !isfinite(r[i])) return POTREF_INVALID;
        if (r[i] > 0.0) hr -= r[i] * log(r[i]);
    }
    for (int j = 0; j < m; ++j) {
        if (!(c[j] >= 0.0) || !isfinite(c[j])) return POTREF_INVALID;
        if (c[j] > 0.0) hc -= c[j] * log(c[j]);
    }
    double h = hr < hc ? hr : hc;
    if (!(h > 0.0)) return POTREF_INVALID;
    double gamma = pow(2.0 * eps / (49.0 * h), 1.0 / p);
    out3[0] = gamma;
    out3[1] = h * pow(gamma, p);
    out3[2] = h;
    return POTREF_OK;
}

/* ---------------------------------------------------------------------- */
/* Statistics of B(z).                                                     */
/* ---------------------------------------------------------------------- */
void potref_stats(int n, int m, const double* C, long ldc, double gamma,
                  const double* u, const double* v, double w,
                  double* lR, double* lQ, double* lT) {
    const double ig = 1.0 / gamma;
    /* Row sums: lR_i = log sum_j exp(x_ij), x_ij = u_i + v_j + w - C_ij/gamma. */
#pragma omp parallel
    {
        double* x = (double*)malloc(sizeof(double) * (size_t)m);
#pragma omp for schedule(static)
        for (int i = 0; i < n; ++i) {
            const double* Ci = C + (long)i * ldc;
            double mx = -INFINITY;
            for (int j = 0; j < m; ++j) {
                x[j] = u[i] + v[j] + w - Ci[j] * ig;
                if (x[j] > mx) mx = x[j];
            }
            double acc = 0.0;
            for (int j = 0; j < m; ++j) acc += exp(x[j] - mx);
            lR[i] = mx + log(acc);
        }
        free(x);
    }
    /* Column sums: lQ_j = log sum_i exp(x_ij); a column range per thread,
       first the maxima, then the shifted sums. */
#pragma omp parallel
    {
        int nt = 1, tid = 0;
#ifdef _OPENMP
        nt = omp_get_num_threads();
        tid = omp_get_thread_num();
#endif
        int j0 = (int)((long)m * tid / nt), j1 = (int)((long)m * (tid + 1) / nt);
        int w_ = j1 - j0;
        if (w_ > 0) {
            double* mx = (double*)malloc(sizeof(double) * (size_t)w_);
            double* acc = (double*)malloc(sizeof(double) * (size_t)w_);
            for (int j = 0; j < w_; ++j) { mx[j] = -INFINITY; acc[j] = 0.0; }
            for (int i = 0; i < n; ++i) {
                const double* Ci = C + (long)i * ldc;
                for (int j = j0; j < j1; ++j) {
                    double x = u[i] + v[j] + w - Ci[j] * ig;
                    if (x > mx[j - j0]) mx[j - j0] = x;
                }
            }
            for (int i = 0; i < n; ++i) {
                const double* Ci = C + (long)i * ldc;
                for (int j = j0; j < j1; ++j) {
                    double x = u[i] + v[j] + w - Ci[j] * ig;
                    acc[j - j0] += exp(x - mx[j - j0]);
                }
            }
            for (int j = j0; j < j1; ++j) lQ[j] = mx[j - j0] + log(acc[j - j0]);
            free(mx);
            free(acc);
        }
    }
    /* Total: lT = log sum_i exp(lR_i). */
    double mx = -INFINITY;
    for (int i = 0; i < n; ++i) if (lR[i] > mx) mx = lR[i];
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += exp(lR[i] - mx);
    *lT = mx + log(acc);
}

/* phi from the statistics and the point (Section 2.1). */
static double phi_from(int n, int m, const double* rt, const double* ct, double s,
                       const double* u, const double* v, double w, double lT) {
    return exp(lT) + sum_exp(n, u) + sum_exp(m, v) - dot_vec(n, u, rt) - dot_vec(m, v, ct) - w * s;
}

double potref_phi(int n, int m, const double* C, long ldc, double gamma,
                  const double* rt, const double* ct, double s,
                  const double* u, const double* v, double w) {
    double* lR = (double*)malloc(sizeof(double) * (size_t)n);
    double* lQ = (double*)malloc(sizeof(double) * (size_t)m);
    double lT;
    potref_stats(n, m, C, ldc, gamma, u, v, w, lR, lQ, &lT);
    double ph = phi_from(n, m, rt, ct, s, u, v, w, lT);
    free(lR);
    free(lQ);
    return ph;
}

/* E(z) = |1^T B 1 - s| + |B 1 + p~ - r~|_1 + |B^T 1 + q~ - c~|_1, p~ = e^u, q~ = e^v. */
static double error_from(int n, int m, const double* rt, const double* ct, double s,
                         const double* u, const double* v, const double* lR,
                         const double* lQ, double lT) {
    double e = fabs(exp(lT) - s);
    for (int i = 0; i < n; ++i) e += fabs(exp(lR[i]) + exp(u[i]) - rt[i]);
    for (int j = 0; j < m; ++j) e += fabs(exp(lQ[j]) + exp(v[j]) - ct[j]);
    return e;
}

double potref_error(int n, int m, const double* C, long ldc, double gamma,
                    const double* rt, const double* ct, double s,
                    const double* u, const double* v, double w) {
    double* lR = (double*)malloc(sizeof(double) * (size_t)n);
    double* lQ = (double*)malloc(sizeof(double) * (size_t)m);
    double lT;
    potref_stats(n, m, C, ldc, gamma, u, v, w, lR, lQ, &lT);
    double e = error_from(n, m, rt, ct, s, u, v, lR, lQ, lT);
    free(lR);
    free(lQ);
    return e;
}

/* ---------------------------------------------------------------------- */
/* Greenkhorn step (Algorithm 1).                                          */
/* ---------------------------------------------------------------------- */
/* Decrease scores of the three blocks: exact minimisation over a block lowers
   phi by sum_i rho(r~_i, R_i + e^{u_i}) (u block), by the column analogue
   (v block) and by rho(s, T) (w block), as in the proof of Theorem 3. */
static void gk_scores(int n, int m, const double* rt, const double* ct, double s,
                      const double* u, const double* v, const double* lR,
                      const double* lQ, double lT, double* sc) {
    double su = 0.0, sv = 0.0;
    for (int i = 0; i < n; ++i) su += rho_log(rt[i], logaddexp(lR[i], u[i]));
    for (int j = 0; j < m; ++j) sv += rho_log(ct[j], logaddexp(lQ[j], v[j]));
    sc[0] = su;
    sc[1] = sv;
    sc[2] = rho_log(s, lT);
}

static int pick_block(const double* sc) {
    int b = 0;
    if (sc[1] > sc[b]) b = 1;
    if (sc[2] > sc[b]) b = 2;
    return b;
}

/* u <- u + log r~ - log(B 1 + e^u);  v <- v + log c~ - log(B^T 1 + e^v);
   w <- w + log s - log |B|_1. */
static void gk_apply(int block, int n, int m, const double* rt, const double* ct, double s,
                     double* u, double* v, double* w, const double* lR,
                     const double* lQ, double lT) {
    if (block == 0) {
        for (int i = 0; i < n; ++i) u[i] = u[i] + log(rt[i]) - logaddexp(lR[i], u[i]);
    } else if (block == 1) {
        for (int j = 0; j < m; ++j) v[j] = v[j] + log(ct[j]) - logaddexp(lQ[j], v[j]);
    } else {
        *w = *w + log(s) - lT;
    }
}

int potref_greenkhorn(int n, int m, const double* C, long ldc, double gamma,
                      const double* rt, const double* ct, double s,
                      double* u, double* v, double* w, int block, double* scores3) {
    double* lR = (double*)malloc(sizeof(double) * (size_t)n);
    double* lQ = (double*)malloc(sizeof(double) * (size_t)m);
    double lT, sc[3];
    potref_stats(n, m, C, ldc, gamma, u, v, *w, lR, lQ, &lT);
    gk_scores(n, m, rt, ct, s, u, v, lR, lQ, lT, sc);
    int b = block >= 0 ? block : pick_block(sc);
    gk_apply(b, n, m, rt, ct, s, u, v, w, lR, lQ, lT);
    if (scores3) memcpy(scores3, sc, sizeof(sc));
    free(lR);
    free(lQ);
    return b;
}

/* ---------------------------------------------------------------------- */
/* ASPOT (Algorithm 2).                                                    */
/* ---------------------------------------------------------------------- */
typedef struct {
    double* u;
    double* v;
    double w;
} zvec;

static zvec z_alloc(int n, int m) {
    zvec z;
    z.u = (double*)calloc((size_t)n, sizeof(double));
    z.v = (double*)calloc((size_t)m, sizeof(double));
    z.w = 0.0;
    return z;
}
static void z_free(zvec* z) { free(z->u); free(z->v); }
static void z_copy(int n, int m, zvec* dst, const zvec* src) {
    memcpy(dst->u, src->u, sizeof(double) * (size_t)n);
    memcpy(dst->v, src->v, sizeof(double) * (size_t)m);
    dst->w = src->w;
}

int potref_aspot(int n, int m, const double* C, long ldc, double gamma, double tol,
                 const double* rt, const double* ct, double s, double M,
                 const double* u0, const double* v0, double w0,
                 const potref_aspot_opts* o,
                 double* u_out, double* v_out, double* w_out,
                 int* iters_out, double* E_out) {
    const int max_iter = o ? o->max_iter : 1000;
    const int block_rule = o ? o->block_rule : 0;
    const int step_rule = o ? o->step_rule : 0;
    const int cap = (o && o->trace_cap > 0) ? o->trace_cap : 0;

    zvec zchk = z_alloc(n, m), ztil = z_alloc(n, m), zbar = z_alloc(n, m);
    zvec ztil1 = z_alloc(n, m), zgrave = z_alloc(n, m), zhat = z_alloc(n, m), z = z_alloc(n, m);
    double* lR = (double*)malloc(sizeof(double) * (size_t)n);
    double* lQ = (double*)malloc(sizeof(double) * (size_t)m);
    double* gu = (double*)malloc(sizeof(double) * (size_t)n);
    double* gv = (double*)malloc(sizeof(double) * (size_t)m);
    double lT;

    /* theta_0 = 1, z~^0 = z-check^0 = z0 (zero unless a start point is given). */
    if (u0) memcpy(zchk.u, u0, sizeof(double) * (size_t)n);
    if (v0) memcpy(zchk.v, v0, sizeof(double) * (size_t)m);
    zchk.w = w0;
    z_copy(n, m, &ztil, &zchk);
    double theta = 1.0;
    double phichk = potref_phi(n, m, C, ldc, gamma, rt, ct, s, zchk.u, zchk.v, zchk.w);
    int cyc = 0;  /* per-call counter of the cyclic block rule */

    int status = POTREF_NOCONV, t = 0;
    double E = INFINITY;
    for (t = 0; t < max_iter; ++t) {
        /* zbar^t = (1 - theta_t) zcheck^t + theta_t z~^t */
        for (int i = 0; i < n; ++i) zbar.u[i] = (1.0 - theta) * zchk.u[i] + theta * ztil.u[i];
        for (int j = 0; j < m; ++j) zbar.v[j] = (1.0 - theta) * zchk.v[j] + theta * ztil.v[j];
        zbar.w = (1.0 - theta) * zchk.w + theta * ztil.w;

        /* grad phi(zbar) = (B1 + e^u - r~, B^T 1 + e^v - c~, 1^T B 1 - s) */
        potref_stats(n, m, C, ldc, gamma, zbar.u, zbar.v, zbar.w, lR, lQ, &lT);
        for (int i = 0; i < n; ++i) gu[i] = exp(lR[i]) + exp(zbar.u[i]) - rt[i];
        for (int j = 0; j < m; ++j) gv[j] = exp(lQ[j]) + exp(zbar.v[j]) - ct[j];
        double gw = exp(lT) - s;
        double phibar = phi_from(n, m, rt, ct, s, zbar.u, zbar.v, zbar.w, lT);

        /* z~^{t+1}: printed form zbar - gamma/(3 M theta) grad; mirror form
           z~ - 1/(3 M theta) grad. */
        const zvec* base = step_rule == 0 ? &zbar : &ztil;
        double eta = step_rule == 0 ? gamma / (3.0 * M * theta) : 1.0 / (3.0 * M * theta);
        for (int i = 0; i < n; ++i) ztil1.u[i] = base->u[i] - eta * gu[i];
        for (int j = 0; j < m; ++j) ztil1.v[j] = base->v[j] - eta * gv[j];
        ztil1.w = base->w - eta * gw;

        /* z-grave^t = zbar^t + theta_t (z~^{t+1} - z~^t) */
        double gdot = 0.0, step2 = 0.0;
        for (int i = 0; i < n; ++i) {
            double d = ztil1.u[i] - ztil.u[i];
            zgrave.u[i] = zbar.u[i] + theta * d;
            gdot += d * gu[i];
            step2 += d * d;
        }
        for (int j = 0; j < m; ++j) {
            double d = ztil1.v[j] - ztil.v[j];
            zgrave.v[j] = zbar.v[j] + theta * d;
            gdot += d * gv[j];
            step2 += d * d;
        }
        {
            double d = ztil1.w - ztil.w;
            zgrave.w = zbar.w + theta * d;
            gdot += d * gw;
            step2 += d * d;
        }
        gdot *= theta;

        /* z-hat^t = GreenkhornStep(z-grave^t) */
        double sc[3];
        potref_stats(n, m, C, ldc, gamma, zgrave.u, zgrave.v, zgrave.w, lR, lQ, &lT);
        double phigrave = phi_from(n, m, rt, ct, s, zgrave.u, zgrave.v, zgrave.w, lT);
        gk_scores(n, m, rt, ct, s, zgrave.u, zgrave.v, lR, lQ, lT, sc);
        int bhat = block_rule == 0 ? pick_block(sc) : (cyc++ % 3);
        z_copy(n, m, &zhat, &zgrave);
        gk_apply(bhat, n, m, rt, ct, s, zhat.u, zhat.v, &zhat.w, lR, lQ, lT);
        double phihat = potref_phi(n, m, C, ldc, gamma, rt, ct, s, zhat.u, zhat.v, zhat.w);

        /* z^t = argmin { phi(z) : z in { z-check^t, z-hat^t } }, ties keep z-check */
        int pick = phihat < phichk ? 1 : 0;
        z_copy(n, m, &z, pick ? &zhat : &zchk);
        double phiz = pick ? phihat : phichk;

        /* E(z^t); stop and output z^t once E <= eps~ */
        potref_stats(n, m, C, ldc, gamma, z.u, z.v, z.w, lR, lQ, &lT);
        E = error_from(n, m, rt, ct, s, z.u, z.v, lR, lQ, lT);
        if (t < cap) {
            if (o->tr_bhat) o->tr_bhat[t] = bhat;
            if (o->tr_pick) o->tr_pick[t] = pick;
            if (o->tr_E) o->tr_E[t] = E;
            if (o->tr_theta) o->tr_theta[t] = theta;
            if (o->tr_phibar) o->tr_phibar[t] = phibar;
            if (o->tr_phigrave) o->tr_phigrave[t] = phigrave;
            if (o->tr_phihat) o->tr_phihat[t] = phihat;
            if (o->tr_phichk) o->tr_phichk[t] = phichk;
            if (o->tr_phiz) o->tr_phiz[t] = phiz;
            if (o->tr_gdot) o->tr_gdot[t] = gdot;
            if (o->tr_step2) o->tr_step2[t] = step2;
            if (o->tr_ztil) {
                double* h = o->tr_ztil + (size_t)t * (size_t)(n + m + 1);
                memcpy(h, ztil.u, sizeof(double) * (size_t)n);
                memcpy(h + n, ztil.v, sizeof(double) * (size_t)m);
                h[n + m] = ztil.w;
            }
        }
        if (E <= tol) {
            if (t < cap) {
                if (o->tr_bchk) o->tr_bchk[t] = -1;
                if (o->tr_phinext) o->tr_phinext[t] = NAN;
            }
            status = POTREF_OK;
            ++t;
            break;
        }

        /* z-check^{t+1} = GreenkhornStep(z^t) */
        gk_scores(n, m, rt, ct, s, z.u, z.v, lR, lQ, lT, sc);
        int bchk = block_rule == 0 ? pick_block(sc) : (cyc++ % 3);
        z_copy(n, m, &zchk, &z);
        gk_apply(bchk, n, m, rt, ct, s, zchk.u, zchk.v, &zchk.w, lR, lQ, lT);
        phichk = potref_phi(n, m, C, ldc, gamma, rt, ct, s, zchk.u, zchk.v, zchk.w);
        if (t < cap) {
            if (o->tr_bchk) o->tr_bchk[t] = bchk;
            if (o->tr_phinext) o->tr_phinext[t] = phichk;
        }

        /* theta_{t+1} = theta_t (sqrt(theta_t^2 + 4) - theta_t) / 2 */
        z_copy(n, m, &ztil, &ztil1);
        theta = theta * (sqrt(theta * theta + 4.0) - theta) / 2.0;
    }

    memcpy(u_out, z.u, sizeof(double) * (size_t)n);
    memcpy(v_out, z.v, sizeof(double) * (size_t)m);
    *w_out = z.w;
    if (iters_out) *iters_out = t;
    if (E_out) *E_out = E;

    z_free(&zchk); z_free(&ztil); z_free(&zbar); z_free(&ztil1);
    z_free(&zgrave); z_free(&zhat); z_free(&z);
    free(lR); free(lQ); free(gu); free(gv);
    return status;
}

/* ---------------------------------------------------------------------- */
/* Feasible Sinkhorn on the extended instance (Algorithm 3 loop).          */
/* ---------------------------------------------------------------------- */
int potref_sinkhorn(int n, int m, const double* C, long ldc, double gamma, double tol,
                    const double* rt, const double* ct, double s, double A, int max_iter,
                    double* a_out, double* b_out, int* iters_out, double* err_out,
                    double* tr_err) {
    const int n1 = n + 1, m1 = m + 1;
    const double ig = 1.0 / gamma;
    /* C^ = [[C, 0], [0^T, A]] */
    double* Ce = (double*)malloc(sizeof(double) * (size_t)n1 * (size_t)m1);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < m; ++j) Ce[(size_t)i * m1 + j] = C[(long)i * ldc + j];
        Ce[(size_t)i * m1 + m] = 0.0;
    }
    for (int j = 0; j < m; ++j) Ce[(size_t)n * m1 + j] = 0.0;
    Ce[(size_t)n * m1 + m] = A;
    /* r^ = (r~, |c~|_1 - s), c^ = (c~, |r~|_1 - s) */
    double* rh = (double*)malloc(sizeof(double) * (size_t)n1);
    double* chh = (double*)malloc(sizeof(double) * (size_t)m1);
    memcpy(rh, rt, sizeof(double) * (size_t)n);
    memcpy(chh, ct, sizeof(double) * (size_t)m);
    rh[n] = sum_vec(m, ct) - s;
    chh[m] = sum_vec(n, rt) - s;
    if (rh[n] < 0.0) rh[n] = 0.0;
    if (chh[m] < 0.0) chh[m] = 0.0;

    double* a = (double*)calloc((size_t)n1, sizeof(double));
    double* b = (double*)calloc((size_t)m1, sizeof(double));
    double* colmx = (double*)malloc(sizeof(double) * (size_t)m1);
    double* colacc = (double*)malloc(sizeof(double) * (size_t)m1);
    double* rows = (double*)malloc(sizeof(double) * (size_t)n1);
    double* cols = (double*)malloc(sizeof(double) * (size_t)m1);

    int status = POTREF_NOCONV, it = 0;
    double err = INFINITY;
    for (it = 0; it < max_iter; ++it) {
        /* u <- log r^ - LSE_j (v_j - C^_ij / gamma) */
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n1; ++i) {
            const double* Ci = Ce + (size_t)i * m1;
            double mx = -INFINITY;
            for (int j = 0; j < m1; ++j) {
                double x = b[j] - Ci[j] * ig;
                if (x > mx) mx = x;
            }
            double acc = 0.0;
            for (int j = 0; j < m1; ++j) acc += exp(b[j] - Ci[j] * ig - mx);
            a[i] = log(rh[i]) - (mx + log(acc));
        }
        /* v <- log c^ - LSE_i (u_i - C^_ij / gamma) */
        for (int j = 0; j < m1; ++j) { colmx[j] = -INFINITY; colacc[j] = 0.0; }
        for (int i = 0; i < n1; ++i) {
            const double* Ci = Ce + (size_t)i * m1;
            for (int j = 0; j < m1; ++j) {
                double x = a[i] - Ci[j] * ig;
                if (x > colmx[j]) colmx[j] = x;
            }
        }
        for (int i = 0; i < n1; ++i) {
            const double* Ci = Ce + (size_t)i * m1;
            for (int j = 0; j < m1; ++j) colacc[j] += exp(a[i] - Ci[j] * ig - colmx[j]);
        }
        for (int j = 0; j < m1; ++j) b[j] = log(chh[j]) - (colmx[j] + log(colacc[j]));

        /* |X^ 1 - r^|_1 + |X^T 1 - c^|_1 at the new (u, v) */
        for (int j = 0; j < m1; ++j) cols[j] = 0.0;
        for (int i = 0; i < n1; ++i) {
            const double* Ci = Ce + (size_t)i * m1;
            double acc = 0.0;
            for (int j = 0; j < m1; ++j) {
                double x = exp(a[i] + b[j] - Ci[j] * ig);
                acc += x;
                cols[j] += x;
            }
            rows[i] = acc;
        }
        err = 0.0;
        for (int i = 0; i < n1; ++i) err += fabs(rows[i] - rh[i]);
        for (int j = 0; j < m1; ++j) err += fabs(cols[j] - chh[j]);
        if (tr_err) tr_err[it] = err;
        if (err <= tol) {
            status = POTREF_OK;
            ++it;
            break;
        }
    }
    memcpy(a_out, a, sizeof(double) * (size_t)n1);
    memcpy(b_out, b, sizeof(double) * (size_t)m1);
    if (iters_out) *iters_out = it;
    if (err_out) *err_out = err;
    free(Ce); free(rh); free(chh); free(a); free(b);
    free(colmx); free(colacc); free(rows); free(cols);
    return status;
}

/* ---------------------------------------------------------------------- */
/* Rounding onto U(r, c, s).                                               */
/* ---------------------------------------------------------------------- */
/* The paper cites ROUND-POT without printing it.  Reading used here, on the
   original r, c, s:
     1. alpha_i = min(1, r_i / (X 1)_i), X' = diag(alpha) X;
     2. beta_j = min(1, c_j / (X'^T 1)_j), X'' = X' diag(beta), T'' = |X''|_1;
     3. if T'' > s: Xbar = (s / T'') X'';
        if T'' < s: p' = r - X'' 1, q' = c - X''^T 1, delta = s - T'',
                    Xbar = X'' + delta p' q'^T / (|p'|_1 |q'|_1);
        else Xbar = X''.
   (0/0 is read as 1 in steps 1 and 2.) */
static int round_core(int n, int m, double* X /* in: X~, out: Xbar */,
                      const double* r, const double* c, double s,
                      double* alpha, double* beta, double* pp, double* qq, double* out3) {
    double* rs = (double*)malloc(sizeof(double) * (size_t)n);
    double* cs = (double*)calloc((size_t)m, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) rs[i] = sum_vec(m, X + (size_t)i * m);
    for (int i = 0; i < n; ++i) {
        double a = rs[i] > r[i] ? r[i] / rs[i] : 1.0;
        alpha[i] = a;
        double* Xi = X + (size_t)i * m;
        for (int j = 0; j < m; ++j) Xi[j] *= a;
    }
    for (int i = 0; i < n; ++i) {
        const double* Xi = X + (size_t)i * m;
        for (int j = 0; j < m; ++j) cs[j] += Xi[j];
    }
    for (int j = 0; j < m; ++j) beta[j] = cs[j] > c[j] ? c[j] / cs[j] : 1.0;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double* Xi = X + (size_t)i * m;
        for (int j = 0; j < m; ++j) Xi[j] *= beta[j];
        rs[i] = sum_vec(m, Xi);
    }
    for (int j = 0; j < m; ++j) cs[j] = 0.0;
    for (int i = 0; i < n; ++i) {
        const double* Xi = X + (size_t)i * m;
        for (int j = 0; j < m; ++j) cs[j] += Xi[j];
    }
    double T2 = sum_vec(n, rs);
    double kappa = 1.0, lambda = 0.0;
    for (int i = 0; i < n; ++i) pp[i] = 0.0;
    for (int j = 0; j < m; ++j) qq[j] = 0.0;
    if (T2 > s) {
        kappa = s / T2;
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            double* Xi = X + (size_t)i * m;
            for (int j = 0; j < m; ++j) Xi[j] *= kappa;
        }
    } else if (T2 < s) {
        for (int i = 0; i < n; ++i) pp[i] = r[i] - rs[i] > 0.0 ? r[i] - rs[i] : 0.0;
        for (int j = 0; j < m; ++j) qq[j] = c[j] - cs[j] > 0.0 ? c[j] - cs[j] : 0.0;
        double np = sum_vec(n, pp), nq = sum_vec(m, qq);
        /* np >= |r|_1 - T'' > 0 and nq > 0 whenever s <= min(|r|_1, |c|_1) */
        lambda = np * nq > 0.0 ? (s - T2) / (np * nq) : 0.0;
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            double* Xi = X + (size_t)i * m;
            for (int j = 0; j < m; ++j) Xi[j] += lambda * pp[i] * qq[j];
        }
    }
    out3[0] = kappa;
    out3[1] = lambda;
    out3[2] = T2;
    free(rs);
    free(cs);
    return POTREF_OK;
}

double potref_cost(int n, int m, const double* C, long ldc, const double* X) {
    double* part = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp parallel
    {
        double* pr = (double*)malloc(sizeof(double) * (size_t)m);
#pragma omp for schedule(static)
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < m; ++j) pr[j] = C[(long)i * ldc + j] * X[(size_t)i * m + j];
            part[i] = sum_vec(m, pr);
        }
        free(pr);
    }
    double tot = sum_vec(n, part);
    free(part);
    return tot;
}

int potref_round(int n, int m, const double* C, long ldc, double gamma,
                 const double* f, const double* g,
                 const double* r, const double* c, double s,
                 double* alpha, double* beta, double* pp, double* qq,
                 double* out5, double* X_out) {
    const double ig = 1.0 / gamma;
    double* X = (double*)malloc(sizeof(double) * (size_t)n * (size_t)m);
    /* Form primal: X~_ij = exp(f_i + g_j - C_ij / gamma) */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < m; ++j)
            X[(size_t)i * m + j] = exp(f[i] + g[j] - C[(long)i * ldc + j] * ig);
    double o3[3];
    round_core(n, m, X, r, c, s, alpha, beta, pp, qq, o3);
    out5[0] = o3[0];
    out5[1] = o3[1];
    out5[2] = o3[2];
    out5[3] = potref_cost(n, m, C, ldc, X);
    double* rs = (double*)malloc(sizeof(double) * (size_t)n);
    for (int i = 0; i < n; ++i) rs[i] = sum_vec(m, X + (size_t)i * m);
    out5[4] = sum_vec(n, rs);
    free(rs);
    if (X_out) memcpy(X_out, X, sizeof(double) * (size_t)n * (size_t)m);
    free(X);
    return POTREF_OK;
}

int potref_round_dense(int n, int m, const double* X, const double* r,
                       const double* c, double s, double* X_out) {
    double* alpha = (double*)malloc(sizeof(double) * (size_t)n);
    double* beta = (double*)malloc(sizeof(double) * (size_t)m);
    double* pp = (double*)malloc(sizeof(double) * (size_t)n);
    double* qq = (double*)malloc(sizeof(double) * (size_t)m);
    double o3[3];
    memcpy(X_out, X, sizeof(double) * (size_t)n * (size_t)m);
    round_core(n, m, X_out, r, c, s, alpha, beta, pp, qq, o3);
    free(alpha); free(beta); free(pp); free(qq);
    return POTREF_OK;
}

/* ---------------------------------------------------------------------- */
/* Checks of a solver's output point (used to judge another solver's       */
/* result against the definitions, not by the algorithms above).           */
/* ---------------------------------------------------------------------- */
/* Stopping error of feasible Sinkhorn (Algorithm 3) at the extended
   log-scalings a (n+1), b (m+1): |X^ 1 - r^|_1 + |X^T 1 - c^|_1 with
   X^_ij = exp(a_i + b_j - C^_ij / gamma), C^ = [[C, 0], [0^T, A]],
   r^ = (r~, |c~|_1 - s), c^ = (c~, |r~|_1 - s).  Every entry is summed
   directly; no dummy row or column is treated in closed form. */
double potref_sk_error(int n, int m, const double* C, long ldc, double gamma,
                       const double* rt, const double* ct, double s, double A,
                       const double* a, const double* b) {
    const int n1 = n + 1, m1 = m + 1;
    const double ig = 1.0 / gamma;
    double* rows = (double*)malloc(sizeof(double) * (size_t)n1);
    double* cols = (double*)calloc((size_t)m1, sizeof(double));
    double rh_d = sum_vec(m, ct) - s, ch_d = sum_vec(n, rt) - s;
    if (rh_d < 0.0) rh_d = 0.0;
    if (ch_d < 0.0) ch_d = 0.0;
#pragma omp parallel
    {
        double* cl = (double*)calloc((size_t)m1, sizeof(double));
#pragma omp for schedule(static)
        for (int i = 0; i < n1; ++i) {
            double acc = 0.0;
            for (int j = 0; j < m1; ++j) {
                double cij = (i < n && j < m) ? C[(long)i * ldc + j] : ((i == n && j == m) ? A : 0.0);
                double x = exp(a[i] + b[j] - cij * ig);
                acc += x;
                cl[j] += x;
            }
            rows[i] = acc;
        }
#pragma omp critical
        for (int j = 0; j < m1; ++j) cols[j] += cl[j];
        free(cl);
    }
    double e = 0.0;
    for (int i = 0; i < n1; ++i) e += fabs(rows[i] - (i < n ? rt[i] : rh_d));
    for (int j = 0; j < m1; ++j) e += fabs(cols[j] - (j < m ? ct[j] : ch_d));
    free(rows);
    free(cols);
    return e;
}

/* A plan given in factored form,
     Xbar_ij = kappa alpha_i exp(f_i + g_j - Cp_ij / gamma) beta_j + lambda p'_i q'_j,
   evaluated entry by entry: its row sums (rows_out, n), column sums
   (cols_out, m), out3 = {<Ce, Xbar>, 1^T Xbar 1, min_ij Xbar_ij}.  Cp is the
   cost inside the exponent, Ce the cost the plan is priced with (they differ
   when a plan computed on a rounded cost is priced on the exact one). */
int potref_plan_eval(int n, int m, const double* Cp, long ldp, const double* Ce, long lde,
                     double gamma, const double* f, const double* g,
                     const double* alpha, const double* beta, double kappa, double lambda,
                     const double* pp, const double* qq,
                     double* rows_out, double* cols_out, double* out3) {
    const double ig = 1.0 / gamma;
    double* part = (double*)malloc(sizeof(double) * (size_t)n);
    double* cols = (double*)calloc((size_t)m, sizeof(double));
    double mn = INFINITY;
#pragma omp parallel
    {
        double* x = (double*)malloc(sizeof(double) * (size_t)m);
        double* cx = (double*)malloc(sizeof(double) * (size_t)m);
        double* cl = (double*)calloc((size_t)m, sizeof(double));
        double lmn = INFINITY;
#pragma omp for schedule(static)
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < m; ++j) {
                double xt = exp(f[i] + g[j] - Cp[(long)i * ldp + j] * ig);
                double v = kappa * (alpha[i] * xt * beta[j]) + lambda * pp[i] * qq[j];
                x[j] = v;
                cx[j] = Ce[(long)i * lde + j] * v;
                cl[j] += v;
                if (v < lmn) lmn = v;
            }
            rows_out[i] = sum_vec(m, x);
            part[i] = sum_vec(m, cx);
        }
#pragma omp critical
        {
            for (int j = 0; j < m; ++j) cols[j] += cl[j];
            if (lmn < mn) mn = lmn;
        }
        free(x);
        free(cx);
        free(cl);
    }
    for (int j = 0; j < m; ++j) cols_out[j] = cols[j];
    out3[0] = sum_vec(n, part);
    out3[1] = sum_vec(n, rows_out);
    out3[2] = mn;
    free(part);
    free(cols);
    return POTREF_OK;
}
