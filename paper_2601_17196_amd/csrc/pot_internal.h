// pot_internal.h -- shared device/host definitions of libpot (gfx950).
//
// Layout of one solve's workspace, the control block the device-side
// decision logic keeps, and the argument block of the statistics pass.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pot.h"

namespace pot {

constexpr int kThreads = 256;         // workgroup size of the tiled passes (4 wave64s)
constexpr int kScal = 8;              // FP64 per-strip partial sums carried to the decider
constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLn2 = 0.6931471805599453094;

// Passes of the solver.  One launch of the statistics kernel is one pass.
enum Phase : int {
    PH_INIT = 0,     // phi at the start point
    PH_BAR = 1,      // ASPOT: statistics at zbar^t -> gradient
    PH_GRAVE = 2,    // ASPOT: statistics at z-grave^t -> Greenkhorn step -> z-hat^t, argmin
    PH_Z = 3,        // ASPOT: statistics at z^t -> E(z^t), stop, Greenkhorn step -> z-check^{t+1}
    PH_SK_ROW = 4,   // Sinkhorn: row sums at (a^k, b^k) -> error of iterate k, a^{k+1}
    PH_SK_COL = 5,   // Sinkhorn: column sums at (a^{k+1}, b^k) -> b^{k+1}
    PH_R1 = 6,       // rounding: FP64 row sums of X~ -> alpha
    PH_R2 = 7,       // rounding: FP64 column sums of diag(alpha) X~ -> beta, q'
    PH_R3 = 8,       // rounding: FP64 row sums of X'' and C X'', C q' -> p', cost
    PH_R4 = 9,       // rounding: dense plan
    PH_R5 = 10,      // plan moments (points cost): z_i = sum_j X~_ij beta_j y_j
};

// Device control block: every scalar of the algorithm lives here, written
// only by the deciding workgroup of a pass (or the setup kernel) and read by
// the next pass.
struct Ctl {
    // setup (Algorithm 2, "Approximating POT")
    double gamma, tol, M, eps, s, cmax, cost_scale;
    double G;              // log2(e) * cost_scale / gamma: exponent slope per unit of stored cost
    double sum_r, sum_c, sum_rt, sum_ct, log_s, A;
    double rhat_d, chat_d, lrhat_d, lchat_d;   // Sinkhorn dummy masses and their logs
    // ASPOT scalar state
    double theta;
    double wchk[2], wtil[2], wbar, wgrave, wz;
    double phichk, phihat, E, T;
    // Sinkhorn scalar state: a_{n+1} by parity, b_{m+1}, LSE of a_1..a_n and b_1..b_m
    double ad[2], bd, lse_a, lse_b;
    // rounding
    double T2, nq, np, cost1, pcq, kappa, lambda, cost, mass;
    double viol_row, viol_col, viol_mass;   // excess of the rounded plan's sums over r, c and |mass - s|
    double phi0;           // warm-start check: phi at the zero start
    int32_t t, done, status, bhat, pick, bchk, iters, nonfinite;
    int32_t out_par;       // Sinkhorn: parity slot of the output a
    int32_t cyc;           // cyclic block counter
    int32_t valid;         // setup status (0 ok)
    int32_t wide;          // a tile of the pass just made had its shift beyond the normal
                           // FP64 window (set by the tile pass, cleared by the decider)
    int32_t cold;          // the start pass evaluates the zero start instead of (u0, v0, w0)
    int32_t used_warm;     // the solve runs from the caller's warm start
    int32_t rounded;       // the rounding passes ran (factors, cost and mass are set)
    int32_t pad0;
};

// The result block of a solve from its control block (host and device).
__host__ __device__ inline void fill_result(const Ctl& c, int algo, pot_result& R) {
    R.status = c.done ? c.status : POT_ERR_DEVICE;
    R.iters = c.iters;
    R.algo = algo;
    R.used_warm = c.used_warm;
    R.cost = c.cost;
    R.E = c.E;
    R.gamma = c.gamma;
    R.tol = c.tol;
    R.phi = c.phichk;
    R.mass = c.mass;
    R.kappa = c.kappa;
    R.lambda = c.lambda;
    R.T2 = c.T2;
    R.cost_scale = c.cost_scale;
    R.cmax = c.cmax;
    R.w = algo == POT_ASPOT ? c.wz : 0.0;
    R.viol_row = c.viol_row;
    R.viol_col = c.viol_col;
    R.viol_mass = c.viol_mass;
    R.ext_a = algo == POT_SINKHORN ? (c.out_par ? c.ad[1] : c.ad[0]) : 0.0;
    R.ext_b = algo == POT_SINKHORN ? c.bd : 0.0;
}

// Pointers into one solve's workspace.
struct Ws {
    Ctl* ctl;
    int32_t* rowcnt;       // [ny]  arrivals per row strip
    int32_t* colcnt;       // [nx]  arrivals per column strip
    int32_t* glob;         // [4]   arrivals of strip finalisers
    int32_t* tshift;       // [nx * ny] per-tile exponent shift, kept across passes
    void* rowpart;         // [nx * n] FP64 row partial sums ([3 * nx * n] in rounding passes)
    void* colpart;         // [ny * m] FP64 column partial sums
    double* rowscal;       // [nrb * kScal] block sums of the finalising pass (rows)
    double* colscal;       // [ncb * kScal] (columns); the rounding passes use [ny] / [nx]
    // per-row FP64 vectors (n)
    double *rt, *lrt, *uchk0, *uchk1, *util0, *util1, *ubar, *ugrave, *uz, *du, *alpha, *pp;
    // per-column FP64 vectors (m)
    double *ct, *lct, *vchk0, *vchk1, *vtil0, *vtil1, *vbar, *vgrave, *vz, *dv, *beta, *qq;
};

struct PassArgs {
    const void* C;
    int64_t ldc;
    const float* x;
    const float* y;
    const double* r;       // original masses (rounding)
    const double* c;
    int32_t n, m, d, kind;
    int32_t br, bc;        // tile rows, tile columns
    int32_t nx, ny;        // column strips, row strips
    int32_t nrb, ncb;      // 64-row and 64-column blocks of the finalising pass
    int32_t phase;
    int32_t max_iter, block_rule, step_rule;
    const double* u0;
    const double* v0;
    double w0;
    const int32_t* force;
    int32_t force_len;
    int32_t* trace_i;
    double* trace_d;
    int32_t trace_cap;
    double* plan;          // PH_R4 output
    int32_t* host_done;    // pinned host flag set to 1 by the decider when the solve finishes (or NULL)
    Ws ws;
};

// Arguments of the setup kernel.
struct SetupArgs {
    int32_t n, m, algo, nx, ny;
    int32_t gamma_rule;    // 0 default (Algorithm 2 setup), 1 tuned (Algorithm 3)
    double p;              // exponent of the tuned rule
    double s, eps, gamma_user, tol_user, A_user, cmax, cost_scale, w0;
    const double* r;
    const double* c;
    // device-computed cost maximum {FP64 bits of max C (or max |x - y|^2), count of bad
    // entries}, or NULL when cmax and cost_scale are given
    const unsigned long long* maxbuf;
    int32_t kind;          // pot_cost_kind (how maxbuf is read)
    int32_t warm;          // u0 or v0 given
    Ws ws;
};

// ---------------------------------------------------------------------------
// batched solver (pot_solve_batched): one persistent launch; an instance is
// solved by a group of G workgroups ("members") that split its rows
// ---------------------------------------------------------------------------
constexpr int kBMax = 1024;           // rows and columns per instance
constexpr int kBMaxGroup = 8;         // members per instance

struct BDesc {
    const void* C;                    // dense cost (F32 or BF16), n x m, ld = ldc
    int64_t ldc;
    const double* r;
    const double* c;
    const double* u0;                 // warm start (n), or NULL
    const double* v0;                 // warm start (m), or NULL
    double* f_out;                    // log scalings out (n), or NULL
    double* g_out;                    // (m), or NULL
    double* u_out;                    // duals out (n), or NULL
    double* v_out;                    // (m), or NULL
    double s, cmax, w0;
    int32_t n, m, G, vec;             // vec: 16-byte vector loads of C allowed
    int64_t off;                      // byte offset of the instance's region in the workspace
};

struct BSlot {
    int32_t inst, member;
};

struct BArgs {
    const BDesc* desc;
    const BSlot* slot;                // members of all instances, largest instance first
    int32_t nslot;
    int32_t batch;
    int32_t* queue;                   // next slot to take
    pot_result* res;                  // per-instance results (device)
    char* base;                       // workspace base (instance regions)
    int32_t algo, max_iter, block_rule, step_rule;
    int32_t warm_check;               // 1: keep a warm start only if phi(z0) < phi(0)
    int32_t spin_limit;               // bound of every wait of a group barrier
    int32_t do_round;                 // 0: skip the rounding (timing runs of the autotuner)
    int32_t gamma_rule;               // 0 default, 1 tuned (Algorithm 3)
    double p;                         // exponent of the tuned rule
    double eps, gamma_user, tol_user, A_user;
};

// byte layout of one instance's region (the same on the host and the device)
struct BLayout {
    int64_t sync, rows, cols, colpart, rowsc, total;
};
__host__ __device__ inline BLayout blayout(int n, int m, int G) {
    auto al = [](int64_t x) { return (x + 255) & ~(int64_t)255; };
    BLayout L;
    L.sync = 0;                                          // int32 [2]: barrier count, error
    L.rows = 256;                                        // 12 FP64 row vectors of length n
    L.cols = L.rows + al(12 * 8 * (int64_t)n);           // per member: 12 FP64 column vectors of length m
    L.colpart = L.cols + al(12 * 8 * (int64_t)m) * G;    // FP64 [G][m] column partials
    L.rowsc = L.colpart + al(8 * (int64_t)m * G);        // FP64 [G][kScal] row-side scalars
    L.total = L.rowsc + al(8 * (int64_t)kScal * G);
    return L;
}

// per-member state of a shared-cost batch (pot_solve_shared), device arrays
struct SharedCtl {
    int32_t* done;         // [B] finished (converged, stopped at max_iter, invalid or not representable)
    int32_t* iters;        // [B]
    int32_t* status;       // [B] pot_status
    int32_t* out_par;      // [B] parity slot of the output row scalings
    double* E;             // [B] stopping error of the output iterate
    const double* tol;     // [B] threshold
    int32_t* ndone;        // [1] members finished
    int32_t* host_done;    // pinned host flag set when every member has finished, or NULL
};

// a rigid map F(y) = R y + t (R row-major), passed to kernels by value
struct RigidMap {
    double R[9];
    double t[3];
};

// one instance of the warm-start inference (pot_warm_predict)
struct WDesc {
    const float* x;
    const float* y;
    const double* r;
    const double* c;
    double* u0;
    double* v0;
    double cost_scale, inv_gamma;
    int32_t n, m;
};

}  // namespace pot
