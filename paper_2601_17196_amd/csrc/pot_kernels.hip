// pot_kernels.hip -- device code of libpot for gfx950 (MI355X).
//
// One pass over the cost is two launches.  In `stats_pass` every workgroup
// (WG) owns a tile of BR rows x BC columns, forms the exponent
//     t_ij = log2(e) (u_i + v_j + w - C_ij / gamma)   (in FP64)
// takes 2^t in FP32 and accumulates FP64 row and column partial sums of the
// tile (B(z)'s row sums R, column sums Q and total T, Section 2.1).  In
// `fin_pass` each WG reduces the partials of 64 rows or columns and applies
// the per-row (per-column) step of the algorithm; the last WG makes the
// scalar decisions of the iteration (block choice, argmin, stopping) for the
// next pass.  No host round trip per iteration.
//
// The FP64 rounding passes (`round_pass`) use the same tile/strip scheme with
// an FP64 exponential and FP64 accumulation.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <math.h>

#include <type_traits>

#include "pot_internal.h"

namespace pot {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
// Wave reductions with DPP lane moves (VALU only; no LDS round trips).  A
// double moves as its two 32-bit halves.  `old` is what lanes outside the
// row mask receive.  Every lane of the wave must be active.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_d(double v, double old) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, ROW_MASK, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp_f(float v, float old) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}
constexpr int kQuadX1 = 0xB1;      // quad_perm [1, 0, 3, 2]
constexpr int kQuadX2 = 0x4E;      // quad_perm [2, 3, 0, 1]
constexpr int kHalfMirror = 0x141; // row_half_mirror
constexpr int kMirror = 0x140;     // row_mirror
constexpr int kBcast15 = 0x142;    // row_bcast:15 (lane 15 of a row into the next row)
constexpr int kBcast31 = 0x143;    // row_bcast:31 (lane 31 into rows 2 and 3)

__device__ __forceinline__ double readlane_d(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// fixed combination order: deterministic; the total is returned to every lane
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_d<kQuadX1>(v, 0.0);
    v += dpp_d<kQuadX2>(v, 0.0);
    v += dpp_d<kHalfMirror>(v, 0.0);
    v += dpp_d<kMirror>(v, 0.0);            // every lane: its row's sum
    v += dpp_d<kBcast15, 0xA>(v, 0.0);      // rows 1, 3 add rows 0, 2
    v += dpp_d<kBcast31, 0xC>(v, 0.0);      // rows 2, 3 add rows 0 + 1
    return readlane_d(v, 63);
}

__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_f<kQuadX1>(v, 0.0f);
    v += dpp_f<kQuadX2>(v, 0.0f);
    v += dpp_f<kHalfMirror>(v, 0.0f);
    v += dpp_f<kMirror>(v, 0.0f);
    v += dpp_f<kBcast15, 0xA>(v, 0.0f);
    v += dpp_f<kBcast31, 0xC>(v, 0.0f);
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_d<kQuadX1>(v, v));
    v = fmax(v, dpp_d<kQuadX2>(v, v));
    v = fmax(v, dpp_d<kHalfMirror>(v, v));
    v = fmax(v, dpp_d<kMirror>(v, v));
    v = fmax(v, dpp_d<kBcast15, 0xA>(v, v));
    v = fmax(v, dpp_d<kBcast31, 0xC>(v, v));
    return readlane_d(v, 63);
}

// Sum K doubles over the 256 threads of the block (fixed order: deterministic).
// The result is returned to every thread.
template <int K>
__device__ void block_sum(double (&v)[K], double* lds /* >= 4*K */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) lds[wave * K + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = (lds[k] + lds[K + k]) + (lds[2 * K + k] + lds[3 * K + k]);
    __syncthreads();
}

// Merge (max, sum-of-exp) pairs: log-sum-exp in two numbers.
__device__ __forceinline__ void lse_merge(double& m1, double& s1, double m2, double s2) {
    if (m2 == -INFINITY) return;
    if (m1 == -INFINITY) { m1 = m2; s1 = s2; return; }
    if (m2 > m1) { s1 = s1 * exp(m1 - m2) + s2; m1 = m2; }
    else s1 = s1 + s2 * exp(m2 - m1);
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ void lse_step(double& m, double& s) {
    const double m2 = dpp_d<CTRL, ROW_MASK>(m, -INFINITY), s2 = dpp_d<CTRL, ROW_MASK>(s, 0.0);
    lse_merge(m, s, m2, s2);
}

// log-sum-exp pair over the block; the result is returned to every thread
__device__ void block_lse(double& m, double& s, double* lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    lse_step<kQuadX1>(m, s);
    lse_step<kQuadX2>(m, s);
    lse_step<kHalfMirror>(m, s);
    lse_step<kMirror>(m, s);
    lse_step<kBcast15, 0xA>(m, s);
    lse_step<kBcast31, 0xC>(m, s);
    m = readlane_d(m, 63);
    s = readlane_d(s, 63);
    if (lane == 0) { lds[2 * wave] = m; lds[2 * wave + 1] = s; }
    __syncthreads();
    m = lds[0];
    s = lds[1];
    for (int w = 1; w < 4; ++w) lse_merge(m, s, lds[2 * w], lds[2 * w + 1]);
    __syncthreads();
}

// two-slot state by parity with constant indices (lets a copy of the control block
// live in registers)
__device__ __forceinline__ double pick2(const double (&a)[2], int k) { return k ? a[1] : a[0]; }
__device__ __forceinline__ void put2(double (&a)[2], int k, double v) {
    if (k) a[1] = v;
    else a[0] = v;
}

// Cross-workgroup data inside one launch (tile partials, the points a strip's
// writer stores, strip sums) is written with agent-scope stores and read with
// agent-scope loads, which are coherent across the XCDs' L2 caches; the
// stores are waited for (s_waitcnt vmcnt(0)) before the arrival counter is
// incremented.  This avoids an L2 write-back and invalidate in every
// workgroup, which an agent-scope fence costs.  Data consumed by a later
// launch needs nothing: the kernel boundary orders it.
template <typename T>
__device__ __forceinline__ void st_agent(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_agent(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// s_waitcnt vmcnt(0): every store of this wave has completed
__device__ __forceinline__ void wait_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__device__ __forceinline__ double logaddexp(double a, double b) {
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    double hi = fmax(a, b), lo = fmin(a, b);
    return hi + log1p(exp(lo - hi));
}

// rho(a, b) = b - a + a log(a / b) (Section 2.1 notation) as a * h(d),
// d = b/a - 1, h(d) = d - log(1 + d).  For |d| < 1/2 with y = d / (2 + d):
// log(1 + d) = 2 atanh(y), so h = 2 y^2 / (1 - y) - 2 y^3 sum_k y^{2k} / (2k + 3),
// free of cancellation; |y| <= 1/3 and 18 terms leave a relative error below
// 1e-17.  lb = log b, la = log a.
__device__ double rho_log(double a, double la, double lb) {
    const double d = expm1(lb - la);
    double h;
    if (fabs(d) < 0.5) {
        const double y = d / (2.0 + d), y2 = y * y;
        double p = 1.0 / 39.0;             // k = 18
#pragma unroll
        for (int k = 17; k >= 0; --k) p = fma(p, y2, 1.0 / (2 * k + 3));
        // p = sum_{k=0}^{18} y^{2k} / (2k + 3) (Horner)
        h = 2.0 * y2 / (1.0 - y) - 2.0 * y * y2 * p;
    } else {
        h = d - log1p(d);
    }
    return a * h;
}

// ---------------------------------------------------------------------------
// cost access
// ---------------------------------------------------------------------------
// elements per thread per row: 4 (FP32, points) or 8 (BF16); BC = 64 * VW
template <int KIND> struct Vw { static constexpr int v = 4; };
template <> struct Vw<POT_COST_BF16> { static constexpr int v = 8; };

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
    return __uint_as_float(((uint32_t)b) << 16);
}

// 2^t for an FP64 exponent t, accurate to about one FP32 ulp whatever |t|:
// t = k + f with k = rint(t) taken from the low word of t + 1.5 * 2^52 (exact
// for |t| < 2^31) and f = t - k in [-1/2, 1/2] exact in FP64; 2^f in FP32,
// then scaled by 2^k.  Rounding t itself to FP32 would cost |t| * 2^-24.
// Callers keep |t| < 2^31 (the duals are clamped, |G C| is bounded).
__device__ __forceinline__ float exp2_split(double t) {
    const double magic = 6755399441055744.0;   // 1.5 * 2^52
    const double mm = t + magic;
    const int k = __double2loint(mm);
    const double f = t - (mm - magic);
    return ldexpf(__builtin_amdgcn_exp2f((float)f), k);
}

// Load VW consecutive costs of row i starting at column j (j < m); columns
// >= m are returned as 0 and their terms are zeroed by the caller.
template <int KIND>
__device__ __forceinline__ void load_costs(const PassArgs& A, int i, int j, bool vec_ok, float* c) {
    constexpr int VW = Vw<KIND>::v;
    if (KIND == POT_COST_F32) {
        const float* row = (const float*)A.C + (int64_t)i * A.ldc;
        if (vec_ok && j + VW <= A.m) {
            float4 q = *(const float4*)(row + j);
            c[0] = q.x; c[1] = q.y; c[2] = q.z; c[3] = q.w;
        } else {
#pragma unroll
            for (int k = 0; k < VW; ++k) c[k] = (j + k < A.m) ? row[j + k] : 0.0f;
        }
    } else if (KIND == POT_COST_BF16) {
        const uint16_t* row = (const uint16_t*)A.C + (int64_t)i * A.ldc;
        if (vec_ok && j + VW <= A.m) {
            uint4 q = *(const uint4*)(row + j);
            uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                c[2 * k] = __uint_as_float(w4[k] << 16);
                c[2 * k + 1] = __uint_as_float(w4[k] & 0xffff0000u);
            }
        } else {
#pragma unroll
            for (int k = 0; k < VW; ++k) c[k] = (j + k < A.m) ? bf16_to_f32(row[j + k]) : 0.0f;
        }
    }
}

// ---------------------------------------------------------------------------
// points of the passes: the value of a row (u) or column (v) dual variable at
// the point a pass evaluates, with the state writes of that phase, done by
// the strip's "writer" workgroup only (every WG of the strip computes the same
// value).  The candidate state values are loaded first (`load_cand`), before
// the control block is read, and combined with its scalars afterwards
// (`eval_point`).  side 0 = rows (u, block u), side 1 = columns (v, block v).
// ---------------------------------------------------------------------------
struct SideVecs {
    const double* init;
    double *chk0, *chk1, *til0, *til1, *bar, *grave, *z, *d;
};

__device__ __forceinline__ SideVecs side_vecs(const PassArgs& A, int side) {
    const Ws& w = A.ws;
    if (side == 0) return {A.u0, w.uchk0, w.uchk1, w.util0, w.util1, w.ubar, w.ugrave, w.uz, w.du};
    return {A.v0, w.vchk0, w.vchk1, w.vtil0, w.vtil1, w.vbar, w.vgrave, w.vz, w.dv};
}

struct Cand {
    double q0, q1, q2, q3, q4;
};

// select by value (a conditional on two members would select their addresses
// and keep the struct in scratch memory)
__device__ __forceinline__ double sel(int p, double a, double b) { return p ? a : b; }

template <int PH>
__device__ __forceinline__ Cand load_cand(const PassArgs& A, const SideVecs& V, int side, int i) {
    Cand q = {0.0, 0.0, 0.0, 0.0, 0.0};
    switch (PH) {
    case PH_INIT: q.q0 = V.init ? V.init[i] : 0.0; break;
    case PH_BAR: q.q0 = V.chk0[i]; q.q1 = V.z[i]; q.q2 = V.d[i]; q.q3 = V.til0[i]; q.q4 = V.til1[i]; break;
    case PH_GRAVE: q.q0 = V.bar[i]; q.q1 = V.til0[i]; q.q2 = V.til1[i]; q.q3 = V.d[i]; break;
    case PH_Z: q.q0 = V.grave[i]; q.q1 = V.d[i]; q.q2 = V.chk0[i]; q.q3 = V.chk1[i]; break;
    case PH_SK_ROW:
    case PH_SK_COL:
        if (side == 0) { q.q0 = V.chk0[i]; q.q1 = V.chk1[i]; }   // a^k by parity
        else q.q0 = V.z[i];                                      // b^k
        break;
    default: break;
    }
    return q;
}

template <int PH>
__device__ __forceinline__ double eval_point(const PassArgs& A, const Ctl& c, const SideVecs& V, const Cand& q,
                                           int side, int i, bool writer) {
    const int par = c.t & 1;
    switch (PH) {
    case PH_INIT:
        if (writer) { V.chk0[i] = q.q0; V.til0[i] = q.q0; }
        return q.q0;
    case PH_BAR: {
        // z-check^t = GreenkhornStep(z^{t-1}): d holds this block's delta at z^{t-1}
        double xc = q.q0;
        if (c.t != 0) {
            xc = q.q1 + (c.bchk == side ? q.q2 : 0.0);
            if (writer) (par ? V.chk1 : V.chk0)[i] = xc;
        }
        const double xt = sel(par, q.q4, q.q3);
        const double xb = (1.0 - c.theta) * xc + c.theta * xt;    // zbar^t
        if (writer) V.bar[i] = xb;
        return xb;
    }
    case PH_GRAVE: {
        // z~^{t+1} = base - eta grad phi(zbar); z-grave = zbar + theta (z~^{t+1} - z~^t)
        const double xb = q.q0, xt = sel(par, q.q2, q.q1), g = q.q3;
        const double eta = (A.step_rule == 0 ? c.gamma : 1.0) / (3.0 * c.M * c.theta);
        const double xt1 = (A.step_rule == 0 ? xb : xt) - eta * g;
        const double xg = xb + c.theta * (xt1 - xt);
        if (writer) { (par ? V.til0 : V.til1)[i] = xt1; V.grave[i] = xg; }
        return xg;
    }
    case PH_Z: {
        // z-hat^t = GreenkhornStep(z-grave^t); z^t = argmin phi over {z-check^t, z-hat^t}
        const double xh = q.q0 + (c.bhat == side ? q.q1 : 0.0);
        const double z = c.pick ? xh : sel(par, q.q3, q.q2);
        if (writer) V.z[i] = z;
        return z;
    }
    case PH_SK_ROW: return side == 0 ? sel(par, q.q1, q.q0) : q.q0;   // a^k, b^k
    case PH_SK_COL: return side == 0 ? sel(par, q.q0, q.q1) : q.q0;   // a^{k+1}, b^k
    default: return 0.0;
    }
}

// scalar w of the point of each ASPOT pass
template <int PH>
__device__ __forceinline__ double w_point(const PassArgs& A, const Ctl& c) {
    const int par = c.t & 1;
    switch (PH) {
    case PH_INIT: return A.w0;
    case PH_BAR: return (1.0 - c.theta) * pick2(c.wchk, par) + c.theta * pick2(c.wtil, par);
    case PH_GRAVE: return c.wgrave;
    case PH_Z: return c.wz;
    default: return 0.0;
    }
}

// ---------------------------------------------------------------------------
// per-row and per-column steps of the finalising pass.  The state a step
// reads is loaded (`load_step`) before the control block, together with the
// tile partials, so that the pass makes a single round trip to memory.
// acc slots: 0 T-part, 1 sum e^u, 2 <u, r~>, 3 <du, r~>, 4 rho score,
//            5 E part, 6 spare, 7 non-finite count
// ---------------------------------------------------------------------------
struct StepPre {
    double x0, x1, x2, x3;
};

template <int PH>
__device__ __forceinline__ StepPre load_step(const PassArgs& A, bool row, int i) {
    const Ws& w = A.ws;
    StepPre p = {0.0, 0.0, 0.0, 0.0};
    const double* tv = row ? w.rt : w.ct;          // r~ or c~
    const double* lv = row ? w.lrt : w.lct;        // their logs
    switch (PH) {
    case PH_INIT: p.x0 = (row ? w.uchk0 : w.vchk0)[i]; p.x1 = tv[i]; break;
    case PH_BAR: p.x0 = (row ? w.ubar : w.vbar)[i]; p.x1 = tv[i]; break;
    case PH_GRAVE: p.x0 = (row ? w.ugrave : w.vgrave)[i]; p.x1 = tv[i]; p.x2 = lv[i]; break;
    case PH_Z: p.x0 = (row ? w.uz : w.vz)[i]; p.x1 = tv[i]; p.x2 = lv[i]; break;
    case PH_SK_ROW: p.x0 = w.uchk0[i]; p.x1 = w.uchk1[i]; p.x2 = w.rt[i]; p.x3 = w.lrt[i]; break;
    case PH_SK_COL: p.x0 = w.vz[i]; p.x1 = w.lct[i]; break;
    default: break;
    }
    return p;
}

// ASPOT step of row i (row) or column i: R is the row (column) sum of B at
// the point of the pass, x0 the dual there, x1 the smoothed mass, x2 its log.
template <int PH>
__device__ __forceinline__ void aspot_step(const PassArgs& A, bool row, int i, double R, const StepPre& p,
                                           double* acc) {
    const Ws& w = A.ws;
    const double x = p.x0, t = p.x1;
    acc[7] += isfinite(R) ? 0.0 : 1.0;
    if (row) acc[0] += R;
    switch (PH) {
    case PH_INIT:
        acc[1] += exp(x); acc[2] += t * x;
        break;
    case PH_BAR:
        // gradient of phi at zbar (Section 2.1): R + e^u - r~
        (row ? w.du : w.dv)[i] = R + exp(x) - t;
        break;
    case PH_GRAVE:
    case PH_Z: {
        const double ex = exp(x), b = R + ex, lb = log(b);
        const double d = p.x2 - lb;                 // Greenkhorn step: u + log r~ - log(B 1 + e^u)
        (row ? w.du : w.dv)[i] = d;
        acc[1] += ex; acc[2] += t * x; acc[3] += t * d;
        acc[4] += rho_log(t, p.x2, lb);
        acc[5] += fabs(b - t);
        break;
    }
    default: break;
    }
}

// ---------------------------------------------------------------------------
// the deciding workgroup: scalar logic of the iteration
// ---------------------------------------------------------------------------
// Sum the per-strip partials in a fixed order.
// (agent-scope loads: the rounding passes gather inside the launch that
// wrote the partials)
__device__ void gather_strips(const double* part, int nstrips, double (&tot)[kScal], double* lds) {
#pragma unroll
    for (int k = 0; k < kScal; ++k) tot[k] = 0.0;
    for (int sidx = threadIdx.x; sidx < nstrips; sidx += kThreads)
#pragma unroll
        for (int k = 0; k < kScal; ++k) tot[k] += ld_agent(&part[(int64_t)sidx * kScal + k]);
    block_sum<kScal>(tot, lds);
}

__device__ int argmax3(double a, double b, double d) {
    int k = 0;
    double best = a;
    if (b > best) { k = 1; best = b; }
    if (d > best) k = 2;
    return k;
}

// phi after a block step from a point with sums S (Section 2.1 with the
// stationarity of the updated block, as in the proof of Theorem 3):
//   u-step: |r~|_1 + sum e^v - <u', r~> - <v, c~> - w s
//   v-step: |c~|_1 + sum e^u - <u, r~> - <v', c~> - w s
//   w-step: s + sum e^u + sum e^v - <u, r~> - <v, c~> - w' s
__device__ double phi_after(const Ctl& c, int block, const double* R, const double* Cc, double w) {
    switch (block) {
    case 0: return c.sum_rt + Cc[1] - (R[2] + R[3]) - Cc[2] - w * c.s;
    case 1: return c.sum_ct + R[1] - R[2] - (Cc[2] + Cc[3]) - w * c.s;
    default: {
        double w1 = w + c.log_s - log(R[0]);
        return c.s + R[1] + Cc[1] - R[2] - Cc[2] - w1 * c.s;
    }
    }
}

__device__ __forceinline__ void decide_logic(const PassArgs& A, Ctl& c, const double* Rs, const double* Cs);

// The deciding block: gathers every block's sums (all threads), then thread 0
// runs the iteration's scalar logic on the LDS snapshot of the control block
// and the block writes the snapshot back.
__device__ void decide(const PassArgs& A, Ctl& cs, double* lds) {
    double Rs[kScal], Cs[kScal];
    const bool rows = A.phase != PH_SK_COL;
    const bool cols = A.phase != PH_SK_ROW;
    const bool sk = A.phase == PH_SK_ROW || A.phase == PH_SK_COL;
    {
        // every block's sums in one batch of loads; Sinkhorn passes also merge
        // the blocks' (max, sum of exp) pairs (one side only) in a fixed tree
        const int nr = rows ? A.nrb : 0, nb = nr + (cols ? A.ncb : 0);
        double v[2 * kScal];
#pragma unroll
        for (int k = 0; k < 2 * kScal; ++k) v[k] = 0.0;
        double mx = -INFINITY, se = 0.0;
        for (int b = threadIdx.x; b < nb; b += kThreads) {
            const bool isr = b < nr;
            const double* p = isr ? A.ws.rowscal + (int64_t)b * kScal : A.ws.colscal + (int64_t)(b - nr) * kScal;
            double x[kScal];
#pragma unroll
            for (int k = 0; k < kScal; ++k) x[k] = ld_agent(&p[k]);
#pragma unroll
            for (int k = 0; k < kScal; ++k) {
                v[k] += isr ? x[k] : 0.0;
                v[kScal + k] += isr ? 0.0 : x[k];
            }
            if (sk) lse_merge(mx, se, x[1], x[2]);
        }
        block_sum<2 * kScal>(v, lds);
        if (sk) block_lse(mx, se, lds);
#pragma unroll
        for (int k = 0; k < kScal; ++k) { Rs[k] = v[k]; Cs[k] = v[kScal + k]; }
        if (sk) {
            if (rows) { Rs[1] = mx; Rs[2] = se; }
            else { Cs[1] = mx; Cs[2] = se; }
        }
    }
    if (threadIdx.x == 0) decide_logic(A, cs, Rs, Cs);
    __syncthreads();
    constexpr int kCtlWords = sizeof(Ctl) / 8;
    if (threadIdx.x < kCtlWords)
        reinterpret_cast<uint64_t*>(A.ws.ctl)[threadIdx.x] = reinterpret_cast<const uint64_t*>(&cs)[threadIdx.x];
}

__device__ __forceinline__ void decide_logic(const PassArgs& A, Ctl& c, const double* Rs, const double* Cs) {
    const bool rows = A.phase != PH_SK_COL;
    const bool cols = A.phase != PH_SK_ROW;
    const int t = c.t, par = t & 1;
    // a non-finite sum, or (ASPOT) a total that underflowed even the FP64
    // range after the tiles' shifts: the statistics cannot be represented
    const bool aspot_phase = A.phase == PH_INIT || A.phase == PH_BAR || A.phase == PH_GRAVE || A.phase == PH_Z;
    const bool bad = (rows && Rs[7] > 0.0) || (cols && Cs[7] > 0.0) ||
                     (aspot_phase && !(Rs[0] > 0.0 && isfinite(Rs[0])));
    if (bad) {
        c.nonfinite = 1;
        c.status = POT_ERR_NUMERIC;
        c.done = 1;
        c.iters = t;
        return;
    }
    switch (A.phase) {
    case PH_INIT: {
        c.T = Rs[0];
        c.phichk = Rs[0] + Rs[1] + Cs[1] - Rs[2] - Cs[2] - A.w0 * c.s;
        c.wchk[0] = A.w0;
        c.wtil[0] = A.w0;
        c.theta = 1.0;
        c.t = 0;
        break;
    }
    case PH_BAR: {
        double gw = Rs[0] - c.s;                         // d phi / d w at zbar
        double wb = (1.0 - c.theta) * pick2(c.wchk, par) + c.theta * pick2(c.wtil, par);
        double eta = (A.step_rule == 0 ? c.gamma : 1.0) / (3.0 * c.M * c.theta);
        double wt1 = (A.step_rule == 0 ? wb : pick2(c.wtil, par)) - eta * gw;
        c.wbar = wb;
        put2(c.wtil, par ^ 1, wt1);
        c.wgrave = wb + c.theta * (wt1 - pick2(c.wtil, par));
        break;
    }
    case PH_GRAVE: {
        double T = Rs[0];
        double rho_w = rho_log(c.s, c.log_s, log(T));
        int b = A.block_rule == 0 ? argmax3(Rs[4], Cs[4], rho_w) : (c.cyc++ % 3);
        if (A.force && t < A.force_len) b = A.force[3 * t + 0];
        double ph = phi_after(c, b, Rs, Cs, c.wgrave);
        double wh = c.wgrave + (b == 2 ? c.log_s - log(T) : 0.0);
        int pick = ph < c.phichk ? 1 : 0;                // argmin, ties keep z-check
        if (A.force && t < A.force_len) pick = A.force[3 * t + 1];
        c.bhat = b;
        c.pick = pick;
        c.phihat = ph;
        c.wz = pick ? wh : pick2(c.wchk, par);
        if (A.trace_i && t < A.trace_cap) {
            A.trace_i[3 * t + 0] = b;
            A.trace_i[3 * t + 1] = pick;
        }
        if (A.trace_d && t < A.trace_cap) {
            A.trace_d[4 * t + 1] = c.phichk;
            A.trace_d[4 * t + 2] = ph;
            A.trace_d[4 * t + 3] = c.theta;
        }
        break;
    }
    case PH_Z: {
        double T = Rs[0];
        double E = fabs(T - c.s) + Rs[5] + Cs[5];        // E(z^t), Section 3.1
        c.E = E;
        c.T = T;
        if (A.trace_d && t < A.trace_cap) A.trace_d[4 * t + 0] = E;
        bool stop = E <= c.tol;
        if (A.force && t < A.force_len) stop = A.force[3 * t + 2] < 0;
        if (stop) {
            c.done = 1;
            c.status = POT_OK;
            c.iters = t + 1;
            if (A.trace_i && t < A.trace_cap) A.trace_i[3 * t + 2] = -1;
            break;
        }
        double rho_w = rho_log(c.s, c.log_s, log(T));
        int b = A.block_rule == 0 ? argmax3(Rs[4], Cs[4], rho_w) : (c.cyc++ % 3);
        if (A.force && t < A.force_len) b = A.force[3 * t + 2];
        c.bchk = b;
        c.phichk = phi_after(c, b, Rs, Cs, c.wz);
        put2(c.wchk, par ^ 1, c.wz + (b == 2 ? c.log_s - log(T) : 0.0));
        if (A.trace_i && t < A.trace_cap) A.trace_i[3 * t + 2] = b;
        c.theta = c.theta * (sqrt(c.theta * c.theta + 4.0) - c.theta) / 2.0;
        c.t = t + 1;
        if (t + 1 >= A.max_iter) {
            // out of iterations: output z^t (its duals are still in the z slots)
            c.done = 1;
            c.status = POT_ERR_NO_CONVERGENCE;
            c.iters = t + 1;
            c.t = t;
        }
        break;
    }
    case PH_SK_ROW: {
        // row error of iterate t-1 (columns are exact after the b update)
        double ad = pick2(c.ad, par);
        double rs_d = exp(ad + c.lse_b) + exp(ad + c.bd - c.A / c.gamma);
        double E = Rs[0] + fabs(rs_d - c.rhat_d);
        bool stop = false;
        if (t >= 1) {
            c.E = E;
            if (A.trace_d && t - 1 < A.trace_cap) A.trace_d[4 * (t - 1)] = E;
            stop = E <= c.tol;
            if (A.force && t - 1 < A.force_len) stop = A.force[3 * (t - 1) + 2] < 0;
        }
        if (stop || t >= A.max_iter) {
            c.done = 1;
            c.status = stop ? POT_OK : POT_ERR_NO_CONVERGENCE;
            c.iters = t;
            c.out_par = par;
            break;
        }
        put2(c.ad, par ^ 1, c.lrhat_d - logaddexp(c.lse_b, c.bd - c.A / c.gamma));
        c.lse_a = Rs[1] + log(Rs[2]);
        break;
    }
    case PH_SK_COL: {
        double adn = pick2(c.ad, par ^ 1);
        c.bd = c.lchat_d - logaddexp(c.lse_a, adn - c.A / c.gamma);
        c.lse_b = Cs[1] + log(Cs[2]);
        c.t = t + 1;
        break;
    }
    default: break;
    }
}

// Sinkhorn steps of the finalising pass: one row (column) per thread of the
// first wave; the block's outputs are {error, max, sum of exp, 0.., non-finite}.
__device__ void sk_row_finalise(const PassArgs& A, const Ctl& c, int i0, int rows, const double* R,
                                const StepPre& p, double* out, double* lds) {
    const Ws& w = A.ws;
    const int par = c.t & 1;
    double* an = par ? w.uchk0 : w.uchk1;
    double err = 0.0, nonf = 0.0, mx = -INFINITY, se = 0.0;
    const int r = threadIdx.x;
    if (r < rows) {
        const int i = i0 + r;
        const double a = par ? p.x1 : p.x0;
        const double rs = R[r] + exp(a + c.bd);        // dummy column: cost 0
        err = fabs(rs - p.x2);
        nonf = (isfinite(R[r]) && rs > 0.0) ? 0.0 : 1.0;
        const double anew = a + p.x3 - log(rs);        // u <- u + log r^ - log(X^ 1)
        an[i] = anew;
        mx = anew;
        se = 1.0;
    }
    block_lse(mx, se, lds);
    double v[2] = {err, nonf};
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        st_agent(&out[0], v[0]); st_agent(&out[1], mx); st_agent(&out[2], se);
        for (int k = 3; k < 7; ++k) st_agent(&out[k], 0.0);
        st_agent(&out[7], v[1]);
    }
}

__device__ void sk_col_finalise(const PassArgs& A, const Ctl& c, int j0, int cols, const double* Q,
                                const StepPre& p, double* out, double* lds) {
    const Ws& w = A.ws;
    const int par = c.t & 1;
    const double adn = pick2(c.ad, par ^ 1);
    double nonf = 0.0, mx = -INFINITY, se = 0.0;
    const int q = threadIdx.x;
    if (q < cols) {
        const int j = j0 + q;
        const double cs = Q[q] + exp(adn + p.x0);       // dummy row: cost 0
        nonf = (isfinite(Q[q]) && cs > 0.0) ? 0.0 : 1.0;
        const double bnew = p.x0 + p.x1 - log(cs);
        w.vz[j] = bnew;
        mx = bnew;
        se = 1.0;
    }
    block_lse(mx, se, lds);
    double v[1] = {nonf};
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) {
        st_agent(&out[0], 0.0); st_agent(&out[1], mx); st_agent(&out[2], se);
        for (int k = 3; k < 7; ++k) st_agent(&out[k], 0.0);
        st_agent(&out[7], v[0]);
    }
}

// ---------------------------------------------------------------------------
// the statistics pass
// ---------------------------------------------------------------------------
constexpr int kMaxBR = 256;
typedef float f32x4 __attribute__((ext_vector_type(4)));   // 16-byte vector of the tile loads
constexpr int kMaxBC = 512;

template <int KIND, int PHASE>
__global__ __launch_bounds__(kThreads) void stats_pass(PassArgs A) {
    constexpr bool ROWS = PHASE != PH_SK_COL;     // the pass needs row sums
    constexpr bool COLS = PHASE != PH_SK_ROW;     // ... column sums
    constexpr int VW = (KIND == POT_COST_BF16) ? 8 : 4;
    constexpr bool PTS = (KIND == POT_COST_SQEUCLID_POINTS);
    constexpr int EB = (KIND == POT_COST_BF16) ? 2 : 4;      // bytes per stored cost
    constexpr int U = 4;                                     // rows per load batch
    __shared__ double s_a[kMaxBR];         // row offsets (log2 units, tile shift folded in)
    __shared__ double s_b[kMaxBC];         // column offsets (log2 units)
    __shared__ double s_x[PTS ? kMaxBR * 3 : 1];   // points: source coordinates - tile origin (FP64)
    __shared__ double s_y[PTS ? 256 * 3 : 1];      // points (BC = 256): 2 G (target coordinates - tile origin)
    __shared__ double s_lvl[4];
    // one 16 KB buffer reused by the phases of the kernel:
    //   sweep:     per-lane row partials of a 64-row chunk, float [4][16][64]
    //   columns:   column partials of the 4 waves, double [4][BC]
    __shared__ __align__(16) double s_buf[2048];
    float (*s_rowp)[16][64] = reinterpret_cast<float (*)[16][64]>(s_buf);
    double* s_col = s_buf;                 // [4][bc]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tile = blockIdx.x;
    const int ty = tile % A.ny, tx = tile / A.ny;
    const int i0 = ty * A.br, j0 = tx * A.bc;
    const int rows = min(A.br, A.n - i0), cols = min(A.bc, A.m - j0);
    const int jg = j0 + lane * VW;         // this lane's first column

    // ---- loads, in the order they are needed (vector loads complete in
    // order): the candidate state of this thread's row (tid) and columns
    // (tid, tid + 256) and the tile's shift, then the first batch of costs,
    // which stays in flight while the prologue computes the point of the pass
    // (a converged solve exits below; the hardware drains outstanding loads
    // at the end of a wave)
    // (indices are clamped into range so that the loads are not divergent:
    // a divergent load ends in a wait for every load before it)
    constexpr int NCC = (64 * VW + kThreads - 1) / kThreads;    // column candidates per thread
    const SideVecs RV = side_vecs(A, 0), CV = side_vecs(A, 1);
    const Cand rq = load_cand<PHASE>(A, RV, 0, i0 + min(tid, rows - 1));
    Cand cq[NCC];
#pragma unroll
    for (int h = 0; h < NCC; ++h) cq[h] = load_cand<PHASE>(A, CV, 1, j0 + min(tid + h * kThreads, cols - 1));
    int K = A.ws.tshift[tile];             // this tile's shift, kept from its previous pass
    const bool vec_ok = !PTS && ((A.ldc % VW) == 0) && ((((uintptr_t)A.C) & 15) == 0);
    const bool fast = (PTS || vec_ok) && rows == A.br && (A.br % 64) == 0 && j0 + A.bc <= A.m;
    const char* cbase = (const char*)A.C + ((int64_t)(i0 + wave) * A.ldc + jg) * EB;   // row i0 + wave
    const int64_t rstep = (int64_t)4 * A.ldc * EB;                                      // 4 rows down
    f32x4 pre[U];
    if (!PTS && fast) {
#pragma unroll
        for (int u = 0; u < U; ++u) pre[u] = *(const f32x4*)(cbase + u * rstep);
    }

    Ctl& c = *A.ws.ctl;
    if (c.done) return;                     // converged earlier: nothing to do

    // ---- prologue: the point of this pass on this tile's rows and columns,
    // in log2 units; the duals are clamped to +-2^29 so that every exponent
    // below fits the split of exp2_split (|G * C| < 2^29 is checked on the host)
    const double G = c.G;
    const double wp = w_point<PHASE>(A, c);
    constexpr double kClamp = 536870912.0;  // 2^29
    double ox[3] = {0.0, 0.0, 0.0};        // points: tile origin (first source point)
    if (PTS) {
        for (int k = 0; k < A.d; ++k) ox[k] = (double)A.x[(int64_t)i0 * A.d + k];
    }
    if (tid < rows) {
        double a = fmin(fmax((eval_point<PHASE>(A, c, RV, rq, 0, i0 + tid, tx == 0) + wp) * kLog2e, -kClamp), kClamp);
        if (PTS) {
            // t_ij = a_i + b_j - G |x_i - y_j|^2, with x, y taken relative to the
            // origin o: (a_i - G|x_i - o|^2) + (b_j - G|y_j - o|^2) + 2G (x_i - o).(y_j - o)
            double xx = 0.0;
            for (int k = 0; k < 3; ++k) {
                double xk = k < A.d ? (double)A.x[(int64_t)(i0 + tid) * A.d + k] - ox[k] : 0.0;
                s_x[tid * 3 + k] = xk;
                xx += xk * xk;
            }
            a -= G * xx;
        }
        s_a[tid] = a - (double)K;
    }
#pragma unroll
    for (int h = 0; h < NCC; ++h) {
        const int q = tid + h * kThreads;
        if (q < cols) {
            const int j = j0 + q;
            double v = fmin(fmax(eval_point<PHASE>(A, c, CV, cq[h], 1, j, ty == 0) * kLog2e, -kClamp), kClamp);
            if (PTS) {
                double yy = 0.0;
                for (int k = 0; k < 3; ++k) {
                    double yk = k < A.d ? (double)A.y[(int64_t)j * A.d + k] - ox[k] : 0.0;
                    s_y[q * 3 + k] = 2.0 * G * yk;
                    yy += yk * yk;
                }
                v -= G * yy;
            }
            s_b[q] = v;
        }
    }
    __syncthreads();
    // this lane's VW columns (masked columns get 0 and e = 0 below)
    double b[VW];
    double y2[VW][3];
#pragma unroll
    for (int k = 0; k < VW; ++k) {
        const int q = lane * VW + k;
        const bool in = jg + k < A.m;
        b[k] = in ? s_b[q] : 0.0;
        y2[k][0] = PTS && in ? s_y[q * 3] : 0.0;
        y2[k][1] = PTS && in ? s_y[q * 3 + 1] : 0.0;
        y2[k][2] = PTS && in ? s_y[q * 3 + 2] : 0.0;
    }
    const float Gf = (float)G;
    float bf[VW];
#pragma unroll
    for (int k = 0; k < VW; ++k) bf[k] = (float)b[k];

    // ---- tile.  A sweep forms every term 2^t of the tile, accumulates the
    // column partials (FP32 over a batch of U rows, then FP64) and per-lane
    // row partials, reduced through LDS once per chunk of 64 rows.  It returns
    // the tile's level: the largest row or column sum relative to the shift.
    // A level outside [2^-60, 2^60] (far-apart points, tiny or huge duals at
    // extrapolated ASPOT points) moves the shift and sweeps again; the shift
    // is kept for the tile's next pass, so a far tile re-sweeps once per solve.
    double colacc[VW];

    // terms of one row: returns the row's lane partial and adds to col32
    auto row_terms = [&](auto full_tag, const float* cv, int r, double a, float* col32) __attribute__((always_inline)) -> float {
        constexpr bool FULL = decltype(full_tag)::value;
        float e[VW];
        if constexpr (PTS) {
            const double x0 = s_x[r * 3], x1 = s_x[r * 3 + 1], x2 = s_x[r * 3 + 2];
#pragma unroll
            for (int k = 0; k < VW; ++k)
                e[k] = exp2_split(fma(x0, y2[k][0], fma(x1, y2[k][1], fma(x2, y2[k][2], a + b[k]))));
        } else if constexpr (KIND == POT_COST_BF16) {
            // BF16 costs: FP32 exponent (the BF16 rounding of C dominates its error)
            const float af = (float)a;
#pragma unroll
            for (int k = 0; k < VW; ++k) e[k] = __builtin_amdgcn_exp2f(fmaf(cv[k], -Gf, af + bf[k]));
        } else {
#pragma unroll
            for (int k = 0; k < VW; ++k) e[k] = exp2_split(fma((double)cv[k], -G, a + b[k]));
        }
        if constexpr (!FULL) {
#pragma unroll
            for (int k = 0; k < VW; ++k) e[k] = (jg + k < A.m) ? e[k] : 0.0f;
        }
        float rs = 0.0f;
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            rs += e[k];
            col32[k] += e[k];
        }
        return rs;
    };

    // reduce the per-lane row partials of a 64-row chunk; write them; level
    auto emit_rows = [&](int c0, double scale_d, double& lvl) __attribute__((always_inline)) {
        __syncthreads();
        const int rl = tid >> 2, q = tid & 3;          // row of the chunk, quarter of the lanes
        const int wv = rl & 3, slot = rl >> 2;         // row rl = wave wv's slot-th row
        double sacc = 0.0;
#pragma unroll
        for (int l = 0; l < 16; ++l) sacc += (double)s_rowp[wv][slot][q * 16 + l];
        sacc += dpp_d<kQuadX1>(sacc, 0.0);
        sacc += dpp_d<kQuadX2>(sacc, 0.0);
        const int r = c0 + rl;
        if (r < rows) {
            lvl = fmax(lvl, sacc);                     // (NaN sums reach the finalisers' check)
            if (ROWS && q == 0) ((double*)A.ws.rowpart)[(int64_t)tx * A.n + i0 + r] = sacc * scale_d;
        }
        __syncthreads();
    };

    auto sweep = [&](bool use_pre, double scale_d) __attribute__((always_inline)) -> double {
        double lvl = 0.0;
#pragma unroll
        for (int k = 0; k < VW; ++k) colacc[k] = 0.0;
        for (int c0 = 0; c0 < rows; c0 += 64) {
            // this wave's rows of the chunk: c0 + wave + 4 * slot, slot = 0..15
            if (fast) {
                f32x4 cur[U], nxt[U];
                if (!PTS) {
                    if (use_pre && c0 == 0) {
#pragma unroll
                        for (int u = 0; u < U; ++u) cur[u] = pre[u];
                    } else {
#pragma unroll
                        for (int u = 0; u < U; ++u) cur[u] = *(const f32x4*)(cbase + ((int64_t)c0 / 4 + u) * rstep);
                    }
                }
#pragma unroll
                for (int bb = 0; bb < 16 / U; ++bb) {
                    if (!PTS && bb + 1 < 16 / U) {
#pragma unroll
                        for (int u = 0; u < U; ++u)
                            nxt[u] = *(const f32x4*)(cbase + ((int64_t)c0 / 4 + (bb + 1) * U + u) * rstep);
                    }
                    double av[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) av[u] = s_a[c0 + wave + 4 * (bb * U + u)];
                    float col32[VW];
#pragma unroll
                    for (int k = 0; k < VW; ++k) col32[k] = 0.0f;
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int slot = bb * U + u, r = c0 + wave + 4 * slot;
                        float cv[VW];
                        if constexpr (KIND == POT_COST_BF16) {
                            const uint32_t w4[4] = {__float_as_uint(cur[u][0]), __float_as_uint(cur[u][1]),
                                                    __float_as_uint(cur[u][2]), __float_as_uint(cur[u][3])};
#pragma unroll
                            for (int k = 0; k < 4; ++k) {
                                cv[2 * k] = __uint_as_float(w4[k] << 16);
                                cv[2 * k + 1] = __uint_as_float(w4[k] & 0xffff0000u);
                            }
                        } else if constexpr (KIND == POT_COST_F32) {
                            cv[0] = cur[u][0]; cv[1] = cur[u][1]; cv[2] = cur[u][2]; cv[3] = cur[u][3];
                        }
                        s_rowp[wave][slot][lane] =
                            row_terms(std::integral_constant<bool, true>{}, cv, r, av[u], col32);
                    }
#pragma unroll
                    for (int k = 0; k < VW; ++k) colacc[k] += (double)col32[k];
                    if (!PTS && bb + 1 < 16 / U) {
#pragma unroll
                        for (int u = 0; u < U; ++u) cur[u] = nxt[u];
                    }
                }
            } else {
                for (int slot = 0; slot < 16; ++slot) {
                    const int r = c0 + wave + 4 * slot;
                    float rs = 0.0f;
                    if (r < rows) {
                        float cv[VW];
#pragma unroll
                        for (int k = 0; k < VW; ++k) cv[k] = 0.0f;
                        if (!PTS && jg < A.m) load_costs<KIND>(A, i0 + r, jg, vec_ok, cv);
                        float col32[VW];
#pragma unroll
                        for (int k = 0; k < VW; ++k) col32[k] = 0.0f;
                        rs = row_terms(std::integral_constant<bool, false>{}, cv, r, s_a[r], col32);
#pragma unroll
                        for (int k = 0; k < VW; ++k) colacc[k] += (double)col32[k];
                    }
                    s_rowp[wave][slot][lane] = rs;
                }
            }
            emit_rows(c0, scale_d, lvl);
        }
        if (COLS) {
            // the level also covers this thread's column sums
#pragma unroll
            for (int k = 0; k < VW; ++k) lvl = fmax(lvl, colacc[k]);
        }
        return lvl;
    };

    // largest exponent of the tile's terms (used only when every sum of the
    // tile under- or overflowed, so the level says nothing)
    auto max_exponent = [&]() -> double {
        double mx = -INFINITY;
        for (int r = wave; r < rows; r += 4) {
            float cv[VW];
#pragma unroll
            for (int k = 0; k < VW; ++k) cv[k] = 0.0f;
            if (!PTS && jg < A.m) load_costs<KIND>(A, i0 + r, jg, vec_ok, cv);
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                double t;
                if (PTS) t = fma(s_x[r * 3], y2[k][0], fma(s_x[r * 3 + 1], y2[k][1], fma(s_x[r * 3 + 2], y2[k][2], s_a[r] + b[k])));
                else t = fma((double)cv[k], -G, s_a[r] + b[k]);
                if (jg + k < A.m) mx = fmax(mx, t);
            }
        }
        return mx;
    };

    auto block_level = [&](double v) -> double {
        v = wave_max(v);
        if (lane == 0) s_lvl[wave] = v;
        __syncthreads();
        double l = fmax(fmax(s_lvl[0], s_lvl[1]), fmax(s_lvl[2], s_lvl[3]));
        __syncthreads();
        return l;
    };

    double scale_d = ldexp(1.0, K);
    double lvl = block_level(sweep(true, scale_d));
    const double kHi = 1.152921504606846976e18;   // 2^60
    const double kLo = 8.673617379884035472e-19;  // 2^-60
    if (!(lvl <= kHi && lvl >= kLo)) {
        int delta;
        if (lvl > 0.0 && lvl < INFINITY) delta = ilogb(lvl);
        else {
            // every sum flushed to 0 or overflowed: locate the largest term
            double mx = max_exponent();
            mx = wave_max(mx);
            if (lane == 0) s_lvl[wave] = mx;
            __syncthreads();
            mx = fmax(fmax(s_lvl[0], s_lvl[1]), fmax(s_lvl[2], s_lvl[3]));
            __syncthreads();
            delta = isfinite(mx) ? (int)floor(mx) : 0;
        }
        delta = max(-2000 - K, min(2000 - K, delta));
        if (delta != 0) {
            for (int r = tid; r < rows; r += kThreads) s_a[r] -= (double)delta;
            K += delta;
            __syncthreads();
            scale_d = ldexp(1.0, K);
            sweep(false, scale_d);
            if (tid == 0) A.ws.tshift[tile] = K;
        }
    }
    if (COLS) {
#pragma unroll
        for (int k = 0; k < VW; ++k) s_col[wave * (64 * VW) + lane * VW + k] = colacc[k];
        __syncthreads();
        for (int q = tid; q < cols; q += kThreads) {
            const int B = 64 * VW;
            double v = (s_col[q] + s_col[B + q]) + (s_col[2 * B + q] + s_col[3 * B + q]);
            ((double*)A.ws.colpart)[(int64_t)ty * A.m + j0 + q] = v * scale_d;
        }
    }

}

// ---------------------------------------------------------------------------
// the finalising pass: after the tile pass (the kernel boundary orders its
// partials), each workgroup reduces the partials of 64 rows (or 64 columns)
// in FP64, applies the per-row (per-column) step of the algorithm and writes
// its block's sums; the last block to arrive makes the iteration's scalar
// decisions.
// ---------------------------------------------------------------------------
constexpr int kFinBlock = 64;

template <int PHASE>
__global__ __launch_bounds__(kThreads) void fin_pass(PassArgs A) {
    __shared__ double s_part[4][kFinBlock];
    __shared__ double s_v[kFinBlock];
    __shared__ double s_red[4 * 2 * kScal];
    __shared__ int s_last;
    __shared__ Ctl s_ctl;                              // snapshot of the control block
    static_assert(sizeof(Ctl) % 8 == 0 && sizeof(Ctl) / 8 <= kThreads, "control block copy");
    constexpr int kCtlWords = sizeof(Ctl) / 8;
    const int tid = threadIdx.x;
    constexpr bool rows_pass = PHASE != PH_SK_COL;
    const int blk = blockIdx.x;
    const bool is_row = rows_pass && blk < A.nrb;
    const int cb = rows_pass ? blk - A.nrb : blk;      // column block index
    const int base = is_row ? blk * kFinBlock : cb * kFinBlock;
    const int len = min(kFinBlock, (is_row ? A.n : A.m) - base);
    // loads first, all in one batch: the control block, the tile partials (4
    // threads per row or column, each a quarter of the strips) and the state
    // of the step
    const uint64_t cw = tid < kCtlWords ? reinterpret_cast<const uint64_t*>(A.ws.ctl)[tid] : 0;
    // (indices clamped into range: no divergent loads)
    const int l = tid & (kFinBlock - 1), q = tid / kFinBlock;
    double acc = 0.0;
    {
        const int lc = min(l, len - 1);
        if (is_row) {
            const double* p = (const double*)A.ws.rowpart + base + lc;
#pragma unroll 4
            for (int x = q; x < A.nx; x += 4) acc += p[(int64_t)x * A.n];
        } else {
            const double* p = (const double*)A.ws.colpart + base + lc;
#pragma unroll 4
            for (int y = q; y < A.ny; y += 4) acc += p[(int64_t)y * A.m];
        }
        if (l >= len) acc = 0.0;
    }
    const StepPre pre = load_step<PHASE>(A, is_row, base + min(tid, len - 1));
    if (tid < kCtlWords) reinterpret_cast<uint64_t*>(&s_ctl)[tid] = cw;
    s_part[q][l] = acc;
    __syncthreads();
    const Ctl& c = s_ctl;
    if (c.done) return;              // (uniform: every thread reads the same word)
    // the partials combined in a fixed order
    if (tid < kFinBlock) s_v[tid] = (s_part[0][tid] + s_part[1][tid]) + (s_part[2][tid] + s_part[3][tid]);
    __syncthreads();
    double* out = (is_row ? A.ws.rowscal + (int64_t)blk * kScal : A.ws.colscal + (int64_t)cb * kScal);
    if constexpr (PHASE == PH_SK_ROW) {
        sk_row_finalise(A, c, base, len, s_v, pre, out, s_red);
    } else if constexpr (PHASE == PH_SK_COL) {
        sk_col_finalise(A, c, base, len, s_v, pre, out, s_red);
    } else {
        double sums[kScal];
#pragma unroll
        for (int k = 0; k < kScal; ++k) sums[k] = 0.0;
        if (tid < len) aspot_step<PHASE>(A, is_row, base + tid, s_v[tid], pre, sums);
        block_sum<kScal>(sums, s_red);
        if (tid == 0)
            for (int k = 0; k < kScal; ++k) st_agent(&out[k], sums[k]);
    }
    // arrival: the last block decides
    wait_stores();
    __syncthreads();
    const int total = (rows_pass ? A.nrb : 0) + (PHASE != PH_SK_ROW ? A.ncb : 0);
    if (tid == 0) s_last = (atomicAdd(&A.ws.glob[0], 1) == total - 1);
    __syncthreads();
    if (s_last) {
        decide(A, s_ctl, s_red);
        if (tid == 0) A.ws.glob[0] = 0;
    }
}

// ---------------------------------------------------------------------------
// FP64 rounding passes (form primal and the rounding onto U(r, c, s))
// ---------------------------------------------------------------------------
template <int KIND>
__device__ __forceinline__ double cost64(const PassArgs& A, const Ctl& c, int i, int j) {
    if (KIND == POT_COST_F32) return (double)((const float*)A.C)[(int64_t)i * A.ldc + j];
    if (KIND == POT_COST_BF16) return (double)bf16_to_f32(((const uint16_t*)A.C)[(int64_t)i * A.ldc + j]);
    double s = 0.0;
    for (int k = 0; k < A.d; ++k) {
        double dd = (double)A.x[(int64_t)i * A.d + k] - (double)A.y[(int64_t)j * A.d + k];
        s += dd * dd;
    }
    return c.cost_scale * s;
}

template <int KIND>
__global__ __launch_bounds__(kThreads) void round_pass(PassArgs A) {
    __shared__ double s_red[64];
    __shared__ double s_rows[3][kMaxBR];
    __shared__ double s_cols[4][kMaxBC];
    __shared__ int s_flags[4];
    Ctl& c = *A.ws.ctl;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ty = blockIdx.x % A.ny, tx = blockIdx.x / A.ny;
    const int i0 = ty * A.br, j0 = tx * A.bc;
    const int rows = min(A.br, A.n - i0), cols = min(A.bc, A.m - j0);
    const Ws& w = A.ws;
    const double ig = 1.0 / c.gamma;
    const bool ROWS = A.phase != PH_R2;
    const bool COLS = A.phase == PH_R2;
    // each lane walks columns lane, lane+64, ...; each wave walks rows wave, wave+4, ...
    double colacc[kMaxBC / 64];
    for (int k = 0; k < kMaxBC / 64; ++k) colacc[k] = 0.0;
    for (int r = wave; r < rows; r += 4) {
        const int i = i0 + r;
        const double f = w.ubar[i];
        const double al = (A.phase == PH_R1) ? 1.0 : w.alpha[i];
        double rs = 0.0, rc = 0.0, rq = 0.0;
        int k = 0;
        for (int q = lane; q < cols; q += 64, ++k) {
            const int j = j0 + q;
            const double Cij = cost64<KIND>(A, c, i, j);
            const double x = exp(f + w.vbar[j] - Cij * ig);
            switch (A.phase) {
            case PH_R1: rs += x; break;
            case PH_R2: colacc[k] += al * x; break;
            case PH_R3: {
                double xx = al * w.beta[j] * x;          // X''_ij
                rs += xx;
                rc += Cij * xx;
                rq += Cij * w.qq[j];
                break;
            }
            case PH_R4: {
                double xx = al * w.beta[j] * x;
                A.plan[(int64_t)i * A.m + j] = c.kappa * xx + c.lambda * w.pp[i] * w.qq[j];
                break;
            }
            default: break;
            }
        }
        if (ROWS && A.phase != PH_R4) {
            rs = wave_sum(rs);
            rc = wave_sum(rc);
            rq = wave_sum(rq);
            if (lane == 0) {
                double* rp = (double*)w.rowpart;
                st_agent(&rp[((int64_t)tx * 3 + 0) * A.n + i], rs);
                st_agent(&rp[((int64_t)tx * 3 + 1) * A.n + i], rc);
                st_agent(&rp[((int64_t)tx * 3 + 2) * A.n + i], rq);
            }
        }
    }
    if (A.phase == PH_R4) return;
    if (COLS) {
        int k = 0;
        for (int q = lane; q < cols; q += 64, ++k) s_cols[wave][q] = colacc[k];
        __syncthreads();
        double* cp = (double*)w.colpart;
        for (int q = tid; q < cols; q += kThreads)
            st_agent(&cp[(int64_t)ty * A.m + j0 + q], (s_cols[0][q] + s_cols[1][q]) + (s_cols[2][q] + s_cols[3][q]));
    }
    wait_stores();
    __syncthreads();
    if (tid == 0) {
        s_flags[0] = ROWS ? (atomicAdd(&w.rowcnt[ty], 1) == A.nx - 1) : 0;
        s_flags[1] = COLS ? (atomicAdd(&w.colcnt[tx], 1) == A.ny - 1) : 0;
    }
    __syncthreads();
    int nfin = 0;
    double acc[kScal];
    for (int k = 0; k < kScal; ++k) acc[k] = 0.0;
    if (ROWS && s_flags[0]) {
        const double* rp = (const double*)w.rowpart;
        for (int r = tid; r < rows; r += kThreads) {
            const int i = i0 + r;
            double rs = 0.0, rc = 0.0, rq = 0.0;
            for (int x = 0; x < A.nx; ++x) {
                rs += ld_agent(&rp[((int64_t)x * 3 + 0) * A.n + i]);
                rc += ld_agent(&rp[((int64_t)x * 3 + 1) * A.n + i]);
                rq += ld_agent(&rp[((int64_t)x * 3 + 2) * A.n + i]);
            }
            if (A.phase == PH_R1) {
                // alpha_i = min(1, r_i / (X~ 1)_i), 0/0 read as 1
                w.alpha[i] = rs > A.r[i] ? A.r[i] / rs : 1.0;
                acc[7] += isfinite(rs) ? 0.0 : 1.0;
            } else {
                // p'_i = r_i - (X'' 1)_i
                double p = A.r[i] - rs;
                p = p > 0.0 ? p : 0.0;
                w.pp[i] = p;
                acc[0] += rc;          // <C, X''>
                acc[1] += p;           // |p'|_1
                acc[2] += p * rq;      // p'^T C q'
                acc[3] += rs;          // |X''|_1 (row side)
            }
        }
        block_sum<kScal>(acc, s_red);
        if (tid == 0) {
            for (int k = 0; k < kScal; ++k) st_agent(&w.rowscal[(int64_t)ty * kScal + k], acc[k]);
            w.rowcnt[ty] = 0;
        }
        ++nfin;
    }
    if (COLS && s_flags[1]) {
        const double* cp = (const double*)w.colpart;
        for (int q = tid; q < cols; q += kThreads) {
            const int j = j0 + q;
            double cs = 0.0;
            for (int y = 0; y < A.ny; ++y) cs += ld_agent(&cp[(int64_t)y * A.m + j]);
            // beta_j = min(1, c_j / (X'^T 1)_j); column sums of X'' = beta_j cs
            double be = cs > A.c[j] ? A.c[j] / cs : 1.0;
            w.beta[j] = be;
            double q2 = A.c[j] - be * cs;
            q2 = q2 > 0.0 ? q2 : 0.0;
            w.qq[j] = q2;
            acc[0] += be * cs;        // T''
            acc[1] += q2;             // |q'|_1
            acc[7] += isfinite(cs) ? 0.0 : 1.0;
        }
        block_sum<kScal>(acc, s_red);
        if (tid == 0) {
            for (int k = 0; k < kScal; ++k) st_agent(&w.colscal[(int64_t)tx * kScal + k], acc[k]);
            w.colcnt[tx] = 0;
        }
        ++nfin;
    }
    if (nfin) {
        wait_stores();
        __syncthreads();
        const int total = ROWS ? A.ny : A.nx;
        if (tid == 0) s_flags[2] = (atomicAdd(&w.glob[0], nfin) + nfin == total);
        __syncthreads();
        if (s_flags[2]) {
            double tot[kScal];
            gather_strips(ROWS ? w.rowscal : w.colscal, total, tot, s_red);
            if (tid == 0) {
                if (tot[7] > 0.0) { c.nonfinite = 1; if (c.status == POT_OK) c.status = POT_ERR_NUMERIC; }
                if (A.phase == PH_R2) {
                    c.T2 = tot[0];
                    c.nq = tot[1];
                } else if (A.phase == PH_R3) {
                    c.cost1 = tot[0];
                    c.np = tot[1];
                    c.pcq = tot[2];
                    const double T2 = c.T2;
                    if (T2 > c.s) { c.kappa = c.s / T2; c.lambda = 0.0; }
                    else if (T2 < c.s) {
                        c.kappa = 1.0;
                        double d = c.np * c.nq;
                        c.lambda = d > 0.0 ? (c.s - T2) / d : 0.0;
                    } else { c.kappa = 1.0; c.lambda = 0.0; }
                    c.cost = c.kappa * c.cost1 + c.lambda * c.pcq;
                    c.mass = c.kappa * T2 + c.lambda * c.np * c.nq;
                }
                w.glob[0] = 0;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// setup (Algorithm 2, "Approximating POT"), validation, state initialisation
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void setup_kernel(SetupArgs S) {
    __shared__ double s_red[64];
    __shared__ double s_v[4];
    Ctl& c = *S.ws.ctl;
    const int tid = threadIdx.x, nt = blockDim.x;
    // sums and validity of the masses
    double sr = 0.0, sc = 0.0, bad = 0.0;
    for (int i = tid; i < S.n; i += nt) {
        double x = S.r[i];
        bad += (isfinite(x) && x >= 0.0) ? 0.0 : 1.0;
        sr += x;
    }
    for (int j = tid; j < S.m; j += nt) {
        double x = S.c[j];
        bad += (isfinite(x) && x >= 0.0) ? 0.0 : 1.0;
        sc += x;
    }
    // block reduction over 1024 threads (16 waves)
    {
        const int lane = tid & 63, wave = tid >> 6;
        double v[3] = {sr, sc, bad};
        for (int k = 0; k < 3; ++k) {
            double x = wave_sum(v[k]);
            if (lane == 0) s_red[wave * 3 + k] = x;
        }
        __syncthreads();
        if (tid == 0) {
            double a[3] = {0, 0, 0};
            for (int w = 0; w < nt / 64; ++w)
                for (int k = 0; k < 3; ++k) a[k] += s_red[w * 3 + k];
            s_v[0] = a[0]; s_v[1] = a[1]; s_v[2] = a[2];
        }
        __syncthreads();
    }
    sr = s_v[0];
    sc = s_v[1];
    bad = s_v[2];
    const int N = S.n > S.m ? S.n : S.m;
    double gamma = S.gamma_user > 0.0 ? S.gamma_user : S.eps / (4.0 * log((double)N));
    double et = S.eps / (8.0 * S.cmax);
    if (sr > 1.0) et = fmin(et, 8.0 * (sr - S.s) / (sr - 1.0));
    if (sc > 1.0) et = fmin(et, 8.0 * (sc - S.s) / (sc - 1.0));
    double tol = S.tol_user > 0.0 ? S.tol_user : et;
    int valid = 0;
    if (bad > 0.0) valid = 1;
    else if (!(S.s > 0.0) || S.s > sr || S.s > sc) valid = 2;
    else if (!(gamma > 0.0) || !isfinite(gamma)) valid = 3;
    else if (!(tol > 0.0)) valid = 4;
    // smoothed marginals r~, c~ (and their logs)
    double srt = 0.0, sct = 0.0, nonpos = 0.0;
    for (int i = tid; i < S.n; i += nt) {
        double x = (1.0 - et / 8.0) * S.r[i] + et / (8.0 * S.n);
        S.ws.rt[i] = x;
        S.ws.lrt[i] = log(x);
        nonpos += x > 0.0 ? 0.0 : 1.0;
        srt += x;
    }
    for (int j = tid; j < S.m; j += nt) {
        double x = (1.0 - et / 8.0) * S.c[j] + et / (8.0 * S.m);
        S.ws.ct[j] = x;
        S.ws.lct[j] = log(x);
        nonpos += x > 0.0 ? 0.0 : 1.0;
        sct += x;
    }
    {
        const int lane = tid & 63, wave = tid >> 6;
        double v[3] = {srt, sct, nonpos};
        __syncthreads();
        for (int k = 0; k < 3; ++k) {
            double x = wave_sum(v[k]);
            if (lane == 0) s_red[wave * 3 + k] = x;
        }
        __syncthreads();
        if (tid == 0) {
            double a[3] = {0, 0, 0};
            for (int w = 0; w < nt / 64; ++w)
                for (int k = 0; k < 3; ++k) a[k] += s_red[w * 3 + k];
            s_v[0] = a[0]; s_v[1] = a[1]; s_v[2] = a[2];
        }
        __syncthreads();
    }
    srt = s_v[0];
    sct = s_v[1];
    if (valid == 0 && s_v[2] > 0.0) valid = 5;
    // Sinkhorn state a = 0, b = 0 (b lives in vz)
    if (S.algo == POT_SINKHORN) {
        for (int i = tid; i < S.n; i += nt) S.ws.uchk0[i] = 0.0;
        for (int j = tid; j < S.m; j += nt) S.ws.vz[j] = 0.0;
    }
    for (int k = tid; k < S.ny; k += nt) S.ws.rowcnt[k] = 0;
    for (int k = tid; k < S.nx * S.ny; k += nt) S.ws.tshift[k] = 0;
    for (int k = tid; k < S.nx; k += nt) S.ws.colcnt[k] = 0;
    if (tid < 4) S.ws.glob[tid] = 0;
    if (tid == 0) {
        c.gamma = gamma;
        c.tol = tol;
        c.M = sr + sc - S.s;
        c.eps = S.eps;
        c.s = S.s;
        c.cmax = S.cmax;
        c.cost_scale = S.cost_scale;
        c.G = kLog2e * S.cost_scale / gamma;
        c.sum_r = sr;
        c.sum_c = sc;
        c.sum_rt = srt;
        c.sum_ct = sct;
        c.log_s = log(S.s);
        c.A = S.A_user > 0.0 ? S.A_user : 8.0 * S.cmax / S.eps;
        c.rhat_d = fmax(sct - S.s, 0.0);     // r^ = (r~, |c~|_1 - s)
        c.chat_d = fmax(srt - S.s, 0.0);     // c^ = (c~, |r~|_1 - s)
        c.lrhat_d = log(c.rhat_d);
        c.lchat_d = log(c.chat_d);
        c.theta = 1.0;
        c.wchk[0] = c.wchk[1] = S.w0;
        c.wtil[0] = c.wtil[1] = S.w0;
        c.wbar = c.wgrave = c.wz = S.w0;
        c.phichk = c.phihat = 0.0;
        c.E = INFINITY;
        c.T = 0.0;
        c.ad[0] = 0.0;
        c.ad[1] = 0.0;
        c.bd = 0.0;
        c.lse_a = 0.0;
        c.lse_b = log((double)S.m);
        c.T2 = c.nq = c.np = c.cost1 = c.pcq = 0.0;
        c.kappa = 1.0;
        c.lambda = 0.0;
        c.cost = c.mass = 0.0;
        c.t = 0;
        c.done = valid ? 1 : 0;
        c.status = valid ? POT_ERR_INVALID_ARG : POT_OK;
        c.bhat = c.pick = c.bchk = 0;
        c.iters = 0;
        c.nonfinite = 0;
        c.out_par = 0;
        c.cyc = 0;
        c.valid = valid;
    }
}

// max_ij C_ij and a check that C is finite and >= 0 (dense kinds), or
// max_ij |x_i - y_j|^2 (points): one grid-stride pass.  out[0] receives the
// FP64 bit pattern of the maximum (nonnegative doubles order like their
// bits), out[1] counts bad entries.
template <int KIND>
__global__ __launch_bounds__(kThreads) void cost_max_kernel(const void* C, int64_t ldc, const float* x,
                                                           const float* y, int n, int m, int d,
                                                           unsigned long long* out) {
    double mx = 0.0;
    unsigned long long bad = 0;
    const int64_t total = (int64_t)n * m;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / m), j = (int)(e % m);
        double v;
        if (KIND == POT_COST_F32) v = (double)((const float*)C)[(int64_t)i * ldc + j];
        else if (KIND == POT_COST_BF16) v = (double)bf16_to_f32(((const uint16_t*)C)[(int64_t)i * ldc + j]);
        else {
            v = 0.0;
            for (int k = 0; k < d; ++k) {
                double dd = (double)x[(int64_t)i * d + k] - (double)y[(int64_t)j * d + k];
                v += dd * dd;
            }
        }
        if (!(v >= 0.0) || !isfinite(v)) ++bad;
        else mx = fmax(mx, v);
    }
    mx = wave_max(mx);
    double badd = wave_sum((double)bad);
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&out[0], (unsigned long long)__double_as_longlong(mx));
        if (badd > 0.0) atomicAdd(&out[1], (unsigned long long)badd);
    }
}

// Output duals: f_i, g_j of X~_ij = exp(f_i + g_j - C_ij/gamma) into the
// rounding slots (ubar, vbar) and the optional caller vectors.
__global__ void finish_duals(PassArgs A, int algo, double* fo, double* go, double* uo, double* vo) {
    Ctl& c = *A.ws.ctl;
    const Ws& w = A.ws;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < A.n) {
        const int i = (int)k;
        double u, f;
        if (algo == POT_ASPOT) { u = w.uz[i]; f = u + c.wz; }
        else { u = (c.out_par ? w.uchk1 : w.uchk0)[i]; f = u; }
        w.ubar[i] = f;
        if (fo) fo[i] = f;
        if (uo) uo[i] = u;
    }
    if (k < A.m) {
        const int j = (int)k;
        double g = w.vz[j];
        w.vbar[j] = g;
        if (go) go[j] = g;
        if (vo) vo[j] = g;
    }
}

__global__ void copy_out(PassArgs A, double* alpha, double* beta, double* pp, double* qq) {
    const Ws& w = A.ws;
    const Ctl& c = *A.ws.ctl;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < A.n) {
        if (alpha) alpha[k] = w.alpha[k];
        if (pp) pp[k] = c.lambda > 0.0 ? w.pp[k] : 0.0;
    }
    if (k < A.m) {
        if (beta) beta[k] = w.beta[k];
        if (qq) qq[k] = c.lambda > 0.0 ? w.qq[k] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// host-side launch helpers (C++ linkage, used by pot_api.hip)
// ---------------------------------------------------------------------------
hipError_t launch_setup(const SetupArgs& S, hipStream_t st);

static int fin_blocks(const PassArgs& A) {
    return (A.phase != PH_SK_COL ? A.nrb : 0) + (A.phase != PH_SK_ROW ? A.ncb : 0);
}

template <int KIND, int PHASE>
static hipError_t launch_stats_k(const PassArgs& A, hipStream_t st) {
    stats_pass<KIND, PHASE><<<A.nx * A.ny, kThreads, 0, st>>>(A);
    fin_pass<PHASE><<<fin_blocks(A), kThreads, 0, st>>>(A);
    return hipGetLastError();
}

template <int KIND>
static hipError_t launch_stats_phase(const PassArgs& A, hipStream_t st) {
    switch (A.phase) {
    case PH_INIT: return launch_stats_k<KIND, PH_INIT>(A, st);
    case PH_BAR: return launch_stats_k<KIND, PH_BAR>(A, st);
    case PH_GRAVE: return launch_stats_k<KIND, PH_GRAVE>(A, st);
    case PH_Z: return launch_stats_k<KIND, PH_Z>(A, st);
    case PH_SK_ROW: return launch_stats_k<KIND, PH_SK_ROW>(A, st);
    case PH_SK_COL: return launch_stats_k<KIND, PH_SK_COL>(A, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stats(const PassArgs& A, hipStream_t st) {
    switch (A.kind) {
    case POT_COST_F32: return launch_stats_phase<POT_COST_F32>(A, st);
    case POT_COST_BF16: return launch_stats_phase<POT_COST_BF16>(A, st);
    default: return launch_stats_phase<POT_COST_SQEUCLID_POINTS>(A, st);
    }
}

// Timed launch of the statistics pass: start/stop events recorded around the
// dispatch itself (not around the host call).
template <int KIND>
static hipError_t launch_stats_timed_k(const PassArgs& A, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
                                       hipEvent_t e2, hipEvent_t e3) {
    hipExtLaunchKernelGGL((stats_pass<KIND, PH_INIT>), dim3(A.nx * A.ny), dim3(kThreads), 0, st, e0, e1, 0, A);
    hipExtLaunchKernelGGL(fin_pass<PH_INIT>, dim3(fin_blocks(A)), dim3(kThreads), 0, st, e2, e3, 0, A);
    return hipGetLastError();
}

// Both kernels of one pass, each with start/stop events around its dispatch.
hipError_t launch_stats_timed(const PassArgs& A, hipStream_t st, hipEvent_t e0, hipEvent_t e1, hipEvent_t e2,
                              hipEvent_t e3) {
    switch (A.kind) {
    case POT_COST_F32: return launch_stats_timed_k<POT_COST_F32>(A, st, e0, e1, e2, e3);
    case POT_COST_BF16: return launch_stats_timed_k<POT_COST_BF16>(A, st, e0, e1, e2, e3);
    default: return launch_stats_timed_k<POT_COST_SQEUCLID_POINTS>(A, st, e0, e1, e2, e3);
    }
}

hipError_t launch_round(const PassArgs& A, hipStream_t st) {
    switch (A.kind) {
    case POT_COST_F32: round_pass<POT_COST_F32><<<A.nx * A.ny, kThreads, 0, st>>>(A); break;
    case POT_COST_BF16: round_pass<POT_COST_BF16><<<A.nx * A.ny, kThreads, 0, st>>>(A); break;
    default: round_pass<POT_COST_SQEUCLID_POINTS><<<A.nx * A.ny, kThreads, 0, st>>>(A); break;
    }
    return hipGetLastError();
}

hipError_t launch_setup(const SetupArgs& S, hipStream_t st) {
    setup_kernel<<<1, 1024, 0, st>>>(S);
    return hipGetLastError();
}

hipError_t launch_cost_max(int kind, const void* C, int64_t ldc, const float* x, const float* y, int n,
                           int m, int d, unsigned long long* out, hipStream_t st) {
    const int64_t total = (int64_t)n * m;
    int blocks = (int)((total + kThreads - 1) / kThreads);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    switch (kind) {
    case POT_COST_F32: cost_max_kernel<POT_COST_F32><<<blocks, kThreads, 0, st>>>(C, ldc, x, y, n, m, d, out); break;
    case POT_COST_BF16: cost_max_kernel<POT_COST_BF16><<<blocks, kThreads, 0, st>>>(C, ldc, x, y, n, m, d, out); break;
    default: cost_max_kernel<POT_COST_SQEUCLID_POINTS><<<blocks, kThreads, 0, st>>>(C, ldc, x, y, n, m, d, out); break;
    }
    return hipGetLastError();
}

hipError_t launch_finish(const PassArgs& A, int algo, double* f, double* g, double* u, double* v, hipStream_t st) {
    int len = A.n > A.m ? A.n : A.m;
    finish_duals<<<(len + 255) / 256, 256, 0, st>>>(A, algo, f, g, u, v);
    return hipGetLastError();
}

hipError_t launch_copy_out(const PassArgs& A, double* alpha, double* beta, double* pp, double* qq, hipStream_t st) {
    int len = A.n > A.m ? A.n : A.m;
    copy_out<<<(len + 255) / 256, 256, 0, st>>>(A, alpha, beta, pp, qq);
    return hipGetLastError();
}

}  // namespace pot
