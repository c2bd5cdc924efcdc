// pot_kernels.hip -- device code of libpot for gfx950 (MI355X).
//
// One launch of `stats_pass` is one pass over the cost: every workgroup
// (WG) owns a tile of BR rows x BC columns, forms the exponent
//     t_ij = log2(e) (u_i + v_j + w - C_ij / gamma)   (in FP64)
// takes 2^t in FP32 and accumulates FP64 row and column partial sums of the
// tile (B(z)'s row sums R, column sums Q and total T, Section 2.1).  The last
// WG to finish a row strip (column strip) reduces that strip's partials in
// FP64 and applies the per-row (per-column) step of the algorithm; the last
// strip to finish makes the scalar decisions of the iteration (block choice,
// argmin, stopping) for the next launch.  No host round trip per iteration.
//
// The FP64 rounding passes (`round_pass`) use the same tile/strip scheme with
// an FP64 exponential and FP64 accumulation.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <math.h>

#include "pot_internal.h"

namespace pot {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Sum K doubles over the 256 threads of the block (fixed order: deterministic).
// Result valid in thread 0 (returned to all threads via LDS).
template <int K>
__device__ void block_sum(double (&v)[K], double* lds /* >= 4*K */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = wave_sum(v[k]);
        if (lane == 0) lds[wave * K + k] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = lds[k] + lds[K + k] + lds[2 * K + k] + lds[3 * K + k];
    __syncthreads();
}

// Merge (max, sum-of-exp) pairs: log-sum-exp in two numbers.
__device__ __forceinline__ void lse_merge(double& m1, double& s1, double m2, double s2) {
    if (m2 == -INFINITY) return;
    if (m1 == -INFINITY) { m1 = m2; s1 = s2; return; }
    if (m2 > m1) { s1 = s1 * exp(m1 - m2) + s2; m1 = m2; }
    else s1 = s1 + s2 * exp(m2 - m1);
}

__device__ void block_lse(double& m, double& s, double* lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        double m2 = __shfl_xor(m, o, 64), s2 = __shfl_xor(s, o, 64);
        // combine symmetric pairs in a fixed order (lower lane first)
        if ((lane & o) == 0) lse_merge(m, s, m2, s2);
        else { double mm = m2, ss = s2; lse_merge(mm, ss, m, s); m = mm; s = ss; }
    }
    if (lane == 0) { lds[2 * wave] = m; lds[2 * wave + 1] = s; }
    __syncthreads();
    m = lds[0];
    s = lds[1];
    for (int w = 1; w < 4; ++w) lse_merge(m, s, lds[2 * w], lds[2 * w + 1]);
    __syncthreads();
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
// log(1 + d) = 2 atanh(y), so h = 2 y^2 / (1 - y) - 2 (y^3/3 + y^5/5 + ...),
// free of cancellation.  lb = log b, la = log a.
__device__ double rho_log(double a, double la, double lb) {
    double d = expm1(lb - la);
    double h;
    if (fabs(d) < 0.5) {
        double y = d / (2.0 + d), y2 = y * y;
        double term = y * y2, ser = 0.0;
        for (int k = 3; k < 64; k += 2) {
            double add = term / k;
            ser += add;
            if (fabs(add) <= 1e-17 * fabs(ser)) break;
            term *= y2;
        }
        h = 2.0 * y2 / (1.0 - y) - 2.0 * ser;
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
// The low clamp keeps k in range.  k is returned so that the tile can track
// its largest term's binary exponent.
__device__ __forceinline__ float exp2_split(double t, int& k) {
    const double magic = 6755399441055744.0;   // 1.5 * 2^52
    t = fmax(t, -4096.0);
    const double mm = t + magic;
    k = __double2loint(mm);
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
// points of the passes: the value of the row / column dual variable at the
// point a pass evaluates, with the state writes of that phase (done by the
// strip's "writer" WG only; every WG of the strip computes the same value).
// ---------------------------------------------------------------------------
__device__ double row_point(const PassArgs& A, const Ctl& c, int i, bool writer) {
    const Ws& w = A.ws;
    const int par = c.t & 1;
    switch (A.phase) {
    case PH_INIT: {
        double u0 = A.u0 ? A.u0[i] : 0.0;
        if (writer) { st_agent(&w.uchk0[i], u0); st_agent(&w.util0[i], u0); }
        return u0;
    }
    case PH_BAR: {
        double uc;
        if (c.t == 0) uc = w.uchk0[i];
        else {
            // z-check^t = GreenkhornStep(z^{t-1}); du holds the u-block delta at z^{t-1}
            uc = w.uz[i] + (c.bchk == 0 ? w.du[i] : 0.0);
            if (writer) st_agent(&(par ? w.uchk1 : w.uchk0)[i], uc);
        }
        double ut = (par ? w.util1 : w.util0)[i];
        double ub = (1.0 - c.theta) * uc + c.theta * ut;
        if (writer) st_agent(&w.ubar[i], ub);
        return ub;
    }
    case PH_GRAVE: {
        double ub = w.ubar[i], ut = (par ? w.util1 : w.util0)[i], g = w.du[i];
        double eta = (A.step_rule == 0 ? c.gamma : 1.0) / (3.0 * c.M * c.theta);
        double ut1 = (A.step_rule == 0 ? ub : ut) - eta * g;
        double ug = ub + c.theta * (ut1 - ut);
        if (writer) { st_agent(&(par ? w.util0 : w.util1)[i], ut1); st_agent(&w.ugrave[i], ug); }
        return ug;
    }
    case PH_Z: {
        double uh = w.ugrave[i] + (c.bhat == 0 ? w.du[i] : 0.0);
        double z = c.pick ? uh : (par ? w.uchk1 : w.uchk0)[i];
        if (writer) st_agent(&w.uz[i], z);
        return z;
    }
    case PH_SK_ROW: return (par ? w.uchk1 : w.uchk0)[i];
    case PH_SK_COL: return (par ? w.uchk0 : w.uchk1)[i];
    default: return w.ubar[i];   // rounding passes: f
    }
}

__device__ double col_point(const PassArgs& A, const Ctl& c, int j, bool writer) {
    const Ws& w = A.ws;
    const int par = c.t & 1;
    switch (A.phase) {
    case PH_INIT: {
        double v0 = A.v0 ? A.v0[j] : 0.0;
        if (writer) { st_agent(&w.vchk0[j], v0); st_agent(&w.vtil0[j], v0); }
        return v0;
    }
    case PH_BAR: {
        double vc;
        if (c.t == 0) vc = w.vchk0[j];
        else {
            vc = w.vz[j] + (c.bchk == 1 ? w.dv[j] : 0.0);
            if (writer) st_agent(&(par ? w.vchk1 : w.vchk0)[j], vc);
        }
        double vt = (par ? w.vtil1 : w.vtil0)[j];
        double vb = (1.0 - c.theta) * vc + c.theta * vt;
        if (writer) st_agent(&w.vbar[j], vb);
        return vb;
    }
    case PH_GRAVE: {
        double vb = w.vbar[j], vt = (par ? w.vtil1 : w.vtil0)[j], g = w.dv[j];
        double eta = (A.step_rule == 0 ? c.gamma : 1.0) / (3.0 * c.M * c.theta);
        double vt1 = (A.step_rule == 0 ? vb : vt) - eta * g;
        double vg = vb + c.theta * (vt1 - vt);
        if (writer) { st_agent(&(par ? w.vtil0 : w.vtil1)[j], vt1); st_agent(&w.vgrave[j], vg); }
        return vg;
    }
    case PH_Z: {
        double vh = w.vgrave[j] + (c.bhat == 1 ? w.dv[j] : 0.0);
        double z = c.pick ? vh : (par ? w.vchk1 : w.vchk0)[j];
        if (writer) st_agent(&w.vz[j], z);
        return z;
    }
    case PH_SK_ROW:
    case PH_SK_COL: return w.vz[j];
    default: return w.vbar[j];   // rounding passes: g
    }
}

// scalar w of the point of each ASPOT pass
__device__ double w_point(const PassArgs& A, const Ctl& c) {
    const int par = c.t & 1;
    switch (A.phase) {
    case PH_INIT: return A.w0;
    case PH_BAR: return (1.0 - c.theta) * c.wchk[par] + c.theta * c.wtil[par];
    case PH_GRAVE: return c.wgrave;
    case PH_Z: return c.wz;
    default: return 0.0;
    }
}

// ---------------------------------------------------------------------------
// per-row and per-column steps of the strip finalisers.
// acc slots: 0 T-part, 1 sum e^u, 2 <u, r~>, 3 <du, r~>, 4 rho score,
//            5 E part, 6 spare, 7 non-finite count
// ---------------------------------------------------------------------------
__device__ void row_step(const PassArgs& A, const Ctl& c, int i, double R, double* acc) {
    const Ws& w = A.ws;
    switch (A.phase) {
    case PH_INIT: {
        double u = ld_agent(&w.uchk0[i]);
        acc[0] += R; acc[1] += exp(u); acc[2] += w.rt[i] * u;
        acc[7] += isfinite(R) ? 0.0 : 1.0;
        break;
    }
    case PH_BAR: {
        // gradient of phi at zbar (Section 2.1): R + e^u - r~
        double u = ld_agent(&w.ubar[i]);
        w.du[i] = R + exp(u) - w.rt[i];
        acc[0] += R;
        acc[7] += isfinite(R) ? 0.0 : 1.0;
        break;
    }
    case PH_GRAVE:
    case PH_Z: {
        double u = ld_agent(A.phase == PH_GRAVE ? &w.ugrave[i] : &w.uz[i]);
        double eu = exp(u), b = R + eu, lb = log(b);
        double d = w.lrt[i] - lb;     // Greenkhorn u-step: u + log r~ - log(B1 + e^u)
        w.du[i] = d;
        acc[0] += R; acc[1] += eu; acc[2] += w.rt[i] * u; acc[3] += w.rt[i] * d;
        acc[4] += rho_log(w.rt[i], w.lrt[i], lb);
        acc[5] += fabs(b - w.rt[i]);
        acc[7] += isfinite(R) ? 0.0 : 1.0;
        break;
    }
    default: break;
    }
}

__device__ void col_step(const PassArgs& A, const Ctl& c, int j, double Q, double* acc) {
    const Ws& w = A.ws;
    switch (A.phase) {
    case PH_INIT: {
        double v = ld_agent(&w.vchk0[j]);
        acc[1] += exp(v); acc[2] += w.ct[j] * v;
        acc[7] += isfinite(Q) ? 0.0 : 1.0;
        break;
    }
    case PH_BAR: {
        double v = ld_agent(&w.vbar[j]);
        w.dv[j] = Q + exp(v) - w.ct[j];
        acc[7] += isfinite(Q) ? 0.0 : 1.0;
        break;
    }
    case PH_GRAVE:
    case PH_Z: {
        double v = ld_agent(A.phase == PH_GRAVE ? &w.vgrave[j] : &w.vz[j]);
        double ev = exp(v), b = Q + ev, lb = log(b);
        double d = w.lct[j] - lb;
        w.dv[j] = d;
        acc[1] += ev; acc[2] += w.ct[j] * v; acc[3] += w.ct[j] * d;
        acc[4] += rho_log(w.ct[j], w.lct[j], lb);
        acc[5] += fabs(b - w.ct[j]);
        acc[7] += isfinite(Q) ? 0.0 : 1.0;
        break;
    }
    default: break;
    }
}

// ---------------------------------------------------------------------------
// the deciding workgroup: scalar logic of the iteration
// ---------------------------------------------------------------------------
// Sum the per-strip partials in a fixed order.
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

__device__ void decide(const PassArgs& A, Ctl& c, double* lds) {
    double Rs[kScal], Cs[kScal];
    const bool rows = A.phase != PH_SK_COL;
    const bool cols = A.phase != PH_SK_ROW;
    if (rows) gather_strips(A.ws.rowscal, A.ny, Rs, lds);
    if (cols) gather_strips(A.ws.colscal, A.nx, Cs, lds);
    if (threadIdx.x != 0) return;
    if (A.phase == PH_SK_ROW || A.phase == PH_SK_COL) {
        // slots 1, 2 hold per-strip (max, sum of exp): merge them in strip order
        const double* part = rows ? A.ws.rowscal : A.ws.colscal;
        const int ns = rows ? A.ny : A.nx;
        double mx = -INFINITY, se = 0.0;
        for (int k = 0; k < ns; ++k)
            lse_merge(mx, se, ld_agent(&part[(int64_t)k * kScal + 1]), ld_agent(&part[(int64_t)k * kScal + 2]));
        if (rows) { Rs[1] = mx; Rs[2] = se; }
        else { Cs[1] = mx; Cs[2] = se; }
    }
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
        double wb = (1.0 - c.theta) * c.wchk[par] + c.theta * c.wtil[par];
        double eta = (A.step_rule == 0 ? c.gamma : 1.0) / (3.0 * c.M * c.theta);
        double wt1 = (A.step_rule == 0 ? wb : c.wtil[par]) - eta * gw;
        c.wbar = wb;
        c.wtil[par ^ 1] = wt1;
        c.wgrave = wb + c.theta * (wt1 - c.wtil[par]);
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
        c.wz = pick ? wh : c.wchk[par];
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
        c.wchk[par ^ 1] = c.wz + (b == 2 ? c.log_s - log(T) : 0.0);
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
        double ad = c.ad[par];
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
        c.ad[par ^ 1] = c.lrhat_d - logaddexp(c.lse_b, c.bd - c.A / c.gamma);
        c.lse_a = Rs[1] + log(Rs[2]);
        break;
    }
    case PH_SK_COL: {
        double adn = c.ad[par ^ 1];
        c.bd = c.lchat_d - logaddexp(c.lse_a, adn - c.A / c.gamma);
        c.lse_b = Cs[1] + log(Cs[2]);
        c.t = t + 1;
        break;
    }
    default: break;
    }
}

// Sinkhorn strip finalisers need log-sum-exp partials; they are separate
// because they take two reductions (max, then sum).
__device__ void sk_row_finalise(const PassArgs& A, const Ctl& c, int i0, int rows, const double* R,
                                double* out, double* lds) {
    const Ws& w = A.ws;
    const int par = c.t & 1;
    const double* a = par ? w.uchk1 : w.uchk0;
    double* an = par ? w.uchk0 : w.uchk1;
    double err = 0.0, nonf = 0.0, mx = -INFINITY, se = 0.0;
    for (int r = threadIdx.x; r < rows; r += kThreads) {
        int i = i0 + r;
        double rs = R[r] + exp(a[i] + c.bd);          // dummy column: cost 0
        err += fabs(rs - w.rt[i]);
        nonf += (isfinite(R[r]) && rs > 0.0) ? 0.0 : 1.0;
        double anew = a[i] + w.lrt[i] - log(rs);      // u <- u + log r^ - log(X^ 1)
        an[i] = anew;
        lse_merge(mx, se, anew, 1.0);
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
                                double* out, double* lds) {
    const Ws& w = A.ws;
    const int par = c.t & 1;
    const double adn = c.ad[par ^ 1];
    double nonf = 0.0, mx = -INFINITY, se = 0.0;
    for (int q = threadIdx.x; q < cols; q += kThreads) {
        int j = j0 + q;
        double cs = Q[q] + exp(adn + w.vz[j]);        // dummy row: cost 0
        nonf += (isfinite(Q[q]) && cs > 0.0) ? 0.0 : 1.0;
        double bnew = w.vz[j] + w.lct[j] - log(cs);
        w.vz[j] = bnew;
        lse_merge(mx, se, bnew, 1.0);
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
constexpr int kMaxBC = 512;

template <int KIND, bool ROWS, bool COLS>
__global__ __launch_bounds__(kThreads) void stats_pass(PassArgs A) {
    constexpr int VW = (KIND == POT_COST_BF16) ? 8 : 4;
    constexpr bool PTS = (KIND == POT_COST_SQEUCLID_POINTS);
    __shared__ double s_a[kMaxBR];         // row offsets (log2 units, tile shift folded in)
    __shared__ double s_x[PTS ? kMaxBR * 3 : 1];   // points: source coordinates (FP64)
    __shared__ double s_red[64];
    __shared__ int s_flags[4];
    __shared__ int s_K;
    __shared__ int s_kmx[4];
    // one 16 KB buffer reused by the phases of the kernel:
    //   sweep:     per-lane row partials of a 64-row chunk, float [4][16][64]
    //   columns:   column partials of the 4 waves, double [4][BC]
    //   finalise:  strip sums, double [kMaxBR] (rows) and [kMaxBC] (columns)
    __shared__ __align__(16) double s_buf[2048];
    float (*s_rowp)[16][64] = reinterpret_cast<float (*)[16][64]>(s_buf);
    double* s_col = s_buf;                 // [4][bc]
    double* s_R = s_buf;                   // [br]
    double* s_Q = s_buf + kMaxBR;          // [bc]

    Ctl& c = *A.ws.ctl;
    if (c.done) return;                     // converged earlier: nothing to do

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ty = blockIdx.x % A.ny, tx = blockIdx.x / A.ny;
    const int i0 = ty * A.br, j0 = tx * A.bc;
    const int rows = min(A.br, A.n - i0), cols = min(A.bc, A.m - j0);

    // ---- prologue: the point of this pass on this tile's rows and columns
    const double wp = w_point(A, c);
    if (tid == 0) s_K = -100000;
    __syncthreads();
    for (int r = tid; r < rows; r += kThreads) {
        double u = row_point(A, c, i0 + r, tx == 0);
        s_a[r] = (u + wp) * kLog2e;
        if (PTS) {
            for (int k = 0; k < 3; ++k) s_x[r * 3 + k] = k < A.d ? (double)A.x[(int64_t)(i0 + r) * A.d + k] : 0.0;
        }
        atomicMax(&s_K, ilogb(A.ws.rt[i0 + r]));    // tile shift: sums kept near 2^0
    }
    // each thread's VW columns
    const int jg = j0 + lane * VW;
    double b[VW];
    double y2[VW][3];
#pragma unroll
    for (int k = 0; k < VW; ++k) {
        int j = jg + k;
        y2[k][0] = y2[k][1] = y2[k][2] = 0.0;
        if (j < A.m && lane * VW + k < A.bc) {
            double v = col_point(A, c, j, ty == 0 && wave == 0);
            b[k] = v * kLog2e;
            if (PTS) {
                // t_ij = a_i + b_j - G |x_i - y_j|^2 = (a_i - G|x_i|^2) + (b_j - G|y_j|^2) + 2G x_i.y_j
                double yy = 0.0;
                for (int q = 0; q < A.d; ++q) {
                    double yq = (double)A.y[(int64_t)j * A.d + q];
                    y2[k][q] = 2.0 * c.G * yq;
                    yy += yq * yq;
                }
                b[k] -= c.G * yy;
            }
        } else {
            b[k] = 0.0;    // masked below (e = 0)
        }
    }
    __syncthreads();
    const int K = s_K;
    const double shift = (double)K;
    for (int r = tid; r < rows; r += kThreads) {
        double a = s_a[r] - shift;
        if (PTS) {
            double xx = 0.0;
            for (int k = 0; k < A.d; ++k) xx += s_x[r * 3 + k] * s_x[r * 3 + k];
            a -= c.G * xx;
        }
        s_a[r] = a;
    }
    __syncthreads();
    const double G = c.G;
    const float Gf = (float)G;
    float bf[VW];
#pragma unroll
    for (int k = 0; k < VW; ++k) bf[k] = (float)b[k];
    const bool full = jg + VW <= A.m;   // masked columns only in the last column strip

    // ---- tile.  A sweep forms every term of the tile, accumulates the column
    // partials (FP32 over a batch of U rows, then FP64) and per-lane row
    // partials, which are reduced through LDS once per chunk of 64 rows.  It
    // also returns the largest binary exponent of its terms: if that is out of
    // [-60, 60] (all terms tiny, or some huge: far-apart points at the start,
    // extrapolated ASPOT points), the tile is swept again with its shift moved
    // by that exponent so FP32 holds the dominant terms; the FP64 partials
    // carry the shift's scale.
    double colacc[VW];
    const bool vec_ok = !PTS && ((A.ldc % VW) == 0) && ((((uintptr_t)A.C) & 15) == 0);
    // interior tile: every row and column in range, aligned rows -> branch-free loads
    const bool fast = vec_ok && rows == A.br && (A.br % 64) == 0 && j0 + A.bc <= A.m;
    constexpr int U = 4;

    // one row of VW terms: exponent, 2^t, row and column accumulation
    auto row_terms = [&](const float* cvals, int r, double a, float* col32, int& kmx, float& tmx) -> float {
        float e[VW];
        if (PTS) {
            const double x0 = s_x[r * 3], x1 = s_x[r * 3 + 1], x2 = s_x[r * 3 + 2];
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                int kk;
                double t = fma(x0, y2[k][0], fma(x1, y2[k][1], fma(x2, y2[k][2], a + b[k])));
                e[k] = exp2_split(t, kk);
                kmx = max(kmx, full ? kk : ((jg + k < A.m) ? kk : -1000000));
            }
        } else if (KIND == POT_COST_BF16) {
            // BF16 costs: FP32 exponent (the BF16 rounding of C dominates its error)
            const float af = (float)a;
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                float t = fmaf(cvals[k], -Gf, af + bf[k]);
                e[k] = __builtin_amdgcn_exp2f(t);
                tmx = fmaxf(tmx, (full || jg + k < A.m) ? t : -INFINITY);
            }
        } else {
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                int kk;
                e[k] = exp2_split(fma((double)cvals[k], -G, a + b[k]), kk);
                kmx = max(kmx, full ? kk : ((jg + k < A.m) ? kk : -1000000));
            }
        }
        if (!full) {
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

    // reduce the per-lane row partials of a 64-row chunk and write them
    auto emit_rows = [&](int c0, double scale_d) {
        __syncthreads();
        if (ROWS) {
            const int rl = tid >> 2, q = tid & 3;          // row of the chunk, quarter of the lanes
            const int wv = rl & 3, slot = rl >> 2;         // row rl = wave wv's slot-th row
            double sacc = 0.0;
#pragma unroll
            for (int l = 0; l < 16; ++l) sacc += (double)s_rowp[wv][slot][q * 16 + l];
            sacc += __shfl_xor(sacc, 1, 64);
            sacc += __shfl_xor(sacc, 2, 64);
            const int r = c0 + rl;
            if (q == 0 && r < rows) st_agent(&((double*)A.ws.rowpart)[(int64_t)tx * A.n + i0 + r], sacc * scale_d);
        }
        __syncthreads();
    };

    auto sweep = [&](double scale_d) -> int {
        int kmx = -1000000;
        float tmx = -INFINITY;   // BF16 path: largest FP32 exponent
#pragma unroll
        for (int k = 0; k < VW; ++k) colacc[k] = 0.0;
        for (int c0 = 0; c0 < rows; c0 += 64) {
            // this wave's rows of the chunk: c0 + wave + 4 * slot, slot = 0..15
            if (fast) {
                using VT = float4;   // 16 bytes: 4 FP32 or 8 BF16 costs
                const char* p0 = (const char*)A.C +
                                 ((int64_t)(i0 + c0 + wave) * A.ldc + jg) * (KIND == POT_COST_BF16 ? 2 : 4);
                const int64_t rstep = 4 * A.ldc * (KIND == POT_COST_BF16 ? 2 : 4);
                VT cur[U], nxt[U];
#pragma unroll
                for (int u = 0; u < U; ++u) cur[u] = *(const VT*)(p0 + u * rstep);
#pragma unroll
                for (int bb = 0; bb < 16 / U; ++bb) {
                    if (bb + 1 < 16 / U) {
#pragma unroll
                        for (int u = 0; u < U; ++u) nxt[u] = *(const VT*)(p0 + ((bb + 1) * U + u) * rstep);
                    }
                    float col32[VW];
#pragma unroll
                    for (int k = 0; k < VW; ++k) col32[k] = 0.0f;
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int slot = bb * U + u, r = c0 + wave + 4 * slot;
                        float cvals[VW];
                        if (KIND == POT_COST_BF16) {
                            const uint32_t w4[4] = {__float_as_uint(cur[u].x), __float_as_uint(cur[u].y),
                                                    __float_as_uint(cur[u].z), __float_as_uint(cur[u].w)};
#pragma unroll
                            for (int k = 0; k < 4; ++k) {
                                cvals[2 * k] = __uint_as_float(w4[k] << 16);
                                cvals[2 * k + 1] = __uint_as_float(w4[k] & 0xffff0000u);
                            }
                        } else {
                            cvals[0] = cur[u].x; cvals[1] = cur[u].y; cvals[2] = cur[u].z; cvals[3] = cur[u].w;
                        }
                        s_rowp[wave][slot][lane] = row_terms(cvals, r, s_a[r], col32, kmx, tmx);
                    }
#pragma unroll
                    for (int k = 0; k < VW; ++k) colacc[k] += (double)col32[k];
                    if (bb + 1 < 16 / U) {
#pragma unroll
                        for (int u = 0; u < U; ++u) cur[u] = nxt[u];
                    }
                }
            } else {
                for (int slot = 0; slot < 16; ++slot) {
                    const int r = c0 + wave + 4 * slot;
                    float rs = 0.0f;
                    if (r < rows) {
                        float cvals[VW];
                        if (!PTS) {
                            if (jg < A.m) load_costs<KIND>(A, i0 + r, jg, vec_ok, cvals);
                            else {
#pragma unroll
                                for (int k = 0; k < VW; ++k) cvals[k] = 0.0f;
                            }
                        }
                        float col32[VW];
#pragma unroll
                        for (int k = 0; k < VW; ++k) col32[k] = 0.0f;
                        rs = row_terms(cvals, r, s_a[r], col32, kmx, tmx);
#pragma unroll
                        for (int k = 0; k < VW; ++k) colacc[k] += (double)col32[k];
                    }
                    s_rowp[wave][slot][lane] = rs;
                }
            }
            emit_rows(c0, scale_d);
        }
        if (KIND == POT_COST_BF16 && tmx > -INFINITY)
            kmx = (int)floorf(fmaxf(fminf(tmx, 1.0e6f), -1.0e6f));
        return kmx;
    };
    double scale_d = ldexp(1.0, K);
    int kmx = sweep(scale_d);
    // block max of the terms' exponents
    {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) kmx = max(kmx, __shfl_xor(kmx, o, 64));
        if (lane == 0) s_kmx[wave] = kmx;
        __syncthreads();
        kmx = max(max(s_kmx[0], s_kmx[1]), max(s_kmx[2], s_kmx[3]));
        __syncthreads();
    }
    if (kmx > -1000000 && (kmx > 60 || kmx < -60)) {
        for (int r = tid; r < rows; r += kThreads) s_a[r] -= (double)kmx;
        __syncthreads();
        scale_d = ldexp(1.0, K + kmx);
        sweep(scale_d);
    }
    if (COLS) {
#pragma unroll
        for (int k = 0; k < VW; ++k) s_col[wave * (64 * VW) + lane * VW + k] = colacc[k];
        __syncthreads();
        for (int q = tid; q < cols; q += kThreads) {
            const int B = 64 * VW;
            double v = (s_col[q] + s_col[B + q]) + (s_col[2 * B + q] + s_col[3 * B + q]);
            st_agent(&((double*)A.ws.colpart)[(int64_t)ty * A.m + j0 + q], v * scale_d);
        }
    }

    // ---- arrival: the last WG of a strip finalises it
    wait_stores();
    __syncthreads();
    if (tid == 0) {
        s_flags[0] = ROWS ? (atomicAdd(&A.ws.rowcnt[ty], 1) == A.nx - 1) : 0;
        s_flags[1] = COLS ? (atomicAdd(&A.ws.colcnt[tx], 1) == A.ny - 1) : 0;
    }
    __syncthreads();
    int nfin = 0;
    if (ROWS && s_flags[0]) {
        // R_i = sum over column strips of the partials, in FP64
        for (int r = tid; r < rows; r += kThreads) {
            double R = 0.0;
            const double* p = (const double*)A.ws.rowpart + i0 + r;
#pragma unroll 8
            for (int x = 0; x < A.nx; ++x) R += ld_agent(&p[(int64_t)x * A.n]);
            s_R[r] = R;
        }
        __syncthreads();
        double* out = A.ws.rowscal + (int64_t)ty * kScal;
        if (A.phase == PH_SK_ROW) {
            sk_row_finalise(A, c, i0, rows, s_R, out, s_red);
        } else {
            double acc[kScal];
#pragma unroll
            for (int k = 0; k < kScal; ++k) acc[k] = 0.0;
            for (int r = tid; r < rows; r += kThreads) row_step(A, c, i0 + r, s_R[r], acc);
            block_sum<kScal>(acc, s_red);
            if (tid == 0)
                for (int k = 0; k < kScal; ++k) st_agent(&out[k], acc[k]);
        }
        if (tid == 0) A.ws.rowcnt[ty] = 0;
        ++nfin;
    }
    if (COLS && s_flags[1]) {
        for (int q = tid; q < cols; q += kThreads) {
            double Q = 0.0;
            const double* p = (const double*)A.ws.colpart + j0 + q;
#pragma unroll 8
            for (int y = 0; y < A.ny; ++y) Q += ld_agent(&p[(int64_t)y * A.m]);
            s_Q[q] = Q;
        }
        __syncthreads();
        double* out = A.ws.colscal + (int64_t)tx * kScal;
        if (A.phase == PH_SK_COL) {
            sk_col_finalise(A, c, j0, cols, s_Q, out, s_red);
        } else {
            double acc[kScal];
#pragma unroll
            for (int k = 0; k < kScal; ++k) acc[k] = 0.0;
            for (int q = tid; q < cols; q += kThreads) col_step(A, c, j0 + q, s_Q[q], acc);
            block_sum<kScal>(acc, s_red);
            if (tid == 0)
                for (int k = 0; k < kScal; ++k) st_agent(&out[k], acc[k]);
        }
        if (tid == 0) A.ws.colcnt[tx] = 0;
        ++nfin;
    }
    if (nfin) {
        wait_stores();
        __syncthreads();
        const int total = (ROWS ? A.ny : 0) + (COLS ? A.nx : 0);
        if (tid == 0) s_flags[2] = (atomicAdd(&A.ws.glob[0], nfin) + nfin == total);
        __syncthreads();
        if (s_flags[2]) {
            decide(A, c, s_red);
            if (tid == 0) A.ws.glob[0] = 0;
        }
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

template <int KIND, bool ROWS, bool COLS>
static hipError_t launch_stats_k(const PassArgs& A, hipStream_t st) {
    stats_pass<KIND, ROWS, COLS><<<A.nx * A.ny, kThreads, 0, st>>>(A);
    return hipGetLastError();
}

template <bool ROWS, bool COLS>
static hipError_t launch_stats_kind(const PassArgs& A, hipStream_t st) {
    switch (A.kind) {
    case POT_COST_F32: return launch_stats_k<POT_COST_F32, ROWS, COLS>(A, st);
    case POT_COST_BF16: return launch_stats_k<POT_COST_BF16, ROWS, COLS>(A, st);
    default: return launch_stats_k<POT_COST_SQEUCLID_POINTS, ROWS, COLS>(A, st);
    }
}

hipError_t launch_stats(const PassArgs& A, hipStream_t st) {
    if (A.phase == PH_SK_ROW) return launch_stats_kind<true, false>(A, st);
    if (A.phase == PH_SK_COL) return launch_stats_kind<false, true>(A, st);
    return launch_stats_kind<true, true>(A, st);
}

// Timed launch of the statistics pass: start/stop events recorded around the
// dispatch itself (not around the host call).
template <int KIND>
static hipError_t launch_stats_timed_k(const PassArgs& A, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    hipExtLaunchKernelGGL((stats_pass<KIND, true, true>), dim3(A.nx * A.ny), dim3(kThreads), 0, st, e0, e1, 0, A);
    return hipGetLastError();
}

hipError_t launch_stats_timed(const PassArgs& A, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    switch (A.kind) {
    case POT_COST_F32: return launch_stats_timed_k<POT_COST_F32>(A, st, e0, e1);
    case POT_COST_BF16: return launch_stats_timed_k<POT_COST_BF16>(A, st, e0, e1);
    default: return launch_stats_timed_k<POT_COST_SQEUCLID_POINTS>(A, st, e0, e1);
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
