// pot_device.h -- device functions shared by the single-instance kernels
// (pot_kernels.hip) and the batched persistent kernel (pot_batched.hip):
// wave and block reductions, cross-workgroup coherent accesses, the split
// exponential, the point of each pass, the per-row and per-column steps and
// the scalar decisions of ASPOT and feasible Sinkhorn.
#pragma once

#include <hip/hip_runtime.h>
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

// Lane swaps of gfx950 (v_permlane32_swap, v_permlane16_swap) for reducing
// several values at once.  swap32_add(x, y): lanes 0-31 get x summed over
// lanes l and l + 32, lanes 32-63 get y summed likewise; swap16_add(x, y):
// the even 16-lane groups get x summed over a group and the next, the odd
// groups get y.  Fixed order.
__device__ __forceinline__ double swap32_add(double x, double y) {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(y), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(y), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

__device__ __forceinline__ double swap16_add(double x, double y) {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(x), __double2loint(y), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(x), __double2hiint(y), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

// Eight values summed over the 64 lanes of a wave, all together: two swaps
// (8 -> 4 -> 2 values per lane), one exchange inside 16-lane rows
// (row_mirror: a lane keeps one of the two values and adds its partner's
// copy of it), then row_half_mirror and two quad steps finish the sum.  Lane
// l ends with the total of value 4 b3 + 2 b4 + b5 (b_k: bit k of l); lane 8 j
// holds value ((j & 1) << 2) | (j & 2) | (j >> 2).  Fixed order.
__device__ __forceinline__ double wave_sum8(const double (&v)[8]) {
    const int lane = threadIdx.x & 63;
    double w[4], x[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = swap32_add(v[2 * i], v[2 * i + 1]);
#pragma unroll
    for (int i = 0; i < 2; ++i) x[i] = swap16_add(w[2 * i], w[2 * i + 1]);
    const bool b3 = (lane & 8) != 0;
    const double keep = b3 ? x[1] : x[0], send = b3 ? x[0] : x[1];
    double z = keep + dpp_d<kMirror>(send, 0.0);
    z += dpp_d<kHalfMirror>(z, 0.0);
    z += dpp_d<kQuadX1>(z, 0.0);
    z += dpp_d<kQuadX2>(z, 0.0);
    return z;
}

// Row sums of a sweep step, reduced together.  Each lane holds a partial
// sum of each of the step's U rows.  A swap of the upper and lower 32 lanes
// between two rows' registers (swap32_add) and one add leave row a in lanes
// 0-31 and row b in lanes 32-63, each lane summing two; a swap of odd and
// even 16-lane groups between two such results (swap16_add) leaves one row
// per 16-lane group, each lane summing four; four DPP steps then add the
// group.  Every lane of group g ends with the total of one row:
//   U >= 4: row 4h + ((g & 1) << 1 | g >> 1) in out[h];  U = 2: row g >> 1.
// The order of the additions is fixed (bitwise reproducible).
__device__ __forceinline__ double group16_sum(double v) {
    v += dpp_d<kQuadX1>(v, 0.0);
    v += dpp_d<kQuadX2>(v, 0.0);
    v += dpp_d<kHalfMirror>(v, 0.0);
    v += dpp_d<kMirror>(v, 0.0);
    return v;
}

template <int U>
__device__ __forceinline__ void rows_reduce(const double (&rs)[U], double (&out)[(U + 3) / 4]) {
    static_assert(U == 2 || U == 4 || U == 8, "rows per step");
    if constexpr (U == 2) {
        const double t = swap32_add(rs[0], rs[1]);
        out[0] = group16_sum(swap16_add(t, t));
    } else {
#pragma unroll
        for (int h = 0; h < U / 4; ++h)
            out[h] = group16_sum(swap16_add(swap32_add(rs[4 * h], rs[4 * h + 1]),
                                            swap32_add(rs[4 * h + 2], rs[4 * h + 3])));
    }
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

// sum of lds[w * stride] over waves w in [W0, W0 + NW), as a fixed pairwise tree
template <int NW, int W0 = 0>
__device__ __forceinline__ double wave_tree(const double* lds, int stride) {
    if constexpr (NW == 1) return lds[W0 * stride];
    else return wave_tree<NW / 2, W0>(lds, stride) + wave_tree<NW / 2, W0 + NW / 2>(lds, stride);
}

// Sum K doubles over the NW waves of the block (fixed order: deterministic).
// The result is returned to every thread.
template <int K, int NW = 4>
__device__ inline void block_sum(double (&v)[K], double* lds /* >= NW*K */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) lds[wave * K + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_tree<NW>(lds + k, K);
    __syncthreads();
}

// Merge (max, sum-of-exp) pairs: log-sum-exp in two numbers.
__device__ __forceinline__ void lse_merge(double& m1, double& s1, double m2, double s2) {
    if (m2 == -INFINITY) return;
    if (m1 == -INFINITY) { m1 = m2; s1 = s2; return; }
    if (m2 > m1) { s1 = s1 * exp(m1 - m2) + s2; m1 = m2; }
    else s1 = s1 + s2 * exp(m2 - m1);
}

// log-sum-exp pair over the NW waves of the block; the result is returned
// to every thread.  The block maximum M first (DPP wave maxima, then the
// waves in LDS), then every thread rescales its own pair once,
// s exp(m - M), and the rescaled sums are added in the fixed order of
// block_sum: one exponential per thread instead of a chain of merges.
template <int NW = 4>
__device__ inline void block_lse(double& m, double& s, double* lds /* >= 2*NW */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double M = wave_max(m);
    if (lane == 0) lds[wave] = M;
    __syncthreads();
    M = lds[0];
    for (int w = 1; w < NW; ++w) M = fmax(M, lds[w]);
    const double t = wave_sum(m == -INFINITY ? 0.0 : s * exp(m - M));
    if (lane == 0) lds[NW + wave] = t;
    __syncthreads();
    s = wave_tree<NW>(lds + NW, 1);
    m = M;
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

// rho(a, b) = b - a + a log(a / b) (Section 2.1 notation) as a * h(d) with
// d = (b - a) / a and h(d) = d - log(1 + d).  For |d| < 1/10, with
// y = d / (2 + d) (|y| < 0.048): log(1 + d) = 2 atanh(y), so
// h = 2 y^2 / (1 - y) - 2 y^3 sum_k y^{2k} / (2k + 3), free of cancellation;
// 9 terms leave a relative error below 1e-17, and b - a is exact there
// (b within a factor 2 of a).  Otherwise d - log1p(d) loses at most a factor
// of about 20 to cancellation.
__device__ inline double rho_ab(double a, double b) {
    const double d = (b - a) / a;
    double h;
    if (fabs(d) < 0.1) {
        const double y = d / (2.0 + d), y2 = y * y;
        double p = 1.0 / 19.0;             // k = 8
#pragma unroll
        for (int k = 7; k >= 0; --k) p = fma(p, y2, 1.0 / (2 * k + 3));
        h = 2.0 * y2 / (1.0 - y) - 2.0 * y * y2 * p;
    } else {
        h = d - log1p(d);
    }
    return a * h;
}

// rho(a, b) given also lb = log b, for a b that left the normal FP64 range
// (a total whose every term underflowed): b - a - a (log b - log a)
__device__ inline double rho_abl(double a, double b, double lb) {
    if (b >= 2.2250738585072014e-308 && b <= 1.7976931348623157e308) return rho_ab(a, b);
    return (b - a) - a * (lb - log(a));
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
    case PH_INIT: {
        const double x0 = c.cold ? 0.0 : q.q0;       // (the warm-start check may fall back to zero)
        if (writer) { V.chk0[i] = x0; V.til0[i] = x0; }
        return x0;
    }
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
    case PH_INIT: return c.cold ? 0.0 : A.w0;
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
//            5 E part, 6 binary exponent of slot 0 (T = slot0 * 2^slot6),
//            7 non-finite count
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

// ASPOT step of row i (row) or column i.  The row (column) sum of B at the
// point of the pass is R = Rm 2^Re (its value may leave the FP64 range; its
// log stays exact), Tc the row's share of slot 0 (R scaled by the caller's
// block exponent); x0 the dual there, x1 the smoothed mass, x2 its log.
template <int PH>
__device__ __forceinline__ void aspot_step(const PassArgs& A, bool row, int i, double Rm, int Re, double Tc,
                                           const StepPre& p, double* acc) {
    const Ws& w = A.ws;
    const double x = p.x0, t = p.x1;
    const double R = ldexp(Rm, Re);
    acc[7] += isfinite(R) ? 0.0 : 1.0;
    if (row) acc[0] += Tc;
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
        const double ex = exp(x), b = R + ex;
        double lb = log(b), rh = rho_ab(t, b);
        // R + e^u below the normal range (the row sum underflowed, and e^u
        // with it): log(R + e^u) in the log domain.  (A wave-uniform test, so
        // that the rare path is not evaluated on every row.)
        if (__any(!(b >= 2.2250738585072014e-308))) {
            if (!(b >= 2.2250738585072014e-308)) {
                lb = logaddexp(log(Rm) + Re * kLn2, x);
                rh = rho_abl(t, b, lb);
            }
        }
        const double d = p.x2 - lb;                 // Greenkhorn step: u + log r~ - log(B 1 + e^u)
        (row ? w.du : w.dv)[i] = d;
        acc[1] += ex; acc[2] += t * x; acc[3] += t * d;
        acc[4] += rh;
        acc[5] += fabs(b - t);
        break;
    }
    default: break;
    }
}

// ---------------------------------------------------------------------------
// the scalar logic of an iteration (block choice, argmin, stopping, momentum)
// ---------------------------------------------------------------------------
__device__ inline int argmax3(double a, double b, double d) {
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
// (lT = log T: the w-step stays exact where T itself left the FP64 range)
__device__ inline double phi_after(const Ctl& c, int block, const double* R, const double* Cc, double w,
                                   double lT) {
    switch (block) {
    case 0: return c.sum_rt + Cc[1] - (R[2] + R[3]) - Cc[2] - w * c.s;
    case 1: return c.sum_ct + R[1] - R[2] - (Cc[2] + Cc[3]) - w * c.s;
    default: {
        double w1 = w + c.log_s - lT;
        return c.s + R[1] + Cc[1] - R[2] - Cc[2] - w1 * c.s;
    }
    }
}

__device__ __forceinline__ void decide_logic(const PassArgs& A, Ctl& c, const double* Rs, const double* Cs) {
    const bool rows = A.phase != PH_SK_COL;
    const bool cols = A.phase != PH_SK_ROW;
    const int t = c.t, par = t & 1;
    // a non-finite sum, or (ASPOT) a total that underflowed even the FP64
    // range after the tiles' shifts: the statistics cannot be represented
    // (ASPOT's total arrives as Rs[0] * 2^Rs[6]: its value T may leave the
    // FP64 range while log T stays exact)
    const bool aspot_phase = A.phase == PH_INIT || A.phase == PH_BAR || A.phase == PH_GRAVE || A.phase == PH_Z;
    const bool bad = (rows && Rs[7] > 0.0) || (cols && Cs[7] > 0.0) ||
                     (aspot_phase && !(Rs[0] > 0.0 && isfinite(Rs[0])));
    const double Tv = aspot_phase ? ldexp(Rs[0], (int)Rs[6]) : 0.0;
    const bool T_normal = Tv >= 2.2250738585072014e-308 && Tv <= 1.7976931348623157e308;
    auto logT = [&]() -> double { return T_normal ? log(Tv) : log(Rs[0]) + Rs[6] * kLn2; };
    // rho(s, T): the w block's score
    auto rho_w = [&]() -> double { return T_normal ? rho_ab(c.s, Tv) : (Tv - c.s) - c.s * (logT() - c.log_s); };
    if (bad) {
        c.nonfinite = 1;
        c.status = POT_ERR_NUMERIC;
        c.done = 1;
        c.iters = t;
        return;
    }
    switch (A.phase) {
    case PH_INIT: {
        const double w0 = c.cold ? 0.0 : A.w0;
        c.T = Tv;
        c.phichk = Tv + Rs[1] + Cs[1] - Rs[2] - Cs[2] - w0 * c.s;
        c.wchk[0] = w0;
        c.wtil[0] = w0;
        c.theta = 1.0;
        c.t = 0;
        break;
    }
    case PH_BAR: {
        double gw = Tv - c.s;                            // d phi / d w at zbar
        double wb = (1.0 - c.theta) * pick2(c.wchk, par) + c.theta * pick2(c.wtil, par);
        double eta = (A.step_rule == 0 ? c.gamma : 1.0) / (3.0 * c.M * c.theta);
        double wt1 = (A.step_rule == 0 ? wb : pick2(c.wtil, par)) - eta * gw;
        c.wbar = wb;
        put2(c.wtil, par ^ 1, wt1);
        c.wgrave = wb + c.theta * (wt1 - pick2(c.wtil, par));
        break;
    }
    case PH_GRAVE: {
        int b = A.block_rule == 0 ? argmax3(Rs[4], Cs[4], rho_w()) : (c.cyc++ % 3);
        if (A.force && t < A.force_len) b = A.force[3 * t + 0];
        const double lT = b == 2 ? logT() : 0.0;
        double ph = phi_after(c, b, Rs, Cs, c.wgrave, lT);
        double wh = c.wgrave + (b == 2 ? c.log_s - lT : 0.0);
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
        double T = Tv;
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
        int b = A.block_rule == 0 ? argmax3(Rs[4], Cs[4], rho_w()) : (c.cyc++ % 3);
        if (A.force && t < A.force_len) b = A.force[3 * t + 2];
        c.bchk = b;
        const double lT = b == 2 ? logT() : 0.0;
        c.phichk = phi_after(c, b, Rs, Cs, c.wz, lT);
        put2(c.wchk, par ^ 1, c.wz + (b == 2 ? c.log_s - lT : 0.0));
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

// ---------------------------------------------------------------------------
// setup of Algorithm 2 ("Approximating POT") from the mass sums
// ---------------------------------------------------------------------------
struct SetupIn {
    int n, m, algo, gamma_rule;
    double p, s, eps, gamma_user, tol_user, A_user, cmax, cost_scale, w0;
};

// entropy term of one mass: -x ln x, with 0 ln 0 = 0
__device__ __forceinline__ double ent(double x) { return x > 0.0 ? -x * log(x) : 0.0; }

// gamma, the smoothing weight eps~ (with its two caps) and the stopping
// threshold; returns the validity code (0 ok) from the sums of r and c, the
// count of bad (negative or non-finite) masses and the entropies
// H(r) = -sum r_i ln r_i, H(c).  The default rule is Algorithm 2's setup;
// the tuned rule (Algorithm 3 with Theorem 2) takes
// gamma = (2 eps / (49 H_min))^(1/p) and the threshold eps' = H_min gamma^p,
// H_min = min(H(r), H(c)); a gamma or tol given by the user wins either way.
__device__ inline int setup_params(const SetupIn& S, double sr, double sc, double bad, double hr, double hc,
                                   double& gamma, double& et, double& tol) {
    const int N = S.n > S.m ? S.n : S.m;
    const double hm = fmin(hr, hc);
    const bool tuned = S.gamma_rule == 1;
    if (S.gamma_user > 0.0) gamma = S.gamma_user;
    else if (tuned) gamma = pow(2.0 * S.eps / (49.0 * hm), 1.0 / S.p);
    else gamma = S.eps / (4.0 * log((double)N));
    et = S.eps / (8.0 * S.cmax);
    if (sr > 1.0) et = fmin(et, 8.0 * (sr - S.s) / (sr - 1.0));
    if (sc > 1.0) et = fmin(et, 8.0 * (sc - S.s) / (sc - 1.0));
    tol = S.tol_user > 0.0 ? S.tol_user : (tuned ? hm * pow(gamma, S.p) : et);
    if (bad > 0.0) return 1;
    if (!(S.s > 0.0) || S.s > sr || S.s > sc) return 2;
    if (tuned && !(hm > 0.0 && isfinite(hm))) return 8;
    if (!(gamma > 0.0) || !isfinite(gamma)) return 3;
    if (!(tol > 0.0)) return 4;
    return 0;
}

// r~_i = (1 - eps~/8) r_i + eps~/(8 n) (and c~ with 1/m)
__device__ __forceinline__ double smooth_mass(double x, double et, int len) {
    return (1.0 - et / 8.0) * x + et / (8.0 * len);
}

// the control block at the start of a solve
__device__ inline void setup_fill(Ctl& c, const SetupIn& S, double gamma, double tol, double sr, double sc,
                                  double srt, double sct, int valid) {
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
    c.wide = 0;
    c.iters = 0;
    c.nonfinite = 0;
    c.out_par = 0;
    c.cyc = 0;
    c.valid = valid;
    c.viol_row = c.viol_col = c.viol_mass = 0.0;
    c.phi0 = 0.0;
    c.cold = 0;
    c.used_warm = 0;
    c.rounded = 0;
    c.pad0 = 0;
}

// ---------------------------------------------------------------------------
// feasible Sinkhorn on the extended instance, one row or column
// ---------------------------------------------------------------------------
// row i with row sum R over the real columns: a_i <- a_i + log r^_i -
// log((X^ 1)_i), the dummy column contributing e^{a_i + b_{m+1}} (cost 0);
// returns the new a_i and adds the row's marginal error
__device__ __forceinline__ double sk_row_update(const Ws& w, const Ctl& c, int i, double R, const StepPre& p,
                                                double& err, double& nonf) {
    const int par = c.t & 1;
    double* an = par ? w.uchk0 : w.uchk1;
    const double a = sel(par, p.x1, p.x0);
    const double rs = R + exp(a + c.bd);
    err += fabs(rs - p.x2);
    nonf += (isfinite(R) && rs > 0.0) ? 0.0 : 1.0;
    const double anew = a + p.x3 - log(rs);
    an[i] = anew;
    return anew;
}

// column j with column sum Q over the real rows (at a^{k+1}); the dummy row
// contributes e^{a_{n+1} + b_j}; returns the new b_j
__device__ __forceinline__ double sk_col_update(const Ws& w, const Ctl& c, int j, double Q, const StepPre& p,
                                                double& nonf) {
    const int par = c.t & 1;
    const double adn = pick2(c.ad, par ^ 1);
    const double cs = Q + exp(adn + p.x0);
    nonf += (isfinite(Q) && cs > 0.0) ? 0.0 : 1.0;
    const double bnew = p.x0 + p.x1 - log(cs);
    w.vz[j] = bnew;
    return bnew;
}

}  // namespace pot
