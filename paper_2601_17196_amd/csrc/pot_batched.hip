// pot_batched.hip -- pot_solve_batched on gfx950: many independent POT
// instances (dense FP32 or BF16 costs, up to 1024 x 1024) in one persistent
// launch.
//
// Workgroups take slots from a device queue in which the instances are
// ordered largest first.  An instance is solved by a group of G workgroups
// ("members") that split its rows: a member sweeps its rows against every
// column, keeps the state of its rows and a private copy of the column
// state, and exchanges only column partial sums and row-side scalars through
// the workspace (agent-scope stores and loads, a counting barrier whose every
// wait is bounded).  Each member makes the scalar decisions of the iteration
// itself from the same sums in the same order, so the members stay in step
// without a broadcast.  With G = 1 (most instances) a solve runs inside one
// workgroup without any cross-workgroup traffic: no kernel launch, no grid
// synchronisation and no host round trip per iteration.
//
// The arithmetic is the single-instance path's (the shared device functions
// of pot_device.h): FP64 exponent, split exp2 in FP32, FP64 sums, the same
// per-row steps and decisions, FP64 rounding onto U(r, c, s).
#include <hip/hip_runtime.h>
#include <math.h>

#include "pot_device.h"

namespace pot {

namespace {

// 512 threads (8 waves) per workgroup and one workgroup per CU: an instance
// solved by a single workgroup has two waves on every SIMD.
constexpr int kBThreads = 512;
constexpr int kBWaves = kBThreads / 64;

struct Member {
    PassArgs A;              // phase, options and the member's state pointers (A.ws)
    const BDesc* D;
    int inst, mem, G, n, m, r0, nr;
    int32_t* cnt;            // group barrier: arrivals
    int32_t* err;            // group error flag
    double* colpart;         // [G][m]
    double* rowsc;           // [G][kScal]
    int bar;                 // barriers passed
    int spin_limit;
};

// per-workgroup shared state
struct BShared {
    Member mb;               // the member this workgroup plays (written by thread 0)
    Ctl ctl;                 // control block of the member's instance
    double a[kBMax];         // offsets of the member's rows (log2 units)
    double b[kBMax];         // column offsets (log2 units)
    double R[kBMax];         // row sums of the member's rows (FP64)
    double lR[kBMax];        // their logs (start pass only; exact even where R underflows)
    double Q[kBMax];         // column sums (FP64)
    // the state an ASPOT step reads, kept on chip: the duals at the point of
    // the pass (written by the pass's prologue) and the smoothed masses with
    // their logs (written once by the setup)
    double xr[kBMax], xc[kBMax];
    double rt[kBMax], lrt[kBMax], ct[kBMax], lct[kBMax];
    double colw[kBWaves][kBMax];   // per-wave column partials
    double red[64];
    double lvl[kBWaves];
    int K;                   // exponent shift of the member's sweep, kept across passes
    int slot, ok, used_warm;
};


template <int KIND>
__device__ __forceinline__ double bcost64(const Member& M, int i, int j) {
    if (KIND == POT_COST_BF16) return (double)bf16_to_f32(((const uint16_t*)M.A.C)[(int64_t)i * M.A.ldc + j]);
    return (double)((const float*)M.A.C)[(int64_t)i * M.A.ldc + j];
}

// Counting barrier of the members of one instance.  Every store a member
// made for the others is complete (s_waitcnt) before its arrival; the wait is
// bounded, and a member that gives up raises the group's error flag so that
// the others give up too.  Returns false on failure.
__device__ bool group_sync(Member& M, BShared& S) {
    if (M.G == 1) return true;
    wait_stores();
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        M.bar += 1;
        atomicAdd(M.cnt, 1);
        const int target = M.bar * M.G;
        int spins = 0;
        while (ld_agent(M.cnt) < target) {
            if (ld_agent(M.err) != 0 || ++spins > M.spin_limit) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        if (!ok) __hip_atomic_store(M.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        S.ok = ok;
    }
    __syncthreads();
    return S.ok != 0;
}

// maximum over the workgroup, returned to every thread
__device__ double block_max(double v, BShared& S) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_max(v);
    if (lane == 0) S.lvl[wave] = v;
    __syncthreads();
    v = S.lvl[0];
    for (int w = 1; w < kBWaves; ++w) v = fmax(v, S.lvl[w]);
    __syncthreads();
    return v;
}

// column sum of the per-wave partials (fixed pairwise order)
__device__ __forceinline__ double colw_sum(const BShared& S, int j) {
    return wave_tree<kBWaves>(&S.colw[0][j], kBMax);
}

// Largest |exponent| of the member's terms (used only when every sum of a
// sweep under- or overflowed).
template <int KIND>
__device__ double member_max_exponent(const Member& M, BShared& S, double G2) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double mx = -INFINITY;
    for (int r = wave; r < M.nr; r += kBWaves) {
        const int i = M.r0 + r;
        for (int j = lane; j < M.m; j += 64) mx = fmax(mx, fma(bcost64<KIND>(M, i, j), -G2, S.a[r] + S.b[j]));
    }
    return block_max(mx, S);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));   // 16 bytes: 4 FP32 or 8 BF16 costs

// Costs of one row chunk for this lane: VW consecutive columns from jb.  A
// full chunk (uniform condition) takes one 16-byte load; the last, partial
// chunk takes VW element loads at clamped (always valid) addresses, masked
// later, so that no load is divergent.
template <int KIND, int VW>
__device__ __forceinline__ f32x4 load_chunk(const char* rowp, int jb, int m, bool full) {
    constexpr int EB = (KIND == POT_COST_BF16) ? 2 : 4;
    if (full) return *(const f32x4*)(rowp + (int64_t)jb * EB);
    f32x4 q;
    if constexpr (KIND == POT_COST_BF16) {
        uint32_t h[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) h[e] = ((const uint16_t*)rowp)[min(jb + e, m - 1)];
#pragma unroll
        for (int e = 0; e < 4; ++e) q[e] = __uint_as_float(h[2 * e] | (h[2 * e + 1] << 16));
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) q[e] = ((const float*)rowp)[min(jb + e, m - 1)];
    }
    return q;
}

template <int KIND, int VW>
__device__ __forceinline__ void unpack_chunk(const f32x4& q, float (&cv)[VW]) {
    if constexpr (KIND == POT_COST_BF16) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t wv = __float_as_uint(q[e]);
            cv[2 * e] = __uint_as_float(wv << 16);
            cv[2 * e + 1] = __uint_as_float(wv & 0xffff0000u);
        }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) cv[e] = q[e];
    }
}

// Sixteen values summed over the 64 lanes of a wave, all together: the two
// lane swaps above halve the values each lane carries twice (16 -> 8 -> 4),
// then two exchanges inside 16-lane rows (row_mirror, row_half_mirror: a lane
// keeps one of each pair of values and adds its partner's copy of it) halve
// them to one, and two quad steps finish the sum.  Lane l ends with the total
// of value 8 b2 + 4 b3 + 2 b4 + b5 (b_k: bit k of l).  Fixed order.
__device__ __forceinline__ double wave_sum16(const double (&v)[16]) {
    const int lane = threadIdx.x & 63;
    double w[8], x[4], y[2];
#pragma unroll
    for (int i = 0; i < 8; ++i) w[i] = swap32_add(v[2 * i], v[2 * i + 1]);
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = swap16_add(w[2 * i], w[2 * i + 1]);
    const bool b3 = (lane & 8) != 0, b2 = (lane & 4) != 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double keep = b3 ? x[2 * i + 1] : x[2 * i], send = b3 ? x[2 * i] : x[2 * i + 1];
        y[i] = keep + dpp_d<kMirror>(send, 0.0);
    }
    const double keep = b2 ? y[1] : y[0], send = b2 ? y[0] : y[1];
    double z = keep + dpp_d<kHalfMirror>(send, 0.0);
    z += dpp_d<kQuadX1>(z, 0.0);
    z += dpp_d<kQuadX2>(z, 0.0);
    return z;
}

// The row-side and column-side scalars of the steps (kScal each) summed over
// the workgroup; the totals land on every lane of wave 0 (the lanes that
// exchange and decide).  The waves' totals pass through the column-partial
// area, free once the column sums are formed.
__device__ __forceinline__ void block_sum_rc(double (&Rs)[kScal], double (&Cs)[kScal], BShared& S) {
    static_assert(kScal == 8, "16 values per lane");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double v[16];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[k] = Rs[k];
        v[8 + k] = Cs[k];
    }
    const double z = wave_sum16(v);
    const int q = lane >> 2;
    const int idx = ((q & 1) << 3) | ((q & 2) << 1) | ((q & 4) >> 1) | ((q & 8) >> 3);
    // (in the column offsets' area: the pass does not read them again, while
    // the column partials may still be read by a slower wave's steps)
    double* red = &S.b[0];
    if ((lane & 3) == 0) red[wave * 16 + idx] = z;
    __syncthreads();
    if (wave == 0) {
        const double t = wave_tree<kBWaves>(red + (lane & 15), 16);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            Rs[k] = readlane_d(t, k);
            Cs[k] = readlane_d(t, 8 + k);
        }
    }
}


// One sweep of the member's rows: row sums into S.R (relative to 2^K), column
// partials into per-thread FP64 accumulators; returns the member's level (the
// largest row or column sum relative to 2^K).  Wave w takes rows w,
// w + kBWaves, ... in steps of U rows; the costs of the next step are loaded
// while the current one is computed.
template <int KIND, int VW, int KC>
__device__ double member_sweep(const Member& M, BShared& S, double G2, double Kd, const double (&b)[KC][VW],
                               double (&colacc)[KC][VW]) {
    constexpr int CW = 64 * VW;
    constexpr int U = 8 / KC;                       // rows per step
    constexpr int EB = (KIND == POT_COST_BF16) ? 2 : 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = M.m;
    const bool vec = M.D->vec != 0;
    const char* Cb = (const char*)M.A.C;
    const uint32_t rstride = (uint32_t)(M.A.ldc * EB);     // (below 2^31: checked on the host)
    const int nq = (M.nr - wave + kBWaves - 1) / kBWaves;   // rows of this wave
    double lvl = 0.0;
#pragma unroll
    for (int k = 0; k < KC; ++k)
#pragma unroll
        for (int e = 0; e < VW; ++e) colacc[k][e] = 0.0;
    if (nq > 0) {
        f32x4 cur[U][KC], nxt[U][KC];
        // The loads of step s.  With aligned rows every load is one 16-byte
        // load: a lane past the row's end reads the last group inside the
        // row's stride (its terms are masked).  The choice is made once per
        // step, not per row: the register writes of a per-row partial path
        // would hold each row's load until the previous loads returned.
        const int jlast = (int)M.A.ldc - VW;
        auto fetch = [&](int s, f32x4 (&buf)[U][KC]) __attribute__((always_inline)) {
            if (vec) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int q = min(s * U + u, nq - 1);
                    const char* rowp = Cb + (uint64_t)(uint32_t)(M.r0 + wave + kBWaves * q) * rstride;
#pragma unroll
                    for (int k = 0; k < KC; ++k)
                        buf[u][k] = *(const f32x4*)(rowp + (int64_t)min(k * CW + lane * VW, jlast) * EB);
                }
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int q = min(s * U + u, nq - 1);
                    const char* rowp = Cb + (uint64_t)(uint32_t)(M.r0 + wave + kBWaves * q) * rstride;
#pragma unroll
                    for (int k = 0; k < KC; ++k)
                        buf[u][k] = load_chunk<KIND, VW>(rowp, min(k * CW + lane * VW, m - 1), m, false);
                }
            }
        };
        // one step of U rows from its loads
        auto step = [&](int s, const f32x4 (&buf)[U][KC]) __attribute__((always_inline)) {
            // (every sum starts from its first term: the terms are >= 0, so
            // the results are those of sums started from zero)
            double rsum[U];
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                float col32[VW];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int q = s * U + u;
                    const bool rv = q < nq;
                    const double ar = S.a[wave + kBWaves * min(q, nq - 1)] - Kd;
                    float cv[VW];
                    unpack_chunk<KIND, VW>(buf[u][k], cv);
                    float rs;
#pragma unroll
                    for (int e = 0; e < VW; ++e) {
                        const int j = k * CW + lane * VW + e;
                        float ex;
                        if constexpr (KIND == POT_COST_BF16)
                            ex = __builtin_amdgcn_exp2f(fmaf(cv[e], -(float)G2, (float)ar + (float)b[k][e]));
                        else
                            ex = exp2_split(fma((double)cv[e], -G2, ar + b[k][e]));
                        // (every term is computed, then masked: the empty
                        // barrier keeps the mask from becoming a branch
                        // around the term)
                        asm volatile("" : "+v"(ex));
                        ex = (rv && j < m) ? ex : 0.0f;
                        rs = e == 0 ? ex : rs + ex;
                        col32[e] = u == 0 ? ex : col32[e] + ex;
                    }
                    rsum[u] = k == 0 ? (double)rs : rsum[u] + (double)rs;
                }
#pragma unroll
                for (int e = 0; e < VW; ++e) colacc[k][e] += (double)col32[e];
            }
            {
                double tot[(U + 3) / 4];
                rows_reduce<U>(rsum, tot);
                const int g = lane >> 4;
                const int rsel = U == 2 ? (g >> 1) : (((g & 1) << 1) | (g >> 1));
#pragma unroll
                for (int h = 0; h < (U + 3) / 4; ++h) {
                    const int q = s * U + 4 * h + rsel;
                    if (q < nq) {
                        if ((lane & 15) == 0) S.R[wave + kBWaves * q] = tot[h];
                        lvl = fmax(lvl, tot[h]);
                    }
                }
            }
        };
        // two buffers in turn (no register copies)
        fetch(0, cur);
        for (int s = 0; s * U < nq; s += 2) {
            if ((s + 1) * U < nq) fetch(s + 1, nxt);
            step(s, cur);
            if ((s + 1) * U >= nq) break;
            if ((s + 2) * U < nq) fetch(s + 2, cur);
            step(s + 1, nxt);
        }
    }
#pragma unroll
    for (int k = 0; k < KC; ++k)
#pragma unroll
        for (int e = 0; e < VW; ++e) lvl = fmax(lvl, colacc[k][e]);
    return block_max(lvl, S);
}

// One pass of the algorithm on the member's share of the instance: the point
// of the pass, the sweep, the column exchange, the per-row and per-column
// steps, the row-side scalar exchange and the decisions (thread 0, on the
// member's copy of the control block).  Returns false if a group barrier
// failed.
template <int KIND, int KC, int PH>
__device__ bool member_pass(Member& M, BShared& S) {
    constexpr bool ROWS = PH != PH_SK_COL;
    constexpr bool COLS = PH != PH_SK_ROW;
    constexpr int VW = (KIND == POT_COST_BF16) ? 8 : 4;
    constexpr int CW = 64 * VW;
    PassArgs& A = M.A;
    const Ctl& c = S.ctl;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = M.m, r0 = M.r0, nr = M.nr;
    const SideVecs RV = side_vecs(A, 0), CV = side_vecs(A, 1);

    // ---- the point of the pass, clamped as in the tile kernel
    constexpr double kClamp = 536870912.0;  // 2^29
    const double wp = w_point<PH>(A, c);
    // (rows and columns side by side: one round trip for the duals' loads)
    for (int k = tid; k < nr + m; k += kBThreads) {
        if (k < nr) {
            const int i = r0 + k;
            const Cand q = load_cand<PH>(A, RV, 0, i);
            const double x = eval_point<PH>(A, c, RV, q, 0, i, true);
            S.xr[k] = x;
            S.a[k] = fmin(fmax((x + wp) * kLog2e, -kClamp), kClamp);
        } else {
            const int j = k - nr;
            const Cand q = load_cand<PH>(A, CV, 1, j);
            const double x = eval_point<PH>(A, c, CV, q, 1, j, true);
            S.xc[j] = x;
            S.b[j] = fmin(fmax(x * kLog2e, -kClamp), kClamp);
        }
    }
    __syncthreads();

    // ---- sweep, with the level check and re-sweep of the tile kernel
    const double G2 = c.G;
    double b[KC][VW];
#pragma unroll
    for (int k = 0; k < KC; ++k)
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            const int j = k * CW + lane * VW + e;
            b[k][e] = j < m ? S.b[j] : 0.0;
        }
    double colacc[KC][VW];
    int K = S.K;
    double lvl = member_sweep<KIND, VW, KC>(M, S, G2, (double)K, b, colacc);
    const double kHi = 1.152921504606846976e18;   // 2^60
    const double kLo = 8.673617379884035472e-19;  // 2^-60
    if (!(lvl <= kHi && lvl >= kLo)) {
        int delta;
        if (lvl > 0.0 && lvl < INFINITY) delta = ilogb(lvl);
        else {
            const double mx = member_max_exponent<KIND>(M, S, G2) - (double)K;
            delta = isfinite(mx) ? (int)floor(mx) : 0;
        }
        // (a lone member of an ASPOT pass may go as far as the duals' clamp:
        // its sums are then kept relative to 2^K below)
        const int kmax = (M.G == 1 && ROWS && COLS) ? (1 << 29) : 2000;
        delta = max(-kmax - K, min(kmax - K, delta));
        if (delta != 0) {
            K += delta;
            lvl = member_sweep<KIND, VW, KC>(M, S, G2, (double)K, b, colacc);
        }
    }
    // Sums are scaled by 2^K while |K| <= 800 (normal FP64 values); a lone
    // member of an ASPOT pass beyond that keeps them relative to 2^K and
    // hands the steps and the decisions the exponent Ke (a group's members
    // exchange plain FP64 sums).
    const bool rel = M.G == 1 && ROWS && COLS && (K > 800 || K < -800);
    const int Ke = rel ? K : 0;
    const double scale_d = rel ? 1.0 : ldexp(1.0, K);
    if (COLS) {
#pragma unroll
        for (int k = 0; k < KC; ++k)
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                const int j = k * CW + lane * VW + e;
                if (j < m) S.colw[wave][j] = colacc[k][e];
            }
    }
    __syncthreads();
    if (tid == 0) S.K = K;
    // A lone member's ASPOT pass forms each row's and column's scaled sum in
    // the thread that steps it (below); otherwise they are combined here,
    // behind one more barrier.
    const bool fused = ROWS && COLS && M.G == 1;
    if (!fused) {
        if (PH == PH_INIT)
            for (int r = tid; r < nr; r += kBThreads) S.lR[r] = log(S.R[r]) + (double)K * kLn2;
        if (ROWS)
            for (int r = tid; r < nr; r += kBThreads) S.R[r] *= scale_d;
        if (COLS) {
            for (int j = tid; j < m; j += kBThreads) {
                const double q = colw_sum(S, j) * scale_d;
                if (M.G == 1) S.Q[j] = q;
                else st_agent(&M.colpart[(int64_t)M.mem * m + j], q);
            }
            if (M.G > 1) {
                if (!group_sync(M, S)) return false;
                for (int j = tid; j < m; j += kBThreads) {
                    double q = 0.0;
                    for (int g = 0; g < M.G; ++g) q += ld_agent(&M.colpart[(int64_t)g * m + j]);
                    S.Q[j] = q;
                }
            }
        }
        __syncthreads();
    }

    // ---- steps and the scalars of the decisions
    double Rs[kScal], Cs[kScal];
#pragma unroll
    for (int k = 0; k < kScal; ++k) { Rs[k] = 0.0; Cs[k] = 0.0; }
    if constexpr (PH == PH_SK_ROW) {
        double err = 0.0, nonf = 0.0, mx = -INFINITY, se = 0.0;
        for (int r = tid; r < nr; r += kBThreads) {
            const int i = r0 + r;
            const double an = sk_row_update(A.ws, c, i, S.R[r], load_step<PH>(A, true, i), err, nonf);
            lse_merge(mx, se, an, 1.0);
        }
        block_lse<kBWaves>(mx, se, S.red);
        double v[2] = {err, nonf};
        block_sum<2, kBWaves>(v, S.red);
        Rs[0] = v[0]; Rs[1] = mx; Rs[2] = se; Rs[7] = v[1];
    } else if constexpr (PH == PH_SK_COL) {
        double nonf = 0.0, mx = -INFINITY, se = 0.0;
        for (int j = tid; j < m; j += kBThreads) {
            const double bn = sk_col_update(A.ws, c, j, S.Q[j], load_step<PH>(A, false, j), nonf);
            lse_merge(mx, se, bn, 1.0);
        }
        block_lse<kBWaves>(mx, se, S.red);
        double v[1] = {nonf};
        block_sum<1, kBWaves>(v, S.red);
        Cs[1] = mx; Cs[2] = se; Cs[7] = v[0];
    } else {
        // rows and columns side by side (one element per thread at the sizes
        // of a batch); the state comes from LDS (the point's duals, the masses)
        for (int k = tid; k < nr + m; k += kBThreads) {
            if (k < nr) {
                const StepPre p = {S.xr[k], S.rt[k], S.lrt[k], 0.0};
                double R = S.R[k];
                if (fused) {
                    if (PH == PH_INIT) S.lR[k] = log(R) + (double)K * kLn2;
                    R *= scale_d;
                }
                aspot_step<PH>(A, true, r0 + k, R, Ke, R, p, Rs);
            } else {
                const int j = k - nr;
                const StepPre p = {S.xc[j], S.ct[j], S.lct[j], 0.0};
                const double Q = fused ? colw_sum(S, j) * scale_d : S.Q[j];
                aspot_step<PH>(A, false, j, Q, Ke, 0.0, p, Cs);
            }
        }
        block_sum_rc(Rs, Cs, S);
    }
    // ---- row-side scalars of the whole instance (fixed member order)
    if (ROWS && M.G > 1) {
        // every member's scalars in one load per thread, summed in member order
#pragma unroll
        for (int k = 0; k < kScal; ++k)
            if (tid == k) st_agent(&M.rowsc[(int64_t)M.mem * kScal + k], Rs[k]);
        if (!group_sync(M, S)) return false;
        if (tid < M.G * kScal) S.red[tid] = ld_agent(&M.rowsc[tid]);
        __syncthreads();
        if (tid == 0) {
            double mx = -INFINITY, se = 0.0;
#pragma unroll
            for (int k = 0; k < kScal; ++k) Rs[k] = 0.0;
            for (int g = 0; g < M.G; ++g) {
#pragma unroll
                for (int k = 0; k < kScal; ++k) Rs[k] += S.red[g * kScal + k];
                if (PH == PH_SK_ROW) lse_merge(mx, se, S.red[g * kScal + 1], S.red[g * kScal + 2]);
            }
            if (PH == PH_SK_ROW) { Rs[1] = mx; Rs[2] = se; }
        }
    }
    if (tid == 0) {
        A.phase = PH;
        if (ROWS && COLS) Rs[6] = (double)Ke;      // T = Rs[0] 2^Ke
        decide_logic(A, S.ctl, Rs, Cs);
    }
    __syncthreads();
    return true;
}

// setup of the instance (Algorithm 2, "Approximating POT"); |C|_max scanned
// when not given.  Returns the validity code (0 ok).
template <int KIND>
__device__ int member_setup(Member& M, BShared& S, const BArgs& B) {
    const BDesc& D = *M.D;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = M.n, m = M.m;
    const Ws& w = M.A.ws;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};      // |r|_1, |c|_1, bad masses, H(r), H(c)
    for (int i = tid; i < n; i += kBThreads) {
        const double x = D.r[i];
        v[2] += (isfinite(x) && x >= 0.0) ? 0.0 : 1.0;
        v[0] += x;
        v[3] += ent(x);
    }
    for (int j = tid; j < m; j += kBThreads) {
        const double x = D.c[j];
        v[2] += (isfinite(x) && x >= 0.0) ? 0.0 : 1.0;
        v[1] += x;
        v[4] += ent(x);
    }
    block_sum<5, kBWaves>(v, S.red);
    double cmax = D.cmax;
    int bad_cost = 0;
    if (!(cmax > 0.0)) {
        double mx = 0.0, nb = 0.0;
        for (int64_t e = tid; e < (int64_t)n * m; e += kBThreads) {
            const double x = bcost64<KIND>(M, (int)(e / m), (int)(e % m));
            if (!(x >= 0.0) || !isfinite(x)) nb += 1.0;
            else mx = fmax(mx, x);
        }
        cmax = block_max(mx, S);
        double q[1] = {nb};
        block_sum<1, kBWaves>(q, S.red);
        bad_cost = q[0] > 0.0 || !(cmax > 0.0);
    }
    const SetupIn in = {n, m, B.algo, B.gamma_rule, B.p, D.s, B.eps, B.gamma_user, B.tol_user, B.A_user, cmax, 1.0,
                        D.w0};
    double gamma, et, tol;
    int valid = setup_params(in, v[0], v[1], v[2], v[3], v[4], gamma, et, tol);
    if (valid == 0 && bad_cost) valid = 6;
    // every exponent log2(e) C_ij / gamma must stay below 2^29 (exponent split)
    if (valid == 0 && !(kLog2e * cmax / gamma < 536870912.0)) valid = 7;
    double u[3] = {0.0, 0.0, 0.0};      // |r~|_1, |c~|_1, non-positive entries
    for (int i = tid; i < n; i += kBThreads) {
        const double x = smooth_mass(D.r[i], et, n);
        if (i >= M.r0 && i < M.r0 + M.nr) {
            w.rt[i] = x;
            w.lrt[i] = log(x);
            S.rt[i - M.r0] = x;
            S.lrt[i - M.r0] = w.lrt[i];
            if (B.algo == POT_SINKHORN) w.uchk0[i] = 0.0;
        }
        u[2] += x > 0.0 ? 0.0 : 1.0;
        u[0] += x;
    }
    for (int j = tid; j < m; j += kBThreads) {
        const double x = smooth_mass(D.c[j], et, m);
        w.ct[j] = x;
        w.lct[j] = log(x);
        S.ct[j] = x;
        S.lct[j] = w.lct[j];
        if (B.algo == POT_SINKHORN) w.vz[j] = 0.0;
        u[2] += x > 0.0 ? 0.0 : 1.0;
        u[1] += x;
    }
    block_sum<3, kBWaves>(u, S.red);
    if (valid == 0 && u[2] > 0.0) valid = 5;
    if (tid == 0) {
        setup_fill(S.ctl, in, gamma, tol, v[0], v[1], u[0], u[1], valid);
        S.K = 0;
    }
    __syncthreads();
    return valid;
}

// FP64 rounding onto U(r, c, s) (the three rounding passes of the
// single-instance path) and the objective, at the duals in ubar / vbar.
template <int KIND>
__device__ bool member_round(Member& M, BShared& S) {
    Ctl& c = S.ctl;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = M.m, r0 = M.r0, nr = M.nr;
    const Ws& w = M.A.ws;
    const double ig = 1.0 / c.gamma;
    const double* r = M.A.r;
    const double* cm = M.A.c;
    double nonf = 0.0;
    // alpha_i = min(1, r_i / (X~ 1)_i), 0/0 read as 1
    for (int rr = wave; rr < nr; rr += kBWaves) {
        const int i = r0 + rr;
        const double fi = w.ubar[i];
        double rs = 0.0;
        for (int j = lane; j < m; j += 64) rs += exp(fi + w.vbar[j] - bcost64<KIND>(M, i, j) * ig);
        rs = wave_sum(rs);
        if (lane == 0) {
            w.alpha[i] = rs > r[i] ? r[i] / rs : 1.0;
            nonf += isfinite(rs) ? 0.0 : 1.0;
        }
    }
    // column sums of X' = diag(alpha) X~ over the member's rows
    constexpr int KQ = kBMax / 64;
    double cacc[KQ];
#pragma unroll
    for (int k = 0; k < KQ; ++k) cacc[k] = 0.0;
    __syncthreads();
    for (int rr = wave; rr < nr; rr += kBWaves) {
        const int i = r0 + rr;
        const double fi = w.ubar[i], al = w.alpha[i];
#pragma unroll
        for (int k = 0; k < KQ; ++k) {
            const int j = lane + 64 * k;
            if (j < m) cacc[k] += al * exp(fi + w.vbar[j] - bcost64<KIND>(M, i, j) * ig);
        }
    }
#pragma unroll
    for (int k = 0; k < KQ; ++k) {
        const int j = lane + 64 * k;
        if (j < m) S.colw[wave][j] = cacc[k];
    }
    __syncthreads();
    for (int j = tid; j < m; j += kBThreads) {
        const double q = colw_sum(S, j);
        if (M.G == 1) S.Q[j] = q;
        else st_agent(&M.colpart[(int64_t)M.mem * m + j], q);
    }
    if (M.G > 1) {
        if (!group_sync(M, S)) return false;
        for (int j = tid; j < m; j += kBThreads) {
            double q = 0.0;
            for (int g = 0; g < M.G; ++g) q += ld_agent(&M.colpart[(int64_t)g * m + j]);
            S.Q[j] = q;
        }
    }
    __syncthreads();
    // beta_j = min(1, c_j / (X'^T 1)_j); q'_j = c_j - (X''^T 1)_j; T'' and |q'|_1
    double v2[3] = {0.0, 0.0, nonf};
    for (int j = tid; j < m; j += kBThreads) {
        const double cs = S.Q[j];
        const double be = cs > cm[j] ? cm[j] / cs : 1.0;
        w.beta[j] = be;
        double q2 = cm[j] - be * cs;
        q2 = q2 > 0.0 ? q2 : 0.0;
        w.qq[j] = q2;
        w.dv[j] = be * cs;                 // (X''^T 1)_j, for the marginal check
        v2[0] += be * cs;
        v2[1] += q2;
        v2[2] += isfinite(cs) ? 0.0 : 1.0;
    }
    block_sum<3, kBWaves>(v2, S.red);
    // rows of X'' = diag(alpha) X~ diag(beta): p'_i = r_i - (X'' 1)_i, <C, X''>, C q'
    for (int rr = wave; rr < nr; rr += kBWaves) {
        const int i = r0 + rr;
        const double fi = w.ubar[i], al = w.alpha[i];
        double rs = 0.0, rc = 0.0, rq = 0.0;
        for (int j = lane; j < m; j += 64) {
            const double Cij = bcost64<KIND>(M, i, j);
            const double xx = al * w.beta[j] * exp(fi + w.vbar[j] - Cij * ig);
            rs += xx;
            rc += Cij * xx;
            rq += Cij * w.qq[j];
        }
        rs = wave_sum(rs);
        rc = wave_sum(rc);
        rq = wave_sum(rq);
        if (lane == 0) {
            double p = r[i] - rs;
            p = p > 0.0 ? p : 0.0;
            w.pp[i] = p;
            w.du[i] = rs;                  // (X'' 1)_i
            S.R[rr] = rc;
            S.a[rr] = p;
            S.b[rr] = p * rq;
        }
    }
    __syncthreads();
    double v3[4] = {0.0, 0.0, 0.0, 0.0};   // <C, X''>, |p'|_1, p'^T C q', (spare)
    for (int rr = tid; rr < nr; rr += kBThreads) {
        v3[0] += S.R[rr];
        v3[1] += S.a[rr];
        v3[2] += S.b[rr];
    }
    block_sum<4, kBWaves>(v3, S.red);
    if (M.G > 1) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (tid == k) st_agent(&M.rowsc[(int64_t)M.mem * kScal + k], v3[k]);
        if (!group_sync(M, S)) return false;
        if (tid < M.G * kScal) S.red[tid] = ld_agent(&M.rowsc[tid]);
        __syncthreads();
        if (tid == 0) {
            v3[0] = v3[1] = v3[2] = 0.0;
            for (int g = 0; g < M.G; ++g)
#pragma unroll
                for (int k = 0; k < 3; ++k) v3[k] += S.red[g * kScal + k];
        }
    }
    if (tid == 0) {
        if (v2[2] > 0.0) { c.nonfinite = 1; if (c.status == POT_OK) c.status = POT_ERR_NUMERIC; }
        const double T2 = v2[0];
        c.T2 = T2;
        c.nq = v2[1];
        c.cost1 = v3[0];
        c.np = v3[1];
        c.pcq = v3[2];
        if (T2 > c.s) { c.kappa = c.s / T2; c.lambda = 0.0; }
        else if (T2 < c.s) {
            c.kappa = 1.0;
            const double d = c.np * c.nq;
            c.lambda = d > 0.0 ? (c.s - T2) / d : 0.0;
        } else { c.kappa = 1.0; c.lambda = 0.0; }
        c.cost = c.kappa * c.cost1 + c.lambda * c.pcq;
        c.mass = c.kappa * T2 + c.lambda * c.np * c.nq;
    }
    __syncthreads();
    // marginal violations of Xbar = kappa X'' + lambda p' q'^T from its FP64
    // sums: (Xbar 1)_i = kappa (X'' 1)_i + lambda |q'|_1 p'_i, and the columns
    // likewise (every member holds every column; the rows are summed over
    // the group)
    {
        const double lr = c.lambda > 0.0 ? c.lambda * c.nq : 0.0;
        const double lc = c.lambda > 0.0 ? c.lambda * c.np : 0.0;
        double vv[2] = {0.0, 0.0};
        for (int rr = tid; rr < nr; rr += kBThreads) {
            const int i = r0 + rr;
            vv[0] += fmax(c.kappa * w.du[i] + lr * w.pp[i] - r[i], 0.0);
        }
        for (int j = tid; j < m; j += kBThreads) vv[1] += fmax(c.kappa * w.dv[j] + lc * w.qq[j] - cm[j], 0.0);
        block_sum<2, kBWaves>(vv, S.red);
        if (M.G > 1) {
            if (tid == 0) st_agent(&M.rowsc[(int64_t)M.mem * kScal + 4], vv[0]);
            if (!group_sync(M, S)) return false;
            if (tid == 0) {
                vv[0] = 0.0;
                for (int g = 0; g < M.G; ++g) vv[0] += ld_agent(&M.rowsc[(int64_t)g * kScal + 4]);
            }
        }
        if (tid == 0) {
            c.viol_row = vv[0];
            c.viol_col = vv[1];
            c.viol_mass = fabs(c.mass - c.s);
            c.rounded = 1;
        }
        __syncthreads();
    }
    return true;
}

// one member's share of one instance's solve; KC = column chunks of 64 * VW
template <int KIND, int KC>
__device__ void member_solve(const BArgs& B, BShared& S, int inst, int mem) {
    const BDesc* D = &B.desc[inst];
    const int tid = threadIdx.x;
    Member& M = S.mb;
    PassArgs& A = M.A;
    Ws& w = A.ws;
    const int n = D->n, m = D->m;
    if (tid == 0) {
        M.D = D;
        M.inst = inst;
        M.mem = mem;
        M.G = D->G;
        M.n = n;
        M.m = m;
        M.r0 = (int)((int64_t)n * mem / D->G);
        M.nr = (int)((int64_t)n * (mem + 1) / D->G) - M.r0;
        M.bar = 0;
        M.spin_limit = B.spin_limit;
        const BLayout L = blayout(n, m, D->G);
        char* region = B.base + D->off;
        M.cnt = (int32_t*)(region + L.sync);
        M.err = M.cnt + 1;
        M.colpart = (double*)(region + L.colpart);
        M.rowsc = (double*)(region + L.rowsc);
        double* rows = (double*)(region + L.rows);
        double* cols = (double*)(region + L.cols + ((12 * 8 * (int64_t)m + 255) & ~(int64_t)255) * mem);
        A = PassArgs{};
        A.C = D->C;
        A.ldc = D->ldc;
        A.r = D->r;
        A.c = D->c;
        A.n = n;
        A.m = m;
        A.kind = KIND;
        A.max_iter = B.max_iter;
        A.block_rule = B.block_rule;
        A.step_rule = B.step_rule;
        A.u0 = D->u0;
        A.v0 = D->v0;
        A.w0 = D->w0;
        w.rt = rows; w.lrt = rows + n; w.uchk0 = rows + 2 * n; w.uchk1 = rows + 3 * n;
        w.util0 = rows + 4 * n; w.util1 = rows + 5 * n; w.ubar = rows + 6 * n; w.ugrave = rows + 7 * n;
        w.uz = rows + 8 * n; w.du = rows + 9 * n; w.alpha = rows + 10 * n; w.pp = rows + 11 * n;
        w.ct = cols; w.lct = cols + m; w.vchk0 = cols + 2 * m; w.vchk1 = cols + 3 * m;
        w.vtil0 = cols + 4 * m; w.vtil1 = cols + 5 * m; w.vbar = cols + 6 * m; w.vgrave = cols + 7 * m;
        w.vz = cols + 8 * m; w.dv = cols + 9 * m; w.beta = cols + 10 * m; w.qq = cols + 11 * m;
        S.used_warm = 0;
    }
    __syncthreads();

    int valid = member_setup<KIND>(M, S, B);
    bool ok = true;
    // a second attempt runs only as the cold fallback of a warm start (below)
    for (int attempt = 0; attempt < 2; ++attempt) {
    const bool cold_retry = attempt > 0;
    if (valid == 0) {
        if (B.algo == POT_ASPOT) {
            const bool warm = (D->u0 || D->v0) && !cold_retry;
            // A warm start (u0, v0, w0) is first made safe by one exact u-block
            // step (Algorithm 1): u <- u0 + log r~ - log(R + e^u0).  Afterwards
            // every row sum is at most r~_i and every column sum and the total at
            // most |r~|_1, whatever the error of the prediction, so the first
            // momentum step stays in range as from the cold start.  Then one
            // exact w-block step (w <- w + log s - log T, so that T = s; phi
            // drops by T - s - s log(s / T)).  A start whose sums are not
            // representable counts as worse than the cold start.
            auto warm_init = [&]() __attribute__((always_inline)) -> double {
                __syncthreads();
                if (tid == 0) {
                    A.u0 = D->u0;
                    A.v0 = D->v0;
                    A.w0 = D->w0;
                }
                __syncthreads();
                ok = member_pass<KIND, KC, PH_INIT>(M, S);
                if (!ok || S.ctl.done) return INFINITY;
                for (int r = tid; r < M.nr; r += kBThreads) {
                    const int i = M.r0 + r;
                    const double u = D->u0 ? D->u0[i] : 0.0;
                    w.du[i] = u + w.lrt[i] - logaddexp(S.lR[r], u);      // log(R + e^u) in the log domain
                }
                __syncthreads();
                if (tid == 0) A.u0 = w.du;
                __syncthreads();
                ok = member_pass<KIND, KC, PH_INIT>(M, S);
                if (tid == 0 && !S.ctl.done) {
                    Ctl& c = S.ctl;
                    const double dw = c.log_s - log(c.T);
                    c.phichk = c.phichk - c.T + c.s - dw * c.s;
                    c.wchk[0] += dw;
                    c.wtil[0] += dw;
                    c.T = c.s;
                }
                __syncthreads();
                return S.ctl.done ? INFINITY : S.ctl.phichk;
            };
            auto cold_init = [&]() __attribute__((always_inline)) -> double {
                __syncthreads();
                if (tid == 0) {
                    A.u0 = nullptr;
                    A.v0 = nullptr;
                    A.w0 = 0.0;
                    S.ctl.done = 0;
                    S.ctl.status = POT_OK;
                    S.ctl.nonfinite = 0;
                }
                __syncthreads();
                ok = member_pass<KIND, KC, PH_INIT>(M, S);
                return S.ctl.phichk;
            };
            if (warm && B.warm_check) {
                // keep the warm start only if phi(z0) < phi(0): cold point first,
                // then the warm one, which stays unless it is not better
                const double phi_0 = cold_init();
                const double phi_w = ok ? warm_init() : INFINITY;
                if (ok && phi_w < phi_0) {
                    if (tid == 0) S.used_warm = 1;
                } else if (ok) {
                    cold_init();
                }
            } else if (warm) {
                if (tid == 0) S.used_warm = 1;
                warm_init();
            } else {
                ok = member_pass<KIND, KC, PH_INIT>(M, S);
            }
            __syncthreads();
            while (ok && !S.ctl.done) {
                ok = member_pass<KIND, KC, PH_BAR>(M, S);
                if (!ok || S.ctl.done) break;
                ok = member_pass<KIND, KC, PH_GRAVE>(M, S);
                if (!ok || S.ctl.done) break;
                ok = member_pass<KIND, KC, PH_Z>(M, S);
            }
        } else {
            while (ok && !S.ctl.done) {
                ok = member_pass<KIND, KC, PH_SK_ROW>(M, S);
                if (!ok || S.ctl.done) break;
                ok = member_pass<KIND, KC, PH_SK_COL>(M, S);
            }
        }
        // cold-start ASPOT is the fallback of a warm start whose run left the
        // representable range (every member takes the same decision)
        if (B.algo == POT_ASPOT && ok && S.used_warm && S.ctl.status == POT_ERR_NUMERIC && !cold_retry) {
            __syncthreads();
            valid = member_setup<KIND>(M, S, B);
            if (tid == 0) {
                S.used_warm = 0;
                A.u0 = nullptr;
                A.v0 = nullptr;
                A.w0 = 0.0;
            }
            __syncthreads();
            continue;
        }
        // form primal: f = u + w (ASPOT) or a (Sinkhorn); g = v or b
        if (ok) {
            const Ctl& c = S.ctl;
            for (int r = tid; r < M.nr; r += kBThreads) {
                const int i = M.r0 + r;
                const double u = B.algo == POT_ASPOT ? w.uz[i] : (c.out_par ? w.uchk1 : w.uchk0)[i];
                const double f = B.algo == POT_ASPOT ? u + c.wz : u;
                w.ubar[i] = f;
                if (D->f_out) D->f_out[i] = f;
                if (D->u_out) D->u_out[i] = u;
            }
            for (int j = tid; j < m; j += kBThreads) {
                const double g = w.vz[j];
                w.vbar[j] = g;
                if (mem == 0 && D->g_out) D->g_out[j] = g;
                if (mem == 0 && D->v_out) D->v_out[j] = g;
            }
            __syncthreads();
            if (S.ctl.status != POT_ERR_NUMERIC && B.do_round) ok = member_round<KIND>(M, S);
        }
    }
    break;
    }
    if (mem == 0 && tid == 0) {
        const Ctl& c = S.ctl;
        pot_result R;
        fill_result(c, B.algo, R);
        R.status = !ok ? POT_ERR_DEVICE : (valid ? POT_ERR_INVALID_ARG : c.status);
        R.used_warm = S.used_warm;
        R.cost_scale = 1.0;
        B.res[inst] = R;
    }
    __syncthreads();
}

template <int KIND>
__global__ __launch_bounds__(kBThreads) void batched_kernel(BArgs B) {
    __shared__ BShared S;
    // every workgroup takes slots until the queue is empty (each instance's
    // loop is bounded by max_iter and every group wait by spin_limit)
    for (;;) {
        if (threadIdx.x == 0) S.slot = atomicAdd(B.queue, 1);
        __syncthreads();
        const int sl = S.slot;
        __syncthreads();
        if (sl >= B.nslot) return;
        const BSlot slot = B.slot[sl];
        constexpr int CW = 64 * ((KIND == POT_COST_BF16) ? 8 : 4);
        const int m = B.desc[slot.inst].m;
        if (m <= CW) member_solve<KIND, 1>(B, S, slot.inst, slot.member);
        else if (m <= 2 * CW) member_solve<KIND, 2>(B, S, slot.inst, slot.member);
        else member_solve<KIND, (kBMax + CW - 1) / CW>(B, S, slot.inst, slot.member);
    }
}

// the queue and every instance's barrier counter and error flag start at 0
__global__ void batched_init(BArgs B) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < B.batch; k += gridDim.x * blockDim.x) {
        int32_t* sync = (int32_t*)(B.base + B.desc[k].off);
        sync[0] = 0;
        sync[1] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *B.queue = 0;
}

}  // namespace

// workgroups per CU the batched kernel can keep resident
int batched_blocks_per_cu(int kind) {
    int nb = 0;
    hipError_t e = kind == POT_COST_BF16
                       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batched_kernel<POT_COST_BF16>, kBThreads, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batched_kernel<POT_COST_F32>, kBThreads, 0);
    return e == hipSuccess ? nb : 0;
}

hipError_t launch_batched(const BArgs& B, int kind, int grid, hipStream_t st) {
    batched_init<<<(B.batch + 255) / 256, 256, 0, st>>>(B);
    if (kind == POT_COST_BF16) batched_kernel<POT_COST_BF16><<<grid, kBThreads, 0, st>>>(B);
    else batched_kernel<POT_COST_F32><<<grid, kBThreads, 0, st>>>(B);
    return hipGetLastError();
}

}  // namespace pot
