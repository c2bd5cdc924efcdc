// pot_kernels.hip -- device code of libpot for gfx950 (MI355X).
//
// One pass over the cost is two launches.  In `stats_pass` every workgroup
// (WG) owns a tile of BR rows x BC columns, forms the exponent
//     t_ij = log2(e) (u_i + v_j + w - C_ij / gamma)   (in FP64)
// takes 2^t in FP32 and accumulates FP64 row and column partial sums of the
// tile (B(z)'s row sums R, column sums Q and total T, Section 2.1), formed
// relative to the tile's binary shift K (kept per tile) and stored scaled by
// 2^K while that stays in the normal FP64 range; a tile beyond it stores them
// relative to 2^K and marks the pass wide.  In `fin_pass` each WG sums the
// partials of 64 rows or columns (in a wide pass exactly, as mantissa and
// exponent, so that sums beyond the FP64 range keep their logarithm) and
// applies the per-row (per-column) step of the algorithm; the last WG makes
// the scalar decisions of the iteration (block choice, argmin, stopping) for
// the next pass.  No host round trip per iteration.
//
// The FP64 rounding passes (`round_pass`) use the same tile/strip scheme with
// an FP64 exponential and FP64 accumulation.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <math.h>

#include <type_traits>

#include "pot_device.h"

namespace pot {

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

__device__ void decide(const PassArgs& A, Ctl& cs, double* lds /* >= 17 */, bool wide) {
    double Rs[kScal], Cs[kScal];
    const bool rows = A.phase != PH_SK_COL;
    const bool cols = A.phase != PH_SK_ROW;
    const bool sk = A.phase == PH_SK_ROW || A.phase == PH_SK_COL;
    {
        // Every block's sums, added in a fixed order.  The 16 groups of 16
        // lanes (one DPP row each) take one slot each: group k, lane g sums
        // slot k % 8 of side k / 8 (row blocks, column blocks) over blocks g,
        // g + 16, ..., loading 8 blocks per batch, and the row is then reduced
        // in 4 DPP steps.  A Sinkhorn pass has one side (groups 0..7).  One
        // group merges pairs (x, y) whose value is y scaled by x: in a
        // Sinkhorn pass group 1, the blocks' (max, sum of exp) of slots 1 and
        // 2 (y e^x); in a wide ASPOT pass group 0, the total's share and its
        // binary exponent, slots 0 and 6 (y 2^x, rescaled exactly).  Running
        // maximum of x per lane, then the row maximum, then one rescaling per
        // lane before the row sum.
        const int tid = threadIdx.x, k = tid >> 4, g = tid & 15;
        const int side = sk ? (rows ? 0 : 1) : (k >> 3);
        const int slot = k & 7;
        const bool pair = sk ? slot == 1 : (wide && side == 0 && slot == 0);
        const int xs = pair ? (sk ? 1 : 6) : slot, ys = sk ? 2 : 0;
        const int nside = (sk && k >= 8) ? 0 : (side == 0 ? (rows ? A.nrb : 0) : (cols ? A.ncb : 0));
        const double* base = side == 0 ? A.ws.rowscal : A.ws.colscal;
        // y scaled by x - top (x <= top): e^(x - top) or 2^(x - top)
        auto scaled = [&](double y, double x, double top) -> double {
            if (sk) return x == -INFINITY ? 0.0 : y * exp(x - top);
            return ldexp(y, (int)fmax(x - top, -4096.0));
        };
        double v = 0.0, m = -INFINITY;
        for (int b0 = g; b0 < nside; b0 += 16 * 8) {
            double x[8], y[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int b = b0 + 16 * u;
                x[u] = b < nside ? ld_agent(&base[(int64_t)b * kScal + xs]) : (pair ? -INFINITY : 0.0);
                y[u] = (pair && b < nside) ? ld_agent(&base[(int64_t)b * kScal + ys]) : 0.0;
            }
            if (pair) {
                double bm = m;
#pragma unroll
                for (int u = 0; u < 8; ++u) bm = fmax(bm, x[u]);
                if (bm != -INFINITY) {
                    double acc = scaled(v, m, bm);
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc += scaled(y[u], x[u], bm);
                    m = bm;
                    v = acc;
                }
            } else {
#pragma unroll
                for (int u = 0; u < 8; ++u) v += x[u];
            }
        }
        double M = m;
        if (sk || wide) {
            M = fmax(M, dpp_d<kQuadX1>(M, M));
            M = fmax(M, dpp_d<kQuadX2>(M, M));
            M = fmax(M, dpp_d<kHalfMirror>(M, M));
            M = fmax(M, dpp_d<kMirror>(M, M));
            if (pair) v = M == -INFINITY ? 0.0 : scaled(v, m, M);
        }
        v += dpp_d<kQuadX1>(v, 0.0);
        v += dpp_d<kQuadX2>(v, 0.0);
        v += dpp_d<kHalfMirror>(v, 0.0);
        v += dpp_d<kMirror>(v, 0.0);
        if (g == 0) lds[k] = v;
        if (pair && g == 0) lds[16] = M;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kScal; ++j) {
            Rs[j] = sk ? (rows ? lds[j] : 0.0) : lds[j];
            Cs[j] = sk ? (cols ? lds[j] : 0.0) : lds[kScal + j];
        }
        if (sk) {
            if (rows) { Rs[1] = lds[16]; Rs[2] = lds[1]; }
            else { Cs[1] = lds[16]; Cs[2] = lds[1]; }
        } else {
            Rs[6] = wide ? lds[16] : 0.0;    // T = Rs[0] 2^Rs[6]
        }
    }
    if (threadIdx.x == 0) {
        decide_logic(A, cs, Rs, Cs);
        cs.wide = 0;                 // the next tile pass marks itself
        // the host polls this flag between chunks of iterations (system
        // scope: host memory)
        if (cs.done && A.host_done) __hip_atomic_store(A.host_done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __syncthreads();
    constexpr int kCtlWords = sizeof(Ctl) / 8;
    if (threadIdx.x < kCtlWords)
        reinterpret_cast<uint64_t*>(A.ws.ctl)[threadIdx.x] = reinterpret_cast<const uint64_t*>(&cs)[threadIdx.x];
}

// Sinkhorn steps of the finalising pass: one row (column) per thread of the
// first wave; the block's outputs are {error, max, sum of exp, 0.., non-finite}.
__device__ void sk_row_finalise(const PassArgs& A, const Ctl& c, int i0, int rows, const double* R,
                                const StepPre& p, double* out, double* lds) {
    double err = 0.0, nonf = 0.0, mx = -INFINITY, se = 0.0;
    const int r = threadIdx.x;
    if (r < rows) {
        mx = sk_row_update(A.ws, c, i0 + r, R[r], p, err, nonf);
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
    double nonf = 0.0, mx = -INFINITY, se = 0.0;
    const int q = threadIdx.x;
    if (q < cols) {
        mx = sk_col_update(A.ws, c, j0 + q, Q[q], p, nonf);
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

// Tile of this workgroup.  Tiles are numbered along rows (column index
// fastest).  The launch deals workgroups to the 8 XCDs round robin, so the
// first 8 floor(T / 8) workgroups are renumbered to give each XCD a
// contiguous run of tiles: the XCDs stream disjoint bands of whole rows.
__device__ __forceinline__ int tile_index() {
    const unsigned b = blockIdx.x, q = gridDim.x / 8u;
    return (int)(b < 8u * q ? (b % 8u) * q + b / 8u : b);
}

// ---------------------------------------------------------------------------
// the statistics pass
// ---------------------------------------------------------------------------
constexpr int kMaxBR = 256;
typedef float f32x4 __attribute__((ext_vector_type(4)));   // 16-byte vector of the tile loads
constexpr int kMaxBC = 512;
constexpr int kShiftMax = 1 << 29;   // |tile shift| bound (log2 units), as the duals' clamp
// Within +-kWideShift every nonzero scaled partial (>= 2^-149 2^K, <= 2^62
// 2^K) and every sum of them stays in the normal FP64 range.
constexpr int kWideShift = 800;

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
    // per-lane row partials of a 64-row chunk, float [4][16][64]
    __shared__ __align__(16) double s_buf[2048];
    float (*s_rowp)[16][64] = reinterpret_cast<float (*)[16][64]>(s_buf);
    // column partials of the 4 waves, double [4][BC] (an area of their own,
    // so that the kernel's tail needs one barrier)
    __shared__ double s_col[4 * kMaxBC];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tile = tile_index();
    const int tx = tile % A.nx, ty = tile / A.nx;
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
    // Within the normal window of the shift the partials are written scaled
    // by 2^K; beyond it they are written relative to 2^K, the pass is marked
    // wide, and the finalising pass reads the shift beside them.
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
    // (the last chunk skips the trailing barrier: what follows writes other
    // LDS areas, and a re-sweep synchronises before its first chunk)
    auto emit_rows = [&](int c0, double scale_d, double& lvl, bool last) __attribute__((always_inline)) {
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
        if (!last) __syncthreads();
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
            emit_rows(c0, scale_d, lvl, c0 + 64 >= rows);
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

    // the waves' column partials and levels into LDS, one barrier, the
    // tile's level
    auto stage = [&](double v) -> double {
        if (COLS) {
#pragma unroll
            for (int k = 0; k < VW; ++k) s_col[wave * (64 * VW) + lane * VW + k] = colacc[k];
        }
        v = wave_max(v);
        if (lane == 0) s_lvl[wave] = v;
        __syncthreads();
        return fmax(fmax(s_lvl[0], s_lvl[1]), fmax(s_lvl[2], s_lvl[3]));
    };

    // partials are stored times 2^K while |K| <= kWideShift (normal FP64
    // values), else as computed (relative to 2^K)
    auto out_scale = [](int k) { return (k > kWideShift || k < -kWideShift) ? 1.0 : ldexp(1.0, k); };
    double scale_d = out_scale(K);
    double lvl = stage(sweep(true, scale_d));
    const double kHi = 1.152921504606846976e18;   // 2^60
    const double kLo = 8.673617379884035472e-19;  // 2^-60
    if (!(lvl <= kHi && lvl >= kLo)) {
        __syncthreads();                   // every wave has read the levels
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
        delta = max(-kShiftMax - K, min(kShiftMax - K, delta));
        if (delta != 0) {
            for (int r = tid; r < rows; r += kThreads) s_a[r] -= (double)delta;
            K += delta;
            __syncthreads();
            scale_d = out_scale(K);
            stage(sweep(false, scale_d));  // the new column partials
            if (tid == 0) A.ws.tshift[tile] = K;
        }
    }
    // a shift beyond +-kWideShift can take the scaled partials or their sums
    // out of the normal FP64 range: the finalising pass then combines them
    // as mantissa and exponent
    if (tid == 0 && (K > kWideShift || K < -kWideShift)) A.ws.ctl->wide = 1;
    if (COLS) {
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
constexpr int kNoExp = -(1 << 30);   // exponent of a sum with no positive finite term

// acc 2^e += v 2^K, exactly (a change of e only rescales acc by a power of
// two): e follows the largest term, so terms far below it vanish and nothing
// overflows.  Zero adds nothing; a non-finite v propagates.  Branch-free, so
// that a batch of partial loads stays in flight ahead of the arithmetic.
__device__ __forceinline__ void add_shifted(double& acc, int& e, double v, int K) {
    const bool pos = v > 0.0 && v <= 1.7976931348623157e308;
    const int ev = pos ? K + ilogb(pos ? v : 1.0) : kNoExp;
    const int en = max(e, ev);
    acc = ldexp(acc, e - en) + (pos ? ldexp(v, K - en) : v);
    e = en;
}

// Plain sum of this thread's strips q, q + 4, ... < cnt of one row or column
// (partial of strip x at p[x ps]), in strip order.  Loads go out 4 strips at
// a time (indices clamped into range) before any arithmetic; the first batch
// is straight-line code, since a loop header waits for every load in flight.
__device__ __forceinline__ double sum_strips(const double* p, int64_t ps, int q, int cnt) {
    double acc = 0.0;
    auto batch = [&](int x0) __attribute__((always_inline)) {
        double pv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) pv[u] = p[(int64_t)min(x0 + 4 * u, cnt - 1) * ps];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += x0 + 4 * u < cnt ? pv[u] : 0.0;   // (sums are >= 0: + 0 is exact)
    };
    batch(q);
    for (int x0 = q + 4 * 4; x0 < cnt; x0 += 4 * 4) batch(x0);
    return acc;
}

// The same sum in a wide pass, exactly, as acc 2^ex: a partial whose tile
// shift K lies beyond +-kWideShift is relative to 2^K, the others are stored
// scaled.  A sum with no positive or non-finite term keeps ex = kNoExp.
// (Inline: out of line, its reference arguments would give every finalising
// launch a scratch segment.)
__device__ __forceinline__ void sum_strips_exact(const double* p, int64_t ps, const int32_t* ks, int64_t kst, int q,
                                                 int cnt, double& acc, int& ex) {
    acc = 0.0;
    ex = kNoExp;
    for (int x = q; x < cnt; x += 4) {
        const int K = ks[(int64_t)x * kst];
        add_shifted(acc, ex, p[(int64_t)x * ps], (K > kWideShift || K < -kWideShift) ? K : 0);
    }
}

template <int PHASE>
__global__ __launch_bounds__(kThreads) void fin_pass(PassArgs A) {
    __shared__ double s_part[4][kFinBlock];
    __shared__ int s_pe[4][kFinBlock];
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
    // loads first, in one batch: the control block, the state of the step,
    // then the tile partials (4 threads per row or column, each a quarter of
    // the strips); a wide pass reloads the partials with their tiles' shifts
    const uint64_t cw = tid < kCtlWords ? reinterpret_cast<const uint64_t*>(A.ws.ctl)[tid] : 0;
    // (indices clamped into range: no divergent loads)
    const StepPre pre = load_step<PHASE>(A, is_row, base + min(tid, len - 1));
    const int l = tid & (kFinBlock - 1), q = tid / kFinBlock;
    const int lc = min(l, len - 1), idx = base + lc;
    double acc = is_row ? sum_strips((const double*)A.ws.rowpart + idx, A.n, q, A.nx)
                        : sum_strips((const double*)A.ws.colpart + idx, A.m, q, A.ny);
    if (tid < kCtlWords) reinterpret_cast<uint64_t*>(&s_ctl)[tid] = cw;
    s_part[q][l] = l < len ? acc : 0.0;
    __syncthreads();
    const Ctl& c = s_ctl;
    if (c.done) return;              // (uniform: every thread reads the same word)
    // a wide pass: the exact sums as acc 2^ex (partial x of row idx: tile
    // (idx / br, x); partial y of column idx: tile (y, idx / bc))
    const bool wide = c.wide != 0;
    if (wide) {
        int ex;
        if (is_row)
            sum_strips_exact((const double*)A.ws.rowpart + idx, A.n, A.ws.tshift + (int64_t)(idx / A.br) * A.nx, 1,
                             q, A.nx, acc, ex);
        else
            sum_strips_exact((const double*)A.ws.colpart + idx, A.m, A.ws.tshift + idx / A.bc, A.nx, q, A.ny, acc,
                             ex);
        s_part[q][l] = l < len ? acc : 0.0;
        s_pe[q][l] = l < len ? ex : kNoExp;
        __syncthreads();
    }
    // the quarters combined in a fixed order, on the largest exponent (the
    // rescalings are exact: in the FP64 range these are the plain sums).
    // An ASPOT pass keeps them in wave 0's registers (the lanes that step
    // them); a Sinkhorn pass shares them through LDS.
    constexpr bool skp = PHASE == PH_SK_ROW || PHASE == PH_SK_COL;
    double Rv = 0.0;
    int Re = 0;
    if (tid < kFinBlock) {
        int e = 0;
        double v;
        if (!wide) {
            v = (s_part[0][tid] + s_part[1][tid]) + (s_part[2][tid] + s_part[3][tid]);
        } else {
            e = max(max(s_pe[0][tid], s_pe[1][tid]), max(s_pe[2][tid], s_pe[3][tid]));
            v = (ldexp(s_part[0][tid], s_pe[0][tid] - e) + ldexp(s_part[1][tid], s_pe[1][tid] - e)) +
                (ldexp(s_part[2][tid], s_pe[2][tid] - e) + ldexp(s_part[3][tid], s_pe[3][tid] - e));
            if (e == kNoExp) e = 0;
        }
        // (the Sinkhorn steps take the value itself)
        if (skp) s_v[tid] = ldexp(v, e);
        Rv = v;
        Re = e;
    }
    if (skp) __syncthreads();
    double* out = (is_row ? A.ws.rowscal + (int64_t)blk * kScal : A.ws.colscal + (int64_t)cb * kScal);
    if constexpr (PHASE == PH_SK_ROW) {
        sk_row_finalise(A, c, base, len, s_v, pre, out, s_red);
    } else if constexpr (PHASE == PH_SK_COL) {
        sk_col_finalise(A, c, base, len, s_v, pre, out, s_red);
    } else {
        double sums[kScal];
#pragma unroll
        for (int k = 0; k < kScal; ++k) sums[k] = 0.0;
        // slot 0 (the block's share of T) is carried as sums[0] 2^eref, eref
        // the largest exponent of the block's row sums (slot 6)
        double eref = 0.0;
        if (tid < kFinBlock) {       // wave 0: the block's rows or columns
            const double Rm = Rv;
            if (wide) {
                const bool pos = tid < len && Rm > 0.0 && Rm <= 1.7976931348623157e308;
                eref = wave_max(pos ? (double)(Re + ilogb(pos ? Rm : 1.0)) : -INFINITY);
                if (!(eref > -INFINITY)) eref = 0.0;
            }
            if (tid < len)
                aspot_step<PHASE>(A, is_row, base + tid, Rm, Re, ldexp(Rm, Re - (int)eref), pre, sums);
            // the block's sums, all slots over the wave at once (no barrier:
            // the other waves hold nothing); lane 8 j stores one slot
            const double z = wave_sum8(sums);
            if ((tid & 7) == 0) {
                const int j = tid >> 3, k = ((j & 1) << 2) | (j & 2) | (j >> 2);
                st_agent(&out[k], k == 6 ? (is_row ? eref : 0.0) : z);
            }
        }
    }
    // arrival: the last block decides (an ASPOT pass stored from wave 0
    // only: that wave's own wait orders its stores before the arrival)
    const int total = (rows_pass ? A.nrb : 0) + (PHASE != PH_SK_ROW ? A.ncb : 0);
    if (skp) {
        wait_stores();
        __syncthreads();
    }
    if (tid < kFinBlock) {
        wait_stores();
        if (tid == 0) s_last = (atomicAdd(&A.ws.glob[0], 1) == total - 1);
    }
    __syncthreads();
    if (s_last) {
        decide(A, s_ctl, s_red, wide);
        if (tid == 0) st_agent(&A.ws.glob[0], 0);
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
    // no rounding without a finished loop and representable statistics (a
    // uniform test: every workgroup reads the same words)
    if (c.valid != 0 || !c.done || c.status == POT_ERR_NUMERIC) return;
    if ((A.phase == PH_R4 || A.phase == PH_R5) && !c.rounded) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tile = tile_index();
    const int tx = tile % A.nx, ty = tile / A.nx;
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
            case PH_R5: {
                // z_i = sum_j X~_ij beta_j y_j (the points' coordinates)
                if constexpr (KIND == POT_COST_SQEUCLID_POINTS) {
                    const double xb = w.beta[j] * x;
                    rs += xb * (double)A.y[(int64_t)j * A.d];
                    rc += xb * (double)A.y[(int64_t)j * A.d + 1];
                    rq += A.d > 2 ? xb * (double)A.y[(int64_t)j * A.d + 2] : 0.0;
                }
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
            } else if (A.phase == PH_R5) {
                w.ugrave[i] = rs;      // z_i (dead ASPOT / Sinkhorn state slots after the loop)
                w.util0[i] = rc;
                w.util1[i] = rq;
            } else {
                // p'_i = r_i - (X'' 1)_i
                double p = A.r[i] - rs;
                p = p > 0.0 ? p : 0.0;
                w.pp[i] = p;
                w.du[i] = rs;          // (X'' 1)_i, for the marginal check of the result
                acc[0] += rc;          // <C, X''>
                acc[1] += p;           // |p'|_1
                acc[2] += p * rq;      // p'^T C q'
                acc[3] += rs;          // |X''|_1 (row side)
            }
        }
        block_sum<kScal>(acc, s_red);
        if (tid == 0) {
            for (int k = 0; k < kScal; ++k) st_agent(&w.rowscal[(int64_t)ty * kScal + k], acc[k]);
            st_agent(&w.rowcnt[ty], 0);        // (atomic, like the increments)
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
            w.dv[j] = be * cs;        // (X''^T 1)_j
            acc[0] += be * cs;        // T''
            acc[1] += q2;             // |q'|_1
            acc[7] += isfinite(cs) ? 0.0 : 1.0;
        }
        block_sum<kScal>(acc, s_red);
        if (tid == 0) {
            for (int k = 0; k < kScal; ++k) st_agent(&w.colscal[(int64_t)tx * kScal + k], acc[k]);
            st_agent(&w.colcnt[tx], 0);
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
                    c.rounded = 1;
                }
                st_agent(&w.glob[0], 0);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// setup (Algorithm 2, "Approximating POT"), validation, state initialisation
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void setup_kernel(SetupArgs S) {
    __shared__ double s_red[16 * 5];
    __shared__ double s_v[5];
    Ctl& c = *S.ws.ctl;
    const int tid = threadIdx.x, nt = blockDim.x;
    SetupIn in = {S.n, S.m, S.algo, S.gamma_rule, S.p, S.s, S.eps, S.gamma_user, S.tol_user, S.A_user,
                  S.cmax, S.cost_scale, S.w0};
    // the cost maximum computed on the device (a solve that does not read it
    // back): |C|_max, or for points the scale 1 / max |x - y|^2 and cmax
    int vmax = 0;
    if (S.maxbuf) {
        const double mx = __longlong_as_double((long long)S.maxbuf[0]);
        const bool bad = S.maxbuf[1] != 0;
        if (S.kind == POT_COST_SQEUCLID_POINTS) {
            if (bad) vmax = 11;
            else if (!(mx > 0.0)) vmax = 12;
            else {
                if (!(in.cost_scale > 0.0)) in.cost_scale = 1.0 / mx;
                if (!(in.cmax > 0.0)) in.cmax = in.cost_scale * mx;
            }
        } else {
            if (bad) vmax = 9;
            else if (!(mx > 0.0)) vmax = 10;
            else in.cmax = mx;
        }
        if (vmax) { in.cmax = 1.0; in.cost_scale = 1.0; }
    }
    // block reduction of K sums over the 1024 threads (16 waves)
    auto reduce = [&](auto& v) {
        constexpr int K = sizeof(v) / sizeof(double);
        const int lane = tid & 63, wave = tid >> 6;
        __syncthreads();
        for (int k = 0; k < K; ++k) {
            double x = wave_sum(v[k]);
            if (lane == 0) s_red[wave * K + k] = x;
        }
        __syncthreads();
        if (tid == 0) {
            for (int k = 0; k < K; ++k) {
                double a = 0.0;
                for (int w = 0; w < nt / 64; ++w) a += s_red[w * K + k];
                s_v[k] = a;
            }
        }
        __syncthreads();
        for (int k = 0; k < K; ++k) v[k] = s_v[k];
    };
    // sums, entropies and validity of the masses
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};      // |r|_1, |c|_1, bad entries, H(r), H(c)
    for (int i = tid; i < S.n; i += nt) {
        double x = S.r[i];
        v[2] += (isfinite(x) && x >= 0.0) ? 0.0 : 1.0;
        v[0] += x;
        v[3] += ent(x);
    }
    for (int j = tid; j < S.m; j += nt) {
        double x = S.c[j];
        v[2] += (isfinite(x) && x >= 0.0) ? 0.0 : 1.0;
        v[1] += x;
        v[4] += ent(x);
    }
    reduce(v);
    const double sr = v[0], sc = v[1];
    double gamma, et, tol;
    int valid = setup_params(in, sr, sc, v[2], v[3], v[4], gamma, et, tol);
    if (vmax) valid = vmax;
    // every exponent log2(e) C_ij / gamma must stay below 2^29 (exponent split)
    if (valid == 0 && !(kLog2e * in.cmax / gamma < 536870912.0)) valid = 7;
    // smoothed marginals r~, c~ (and their logs)
    double u[3] = {0.0, 0.0, 0.0};      // |r~|_1, |c~|_1, non-positive entries
    for (int i = tid; i < S.n; i += nt) {
        double x = smooth_mass(S.r[i], et, S.n);
        S.ws.rt[i] = x;
        S.ws.lrt[i] = log(x);
        u[2] += x > 0.0 ? 0.0 : 1.0;
        u[0] += x;
    }
    for (int j = tid; j < S.m; j += nt) {
        double x = smooth_mass(S.c[j], et, S.m);
        S.ws.ct[j] = x;
        S.ws.lct[j] = log(x);
        u[2] += x > 0.0 ? 0.0 : 1.0;
        u[1] += x;
    }
    reduce(u);
    if (valid == 0 && u[2] > 0.0) valid = 5;
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
        setup_fill(c, in, gamma, tol, sr, sc, u[0], u[1], valid);
        c.used_warm = S.warm;
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
    if (c.valid != 0) return;               // invalid problem: no output is written
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
    if (!c.rounded) return;
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

// Clear `n` 64-bit words (a kernel, not a memset node, so that a captured
// solve replays correctly).
__global__ void zero_words(unsigned long long* p, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = 0ull;
}

// Warm-start check of pot_solve.  mode 0, after the start pass at zero: keep
// phi(0).  mode 1, after the start pass at (u0, v0, w0): keep the warm start
// only if its phi is below phi(0) (a start whose statistics are not
// representable counts as worse); otherwise the next start pass evaluates
// the zero start.
__global__ void warm_decide(PassArgs A, int mode) {
    Ctl& c = *A.ws.ctl;
    if (threadIdx.x != 0 || c.valid != 0) return;
    if (mode == 0) {
        c.phi0 = c.done ? NAN : c.phichk;
        return;
    }
    if (c.phi0 != c.phi0) return;          // the zero start itself ended the solve
    if (c.done) {                          // the warm start's statistics overflowed
        if (A.host_done) __hip_atomic_store(A.host_done, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        c.done = 0;
        c.status = POT_OK;
        c.nonfinite = 0;
        c.iters = 0;
        c.cold = 1;
        c.used_warm = 0;
    } else if (!(c.phichk < c.phi0)) {
        c.cold = 1;
        c.used_warm = 0;
    }
}

// Marginal violations of the rounded plan Xbar = kappa X'' + lambda p' q'^T
// from its FP64 sums, (Xbar 1)_i = kappa (X'' 1)_i + lambda |q'|_1 p'_i and
// the same for the columns, and |1^T Xbar 1 - s|; with res != NULL the
// result block of the solve is written to device memory.
__global__ __launch_bounds__(1024) void result_kernel(PassArgs A, int algo, pot_result* res) {
    __shared__ double s_red[16 * 2];
    Ctl& c = *A.ws.ctl;
    const Ws& w = A.ws;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double v0 = 0.0, v1 = 0.0;
    if (c.rounded) {
        const double lr = c.lambda > 0.0 ? c.lambda * c.nq : 0.0;
        const double lc = c.lambda > 0.0 ? c.lambda * c.np : 0.0;
        for (int i = tid; i < A.n; i += blockDim.x) v0 += fmax(c.kappa * w.du[i] + lr * w.pp[i] - A.r[i], 0.0);
        for (int j = tid; j < A.m; j += blockDim.x) v1 += fmax(c.kappa * w.dv[j] + lc * w.qq[j] - A.c[j], 0.0);
    }
    v0 = wave_sum(v0);
    v1 = wave_sum(v1);
    if (lane == 0) { s_red[wave] = v0; s_red[16 + wave] = v1; }
    __syncthreads();
    if (tid == 0) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) { a += s_red[k]; b += s_red[16 + k]; }
        if (c.rounded) {
            c.viol_row = a;
            c.viol_col = b;
            c.viol_mass = fabs(c.mass - c.s);
        }
        if (res) fill_result(c, algo, *res);
    }
}

// Moments of the rounded plan Xbar = kappa diag(alpha) X~ diag(beta) + lambda
// p' q'^T against the points: M = sum_ij Xbar_ij x_i y_j^T = kappa sum_i
// alpha_i x_i z_i^T + lambda (sum_i p'_i x_i)(sum_j q'_j y_j)^T with z_i of
// the R5 pass, the barycentre sums sum_i (Xbar 1)_i x_i and sum_j
// (Xbar^T 1)_j y_j (row and column sums of Xbar from its factors) and the
// mass: mom[0..8], mom[9..11], mom[12..14], mom[15].
__global__ __launch_bounds__(256) void moments_kernel(PassArgs A, double* mom) {
    __shared__ double s_red[4 * 21];
    const Ctl& c = *A.ws.ctl;
    const Ws& w = A.ws;
    const int tid = threadIdx.x, d = A.d;
    if (!c.rounded) {
        if (tid < 16) mom[tid] = NAN;
        return;
    }
    // 0..8 sum alpha_i x_i z_i^T, 9..11 sum p'_i x_i, 12..14 sum (Xbar 1)_i x_i,
    // 15..17 sum q'_j y_j, 18..20 sum (Xbar^T 1)_j y_j
    double v[21];
#pragma unroll
    for (int k = 0; k < 21; ++k) v[k] = 0.0;
    const double lr = c.lambda > 0.0 ? c.lambda * c.nq : 0.0;
    const double lc = c.lambda > 0.0 ? c.lambda * c.np : 0.0;
    for (int i = tid; i < A.n; i += blockDim.x) {
        double xi[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < d; ++a) xi[a] = (double)A.x[(int64_t)i * d + a];
        const double zi[3] = {w.ugrave[i], w.util0[i], w.util1[i]};
        const double al = w.alpha[i], p = c.lambda > 0.0 ? w.pp[i] : 0.0;
        const double row = c.kappa * w.du[i] + lr * p;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int b = 0; b < 3; ++b) v[3 * a + b] += al * xi[a] * zi[b];
            v[9 + a] += p * xi[a];
            v[12 + a] += row * xi[a];
        }
    }
    for (int j = tid; j < A.m; j += blockDim.x) {
        double yj[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < d; ++a) yj[a] = (double)A.y[(int64_t)j * d + a];
        const double q = c.lambda > 0.0 ? w.qq[j] : 0.0;
        const double col = c.kappa * w.dv[j] + lc * q;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[15 + a] += q * yj[a];
            v[18 + a] += col * yj[a];
        }
    }
    block_sum<21, 4>(v, s_red);
    if (tid == 0) {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) mom[3 * a + b] = c.kappa * v[3 * a + b] + c.lambda * v[9 + a] * v[15 + b];
        for (int a = 0; a < 3; ++a) {
            mom[9 + a] = v[12 + a];
            mom[12 + a] = v[18 + a];
        }
        mom[15] = c.mass;
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

hipError_t launch_moments(const PassArgs& A, double* mom, hipStream_t st) {
    moments_kernel<<<1, 256, 0, st>>>(A, mom);
    return hipGetLastError();
}

hipError_t launch_zero_words(unsigned long long* p, int n, hipStream_t st) {
    zero_words<<<(n + 63) / 64, 64, 0, st>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_warm_decide(const PassArgs& A, int mode, hipStream_t st) {
    warm_decide<<<1, 64, 0, st>>>(A, mode);
    return hipGetLastError();
}

hipError_t launch_result(const PassArgs& A, int algo, pot_result* res, hipStream_t st) {
    result_kernel<<<1, 1024, 0, st>>>(A, algo, res);
    return hipGetLastError();
}

hipError_t launch_copy_out(const PassArgs& A, double* alpha, double* beta, double* pp, double* qq, hipStream_t st) {
    int len = A.n > A.m ? A.n : A.m;
    copy_out<<<(len + 255) / 256, 256, 0, st>>>(A, alpha, beta, pp, qq);
    return hipGetLastError();
}

}  // namespace pot
