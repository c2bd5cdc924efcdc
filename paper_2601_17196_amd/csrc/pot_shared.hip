// pot_shared.hip -- many POT instances on one shared cost: feasible Sinkhorn
// (the loop of Algorithm 3) in the exponential domain, with the kernel of the
// extended instance K~ = exp(-C~ / gamma) built once in BF16 and the
// scalings of all instances multiplied by it on the matrix cores.
//
// Extended instance of each member b (appendix, "Reduction to Extended OT"):
// rows r^_b = (r~_b, |c~_b|_1 - s_b), columns c^_b = (c~_b, |r~_b|_1 - s_b),
// C~ = [[C, 0], [0^T, A]].  One iteration for every member at once:
//     a_b = r^_b / (K~ b_b)        (GEMM 1: K~ (N x M) times [b_1 .. b_B])
//     b_b = c^_b / (K~^T a_b)      (GEMM 2: K~^T (M x N) times [a_1 .. a_B])
// with the row error of iterate t, |a^t (K~ b^t) - r^|_1 (the columns are
// exact after the b update), taken in the a update of iterate t + 1.
//
// Precision: K~ is rounded to BF16 once (it defines the effective cost
// C' = -gamma ln K~_bf16, which differs from C by at most gamma 2^-8); each
// scaling enters the products as the sum of two BF16 numbers (hi + lo, about
// 16 significant bits), so every product K~ b is accumulated in FP32 from an
// operand accurate to about 2^-17: the iteration converges to the fixed point
// of the effective cost.  Scalings are FP32.  The kernel is representable
// only where C / gamma stays inside the FP32 exponent range; the host checks
// max C / gamma <= 80.
//
// Layout: K~ [Np][Mp] and its transpose [Mp][Np], BF16, zero padded to
// multiples of 64; the scalings [Bp][Np] and [Bp][Mp] (FP32, instance-major);
// the BF16 operands [2 Bp][Mp] and [2 Bp][Np] (hi row, lo row per member; Bp
// a multiple of 64);
// GEMM outputs [2 Bp][Np] / [2 Bp][Mp] FP32.
#include <hip/hip_runtime.h>
#include <math.h>

#include "pot_device.h"

namespace pot {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan kept
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

}  // namespace

// K~ and its transpose from the stored cost (FP32 or BF16), cost scale and
// gamma: K~_ij = exp(-C_ij / gamma) for i < n, j < m; 1 on the dummy row and
// column; exp(-A / gamma) at the corner; 0 in the padding.
template <int KIND>
__global__ void shared_build_kernel(const void* C, int64_t ldc, int n, int m, int Np, int Mp, double inv_gamma,
                                    double corner, uint16_t* K, uint16_t* KT) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)Np * Mp) return;
    const int i = (int)(e / Mp), j = (int)(e % Mp);
    float v = 0.0f;
    if (i < n && j < m) {
        double cij;
        if (KIND == POT_COST_F32) cij = (double)((const float*)C)[(int64_t)i * ldc + j];
        else cij = (double)bf16_bits_to_f32(((const uint16_t*)C)[(int64_t)i * ldc + j]);
        v = (float)exp(-cij * inv_gamma);
    } else if ((i < n && j == m) || (i == n && j < m)) {
        v = 1.0f;
    } else if (i == n && j == m) {
        v = (float)corner;
    }
    const uint16_t h = f32_to_bf16_rne(v);
    K[(int64_t)i * Mp + j] = h;
    KT[(int64_t)j * Np + i] = h;
}

// Out[q][i] = sum_k A[i][k] Bop[q][k] for i < rows (multiple of 64), q < cols
// (multiple of TN), k < depth (multiple of 32): both operands K-contiguous,
// BF16, FP32 accumulation on v_mfma_f32_16x16x16_bf16.  A 256-thread
// workgroup owns a 64 x TN output tile (waves 2 x 2, each 32 x TN/2 = 2 x
// TN/32 MFMA tiles); TN = 128 where that still gives a workgroup per compute
// unit, else 64.  Per step of 32 k, every thread brings one 16-byte chunk of
// the A tile and TN/64 of the B tile into registers (the next step's, while
// the current step computes) and stores them to LDS, laid out [k-group of
// 4][row] in 8-byte entries, so that a fragment read (16 rows x 4 k-groups)
// is one ds_read_b64 per lane; two LDS buffers alternate.  MFMA lane layout:
// lane l holds A[row l & 15][k-group l >> 4] and B[col l & 15][k-group l >> 4]
// and receives Out[col l & 15][rows 4 (l >> 4) .. +3].
constexpr int kGM = 64, kGK = 32, kGPad = 4;
template <int TN>
__global__ __launch_bounds__(256) void shared_gemm_kernel(const uint16_t* A, const uint16_t* Bop, float* Out,
                                                          int rows, int cols, int depth, const int32_t* ndone,
                                                          int B) {
    constexpr int NB = TN / 64, NT = TN / 32;
    if (*ndone >= B) return;                 // every member has finished (uniform)
    __shared__ uint2 As[2][kGK / 4][kGM + kGPad];
    __shared__ uint2 Bs[2][kGK / 4][TN + kGPad];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int i0 = blockIdx.x * kGM, q0 = blockIdx.y * TN;
    // global -> register chunks: A row tid >> 2, chunk tid & 3; B rows 64 h + (tid >> 2)
    const int lr = tid >> 2, lc = tid & 3;
    const uint4* ag = (const uint4*)(A + (int64_t)(i0 + lr) * depth + 8 * lc);
    const uint4* bg[NB];
#pragma unroll
    for (int h = 0; h < NB; ++h) bg[h] = (const uint4*)(Bop + (int64_t)(q0 + 64 * h + lr) * depth + 8 * lc);
    uint4 ra, rb[NB];
    auto fetch = [&](int off) __attribute__((always_inline)) {
        ra = ag[off];
#pragma unroll
        for (int h = 0; h < NB; ++h) rb[h] = bg[h][off];
    };
    auto to_lds = [&](int buf) __attribute__((always_inline)) {
        As[buf][2 * lc][lr] = make_uint2(ra.x, ra.y);
        As[buf][2 * lc + 1][lr] = make_uint2(ra.z, ra.w);
#pragma unroll
        for (int h = 0; h < NB; ++h) {
            Bs[buf][2 * lc][64 * h + lr] = make_uint2(rb[h].x, rb[h].y);
            Bs[buf][2 * lc + 1][64 * h + lr] = make_uint2(rb[h].z, rb[h].w);
        }
    };
    f32x4v acc[2][NT];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4v{0.f, 0.f, 0.f, 0.f};
    const int nk = depth / kGK;
    fetch(0);
    to_lds(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) fetch((kt + 1) * kGK / 8);      // offset in 16-byte chunks
#pragma unroll
        for (int ks = 0; ks < kGK / 16; ++ks) {
            const int kg = 4 * ks + (lane >> 4);
            bf16x4 af[2], bf[NT];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                const uint2 v = As[buf][kg][32 * wm + 16 * mt + (lane & 15)];
                af[mt] = *(const bf16x4*)&v;
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const uint2 v = Bs[buf][kg][(TN / 2) * wn + 16 * nt + (lane & 15)];
                bf[nt] = *(const bf16x4*)&v;
            }
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[mt], bf[nt], acc[mt][nt], 0, 0, 0);
        }
        if (kt + 1 < nk) to_lds(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            float* o = Out + (int64_t)(q0 + (TN / 2) * wn + 16 * nt + (lane & 15)) * rows + i0 + 32 * wm + 16 * mt +
                       4 * (lane >> 4);
            *(f32x4v*)o = acc[mt][nt];
        }
}

// The scaling update of one side for every member: s_new = mass / (sum of
// the hi and lo products), written to the other parity slot, and its BF16
// split into the next GEMM's operand.  Row side (err != NULL): the member's
// row error of the current iterate, |s (K~ b) - r^|_1, partial per block.
// Members already finished are left alone.
__global__ __launch_bounds__(256) void shared_update_kernel(const float* prod, const float* mass, const float* scal_cur,
                                                            float* scal_next, uint16_t* op, int len, int ld,
                                                            const int32_t* done, double* err_part) {
    __shared__ double s_red[4];
    const int b = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (done[b]) return;                    // (uniform over the block)
    double e = 0.0;
    if (i < ld) {
        const float p = prod[(int64_t)(2 * b) * ld + i] + prod[(int64_t)(2 * b + 1) * ld + i];
        const float ms = mass[(int64_t)b * ld + i];
        float sn = 0.0f;
        if (i < len) {
            if (err_part) e = fabs((double)scal_cur[(int64_t)b * ld + i] * (double)p - (double)ms);
            sn = ms > 0.0f ? ms / p : 0.0f;
        }
        scal_next[(int64_t)b * ld + i] = sn;
        const uint16_t hi = f32_to_bf16_rne(sn);
        const uint16_t lo = f32_to_bf16_rne(sn - bf16_bits_to_f32(hi));
        op[(int64_t)(2 * b) * ld + i] = hi;
        op[(int64_t)(2 * b + 1) * ld + i] = lo;
    }
    if (err_part) {
        e = wave_sum(e);
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        if (lane == 0) s_red[wave] = e;
        __syncthreads();
        if (threadIdx.x == 0) err_part[(int64_t)b * gridDim.x + blockIdx.x] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
    }
}


// a member has finished: count it; the last one sets the host flag
__device__ __forceinline__ void member_finished(const SharedCtl& S, int B) {
    const int k = atomicAdd(S.ndone, 1);
    if (k + 1 == B && S.host_done) __hip_atomic_store(S.host_done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Per member: the row error of iterate t (t >= 1) against its threshold;
// the stop (or max_iter) freezes the member at iterate t, whose row scalings
// sit in parity slot t & 1 (the update just made wrote the other one).
__global__ void shared_decide_kernel(SharedCtl S, const double* err_part, int nblk, int B, int t, int max_iter) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B || S.done[b]) return;
    double e = 0.0;
    for (int k = 0; k < nblk; ++k) e += err_part[(int64_t)b * nblk + k];
    bool stop = false;
    if (t >= 1) {
        S.E[b] = e;
        stop = e <= S.tol[b];
    }
    if (!(e == e) || (t >= 1 && !isfinite(e))) {
        S.done[b] = 1;
        S.status[b] = POT_ERR_NUMERIC;
        S.iters[b] = t;
        S.out_par[b] = t & 1;
    } else if (stop || t >= max_iter) {
        S.done[b] = 1;
        S.status[b] = stop ? POT_OK : POT_ERR_NO_CONVERGENCE;
        S.iters[b] = t;
        S.out_par[b] = t & 1;
    } else {
        return;
    }
    member_finished(S, B);
}

// Member b's setup results into the batch arrays: r^ and c^ (FP32) and its
// threshold (ws: the single-instance workspace the setup kernel filled).  An
// invalid member is finished at once with POT_ERR_INVALID_ARG.
__global__ void shared_gather_kernel(Ws w, int n, int m, int Np, int Mp, int b, int B, float* rhat, float* chat,
                                     double* tol, SharedCtl S) {
    const Ctl& c = *w.ctl;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = c.valid == 0;
    if (k < Np) rhat[(int64_t)b * Np + k] = (ok && k < n) ? (float)w.rt[k] : ((ok && k == n) ? (float)c.rhat_d : 0.0f);
    if (k < Mp) chat[(int64_t)b * Mp + k] = (ok && k < m) ? (float)w.ct[k] : ((ok && k == m) ? (float)c.chat_d : 0.0f);
    if (k == 0) {
        tol[b] = c.tol;
        if (!ok) {
            S.done[b] = 1;
            S.status[b] = POT_ERR_INVALID_ARG;
            member_finished(S, B);
        }
    }
}

// Start of the loop: b = 1 on every real and dummy column (log b = 0, the
// cold start of Algorithm 3), its BF16 operand, the member flags.
__global__ void shared_init_kernel(float* bsc, uint16_t* bop, int m, int Mp, int B, SharedCtl S) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (k < Mp) {
        const float v = k <= m ? 1.0f : 0.0f;
        bsc[(int64_t)b * Mp + k] = v;
        bop[(int64_t)(2 * b) * Mp + k] = f32_to_bf16_rne(v);
        bop[(int64_t)(2 * b + 1) * Mp + k] = 0;
    }
    if (k == 0) {
        S.done[b] = 0;
        S.iters[b] = 0;
        S.status[b] = POT_OK;
        S.out_par[b] = 0;
        S.E[b] = INFINITY;
        if (b == 0) *S.ndone = 0;
    }
}

// Member b's output scalings as log-scalings of X~_ij = exp(f_i + g_j -
// C_ij / gamma) into the rounding slots of the single-instance workspace
// (ubar, vbar; the dummy entries into the control block), its finish state,
// and the caller's optional f, g.  abuf: [2][Bp][Np] by parity.
__global__ void shared_load_duals_kernel(Ws w, const float* abuf, const float* bsc, int n, int m, int Np, int Mp,
                                         int Bp, int b, SharedCtl S, double* fo, double* go) {
    Ctl& c = *w.ctl;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const float* a = abuf + ((int64_t)S.out_par[b] * Bp + b) * Np;
    const bool out = S.status[b] != POT_ERR_INVALID_ARG;    // an invalid member gets no output
    if (k < n) {
        const double f = log((double)a[k]);
        w.ubar[k] = f;
        if (fo && out) fo[k] = f;
    }
    if (k < m) {
        const double g = log((double)bsc[(int64_t)b * Mp + k]);
        w.vbar[k] = g;
        if (go && out) go[k] = g;
    }
    if (k == 0) {
        c.done = 1;
        c.status = S.status[b];
        c.iters = S.iters[b];
        c.E = S.E[b];
        c.out_par = 0;
        c.ad[0] = c.ad[1] = log((double)a[n]);
        c.bd = log((double)bsc[(int64_t)b * Mp + m]);
    }
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
hipError_t launch_shared_build(int kind, const void* C, int64_t ldc, int n, int m, int Np, int Mp, double inv_gamma,
                               double corner, uint16_t* K, uint16_t* KT, hipStream_t st) {
    const int64_t tot = (int64_t)Np * Mp;
    const int blocks = (int)((tot + 255) / 256);
    if (kind == POT_COST_BF16)
        shared_build_kernel<POT_COST_BF16><<<blocks, 256, 0, st>>>(C, ldc, n, m, Np, Mp, inv_gamma, corner, K, KT);
    else
        shared_build_kernel<POT_COST_F32><<<blocks, 256, 0, st>>>(C, ldc, n, m, Np, Mp, inv_gamma, corner, K, KT);
    return hipGetLastError();
}

hipError_t launch_shared_gemm(const uint16_t* A, const uint16_t* Bop, float* Out, int rows, int cols, int depth,
                              const int32_t* ndone, int B, hipStream_t st) {
    if (rows % kGM || cols % 64 || depth % kGK) return hipErrorInvalidValue;
    if (cols % 128 == 0 && (int64_t)(rows / kGM) * (cols / 128) >= 256)
        shared_gemm_kernel<128><<<dim3(rows / kGM, cols / 128), 256, 0, st>>>(A, Bop, Out, rows, cols, depth, ndone, B);
    else
        shared_gemm_kernel<64><<<dim3(rows / kGM, cols / 64), 256, 0, st>>>(A, Bop, Out, rows, cols, depth, ndone, B);
    return hipGetLastError();
}

hipError_t launch_shared_update(const float* prod, const float* mass, const float* cur, float* next, uint16_t* op,
                                int len, int ld, int B, const int32_t* done, double* err_part, hipStream_t st) {
    shared_update_kernel<<<dim3((ld + 255) / 256, B), 256, 0, st>>>(prod, mass, cur, next, op, len, ld, done, err_part);
    return hipGetLastError();
}

hipError_t launch_shared_gather(const Ws& w, int n, int m, int Np, int Mp, int b, int B, float* rhat, float* chat,
                                double* tol, const SharedCtl& S, hipStream_t st) {
    const int len = Np > Mp ? Np : Mp;
    shared_gather_kernel<<<(len + 255) / 256, 256, 0, st>>>(w, n, m, Np, Mp, b, B, rhat, chat, tol, S);
    return hipGetLastError();
}

hipError_t launch_shared_init(float* bsc, uint16_t* bop, int m, int Mp, int B, const SharedCtl& S, hipStream_t st) {
    shared_init_kernel<<<dim3((Mp + 255) / 256, B), 256, 0, st>>>(bsc, bop, m, Mp, B, S);
    return hipGetLastError();
}

hipError_t launch_shared_load_duals(const Ws& w, const float* abuf, const float* bsc, int n, int m, int Np, int Mp,
                                    int Bp, int b, const SharedCtl& S, double* fo, double* go, hipStream_t st) {
    const int len = n > m ? n : m;
    shared_load_duals_kernel<<<(len + 255) / 256, 256, 0, st>>>(w, abuf, bsc, n, m, Np, Mp, Bp, b, S, fo, go);
    return hipGetLastError();
}

hipError_t launch_shared_decide(const SharedCtl& S, const double* err_part, int nblk, int B, int t, int max_iter,
                                hipStream_t st) {
    shared_decide_kernel<<<(B + 63) / 64, 64, 0, st>>>(S, err_part, nblk, B, t, max_iter);
    return hipGetLastError();
}

}  // namespace pot
