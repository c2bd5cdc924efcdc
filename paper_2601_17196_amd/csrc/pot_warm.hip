// pot_warm.hip -- inference of the warm-start network on gfx950 (BF16 MFMA,
// FP32 accumulation).
//
// Per instance and side ("set"): features of the set's points, encoder
// h = relu(W2 relu(W1 p + b1) + b2), mean pooling; then per point the head
// relu(W3a h + W3b ctx_other + b3) . w4 + b4, divided by gamma.  Two
// launches: `warm_encode` writes every set's pooled context, `warm_head`
// recomputes the encoder of its set (cheaper than storing it) and applies the
// head with the other set's context.  One 256-thread workgroup per set; the
// points go through in tiles of 64, the 64 x 128 x 128 products on the matrix
// cores (v_mfma_f32_16x16x16_bf16: each wave owns 16 rows of a tile).
#include <hip/hip_runtime.h>
#include <math.h>

#include "pot_internal.h"

namespace pot {

namespace {

constexpr int kHid = 128;
constexpr int kTile = 64;              // points per tile
constexpr int kWThreads = 256;
constexpr int kLd = kHid + 8;          // LDS row stride of BF16 activations (elements)
// weight blob: FP32 section (biases, output row), then BF16 matrices
constexpr int kFB1 = 0, kFB2 = kHid, kFB3 = 2 * kHid, kFW4 = 3 * kHid, kFB4 = 4 * kHid;
constexpr int kBf16Off = 2304;         // bytes
constexpr int kHW1 = 0, kHW2 = kHid * 4, kHW3a = kHid * 4 + kHid * kHid, kHW3b = kHid * 4 + 2 * kHid * kHid;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// FP32 -> BF16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

struct WShared {
    uint16_t w2[kHid * kHid];          // out x in
    uint16_t w3a[kHid * kHid];
    uint16_t h1[kTile * kLd];          // BF16 activations of a tile (layer 1, then layer 2)
    float h2[kTile * kHid];            // FP32 layer-2 output of a tile (pooling)
    float feat[kTile][4];
    float hb[kHid];                    // W3b ctx_other + b3
    float out[kTile];
    double red[2 * 8];
};

// mean of the instance's n + m points (FP64), returned to every thread
__device__ void point_mean(const WDesc& D, double* red, double& m0, double& m1) {
    double s0 = 0.0, s1 = 0.0;
    for (int k = threadIdx.x; k < D.n + D.m; k += kWThreads) {
        const float* p = k < D.n ? D.x + 2 * k : D.y + 2 * (k - D.n);
        s0 += (double)p[0];
        s1 += (double)p[1];
    }
    // fixed-order block reduction: waves through LDS, in wave order
    for (int o = 32; o > 0; o >>= 1) {
        s0 += __shfl_xor(s0, o, 64);
        s1 += __shfl_xor(s1, o, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { red[2 * wave] = s0; red[2 * wave + 1] = s1; }
    __syncthreads();
    s0 = (red[0] + red[2]) + (red[4] + red[6]);
    s1 = (red[1] + red[3]) + (red[5] + red[7]);
    __syncthreads();
    m0 = s0 / (D.n + D.m);
    m1 = s1 / (D.n + D.m);
}

// Encoder of one tile: features of points [p0, p0 + 64) of the side (masked
// beyond np), layer 1 (VALU) into S.h1 as BF16, layer 2 on the matrix cores;
// returns the layer-2 output of the wave's 16 rows in acc (8 column blocks of
// 16, lane layout of the MFMA result: rows 4 (lane / 16) + e, column lane % 16).
__device__ void encode_tile(const WDesc& D, int side, int p0, double mu0, double mu1, const float* fw,
                            const uint16_t* hw, WShared& S, f32x4 (&acc)[8]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int np = side == 0 ? D.n : D.m;
    const float* pts = side == 0 ? D.x : D.y;
    const double* mass = side == 0 ? D.r : D.c;
    const double sc = sqrt(D.cost_scale);
    if (tid < kTile) {
        const int p = p0 + tid;
        float f0 = 0.f, f1 = 0.f, f2 = 0.f;
        if (p < np) {
            f0 = (float)(((double)pts[2 * p] - mu0) * sc);
            f1 = (float)(((double)pts[2 * p + 1] - mu1) * sc);
            const double lm = log((double)np * mass[p]);
            f2 = (float)fmin(fmax(lm, -30.0), 30.0);       // (log 0 = -inf clips to -30)
        }
        S.feat[tid][0] = f0;
        S.feat[tid][1] = f1;
        S.feat[tid][2] = f2;
        S.feat[tid][3] = 0.f;
    }
    __syncthreads();
    // layer 1: thread -> hidden unit k = tid % 128, points of one parity
    {
        const int k = tid & (kHid - 1);
        const float w0 = bf2f(hw[kHW1 + 4 * k]), w1 = bf2f(hw[kHW1 + 4 * k + 1]), w2 = bf2f(hw[kHW1 + 4 * k + 2]),
                    w3 = bf2f(hw[kHW1 + 4 * k + 3]);
        const float b = fw[kFB1 + k];
        for (int p = tid >> 7; p < kTile; p += 2) {
            float h = b;
            h = fmaf(w0, S.feat[p][0], h);
            h = fmaf(w1, S.feat[p][1], h);
            h = fmaf(w2, S.feat[p][2], h);
            h = fmaf(w3, S.feat[p][3], h);
            S.h1[p * kLd + k] = f2bf(fmaxf(h, 0.f));
        }
    }
    __syncthreads();
    // layer 2: rows 16 wave .. 16 wave + 15 of the tile, all 128 columns
#pragma unroll
    for (int cb = 0; cb < 8; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int ra = 16 * wave + (lane & 15), kq = 4 * (lane >> 4);
#pragma unroll
    for (int kk = 0; kk < kHid / 16; ++kk) {
        const bf16x4 a = *(const bf16x4*)&S.h1[ra * kLd + 16 * kk + kq];
#pragma unroll
        for (int cb = 0; cb < 8; ++cb) {
            const bf16x4 bv = *(const bf16x4*)&S.w2[(16 * cb + (lane & 15)) * kHid + 16 * kk + kq];
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc[cb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int cb = 0; cb < 8; ++cb) {
        const float b = fw[kFB2 + 16 * cb + (lane & 15)];
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[cb][e] = fmaxf(acc[cb][e] + b, 0.f);
    }
}

__device__ void load_matrix(uint16_t* dst, const uint16_t* src) {
    for (int k = threadIdx.x; k < kHid * kHid / 4; k += kWThreads)
        reinterpret_cast<uint2*>(dst)[k] = reinterpret_cast<const uint2*>(src)[k];
}

// pooled context of every set: ctx[(inst * 2 + side) * 128 + k]
__global__ __launch_bounds__(kWThreads) void warm_encode(const WDesc* desc, const void* blob, float* ctx) {
    __shared__ WShared S;
    const int inst = blockIdx.x >> 1, side = blockIdx.x & 1;
    const WDesc D = desc[inst];
    const float* fw = (const float*)blob;
    const uint16_t* hw = (const uint16_t*)((const char*)blob + kBf16Off);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    load_matrix(S.w2, hw + kHW2);
    double mu0, mu1;
    point_mean(D, S.red, mu0, mu1);
    const int np = side == 0 ? D.n : D.m;
    float pool = 0.f;                  // thread k < 128: running sum of column k
    for (int p0 = 0; p0 < np; p0 += kTile) {
        f32x4 acc[8];
        encode_tile(D, side, p0, mu0, mu1, fw, hw, S, acc);
#pragma unroll
        for (int cb = 0; cb < 8; ++cb)
#pragma unroll
            for (int e = 0; e < 4; ++e) S.h2[(16 * wave + 4 * (lane >> 4) + e) * kHid + 16 * cb + (lane & 15)] = acc[cb][e];
        __syncthreads();
        if (tid < kHid) {
            const int nv = min(kTile, np - p0);
            for (int p = 0; p < nv; ++p) pool += S.h2[p * kHid + tid];
        }
        __syncthreads();
    }
    if (tid < kHid) ctx[(size_t)blockIdx.x * kHid + tid] = pool / (float)np;
}

// predictions of every point of every set
__global__ __launch_bounds__(kWThreads) void warm_head(const WDesc* desc, const void* blob, const float* ctx) {
    __shared__ WShared S;
    const int inst = blockIdx.x >> 1, side = blockIdx.x & 1;
    const WDesc D = desc[inst];
    const float* fw = (const float*)blob;
    const uint16_t* hw = (const uint16_t*)((const char*)blob + kBf16Off);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    load_matrix(S.w2, hw + kHW2);
    load_matrix(S.w3a, hw + kHW3a);
    // head bias of this set: W3b ctx_other + b3
    if (tid < kHid) {
        const float* co = ctx + (size_t)(2 * inst + (side ^ 1)) * kHid;
        float h = fw[kFB3 + tid];
        for (int k = 0; k < kHid; ++k) h = fmaf(bf2f(hw[kHW3b + tid * kHid + k]), co[k], h);
        S.hb[tid] = h;
    }
    double mu0, mu1;
    point_mean(D, S.red, mu0, mu1);
    const int np = side == 0 ? D.n : D.m;
    double* outp = side == 0 ? D.u0 : D.v0;
    for (int p0 = 0; p0 < np; p0 += kTile) {
        f32x4 acc[8];
        encode_tile(D, side, p0, mu0, mu1, fw, hw, S, acc);
        __syncthreads();
        // layer-2 output to BF16 (the head's MFMA input)
#pragma unroll
        for (int cb = 0; cb < 8; ++cb)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                S.h1[(16 * wave + 4 * (lane >> 4) + e) * kLd + 16 * cb + (lane & 15)] = f2bf(acc[cb][e]);
        __syncthreads();
#pragma unroll
        for (int cb = 0; cb < 8; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
        const int ra = 16 * wave + (lane & 15), kq = 4 * (lane >> 4);
#pragma unroll
        for (int kk = 0; kk < kHid / 16; ++kk) {
            const bf16x4 a = *(const bf16x4*)&S.h1[ra * kLd + 16 * kk + kq];
#pragma unroll
            for (int cb = 0; cb < 8; ++cb) {
                const bf16x4 bv = *(const bf16x4*)&S.w3a[(16 * cb + (lane & 15)) * kHid + 16 * kk + kq];
                acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc[cb], 0, 0, 0);
            }
        }
        // z = relu(. + hb); out = z . w4 + b4: each lane holds 4 rows x 8 columns
        float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int cb = 0; cb < 8; ++cb) {
            const int col = 16 * cb + (lane & 15);
            const float hb = S.hb[col], w4 = fw[kFW4 + col];
#pragma unroll
            for (int e = 0; e < 4; ++e) part[e] = fmaf(fmaxf(acc[cb][e] + hb, 0.f), w4, part[e]);
        }
        // sum over the 16 lanes that share rows (fixed xor order)
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) part[e] += __shfl_xor(part[e], o, 64);
        if ((lane & 15) == 0) {
#pragma unroll
            for (int e = 0; e < 4; ++e) S.out[16 * wave + 4 * (lane >> 4) + e] = part[e] + fw[kFB4];
        }
        __syncthreads();
        if (tid < kTile && p0 + tid < np) outp[p0 + tid] = (double)S.out[tid] * D.inv_gamma;
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_warm(const WDesc* desc_dev, int batch, const void* blob, float* ctx, hipStream_t st) {
    warm_encode<<<2 * batch, kWThreads, 0, st>>>(desc_dev, blob, ctx);
    warm_head<<<2 * batch, kWThreads, 0, st>>>(desc_dev, blob, ctx);
    return hipGetLastError();
}

size_t warm_desc_bytes() { return sizeof(WDesc); }

void warm_fill_desc(void* dst, const float* x, const float* y, const double* r, const double* c, double* u0,
                    double* v0, double cost_scale, double inv_gamma, int n, int m) {
    WDesc d;
    d.x = x; d.y = y; d.r = r; d.c = c; d.u0 = u0; d.v0 = v0;
    d.cost_scale = cost_scale;
    d.inv_gamma = inv_gamma;
    d.n = n;
    d.m = m;
    *(WDesc*)dst = d;
}

}  // namespace pot
