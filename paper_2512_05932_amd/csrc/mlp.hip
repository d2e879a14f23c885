// Surrogate network kernels: BF16 matrix products on the MFMA units with
// FP32 accumulation, the elementwise steps around them (bias, GELU and its
// derivative, the loss and its gradient, bias gradients) and the AdamW update.
//
// Network: 1056 -> 256 -> 256 -> 256 -> 16 (inputs 1030..1055 and outputs
// 13..15 are padding), GELU(z) = z/2 (1 + erf(z / sqrt 2)).  Weights are
// kept in FP32 (the optimiser's copy) and in BF16 (the operands of the
// products); activations between layers and the backward operands are BF16.
#include "engine.h"

namespace lidar {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTileM = 64, kTileN = 64, kTileK = 32;
constexpr int kLdsK = kTileK + 8;         // row stride in LDS (elements)

__device__ inline uint16_t to_bf16(float f)
{
    // round to nearest, ties to even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// C = A B over a 64 x 64 tile per workgroup (4 waves of 32 x 32, each 2 x 2
// MFMA 16x16x16 blocks), K in steps of 32 staged through LDS.  Both operands
// are stored in LDS with K contiguous ([row][k] for A, [col][k] for B), so
// every lane's 4 consecutive K values are one 8-byte read.
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g)
{
    __shared__ uint16_t As[kTileM][kLdsK];
    __shared__ uint16_t Bs[kTileN][kLdsK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * kTileM, n0 = blockIdx.x * kTileN;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // load mapping: consecutive threads walk the operand's unit-stride axis
    const bool a_kfast = g.sak == 1;
    const bool b_kfast = g.sbk == 1;
    // this workgroup's share of K (whole tiles)
    const int kchunk = ((g.K + g.ksplit - 1) / g.ksplit + kTileK - 1) / kTileK * kTileK;
    const int kbeg = blockIdx.z * kchunk, kend = min(g.K, kbeg + kchunk);
    for (int k0 = kbeg; k0 < kend; k0 += kTileK) {
#pragma unroll
        for (int q = 0; q < (kTileM * kTileK) / 256; ++q) {
            const int e = tid + 256 * q;
            const int r = a_kfast ? e / kTileK : e % kTileM;
            const int k = a_kfast ? e % kTileK : e / kTileM;
            const int gi = m0 + r, gk = k0 + k;
            As[r][k] = (gi < g.M && gk < kend) ? g.A[(long)gi * g.sam + (long)gk * g.sak] : (uint16_t)0;
        }
#pragma unroll
        for (int q = 0; q < (kTileN * kTileK) / 256; ++q) {
            const int e = tid + 256 * q;
            const int c = b_kfast ? e / kTileK : e % kTileN;
            const int k = b_kfast ? e % kTileK : e / kTileN;
            const int gj = n0 + c, gk = k0 + k;
            Bs[c][k] = (gj < g.N && gk < kend) ? g.B[(long)gk * g.sbk + (long)gj * g.sbn] : (uint16_t)0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kTileK; kk += 16) {
            const int kq = kk + 4 * (lane >> 4);
            bf16x4 a[2], b[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                a[t] = *(const bf16x4*)&As[wm * 32 + t * 16 + (lane & 15)][kq];
                b[t] = *(const bf16x4*)&Bs[wn * 32 + t * 16 + (lane & 15)][kq];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // D block: lane holds column lane % 16, rows 4 (lane / 16) + r
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = n0 + wn * 32 + j * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                if (row < g.M && col < g.N) {
                    if (g.ksplit > 1)
                        atomicAdd(&g.C[(long)row * g.ldc + col], acc[i][j][r]);
                    else
                        g.C[(long)row * g.ldc + col] = acc[i][j][r];
                }
            }
        }
}

// erf by the rational approximation of Abramowitz & Stegun, formula 7.1.26
// (absolute error <= 1.5e-7): for x >= 0, erf(x) = 1 - t (a1 + t (a2 + t (a3
// + t (a4 + t a5)))) exp(-x^2) with t = 1 / (1 + p x); odd in x.  The
// hardware reciprocal and exponential add a few ulp; the result feeds BF16
// activations (relative step 2^-8), far coarser than either error.
__device__ inline float erf_as(float x)
{
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * ax);
    const float poly = t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f +
                       t * (-1.453152027f + t * 1.061405429f))));
    return copysignf(1.0f - poly * __expf(-ax * ax), x);
}

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erf_as(z * 0.70710678118654752f)); }

__device__ inline float gelu_prime(float z)
{
    return 0.5f * (1.0f + erf_as(z * 0.70710678118654752f)) +
           z * __expf(-0.5f * z * z) * 0.39894228040143268f;
}

// Z += bias (in place); H = bf16(gelu(Z)).
__global__ void k_bias_gelu(float* Z, const float* bias, uint16_t* H, long n, int C)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * C) return;
    const float z = Z[i] + bias[i % C];
    Z[i] = z;
    H[i] = to_bf16(gelu(z));
}

__global__ void k_bias(float* Y, const float* bias, long n, int C)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * C) return;
    Y[i] += bias[i % C];
}

__device__ inline float bce(float z, float t) { return fmaxf(z, 0.0f) - z * t + log1pf(expf(-fabsf(z))); }
__device__ inline float sigm(float z) { return 1.0f / (1.0f + expf(-z)); }

// Per-row loss and gradient (scaled by 1/n) with respect to the 16 outputs.
__global__ void k_loss(const float* Y, const float* lab, long n, float inv_n, uint16_t* dYb,
                       float* loss_sum)
{
    const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
    float L = 0.0f;
    if (r < n) {
        const float* y = Y + r * 16;
        const float* l = lab + r * 16;
        float d[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) d[j] = 0.0f;
        bool ok = true;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const float ex = l[e];
            const bool te = ex > 0.5f;
            ok = ok && ((y[e] > 0.0f) == te);
            ok = ok && !(te && fabsf(y[3 + e] - l[3 + e]) * kSurBinScale > 0.5f);
            ok = ok && !(te && fabsf(l[3 + e]) >= kSurDkClip);
            L += bce(y[e], ex);
            d[e] = sigm(y[e]) - ex;
            const float dk = y[3 + e] - l[3 + e];
            const float di = y[6 + e] - l[6 + e];
            const float dw = y[9 + e] - l[9 + e];
            L += ex * (kSurWBin * dk * dk + kSurWInt * di * di + kSurWEpw * dw * dw);
            d[3 + e] = ex * 2.0f * kSurWBin * dk;
            d[6 + e] = ex * 2.0f * kSurWInt * di;
            d[9 + e] = ex * 2.0f * kSurWEpw * dw;
        }
        const float okf = ok ? 1.0f : 0.0f;
        L += bce(y[12], okf);
        d[12] = sigm(y[12]) - okf;
#pragma unroll
        for (int j = 0; j < 16; ++j) dYb[r * 16 + j] = to_bf16(d[j] * inv_n);
    }
    // block sum of the row losses, one atomic per block
    __shared__ float part[256];
    part[threadIdx.x] = L;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss_sum) atomicAdd(loss_sum, part[0] * inv_n);
}

// dZ = bf16(dH * gelu'(Z))
__global__ void k_gelu_back(const float* dH, const float* Z, uint16_t* dZb, long count)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    dZb[i] = to_bf16(dH[i] * gelu_prime(Z[i]));
}

// db[j] += sum over rows of the BF16 operand dZ[r][j]: a workgroup takes 64
// columns x `span` rows (lane = column, wave = every 4th row), sums its waves
// in LDS and adds into the zeroed output (one workgroup per column block
// when span covers every row: then the sum has a fixed order)
__global__ __launch_bounds__(256) void k_colsum(const uint16_t* D, long n, int C, long span, float* out)
{
    __shared__ float part[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    const long r0 = (long)blockIdx.y * span;
    float s = 0.0f;
    if (j < C)
        for (long r = r0 + wave; r < min(n, r0 + span); r += 4) s += from_bf16(D[r * C + j]);
    part[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && j < C) atomicAdd(&out[j], part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane]);
}

__global__ void k_zero_f32(float* p, long n)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// AdamW (decoupled weight decay on the weights, not on the biases), then
// the BF16 operand copy of the parameter.
__global__ void k_adamw(float* theta, const float* grad, float* m, float* v, uint16_t* theta_b,
                        long n, AdamArgs a)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool decay = sur_is_weight(i);
    float t = theta[i];
    if (decay) t *= a.decay_factor;
    const float g = grad[i];
    const float mi = a.beta1 * m[i] + (1.0f - a.beta1) * g;
    const float vi = a.beta2 * v[i] + (1.0f - a.beta2) * g * g;
    m[i] = mi;
    v[i] = vi;
    t -= a.lr * (mi * a.inv_bc1) / (sqrtf(vi * a.inv_bc2) + a.eps);
    theta[i] = t;
    theta_b[i] = to_bf16(t);
}

// ---- minibatches of the training loop -------------------------------------
// Position p of epoch e maps to row perm(p): a four-round Feistel network on
// k-bit values (k even, 2^k >= n; halves of k/2 bits), cycle-walked until the
// value is below n (a bijection of 0 .. n-1).  Round r replaces (L, R) by
// (R, L ^ (mix(key ^ R) & mask)), key = seed ^ ((4 e + r + 1) * golden),
// mix the SplitMix64 output function.
__device__ inline unsigned long long mix64(unsigned long long z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ inline unsigned long long feistel(unsigned long long x, int half, unsigned long long seed,
                                             unsigned long long epoch)
{
    const unsigned long long mask = (1ull << half) - 1ull;
    unsigned long long L = x >> half, R = x & mask;
#pragma unroll
    for (unsigned long long r = 0; r < 4; ++r) {
        const unsigned long long key = seed ^ ((4ull * epoch + r + 1ull) * 0x9e3779b97f4a7c15ull);
        const unsigned long long t = L ^ (mix64(key ^ R) & mask);
        L = R;
        R = t;
    }
    return (L << half) | R;
}

// Rows perm(pos0 + i), i < b, of X [n][1056] BF16 and lab [n][16] into Xb, Lb:
// a wave per row (132 + 4 sixteen-byte pieces).
__global__ __launch_bounds__(256) void k_gather_rows(const uint4* X, const uint4* lab, long n, int half,
                                                     unsigned long long seed, unsigned long long epoch,
                                                     long pos0, int b, uint4* Xb, uint4* Lb)
{
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= b) return;
    unsigned long long r = (unsigned long long)(pos0 + i);
    do {
        r = feistel(r, half, seed, epoch);
    } while (r >= (unsigned long long)n);
    constexpr int kRowX = kSurIn * 2 / 16, kRowL = kSurOut * 4 / 16;
    for (int c = lane; c < kRowX; c += 64) Xb[(long)i * kRowX + c] = X[(long)r * kRowX + c];
    if (lane < kRowL) Lb[(long)i * kRowL + lane] = lab[(long)r * kRowL + lane];
}

__global__ void k_to_bf16(const float* x, uint16_t* y, long n)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = to_bf16(x[i]);
}

// BF16 operand copies transposed to [out][in] (inputs contiguous) for the
// fused inference kernel.
__global__ void k_transpose_bf16(const uint16_t* W, int in, int out, uint16_t* Wt)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)in * out) return;
    const int k = (int)(i / out), n = (int)(i % out);
    Wt[(long)n * in + k] = W[i];
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16v4 __attribute__((ext_vector_type(4)));

// Fused inference with the activations in registers.  The weights are the
// MFMA's A operand (a tile of 16 output features) and the beams its B operand
// (16 rows), so a wave holds all 256 features of its 16 beams.  The output of
// v_mfma_f32_16x16x32_bf16 (lane l: features 4 (l / 16) .. + 3 of row l % 16)
// is the next layer's B operand as it stands once both operands of a K step
// of 32 take the features in the same order: lane quad q and element e stand
// for feature 32 s + 4 q + e (e < 4) or 32 s + 16 + 4 q + (e - 4).  The first
// layer reads its inputs in natural order (8 q + e).  Weight tiles (256 x 32)
// are staged in double-buffered LDS, shared by the workgroup's 8 waves (128
// beams); the tiles of step k + 2 are loaded while step k's MFMAs run.
constexpr int kInfWaves = 8;
constexpr int kInfRows = 16 * kInfWaves;     // rows (beams) per workgroup
constexpr int kInfThreads = 64 * kInfWaves;
constexpr int kInfK = 32;                    // K step
constexpr int kInfLdsK = kInfK + 8;          // staged row stride (elements)
constexpr int kInfAhead = 2;                 // K steps loaded ahead of their use

struct InferLds {
    uint16_t Bs[2][kSurHid][kInfLdsK];       // weight tiles [out][k]
};

__device__ inline bf16x8 ld8(const uint16_t* p) { return *(const bf16x8*)p; }

// the workgroup's share of one weight tile: 1024 chunks of 8 elements,
// kStage per thread (chunk c: row c / 4, elements 8 (c % 4) .. + 7)
constexpr int kStage = 4 * kSurHid / kInfThreads;
__device__ inline void stage_load(const uint16_t* Wt, int K, int k0, int tid, bf16x8 (&r)[kStage])
{
#pragma unroll
    for (int c = 0; c < kStage; ++c) {
        const int q = tid + kInfThreads * c;
        r[c] = ld8(Wt + (long)(q >> 2) * K + k0 + 8 * (q & 3));
    }
}

__device__ inline void stage_store(InferLds& L, int buf, int tid, const bf16x8 (&r)[kStage])
{
#pragma unroll
    for (int c = 0; c < kStage; ++c) {
        const int q = tid + kInfThreads * c;
        *(bf16x8*)&L.Bs[buf][q >> 2][8 * (q & 3)] = r[c];
    }
}

// A fragment of tile t in the permuted order (hidden layers)
__device__ inline bf16x8 frag_perm(const InferLds& L, int buf, int t, int l16, int q)
{
    const bf16v4 lo = *(const bf16v4*)&L.Bs[buf][16 * t + l16][4 * q];
    const bf16v4 hi = *(const bf16v4*)&L.Bs[buf][16 * t + l16][16 + 4 * q];
    return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

__device__ inline __bf16 bf(float x) { return __builtin_bit_cast(__bf16, to_bf16(x)); }

// bias + GELU of the wave's 16 x 256 block into B fragments of the next layer
__device__ inline void to_frags(const f32x4 (&acc)[16], const float* bias, int q, bf16x8 (&h)[8])
{
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const float4 b0 = *(const float4*)(bias + 32 * s + 4 * q);
        const float4 b1 = *(const float4*)(bias + 32 * s + 16 + 4 * q);
        const f32x4 x0 = acc[2 * s], x1 = acc[2 * s + 1];
        h[s] = bf16x8{bf(gelu(x0[0] + b0.x)), bf(gelu(x0[1] + b0.y)), bf(gelu(x0[2] + b0.z)),
                      bf(gelu(x0[3] + b0.w)), bf(gelu(x1[0] + b1.x)), bf(gelu(x1[1] + b1.y)),
                      bf(gelu(x1[2] + b1.z)), bf(gelu(x1[3] + b1.w))};
    }
}

// First layer: acc = W1 x over the 1056 inputs (B fragments straight from X).
__device__ inline void layer_first(const uint16_t* X, long row, long n, InferLds& L,
                                   const uint16_t* Wt, f32x4 (&acc)[16])
{
    const int tid = threadIdx.x, lane = tid & 63, l16 = lane & 15, q = lane >> 4;
    constexpr int S = kSurIn / kInfK;
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8 rb[kInfAhead][kStage], xb[kInfAhead];
    auto xload = [&](int st) { return row < n ? ld8(X + row * kSurIn + st * kInfK + 8 * q) : bf16x8{}; };
#pragma unroll
    for (int u = 0; u < kInfAhead; ++u) {
        stage_load(Wt, kSurIn, u * kInfK, tid, rb[u]);
        xb[u] = xload(u);
    }
    stage_store(L, 0, tid, rb[0]);
    __syncthreads();
    for (int st0 = 0; st0 < S; st0 += kInfAhead) {
#pragma unroll
        for (int u = 0; u < kInfAhead; ++u) {
            const int st = st0 + u;                      // ring slot u
            if (st >= S) break;
            const int buf = st & 1;
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const bf16x8 a = *(const bf16x8*)&L.Bs[buf][16 * t + l16][8 * q];
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, xb[u], acc[t], 0, 0, 0);
            }
            const int un = (u + 1) % kInfAhead;
            if (st + 1 < S) stage_store(L, buf ^ 1, tid, rb[un]);
            if (st + kInfAhead < S) {
                stage_load(Wt, kSurIn, (st + kInfAhead) * kInfK, tid, rb[u]);
                xb[u] = xload(st + kInfAhead);
            }
            __syncthreads();
        }
    }
}

// Hidden layer: acc = W h over 256 inputs held as B fragments.
__device__ inline void layer_hidden(const bf16x8 (&h)[8], InferLds& L, const uint16_t* Wt,
                                    f32x4 (&acc)[16])
{
    const int tid = threadIdx.x, lane = tid & 63, l16 = lane & 15, q = lane >> 4;
    constexpr int S = kSurHid / kInfK;
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8 rb[kInfAhead][kStage];
#pragma unroll
    for (int u = 0; u < kInfAhead; ++u) stage_load(Wt, kSurHid, u * kInfK, tid, rb[u]);
    stage_store(L, 0, tid, rb[0]);
    __syncthreads();
#pragma unroll
    for (int st = 0; st < S; ++st) {
        const int buf = st & 1, u = st % kInfAhead;
#pragma unroll
        for (int t = 0; t < 16; ++t)
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag_perm(L, buf, t, l16, q), h[st],
                                                             acc[t], 0, 0, 0);
        if (st + 1 < S) stage_store(L, buf ^ 1, tid, rb[(u + 1) % kInfAhead]);
        if (st + kInfAhead < S) stage_load(Wt, kSurHid, (st + kInfAhead) * kInfK, tid, rb[u]);
        __syncthreads();
    }
}

// The whole network for 128 rows per workgroup, 16 per wave.
__global__ __launch_bounds__(kInfThreads) void k_mlp_infer(InferArgs a)
{
    extern __shared__ float4 lds_v4[];
    InferLds& L = *(InferLds*)lds_v4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, q = lane >> 4;
    const long row = (long)blockIdx.x * kInfRows + 16 * wave + l16;
    f32x4 acc[16];
    bf16x8 h[8];
    layer_first(a.X, row, a.n, L, a.Wt1, acc);
    to_frags(acc, a.b1, q, h);
    layer_hidden(h, L, a.Wt2, acc);
    to_frags(acc, a.b2, q, h);
    layer_hidden(h, L, a.Wt3, acc);
    to_frags(acc, a.b3, q, h);
    // output layer: one tile of 16 outputs, weights read directly (8 KB)
    f32x4 y = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const uint16_t* w = a.Wt4 + (long)l16 * kSurHid + 32 * s;
        const bf16v4 lo = *(const bf16v4*)(w + 4 * q), hi = *(const bf16v4*)(w + 16 + 4 * q);
        y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7),
                                                    h[s], y, 0, 0, 0);
    }
    if (row < a.n) {
        const float4 b4 = *(const float4*)(a.b4 + 4 * q);
        *(float4*)(a.Y + row * kSurOut + 4 * q) = make_float4(y[0] + b4.x, y[1] + b4.y, y[2] + b4.z,
                                                              y[3] + b4.w);
    }
}

inline unsigned blocks(long n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_transpose_weights(hipStream_t s, const uint16_t* theta_b, uint16_t* wt)
{
    struct L { long off, toff; int in, out; };
    const L ls[4] = {{kSurOffW1, 0, kSurIn, kSurHid},
                     {kSurOffW2, (long)kSurIn * kSurHid, kSurHid, kSurHid},
                     {kSurOffW3, (long)kSurIn * kSurHid + (long)kSurHid * kSurHid, kSurHid, kSurHid},
                     {kSurOffW4, (long)kSurIn * kSurHid + 2L * kSurHid * kSurHid, kSurHid, kSurOut}};
    for (const L& l : ls) {
        const long n = (long)l.in * l.out;
        hipLaunchKernelGGL(k_transpose_bf16, dim3(blocks(n, 256)), dim3(256), 0, s, theta_b + l.off,
                           l.in, l.out, wt + l.toff);
    }
    return hipGetLastError();
}

hipError_t launch_mlp_infer(hipStream_t s, const InferArgs& a)
{
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_infer, dim3(blocks(a.n, kInfRows)), dim3(kInfThreads), sizeof(InferLds), s,
                       a);
    return hipGetLastError();
}

hipError_t launch_gemm_bf16(hipStream_t s, const GemmArgs& g0, bool det)
{
    if (g0.M <= 0 || g0.N <= 0) return hipSuccess;
    GemmArgs g = g0;
    const long tiles = (long)((g.N + kTileN - 1) / kTileN) * ((g.M + kTileM - 1) / kTileM);
    // few output tiles and a long K (weight gradients): split K over the grid
    // (not when deterministic: the atomic adds of the parts come in any order)
    g.ksplit = 1;
    while (!det && tiles * g.ksplit < 512 && g.K / (g.ksplit * 2) >= 4 * kTileK) g.ksplit *= 2;
    if (g.ksplit > 1) {
        if (g.ldc != g.N) return hipErrorInvalidValue;   // split K needs a dense C to zero
        const hipError_t e = launch_zero_f32(s, g.C, (long)g.M * g.N);
        if (e != hipSuccess) return e;
    }
    dim3 grid((g.N + kTileN - 1) / kTileN, (g.M + kTileM - 1) / kTileM, g.ksplit);
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_bias_gelu(hipStream_t s, float* Z, const float* bias, uint16_t* H, long n, int C)
{
    if (n * C == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bias_gelu, dim3(blocks(n * C, 256)), dim3(256), 0, s, Z, bias, H, n, C);
    return hipGetLastError();
}

hipError_t launch_bias(hipStream_t s, float* Y, const float* bias, long n, int C)
{
    if (n * C == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bias, dim3(blocks(n * C, 256)), dim3(256), 0, s, Y, bias, n, C);
    return hipGetLastError();
}

hipError_t launch_loss(hipStream_t s, const float* Y, const float* lab, long n, uint16_t* dYb,
                       float* loss_sum)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_loss, dim3(blocks(n, 256)), dim3(256), 0, s, Y, lab, n, 1.0f / (float)n,
                       dYb, loss_sum);
    return hipGetLastError();
}

hipError_t launch_gelu_back(hipStream_t s, const float* dH, const float* Z, uint16_t* dZb, long count)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gelu_back, dim3(blocks(count, 256)), dim3(256), 0, s, dH, Z, dZb, count);
    return hipGetLastError();
}

hipError_t launch_colsum(hipStream_t s, const uint16_t* D, long n, int C, float* out, bool det)
{
    hipError_t e = launch_zero_f32(s, out, C);
    if (e != hipSuccess || n == 0) return e;
    const long span = det ? n : 256;
    hipLaunchKernelGGL(k_colsum, dim3(blocks(C, 64), (unsigned)((n + span - 1) / span)), dim3(256), 0, s,
                       D, n, C, span, out);
    return hipGetLastError();
}

hipError_t launch_gather_rows(hipStream_t s, const uint16_t* X, const float* lab, long n, int half,
                              unsigned long long seed, unsigned long long epoch, long pos0, int b,
                              uint16_t* Xb, float* Lb)
{
    if (b <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_rows, dim3((b + 3) / 4), dim3(256), 0, s, (const uint4*)X,
                       (const uint4*)lab, n, half, seed, epoch, pos0, b, (uint4*)Xb, (uint4*)Lb);
    return hipGetLastError();
}

hipError_t launch_zero_f32(hipStream_t s, float* p, long n)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_f32, dim3(blocks(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_adamw(hipStream_t s, float* theta, const float* grad, float* m, float* v,
                        uint16_t* theta_b, long n, const AdamArgs& a)
{
    hipLaunchKernelGGL(k_adamw, dim3(blocks(n, 256)), dim3(256), 0, s, theta, grad, m, v, theta_b, n, a);
    return hipGetLastError();
}

hipError_t launch_to_bf16(hipStream_t s, const float* x, uint16_t* y, long n)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks(n, 256)), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

}  // namespace lidar

namespace lidar {

hipError_t SurWork::ensure(long n)
{
    if (n <= cap) return hipSuccess;
    hipError_t e;
    const size_t nh = (size_t)n * kSurHid, no = (size_t)n * kSurOut;
    if ((e = Z1.ensure(nh)) || (e = Z2.ensure(nh)) || (e = Z3.ensure(nh)) || (e = dH.ensure(nh)) ||
        (e = H1.ensure(nh)) || (e = H2.ensure(nh)) || (e = H3.ensure(nh)) || (e = dZb.ensure(nh)) ||
        (e = Y.ensure(no)) || (e = dYb.ensure(no)) || (e = loss.ensure(1)))
        return e;
    cap = n;
    return hipSuccess;
}

#define TRY(x)                                        \
    do {                                              \
        hipError_t e_ = (x);                          \
        if (e_ != hipSuccess) return e_;              \
    } while (0)

// A training product: the library GEMM where it runs (not in the
// deterministic mode, whose products keep a fixed summation order), else the
// own MFMA kernel
static hipError_t gemm(hipStream_t s, const GemmArgs& g, bool det, BlasCtx* blas)
{
    if (!det && blas) {
        const hipError_t e = blas_gemm(blas, s, g);
        if (e != hipErrorNotSupported) return e;
    }
    return launch_gemm_bf16(s, g, det);
}

// Z = A W (+ bias, GELU) with A [n][k] row-major BF16 and W [k][c] BF16
static hipError_t dense(hipStream_t s, const uint16_t* A, int k, const uint16_t* W, int c, long n,
                        float* Z, bool det, BlasCtx* blas)
{
    GemmArgs g{A, k, 1, W, c, 1, Z, c, (int)n, c, k, 1};
    return gemm(s, g, det, blas);
}

hipError_t sur_forward(hipStream_t s, const SurNet& net, const uint16_t* X, long n, SurWork& w)
{
    const uint16_t* Wb = net.theta_b.p;
    const float* th = net.theta.p;
    TRY(dense(s, X, kSurIn, Wb + kSurOffW1, kSurHid, n, w.Z1.p, net.det, w.blas));
    TRY(launch_bias_gelu(s, w.Z1.p, th + kSurOffB1, w.H1.p, n, kSurHid));
    TRY(dense(s, w.H1.p, kSurHid, Wb + kSurOffW2, kSurHid, n, w.Z2.p, net.det, w.blas));
    TRY(launch_bias_gelu(s, w.Z2.p, th + kSurOffB2, w.H2.p, n, kSurHid));
    TRY(dense(s, w.H2.p, kSurHid, Wb + kSurOffW3, kSurHid, n, w.Z3.p, net.det, w.blas));
    TRY(launch_bias_gelu(s, w.Z3.p, th + kSurOffB3, w.H3.p, n, kSurHid));
    TRY(dense(s, w.H3.p, kSurHid, Wb + kSurOffW4, kSurOut, n, w.Y.p, net.det, w.blas));
    TRY(launch_bias(s, w.Y.p, th + kSurOffB4, n, kSurOut));
    return hipSuccess;
}

hipError_t sur_infer(hipStream_t s, SurNet& net, const uint16_t* X, long n, float* Y)
{
    TRY(net.theta_t.ensure(kSurWtSize));
    if (net.t_stale) {
        TRY(launch_transpose_weights(s, net.theta_b.p, net.theta_t.p));
        net.t_stale = false;
    }
    const uint16_t* t = net.theta_t.p;
    InferArgs a;
    a.X = X;
    a.n = n;
    a.Wt1 = t;
    a.Wt2 = t + (long)kSurIn * kSurHid;
    a.Wt3 = a.Wt2 + (long)kSurHid * kSurHid;
    a.Wt4 = a.Wt3 + (long)kSurHid * kSurHid;
    a.b1 = net.theta.p + kSurOffB1;
    a.b2 = net.theta.p + kSurOffB2;
    a.b3 = net.theta.p + kSurOffB3;
    a.b4 = net.theta.p + kSurOffB4;
    a.Y = Y;
    return launch_mlp_infer(s, a);
}

// dW = A^T D (A [n][in] BF16 activations, D [n][out] BF16), db = column sums
static hipError_t weight_grad(hipStream_t s, const uint16_t* A, int in, const uint16_t* D, int out,
                              long n, float* dW, float* db, bool det, BlasCtx* blas)
{
    GemmArgs g{A, 1, in, D, out, 1, dW, out, in, out, (int)n, 1};
    TRY(gemm(s, g, det, blas));
    return launch_colsum(s, D, n, out, db, det);
}

// dH = D W^T (D [n][out], W [in][out]) in FP32
static hipError_t input_grad(hipStream_t s, const uint16_t* D, int out, const uint16_t* W, int in,
                             long n, float* dH, bool det, BlasCtx* blas)
{
    GemmArgs g{D, out, 1, W, 1, out, dH, in, (int)n, in, out, 1};
    return gemm(s, g, det, blas);
}

hipError_t sur_gradients(hipStream_t s, SurNet& net, const uint16_t* X, const float* lab, long n,
                         SurWork& w)
{
    TRY(sur_forward(s, net, X, n, w));
    TRY(launch_loss(s, w.Y.p, lab, n, w.dYb.p, w.loss.p));
    const uint16_t* Wb = net.theta_b.p;
    float* g = net.grad.p;
    const long nh = n * kSurHid;
    // layer 4
    TRY(weight_grad(s, w.H3.p, kSurHid, w.dYb.p, kSurOut, n, g + kSurOffW4, g + kSurOffB4, net.det, w.blas));
    TRY(input_grad(s, w.dYb.p, kSurOut, Wb + kSurOffW4, kSurHid, n, w.dH.p, net.det, w.blas));
    TRY(launch_gelu_back(s, w.dH.p, w.Z3.p, w.dZb.p, nh));
    // layer 3
    TRY(weight_grad(s, w.H2.p, kSurHid, w.dZb.p, kSurHid, n, g + kSurOffW3, g + kSurOffB3, net.det, w.blas));
    TRY(input_grad(s, w.dZb.p, kSurHid, Wb + kSurOffW3, kSurHid, n, w.dH.p, net.det, w.blas));
    TRY(launch_gelu_back(s, w.dH.p, w.Z2.p, w.dZb.p, nh));
    // layer 2
    TRY(weight_grad(s, w.H1.p, kSurHid, w.dZb.p, kSurHid, n, g + kSurOffW2, g + kSurOffB2, net.det, w.blas));
    TRY(input_grad(s, w.dZb.p, kSurHid, Wb + kSurOffW2, kSurHid, n, w.dH.p, net.det, w.blas));
    TRY(launch_gelu_back(s, w.dH.p, w.Z1.p, w.dZb.p, nh));
    // layer 1
    TRY(weight_grad(s, X, kSurIn, w.dZb.p, kSurHid, n, g + kSurOffW1, g + kSurOffB1, net.det, w.blas));
    return hipSuccess;
}

#undef TRY

}  // namespace lidar
