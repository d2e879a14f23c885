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
// columns x 256 rows (lane = column, wave = every 4th row), sums its waves in
// LDS and adds into the zeroed output
__global__ __launch_bounds__(256) void k_colsum(const uint16_t* D, long n, int C, float* out)
{
    __shared__ float part[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    const long r0 = (long)blockIdx.y * 256;
    float s = 0.0f;
    if (j < C)
        for (long r = r0 + wave; r < min(n, r0 + 256); r += 4) s += from_bf16(D[r * C + j]);
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

// Fused inference: 128 rows (beams) per workgroup of 4 waves; wave w computes
// rows 64 (w / 2) .. + 63 and output columns 128 (w % 2) .. + 127 of every
// hidden layer as 4 x 8 tiles of v_mfma_f32_16x16x32_bf16.  Per K step of 32
// the weight tile (256 x 32) and, in the first layer, the input tile
// (128 x 32) are staged in LDS, double buffered: the next step's tiles are
// loaded into registers while the current step's MFMAs run, so one barrier
// per step remains.  Activations stay in LDS between layers.
constexpr int kInfRows = 128;                // rows (beams) per workgroup
constexpr int kInfK = 32;                    // K step
constexpr int kInfLdsK = kInfK + 8;          // staged row stride (elements)
constexpr int kInfAhead = 3;                 // K steps loaded ahead of their use
constexpr int kInfH = kSurHid + 8;           // activation row stride (elements)

__device__ inline bf16x8 ld8(const uint16_t* p) { return *(const bf16x8*)p; }

struct InferLds {
    uint16_t H[kInfRows * kInfH];            // activations (BF16)
    uint16_t Bs[2][kSurHid][kInfLdsK];       // weight tiles [out][k]
    uint16_t As[2][kInfRows][kInfLdsK];      // input tiles of the first layer
};

// One hidden layer: acc = A W for the wave's 64 x 128 block, A = X (global,
// staged) or H (LDS), W^T given as Wt [256][K].  Ends with a barrier: every
// read of H is complete on return.
template <bool A_GLOBAL>
__device__ inline void infer_layer(const uint16_t* Ag, long row0, long n, InferLds& L,
                                   const uint16_t* Wt, int K, f32x4 (&acc)[4][8])
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1, l16 = lane & 15, kq = 8 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int S = K / kInfK;
    // register ring of kInfAhead steps: step k is loaded kInfAhead steps
    // before its tiles are consumed and one step before they are stored
    bf16x8 rb[kInfAhead][4], ra[kInfAhead][2];
    // 16-byte chunk q of a tile: row q / 4, elements 8 (q % 4) .. + 7
    auto load = [&](int st, bf16x8 (&b4)[4], bf16x8 (&a2)[2]) {
        const int k0 = st * kInfK;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int q = tid + 256 * c;
            b4[c] = ld8(Wt + (long)(q >> 2) * K + k0 + 8 * (q & 3));
        }
        if (A_GLOBAL) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int q = tid + 256 * c;
                const long row = row0 + (q >> 2);
                a2[c] = bf16x8{};
                if (row < n) a2[c] = ld8(Ag + row * kSurIn + k0 + 8 * (q & 3));
            }
        }
    };
    auto store = [&](int buf, const bf16x8 (&b4)[4], const bf16x8 (&a2)[2]) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int q = tid + 256 * c;
            *(bf16x8*)&L.Bs[buf][q >> 2][8 * (q & 3)] = b4[c];
        }
        if (A_GLOBAL) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int q = tid + 256 * c;
                *(bf16x8*)&L.As[buf][q >> 2][8 * (q & 3)] = a2[c];
            }
        }
    };
#pragma unroll
    for (int u = 0; u < kInfAhead; ++u)
        if (u < S) load(u, rb[u], ra[u]);
    store(0, rb[0], ra[0]);
    __syncthreads();
    for (int st0 = 0; st0 < S; st0 += kInfAhead) {
#pragma unroll
        for (int u = 0; u < kInfAhead; ++u) {
            const int st = st0 + u;                          // ring slot u
            if (st >= S) break;
            const int buf = st & 1;
            bf16x8 a[4], b[8];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 64 * wr + 16 * i + l16;
                a[i] = A_GLOBAL ? *(const bf16x8*)&L.As[buf][r][kq]
                                : *(const bf16x8*)&L.H[r * kInfH + st * kInfK + kq];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) b[j] = *(const bf16x8*)&L.Bs[buf][128 * wc + 16 * j + l16][kq];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            // the next step's tiles (slot u + 1) into the other buffer; slot u
            // is free again and takes step st + kInfAhead
            const int un = (u + 1) % kInfAhead;
            if (st + 1 < S) store(buf ^ 1, rb[un], ra[un]);
            if (st + kInfAhead < S) load(st + kInfAhead, rb[u], ra[u]);
            __syncthreads();
        }
    }
}

// bias + GELU of the wave's block into H (BF16)
__device__ inline void infer_store(const f32x4 (&acc)[4][8], const float* bias, uint16_t* H)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave >> 1, wc = wave & 1;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int col = 128 * wc + 16 * j + (lane & 15);
        const float bc = bias[col];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 64 * wr + 16 * i + 4 * (lane >> 4) + r;
                H[row * kInfH + col] = to_bf16(gelu(acc[i][j][r] + bc));
            }
    }
}

// The whole network for 128 rows per workgroup.
__global__ __launch_bounds__(256) void k_mlp_infer(InferArgs a)
{
    extern __shared__ float4 lds_v4[];
    InferLds& L = *(InferLds*)lds_v4;
    const long row0 = (long)blockIdx.x * kInfRows;
    f32x4 acc[4][8];
    infer_layer<true>(a.X, row0, a.n, L, a.Wt1, kSurIn, acc);
    infer_store(acc, a.b1, L.H);
    infer_layer<false>(nullptr, row0, a.n, L, a.Wt2, kSurHid, acc);
    infer_store(acc, a.b2, L.H);
    infer_layer<false>(nullptr, row0, a.n, L, a.Wt3, kSurHid, acc);
    infer_store(acc, a.b3, L.H);
    __syncthreads();
    // output layer: wave w takes rows 32 w .. 32 w + 31, all 16 outputs
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = 8 * (lane >> 4);
    f32x4 y[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
    for (int k0 = 0; k0 < kSurHid; k0 += kInfK) {
        const bf16x8 bv = ld8(a.Wt4 + (long)(lane & 15) * kSurHid + k0 + kq);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const bf16x8 av = *(const bf16x8*)&L.H[(wave * 32 + 16 * i + (lane & 15)) * kInfH + k0 + kq];
            y[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, y[i], 0, 0, 0);
        }
    }
    const int col = lane & 15;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long row = row0 + wave * 32 + 16 * i + 4 * (lane >> 4) + r;
            if (row < a.n) a.Y[row * kSurOut + col] = y[i][r] + a.b4[col];
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
    // more than 64 KiB of dynamic LDS: allowed up to the device's per-block limit
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_mlp_infer,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)sizeof(InferLds));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(k_mlp_infer, dim3(blocks(a.n, kInfRows)), dim3(256), sizeof(InferLds), s, a);
    return hipGetLastError();
}

hipError_t launch_gemm_bf16(hipStream_t s, const GemmArgs& g0)
{
    if (g0.M <= 0 || g0.N <= 0) return hipSuccess;
    GemmArgs g = g0;
    const long tiles = (long)((g.N + kTileN - 1) / kTileN) * ((g.M + kTileM - 1) / kTileM);
    // few output tiles and a long K (weight gradients): split K over the grid
    g.ksplit = 1;
    while (tiles * g.ksplit < 512 && g.K / (g.ksplit * 2) >= 4 * kTileK) g.ksplit *= 2;
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

hipError_t launch_colsum(hipStream_t s, const uint16_t* D, long n, int C, float* out)
{
    hipError_t e = launch_zero_f32(s, out, C);
    if (e != hipSuccess || n == 0) return e;
    hipLaunchKernelGGL(k_colsum, dim3(blocks(C, 64), blocks(n, 256)), dim3(256), 0, s, D, n, C, out);
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

// Z = A W (+ bias, GELU) with A [n][k] row-major BF16 and W [k][c] BF16
static hipError_t dense(hipStream_t s, const uint16_t* A, int k, const uint16_t* W, int c, long n,
                        float* Z)
{
    GemmArgs g{A, k, 1, W, c, 1, Z, c, (int)n, c, k, 1};
    return launch_gemm_bf16(s, g);
}

hipError_t sur_forward(hipStream_t s, const SurNet& net, const uint16_t* X, long n, SurWork& w)
{
    const uint16_t* Wb = net.theta_b.p;
    const float* th = net.theta.p;
    TRY(dense(s, X, kSurIn, Wb + kSurOffW1, kSurHid, n, w.Z1.p));
    TRY(launch_bias_gelu(s, w.Z1.p, th + kSurOffB1, w.H1.p, n, kSurHid));
    TRY(dense(s, w.H1.p, kSurHid, Wb + kSurOffW2, kSurHid, n, w.Z2.p));
    TRY(launch_bias_gelu(s, w.Z2.p, th + kSurOffB2, w.H2.p, n, kSurHid));
    TRY(dense(s, w.H2.p, kSurHid, Wb + kSurOffW3, kSurHid, n, w.Z3.p));
    TRY(launch_bias_gelu(s, w.Z3.p, th + kSurOffB3, w.H3.p, n, kSurHid));
    TRY(dense(s, w.H3.p, kSurHid, Wb + kSurOffW4, kSurOut, n, w.Y.p));
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
                              long n, float* dW, float* db)
{
    GemmArgs g{A, 1, in, D, out, 1, dW, out, in, out, (int)n, 1};
    TRY(launch_gemm_bf16(s, g));
    return launch_colsum(s, D, n, out, db);
}

// dH = D W^T (D [n][out], W [in][out]) in FP32
static hipError_t input_grad(hipStream_t s, const uint16_t* D, int out, const uint16_t* W, int in,
                             long n, float* dH)
{
    GemmArgs g{D, out, 1, W, 1, out, dH, in, (int)n, in, out, 1};
    return launch_gemm_bf16(s, g);
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
    TRY(weight_grad(s, w.H3.p, kSurHid, w.dYb.p, kSurOut, n, g + kSurOffW4, g + kSurOffB4));
    TRY(input_grad(s, w.dYb.p, kSurOut, Wb + kSurOffW4, kSurHid, n, w.dH.p));
    TRY(launch_gelu_back(s, w.dH.p, w.Z3.p, w.dZb.p, nh));
    // layer 3
    TRY(weight_grad(s, w.H2.p, kSurHid, w.dZb.p, kSurHid, n, g + kSurOffW3, g + kSurOffB3));
    TRY(input_grad(s, w.dZb.p, kSurHid, Wb + kSurOffW3, kSurHid, n, w.dH.p));
    TRY(launch_gelu_back(s, w.dH.p, w.Z2.p, w.dZb.p, nh));
    // layer 2
    TRY(weight_grad(s, w.H1.p, kSurHid, w.dZb.p, kSurHid, n, g + kSurOffW2, g + kSurOffB2));
    TRY(input_grad(s, w.dZb.p, kSurHid, Wb + kSurOffW2, kSurHid, n, w.dH.p));
    TRY(launch_gelu_back(s, w.dH.p, w.Z1.p, w.dZb.p, nh));
    // layer 1
    TRY(weight_grad(s, X, kSurIn, w.dZb.p, kSurHid, n, g + kSurOffW1, g + kSurOffB1));
    return hipSuccess;
}

#undef TRY

}  // namespace lidar
