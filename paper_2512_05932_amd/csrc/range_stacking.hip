// Range stacking (section II-C, Alg. 2) with a separable kernel
// kappa*eta = H * V: the rendered intensities are split into depth slices
// (time bins); every slice is correlated with the kernel, separably (a pass
// along the rows with H, then along the columns with V); each pixel keeps
// the nearest slice whose correlation reaches rho_min and that value.
//
// Work decomposition: one workgroup per output tile of kTileC x kTileR
// pixels.  It first marks in an LDS bitmap the slices present in the tile's
// input window (tile plus the kernel's half extents) that can reach rho_min
// at all (slice skipping: the largest shade of a slice in the image times
// sum H times sum V bounds every correlation of that slice), and in one
// bitmap per window row the slices the row holds; then it visits the slices
// from the nearest on: the window rows that hold the slice are staged in LDS
// eight at a time (masked to it) and correlated with H into a column buffer
// (other rows are zero), which is correlated with V at the tile's pixels over
// the slice's rows; a pixel takes the first slice that reaches rho_min, and
// the tile stops once every pixel has one.
#include <climits>

#include "engine.h"

namespace lidar {

namespace {

constexpr int kTileC = 32, kTileR = 16;       // output tile: columns x rows
constexpr int kThreads = 256;
constexpr int kStageRows = kThreads / kTileC;  // window rows correlated per step
constexpr int kMaxHalf = kRsMaxHalf;           // M, N <= 127
constexpr int kMaxWords = (kMaxBins + 31) / 32;

static_assert(kTileC * kStageRows == kThreads && kTileC * kTileR == 2 * kThreads,
              "a thread per staged output, two tile pixels per thread");

// Largest shade of every slice (time bin) over the image: FP32 bits of
// non-negative values compare as integers.
__global__ void k_rs_slice_max(const int2* pix, long n, int R, int* smax)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int2 rec = pix[i];
    if (rec.x >= 0 && rec.x < R && rec.y > 0) atomicMax(smax + rec.x, rec.y);
}

__global__ void k_rs_clear(int* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Record of image pixel (u, v) in the 4-column blocks of the pre-pass.
__device__ inline int2 record(const RangeStackArgs& a, int u, int v)
{
    return a.pix[(((long)(u >> 2) * a.H + v) << 2) + (u & 3)];
}

// Dynamic LDS of a workgroup: the column buffer [rows][kTileC], the staged
// rows [kStageRows][scols] and, when it fits (use_bits), the slices present in
// every window row [rows][words] (bit s of row r: the row holds a pixel of
// slice s), so that a slice stages and correlates only its own rows.
constexpr long kRsDynMax = 56 * 1024;         // dynamic LDS with the row bitmaps at most

struct RsLayout {
    int rows, scols, words;
    bool use_bits;
};

__host__ __device__ inline RsLayout rs_layout(int M, int N, int R)
{
    RsLayout l;
    l.rows = kTileR + 2 * N;
    l.scols = kTileC + 2 * M;
    l.words = (R + 31) / 32;
    const long base = 4L * ((long)l.rows * kTileC + (long)kStageRows * l.scols);
    l.use_bits = base + 4L * l.rows * l.words <= kRsDynMax;
    return l;
}

__host__ __device__ inline size_t rs_lds_bytes(const RsLayout& l)
{
    return sizeof(float) * ((size_t)l.rows * kTileC + (size_t)kStageRows * l.scols) +
           (l.use_bits ? sizeof(unsigned) * (size_t)l.rows * l.words : 0);
}

__global__ __launch_bounds__(kThreads)
void k_range_stacking(RangeStackArgs a)
{
    __shared__ float hk[2 * kMaxHalf + 1], vk[2 * kMaxHalf + 1];
    __shared__ unsigned present[kMaxWords];
    __shared__ int rowany[kStageRows];                 // a staged row holds a pixel of the slice
    __shared__ int rlo, rhi;                           // the slice's first and last window rows
    __shared__ int open_count;
    extern __shared__ float4 rs_dyn[];
    const int tid = threadIdx.x;
    const int u0 = blockIdx.x * kTileC, v0 = blockIdx.y * kTileR;
    const int M = a.M, N = a.N, KW = 2 * M + 1, KH = 2 * N + 1;
    const RsLayout ly = rs_layout(M, N, a.R);
    const int rows = ly.rows, scols = ly.scols, words = ly.words;
    float* colbuf = (float*)rs_dyn;                    // [rows][kTileC]
    float* stage = colbuf + rows * kTileC;             // [kStageRows][scols]
    unsigned* rowbits = (unsigned*)(stage + kStageRows * scols);   // [rows][words] (use_bits)
    for (int i = tid; i < KW; i += kThreads) hk[i] = a.hk[i];
    for (int i = tid; i < KH; i += kThreads) vk[i] = a.vk[i];
    for (int i = tid; i < words; i += kThreads) present[i] = 0u;
    if (ly.use_bits)
        for (int i = tid; i < rows * words; i += kThreads) rowbits[i] = 0u;
    if (tid == 0) open_count = 0;
    __syncthreads();
    // slices present in the window that can reach rho_min (and, per window
    // row, every slice it holds)
    const int wr0 = max(0, v0 - N), wr1 = min(a.H - 1, v0 + kTileR - 1 + N);
    const int wc0 = max(0, u0 - M), wc1 = min(a.W - 1, u0 + kTileC - 1 + M);
    const int wcols = wc1 - wc0 + 1, wrows = wr1 - wr0 + 1;
    for (int i = tid; i < wcols * wrows; i += kThreads) {
        const int v = wr0 + i / wcols, u = wc0 + i % wcols;
        const int2 rec = record(a, u, v);
        if (rec.x >= 0 && rec.x < a.R && rec.y > 0) {
            if (ly.use_bits) atomicOr(&rowbits[(v - (v0 - N)) * words + (rec.x >> 5)], 1u << (rec.x & 31));
            if (__int_as_float(a.smax[rec.x]) * a.bound >= a.rho_min)
                atomicOr(&present[rec.x >> 5], 1u << (rec.x & 31));
        }
    }
    // this thread's two tile pixels: column tc, rows tr and tr + kTileR / 2
    const int tc = tid % kTileC, tr = tid / kTileC;
    int best[2] = {a.R, a.R};
    float bval[2] = {0.0f, 0.0f};
    const bool mine[2] = {u0 + tc < a.W && v0 + tr < a.H, u0 + tc < a.W && v0 + tr + kTileR / 2 < a.H};
    if (mine[0] || mine[1]) atomicAdd(&open_count, (int)mine[0] + (int)mine[1]);
    __syncthreads();
    const int srow = tid / kTileC, scol = tid % kTileC;       // staged output of this thread
    for (int w = 0; w < words; ++w) {
        unsigned bits = present[w];
        while (bits) {
            if (open_count == 0) break;                          // uniform (read after a barrier)
            const int s = w * 32 + __builtin_ctz(bits);
            bits &= bits - 1u;
            // whether window row wr can hold a pixel of slice s
            auto holds = [&](int wr) {
                return wr < rows && (!ly.use_bits || ((rowbits[wr * words + w] >> (s & 31)) & 1u));
            };
            // rows with H: window rows v0 - N .. v0 + kTileR - 1 + N, eight at a time
            if (tid == 0) {
                rlo = INT_MAX;
                rhi = -1;
            }
            for (int r0 = 0; r0 < rows; r0 += kStageRows) {
                // a step whose rows hold no pixel of s only zeroes its
                // column-buffer rows (uniform)
                bool any = false;
#pragma unroll
                for (int rr = 0; rr < kStageRows; ++rr) any |= holds(r0 + rr);
                if (!any) {
                    if (r0 + srow < rows) colbuf[(r0 + srow) * kTileC + scol] = 0.0f;
                    continue;
                }
                if (tid < kStageRows) rowany[tid] = 0;
                __syncthreads();
                for (int i = tid; i < kStageRows * scols; i += kThreads) {
                    const int rr = i / scols, cc = i % scols;
                    const int v = v0 - N + r0 + rr, u = u0 - M + cc;
                    float x = 0.0f;
                    if (holds(r0 + rr) && v >= 0 && v < a.H && u >= 0 && u < a.W) {
                        const int2 rec = record(a, u, v);
                        if (rec.x == s) x = __int_as_float(rec.y);
                    }
                    stage[rr * scols + cc] = x;
                    if (x != 0.0f) rowany[rr] = 1;
                }
                __syncthreads();
                // the correlation of a row without a pixel of s is zero
                if (r0 + srow < rows) {
                    float acc = 0.0f;
                    if (rowany[srow]) {
                        const float* st = stage + srow * scols + scol;
                        for (int m = 0; m < KW; ++m) acc += hk[m] * st[m];
                    }
                    colbuf[(r0 + srow) * kTileC + scol] = acc;
                }
                if (tid < kStageRows && rowany[tid]) {
                    atomicMin(&rlo, r0 + tid);
                    atomicMax(&rhi, r0 + tid);
                }
                __syncthreads();
            }
            __syncthreads();                             // the zeroed rows of skipped steps
            // only the window rows rlo .. rhi hold the slice: the other
            // terms of the column correlation are zero
            const int wlo = rlo, whi = rhi;
            // columns with V at the tile's pixels; the first slice that
            // reaches rho_min is the pixel's nearest
            int closed = 0;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int r = tr + k * (kTileR / 2);
                if (!mine[k] || best[k] < a.R) continue;
                float acc = 0.0f;
                const int n0 = max(0, wlo - r), n1 = min(KH - 1, whi - r);
                for (int n = n0; n <= n1; ++n) acc += vk[n] * colbuf[(r + n) * kTileC + tc];
                if (acc >= a.rho_min) {
                    best[k] = s;
                    bval[k] = acc;
                    ++closed;
                }
            }
            if (closed) atomicSub(&open_count, closed);
            __syncthreads();
        }
        if (open_count == 0) break;
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (!mine[k]) continue;
        const long o = (long)(v0 + tr + k * (kTileR / 2)) * a.W + (u0 + tc);
        a.s_nearest[o] = best[k];
        a.xi_nearest[o] = bval[k];
    }
}

}  // namespace

hipError_t launch_range_stacking(hipStream_t s, const RangeStackArgs& a, int* smax_scratch)
{
    if (a.M > kMaxHalf || a.N > kMaxHalf || a.R > kMaxBins) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rs_clear, dim3((a.R + 255) / 256), dim3(256), 0, s, smax_scratch, a.R);
    const long n = (long)a.W4 * a.H;
    hipLaunchKernelGGL(k_rs_slice_max, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a.pix, n,
                       a.R, smax_scratch);
    RangeStackArgs b = a;
    b.smax = smax_scratch;
    dim3 grid((a.W + kTileC - 1) / kTileC, (a.H + kTileR - 1) / kTileR);
    const size_t lds = rs_lds_bytes(rs_layout(a.M, a.N, a.R));
    hipLaunchKernelGGL(k_range_stacking, grid, dim3(kThreads), lds, s, b);
    return hipGetLastError();
}

}  // namespace lidar
