// Per-frame G-buffer pre-pass.
//
// Everything in the footprint weight that depends on the pixel alone is
// folded into one FP32 shade per pixel (Eq. 4: rho_hat = beta cos(theta)/d^2
// for a unit isotropic source at the sensor, times the pixel solid angle of
// Eq. 2), and the pixel's time bin k = floor(2 d / (c dt)) (the Dirac delta
// of Eq. 3) is taken once per pixel in FP64.  Sky, non-finite or
// non-positive depths and ranges beyond the last bin get bin -1 and zero
// shade.  The records are written in blocks of 4 columns ([u/4][v][u%4]) so
// that a footprint-kernel lane, which owns one row, reads 4 consecutive
// columns of its row with one 16-byte access, and the 64 lanes of a wave
// (64 consecutive rows) read one contiguous span; the transpose goes through
// a 64x16 LDS tile.  Columns between W and the next multiple of 4 are sky.
#include "engine.h"

namespace lidar {

namespace {
constexpr int kTileW = 64, kTileH = 16;   // tile of kTileW columns x kTileH rows (256-byte row reads)
constexpr int kThreads = 256;
constexpr int kRowsPerPass = kThreads / kTileW;
static_assert(kTileW % 4 == 0 && kTileH % kRowsPerPass == 0, "whole 4-column blocks and passes");
}

// One kTileW x kTileH tile of a frame, columns u0.., rows v0...
template <bool SUN>
__device__ inline void prepass_tile(const PrepassArgs& a, int u0, int v0)
{
    __shared__ int2 trec[kTileH][kTileW + 1];
    __shared__ float tsun[kTileH][kTileW + 1];
    const int tx = threadIdx.x % kTileW, ty = threadIdx.x / kTileW;
    const float inv_pi = (float)(1.0 / kPi);
    // read rows (coalesced along u), shade, stage in LDS
#pragma unroll
    for (int p = 0; p < kTileH / kRowsPerPass; ++p) {
        int vl = ty + p * kRowsPerPass;
        int u = u0 + tx, v = v0 + vl;
        int bin = -1;
        float shade = 0.0f, sunv = 0.0f;
        if (u < a.W && v < a.H) {
            long px = (long)v * a.pitch + u;
            float d = a.depth[px];
            if (d > 0.0f && isfinite(d)) {
                double kb = floor((double)d * a.to_bin);
                if (kb < (double)a.R) {
                    bin = (int)kb;
                    float2 cs = a.colcs[u];
                    float4 rt = a.rowtab[v];
                    float vx = rt.x * cs.x, vy = rt.x * cs.y, vz = rt.y;
                    float nx = a.nx[px], ny = a.ny[px], nz = a.nz[px];
                    float ct = fmaxf(0.0f, -(nx * vx + ny * vy + nz * vz));
                    float rho = a.refl[px];
                    float g = a.gain[px];
                    shade = rt.z * (g * rho * inv_pi) * ct / (d * d);
                    if (SUN) {
                        float ns = fmaxf(0.0f, nx * a.sun_x + ny * a.sun_y + nz * a.sun_z);
                        sunv = rt.z * (rho * inv_pi) * ns;
                    }
                }
            }
        }
        trec[vl][tx] = make_int2(bin, __float_as_int(shade));
        if (SUN) tsun[vl][tx] = sunv;
    }
    __syncthreads();
    // write kTileW / 4 blocks of 4 columns x kTileH rows, each contiguous in memory
    const int tid = threadIdx.x;
#pragma unroll
    for (int p = 0; p < (kTileW * kTileH) / kThreads; ++p) {
        const int e = p * kThreads + tid;
        const int bi = e / (4 * kTileH), r = (e / 4) % kTileH, j = e % 4;
        const int u = u0 + bi * 4 + j, v = v0 + r;
        if (u < a.W4 && v < a.H) {
            const long o = (((long)(u >> 2) * a.H + v) << 2) + (u & 3);
            // columns past W (padding) were staged as sky above
            a.pix[o] = trec[r][bi * 4 + j];
            if (SUN) a.sun[o] = tsun[r][bi * 4 + j];
        }
    }
}

template <bool SUN>
__global__ __launch_bounds__(kThreads)
void k_prepass(PrepassArgs a)
{
    prepass_tile<SUN>(a, blockIdx.x * kTileW, blockIdx.y * kTileH);
}

// All frames of a batch in one launch: block t is tile t of the frames' tiles
// laid end to end (tile_off[f] = first tile of frame f, tile_off[n] = total).
template <bool SUN>
__global__ __launch_bounds__(kThreads)
void k_prepass_batch(const PrepassArgs* frames, const int* tile_off, int n)
{
    const int t = blockIdx.x;
    int lo = 0, hi = n - 1;                 // last frame with tile_off[f] <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (tile_off[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    const PrepassArgs a = frames[lo];
    const int lt = t - tile_off[lo];
    const int tiles_x = (a.W4 + kTileW - 1) / kTileW;
    prepass_tile<SUN>(a, (lt % tiles_x) * kTileW, (lt / tiles_x) * kTileH);
}

int prepass_tiles(const PrepassArgs& a)
{
    return ((a.W4 + kTileW - 1) / kTileW) * ((a.H + kTileH - 1) / kTileH);
}

hipError_t launch_prepass_batch(hipStream_t s, const PrepassArgs* frames, const int* tile_off,
                                int n, int total_tiles, bool with_sun)
{
    if (total_tiles <= 0) return hipSuccess;
    dim3 block(kThreads);
    if (with_sun)
        hipLaunchKernelGGL(k_prepass_batch<true>, dim3(total_tiles), block, 0, s, frames, tile_off, n);
    else
        hipLaunchKernelGGL(k_prepass_batch<false>, dim3(total_tiles), block, 0, s, frames, tile_off, n);
    return hipGetLastError();
}

hipError_t launch_prepass(hipStream_t s, const PrepassArgs& a, bool with_sun)
{
    dim3 grid((a.W4 + kTileW - 1) / kTileW, (a.H + kTileH - 1) / kTileH);
    dim3 block(kThreads);
    if (with_sun)
        hipLaunchKernelGGL(k_prepass<true>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(k_prepass<false>, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace lidar
