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
#include <climits>

#include "engine.h"

namespace lidar {

namespace {
constexpr int kTileW = 64, kTileH = 16;   // tile of kTileW columns x kTileH rows (256-byte row reads)
constexpr int kThreads = 256;
constexpr int kRowsPerPass = kThreads / kTileW;
static_assert(kTileW % 4 == 0 && kTileH % kRowsPerPass == 0, "whole 4-column blocks and passes");
}

// Range interval of pixel (u, v) of depth d and normal n (FP64): the plane
// through the pixel's centre point with normal n met by its four corner rays
// w, range d (p.n)/(w.n) with the ratio limited to [1/2, 2] (2 where w misses
// the plane's facing side), together with d itself; returns the first and
// last time bin of [min, max] (Alg. 1, pixelRangeInterval).
__device__ inline void pixel_interval(const PrepassArgs& a, int u, int v, double d, double nx,
                                      double ny, double nz, double* k0, double* k1)
{
#pragma clang fp contract(off)
    const double2 cc = a.rt.col[u], rc = a.rt.row[v];
    const double pn = (rc.x * cc.x) * nx + (rc.x * cc.y) * ny + rc.y * nz;
    double lo = d, hi = d;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double2 ce = a.rt.col_edge[u + (c & 1)], re = a.rt.row_edge[v + (c >> 1)];
        const double wn = (re.x * ce.x) * nx + (re.x * ce.y) * ny + re.y * nz;
        double q = pn / wn;
        if (!(q > 0.0)) q = 2.0;
        q = fmin(2.0, fmax(0.5, q));
        const double r = d * q;
        lo = fmin(lo, r);
        hi = fmax(hi, r);
    }
    *k0 = floor(lo * a.to_bin);
    *k1 = floor(hi * a.to_bin);
}

// One kTileW x kTileH tile of a frame, columns u0.., rows v0...  MODE is the
// range mode: CENTRE and CORRECTED store the centre bin (CORRECTED also the
// depth and normal of every pixel), INTERVAL the pixel's first and last bin
// packed as first | last << 16 with the shade divided by the interval's bins.
template <bool SUN, int MODE>
__device__ inline void prepass_tile(const PrepassArgs& a, int u0, int v0, int tile)
{
    __shared__ int2 trec[kTileH][kTileW + 1];
    __shared__ float tsun[kTileH][kTileW + 1];
    __shared__ float4 tr4[MODE == LIDAR_RANGE_CORRECTED ? kTileH : 1][kTileW + 1];
    const int tx = threadIdx.x % kTileW, ty = threadIdx.x / kTileW;
    float st_shade = 0.0f;                      // frame statistics of this thread's pixels
    int st_lo = INT_MAX, st_hi = INT_MIN;
    // read rows (coalesced along u), shade, stage in LDS
#pragma unroll
    for (int p = 0; p < kTileH / kRowsPerPass; ++p) {
        int vl = ty + p * kRowsPerPass;
        int u = u0 + tx, v = v0 + vl;
        int bin = -1;
        float shade = 0.0f, sunv = 0.0f;
        float4 r4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (u < a.W && v < a.H) {
            long px = (long)v * a.pitch + u;
            float d = gptr(a.depth)[px];
            if (d > 0.0f && isfinite(d)) {
                float nx = gptr(a.nx)[px], ny = gptr(a.ny)[px], nz = gptr(a.nz)[px];
                double kb = floor((double)d * a.to_bin), k1 = kb;
                if (MODE == LIDAR_RANGE_INTERVAL)
                    pixel_interval(a, u, v, (double)d, (double)nx, (double)ny, (double)nz, &kb, &k1);
                if (kb < (double)a.R) {
                    bin = (int)kb;
                    const gfloat2 c2 = *gptr((const gfloat2*)(a.colcs + u));
                    const gfloat4 rw = *gptr((const gfloat4*)(a.rowtab + v));
                    const float2 cs = make_float2(c2.x, c2.y);
                    const float4 rt = make_float4(rw.x, rw.y, rw.z, rw.w);
                    const float rho = gptr(a.refl)[px];
                    shade = pixel_shade(rt, cs, nx, ny, nz, rho, gptr(a.gain)[px], d);
                    if (MODE == LIDAR_RANGE_INTERVAL) {
                        // the interval's bins share the pixel's weight; bins
                        // past the last are dropped
                        shade = shade / (float)(k1 - kb + 1.0);
                        bin |= (int)fmin(k1, (double)(a.R - 1)) << 16;
                    }
                    if (SUN) sunv = pixel_sun(a.sun_x, a.sun_y, a.sun_z, rt, nx, ny, nz, rho);
                    if (MODE == LIDAR_RANGE_CORRECTED) r4 = make_float4(d, nx, ny, nz);
                }
            }
        }
        if (MODE == LIDAR_RANGE_CENTRE && bin >= 0) {
            st_shade = fmaxf(st_shade, shade);
            st_lo = min(st_lo, bin);
            st_hi = max(st_hi, bin);
        }
        trec[vl][tx] = make_int2(bin, __float_as_int(shade));
        if (SUN) tsun[vl][tx] = sunv;
        if (MODE == LIDAR_RANGE_CORRECTED) tr4[vl][tx] = r4;
    }
    if (MODE == LIDAR_RANGE_CENTRE && a.stats) {
        // the tile's statistics (wave reductions, the waves combined in LDS)
        // into its own record; k_reduce_stats combines a frame's records.
        // Shades are >= 0, so their FP32 bits order as integers.  Run
        // breaks: valid pixels (past the tile's first column) whose bin
        // differs from their left neighbour's, counted with those pixels
        // as brk | valid << 16 (at most kTileW x kTileH each).
        __shared__ int tstat[4][kThreads / 64];
        __syncthreads();                            // the tile's records are staged
        int nbrk = 0, nval = 0;
        if (tx > 0) {
#pragma unroll
            for (int p = 0; p < kTileH / kRowsPerPass; ++p) {
                const int vl = ty + p * kRowsPerPass;
                const int b = trec[vl][tx].x;
                if (b >= 0) {
                    ++nval;
                    nbrk += trec[vl][tx - 1].x != b ? 1 : 0;
                }
            }
        }
        int sb = __float_as_int(st_shade), cnt = nbrk | nval << 16;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            sb = max(sb, __shfl_xor(sb, m));
            st_lo = min(st_lo, __shfl_xor(st_lo, m));
            st_hi = max(st_hi, __shfl_xor(st_hi, m));
            cnt += __shfl_xor(cnt, m);
        }
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            tstat[0][w] = sb;
            tstat[1][w] = st_lo;
            tstat[2][w] = st_hi;
            tstat[3][w] = cnt;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
#pragma unroll
            for (int i = 1; i < kThreads / 64; ++i) {
                sb = max(sb, tstat[0][i]);
                st_lo = min(st_lo, tstat[1][i]);
                st_hi = max(st_hi, tstat[2][i]);
                cnt += tstat[3][i];
            }
            *gptr((gint4*)a.stats + tile) = gint4{sb, st_lo, st_hi, cnt};
        }
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
            const int2 rec = trec[r][bi * 4 + j];
            *gptr((gint2*)(a.pix + o)) = gint2{rec.x, rec.y};
            if (SUN) gptr(a.sun)[o] = tsun[r][bi * 4 + j];
            if (MODE == LIDAR_RANGE_CORRECTED) {
                const float4 q = tr4[r][bi * 4 + j];
                *gptr((gfloat4*)(a.rec4 + o)) = gfloat4{q.x, q.y, q.z, q.w};
            }
        }
    }
}

template <bool SUN, int MODE>
__global__ __launch_bounds__(kThreads)
void k_prepass(PrepassArgs a)
{
    prepass_tile<SUN, MODE>(a, blockIdx.x * kTileW, blockIdx.y * kTileH, blockIdx.y * gridDim.x + blockIdx.x);
}

// All frames of a batch in one launch: block t is tile t of the frames' tiles
// laid end to end (tile_off[f] = first tile of frame f, tile_off[n] = total).
template <bool SUN, int MODE>
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
    prepass_tile<SUN, MODE>(a, (lt % tiles_x) * kTileW, (lt / tiles_x) * kTileH, lt);
}

// Frame statistics from the tiles' records: a workgroup per frame over
// tiles tile_off[f] .. tile_off[f + 1] - 1 of the batch's records, as
// {largest shade bits, first bin, last bin, short runs}; short runs = 1 when
// more than half of the valid pixels with a left neighbour in their tile
// fall in another bin than it.  Frames without records (no pre-pass) get
// {0, INT_MAX, INT_MIN, 0}.  Workgroup 0 also zeroes the four counters after
// the n frames' statistics.
__global__ __launch_bounds__(256) void k_reduce_stats(const int4* tiles, const int* tile_off, int* stats,
                                                      int n)
{
    __shared__ int red[3][256 / 64];
    __shared__ long long redc[2][256 / 64];
    const int f = blockIdx.x, tid = threadIdx.x;
    int sb = 0, lo = INT_MAX, hi = INT_MIN;
    long long brk = 0, val = 0;
    for (int t = tile_off[f] + tid; t < tile_off[f + 1]; t += 256) {
        const int4 r = tiles[t];
        sb = max(sb, r.x);
        lo = min(lo, r.y);
        hi = max(hi, r.z);
        brk += r.w & 0xffff;
        val += r.w >> 16;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        sb = max(sb, __shfl_xor(sb, m));
        lo = min(lo, __shfl_xor(lo, m));
        hi = max(hi, __shfl_xor(hi, m));
        brk += __shfl_xor(brk, m);
        val += __shfl_xor(val, m);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = sb;
        red[1][tid >> 6] = lo;
        red[2][tid >> 6] = hi;
        redc[0][tid >> 6] = brk;
        redc[1][tid >> 6] = val;
    }
    __syncthreads();
    if (tid == 0) {
        for (int i = 1; i < 256 / 64; ++i) {
            sb = max(sb, red[0][i]);
            lo = min(lo, red[1][i]);
            hi = max(hi, red[2][i]);
            brk += redc[0][i];
            val += redc[1][i];
        }
        reinterpret_cast<int4*>(stats)[f] = make_int4(sb, lo, hi, 2 * brk > val ? 1 : 0);
        if (f == 0) reinterpret_cast<int4*>(stats)[n] = make_int4(0, 0, 0, 0);
    }
}

hipError_t launch_reduce_stats(hipStream_t s, const int* tiles, const int* tile_off, int* stats, int n)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_stats, dim3(n), dim3(256), 0, s, (const int4*)tiles, tile_off, stats, n);
    return hipGetLastError();
}

int prepass_tiles(const PrepassArgs& a)
{
    return ((a.W4 + kTileW - 1) / kTileW) * ((a.H + kTileH - 1) / kTileH);
}

hipError_t launch_prepass_batch(hipStream_t s, const PrepassArgs* frames, const int* tile_off,
                                int n, int total_tiles, bool with_sun, int range_mode)
{
    if (total_tiles <= 0) return hipSuccess;
    dim3 block(kThreads), grid(total_tiles);
    constexpr int C = LIDAR_RANGE_CENTRE, I = LIDAR_RANGE_INTERVAL;
    if (range_mode == C && with_sun)
        hipLaunchKernelGGL((k_prepass_batch<true, C>), grid, block, 0, s, frames, tile_off, n);
    else if (range_mode == C)
        hipLaunchKernelGGL((k_prepass_batch<false, C>), grid, block, 0, s, frames, tile_off, n);
    else if (range_mode == I && with_sun)
        hipLaunchKernelGGL((k_prepass_batch<true, I>), grid, block, 0, s, frames, tile_off, n);
    else if (range_mode == I)
        hipLaunchKernelGGL((k_prepass_batch<false, I>), grid, block, 0, s, frames, tile_off, n);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_prepass(hipStream_t s, const PrepassArgs& a, bool with_sun)
{
    dim3 grid((a.W4 + kTileW - 1) / kTileW, (a.H + kTileH - 1) / kTileH);
    dim3 block(kThreads);
    constexpr int C = LIDAR_RANGE_CENTRE, K = LIDAR_RANGE_CORRECTED, I = LIDAR_RANGE_INTERVAL;
    switch (a.range_mode * 2 + (with_sun ? 1 : 0)) {
    case 2 * C: hipLaunchKernelGGL((k_prepass<false, C>), grid, block, 0, s, a); break;
    case 2 * C + 1: hipLaunchKernelGGL((k_prepass<true, C>), grid, block, 0, s, a); break;
    case 2 * K: hipLaunchKernelGGL((k_prepass<false, K>), grid, block, 0, s, a); break;
    case 2 * K + 1: hipLaunchKernelGGL((k_prepass<true, K>), grid, block, 0, s, a); break;
    case 2 * I: hipLaunchKernelGGL((k_prepass<false, I>), grid, block, 0, s, a); break;
    case 2 * I + 1: hipLaunchKernelGGL((k_prepass<true, I>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lidar
