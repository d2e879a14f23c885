// Per-frame G-buffer pre-pass.
//
// Everything in the footprint weight that depends on the pixel alone is
// folded into one FP32 shade per pixel (Eq. 4: rho_hat = beta cos(theta)/d^2
// for a unit isotropic source at the sensor, times the pixel solid angle of
// Eq. 2), and the pixel's time bin k = floor(2 d / (c dt)) (the Dirac delta
// of Eq. 3) is taken once per pixel in FP64.  Sky, non-finite or
// non-positive depths and ranges beyond the last bin get bin -1 and zero
// shade.  The records are written column-major ([u][v], v contiguous) so that
// the footprint kernel's lanes, which walk rows in parallel, read them
// coalesced; the transpose goes through a 32x32 LDS tile.
#include "engine.h"

namespace lidar {

namespace {
constexpr int kTile = 32;
constexpr int kRowsPerPass = 8;     // 32 x 8 threads, 4 passes per tile
}

template <bool SUN>
__global__ __launch_bounds__(kTile * kRowsPerPass)
void k_prepass(PrepassArgs a)
{
    __shared__ int2 trec[kTile][kTile + 1];
    __shared__ float tsun[kTile][kTile + 1];
    const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;
    const int u0 = blockIdx.x * kTile, v0 = blockIdx.y * kTile;
    const float inv_pi = (float)(1.0 / kPi);
    // read rows (coalesced along u), shade, stage in LDS
#pragma unroll
    for (int p = 0; p < kTile / kRowsPerPass; ++p) {
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
    // write columns (coalesced along v)
#pragma unroll
    for (int p = 0; p < kTile / kRowsPerPass; ++p) {
        int ul = ty + p * kRowsPerPass;
        int u = u0 + ul, v = v0 + tx;
        if (u < a.W && v < a.H) {
            long o = (long)u * a.H + v;
            a.pix[o] = trec[tx][ul];
            if (SUN) a.sun[o] = tsun[tx][ul];
        }
    }
}

hipError_t launch_prepass(hipStream_t s, const PrepassArgs& a, bool with_sun)
{
    dim3 grid((a.W + kTile - 1) / kTile, (a.H + kTile - 1) / kTile);
    dim3 block(kTile * kRowsPerPass);
    if (with_sun)
        hipLaunchKernelGGL(k_prepass<true>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(k_prepass<false>, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace lidar
