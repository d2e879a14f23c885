// Reprojection of a pinhole rendering onto the equiangular raster the
// footprint kernels read (section II-C: a pinhole image makes the kernel
// inhomogeneous; reprojecting the rendered image restores one kernel for
// all beams), with the renderer's depth decoded from a z buffer (section
// II-D).  One thread per output pixel, threads along a row: the six output
// planes are written coalesced; the reads gather the nearest pinhole pixel,
// which neighbouring threads share.
//
// Contraction is off: the index and range decisions are plain IEEE FP64
// operations in the order written, so that an output depth is the FP32
// rounding of the same FP64 value on every implementation.
#pragma clang fp contract(off)

#include "engine.h"

namespace lidar {

namespace {

// Eye-space z or radial range stored at pinhole pixel px (by format); a
// negative result marks sky (non-finite, non-positive, window depth outside
// [0, 1)).
__device__ inline double decode_depth(const ReprojectArgs& a, long px)
{
    double w;
    switch (a.fmt) {
    case LIDAR_DEPTH_RANGE:
    case LIDAR_DEPTH_EYE_Z: {
        const double d = (double)((const float*)a.depth)[px];
        return (d > 0.0 && isfinite(d)) ? d : -1.0;
    }
    case LIDAR_DEPTH_WINDOW_F32: w = (double)((const float*)a.depth)[px]; break;
    case LIDAR_DEPTH_WINDOW_U16: w = (double)((const uint16_t*)a.depth)[px] / 65535.0; break;
    default: w = (double)(((const uint32_t*)a.depth)[px] & 0xFFFFFFu) / 16777215.0; break;
    }
    if (!(w >= 0.0 && w < 1.0)) return -1.0;
    return a.z_near * a.z_far / (a.z_far - w * (a.z_far - a.z_near));
}

__global__ __launch_bounds__(256)
void k_reproject(ReprojectArgs a)
{
    const int u = blockIdx.x * blockDim.x + threadIdx.x, v = blockIdx.y;
    if (u >= a.W) return;
    const double d2r = kPi / 180.0;
    const double az = (a.az_min + ((double)u + 0.5) * a.dphi) * d2r;
    const double el = (a.el_max - ((double)v + 0.5) * a.de) * d2r;
    const double ce = cos(el);
    const double vs[3] = {ce * cos(az), ce * sin(az), sin(el)};
    const double* R = a.rot;                              // row-major, camera -> sensor
    // R^T v: the direction in the camera frame (x right, y down, z forward)
    const double c0 = R[0] * vs[0] + R[3] * vs[1] + R[6] * vs[2];
    const double c1 = R[1] * vs[0] + R[4] * vs[1] + R[7] * vs[2];
    const double c2 = R[2] * vs[0] + R[5] * vs[1] + R[8] * vs[2];
    float depth = INFINITY, refl = 0.0f, gain = 1.0f, nx = 0.0f, ny = 0.0f, nz = 0.0f;
    if (c2 > 0.0) {
        const double x = a.fx * c0 / c2 + a.cx, y = a.fy * c1 / c2 + a.cy;
        const double fi = floor(x), fj = floor(y);
        if (fi >= 0.0 && fi < (double)a.SW && fj >= 0.0 && fj < (double)a.SH) {
            // the pinhole pixel containing the projection, taken as is
            const long px = (long)fj * a.spitch + (long)fi;
            const double dec = decode_depth(a, px);
            if (dec > 0.0) {
                const double rx = (fi + 0.5 - a.cx) / a.fx, ry = (fj + 0.5 - a.cy) / a.fy;
                const double norm = sqrt(rx * rx + ry * ry + 1.0);
                double rng = a.fmt == LIDAR_DEPTH_RANGE ? dec : dec * norm;
                const double n0 = (double)a.nx[px], n1 = (double)a.ny[px], n2 = (double)a.nz[px];
                const double ns0 = R[0] * n0 + R[1] * n1 + R[2] * n2;
                const double ns1 = R[3] * n0 + R[4] * n1 + R[5] * n2;
                const double ns2 = R[6] * n0 + R[7] * n1 + R[8] * n2;
                if (a.correct) {
                    // range on the pixel's plane along the output direction
                    const double p0 = rx / norm, p1 = ry / norm, p2 = 1.0 / norm;
                    const double ps0 = R[0] * p0 + R[1] * p1 + R[2] * p2;
                    const double ps1 = R[3] * p0 + R[4] * p1 + R[5] * p2;
                    const double ps2 = R[6] * p0 + R[7] * p1 + R[8] * p2;
                    const double pn = ps0 * ns0 + ps1 * ns1 + ps2 * ns2;
                    const double vn = vs[0] * ns0 + vs[1] * ns1 + vs[2] * ns2;
                    double q = pn / vn;
                    if (!(q > 0.0)) q = 2.0;
                    rng = rng * fmin(2.0, fmax(0.5, q));
                }
                if (isfinite(rng)) {
                    depth = (float)rng;
                    refl = a.refl[px];
                    gain = a.gain[px];
                    nx = (float)ns0;
                    ny = (float)ns1;
                    nz = (float)ns2;
                }
            }
        }
    }
    const long o = (long)v * a.W + u;
    const long plane = (long)a.W * a.H;
    a.out[o] = depth;
    a.out[plane + o] = refl;
    a.out[2 * plane + o] = gain;
    a.out[3 * plane + o] = nx;
    a.out[4 * plane + o] = ny;
    a.out[5 * plane + o] = nz;
}

}  // namespace

hipError_t launch_reproject(hipStream_t s, const ReprojectArgs& a)
{
    dim3 grid((a.W + 255) / 256, a.H);
    hipLaunchKernelGGL(k_reproject, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace lidar
