// Set-up kernels, run once per (pattern, raster): resample the combined
// emitter x collector pattern onto the pixel-offset grid (Eq. 5's centred
// kernel kappa*eta, Alg. 1 input of size (2M+1) x (2N+1)), reduce it per row,
// and compute every beam's containing pixel and normalisation in FP64.
//
// Floating-point contraction is off in this file: every FP64 decision that
// selects an integer (beam pixel, kernel support) uses plain IEEE operations
// in the order written.
#pragma clang fp contract(off)

#include <climits>

#include "engine.h"

namespace lidar {

// Pattern value at an angular offset (x along azimuth, y along elevation, deg)
// from the beam centre.  Gaussian: exp(-q/2) inside the ellipse q <= trunc^2.
// Table: zero outside [-hx, hx] x [-hy, hy]; inside, bilinear between cell
// centres (row 0 = +elevation) with zero beyond the outermost centres.
__device__ static double pattern_at(const PatternDev& p, double x, double y)
{
    if (p.kind == LIDAR_PATTERN_GAUSS) {
        double a = x / p.sx;
        double b = y / p.sy;
        double q = a * a + b * b;
        return q > p.trunc * p.trunc ? 0.0 : exp(-0.5 * q);
    }
    if (fabs(x) > p.hx || fabs(y) > p.hy) return 0.0;
    double cx = 2.0 * p.hx / (double)p.nx;
    double cy = 2.0 * p.hy / (double)p.ny;
    double fx = (x + p.hx) / cx - 0.5;
    double fy = (p.hy - y) / cy - 0.5;
    double ix = floor(fx);
    double iy = floor(fy);
    double tx = fx - ix;
    double ty = fy - iy;
    int i = (int)ix, j = (int)iy;
    auto at = [&](int ii, int jj) -> double {
        return (ii < 0 || jj < 0 || ii >= p.nx || jj >= p.ny)
                   ? 0.0 : (double)p.table[(long)jj * p.nx + ii];
    };
    double top = (1.0 - tx) * at(i, j) + tx * at(i + 1, j);
    double bot = (1.0 - tx) * at(i, j + 1) + tx * at(i + 1, j + 1);
    return (1.0 - ty) * top + ty * bot;
}

// Solid angle of a pixel of row v (any integer v): dphi (sin e_top - sin e_bot).
__device__ static double row_omega(const RasterDev& r, long v)
{
    const double d2r = kPi / 180.0;
    double e_top = r.el_max - (double)v * r.de;
    double e_bot = r.el_max - (double)(v + 1) * r.de;
    return (r.dphi * d2r) * (sin(e_top * d2r) - sin(e_bot * d2r));
}

// K64[n+N][m+M]: the kernel on the pixel-offset grid (row-major, FP64).
__global__ void k_kernel_grid(PatternDev p, RasterDev r, KernelDev k, double* K64)
{
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long total = (long)k.KW * k.KH;
    if (idx >= total) return;
    int row = (int)(idx / k.KW), col = (int)(idx % k.KW);
    int n = row - k.N, m = col - k.M;
    K64[idx] = pattern_at(p, (double)m * r.dphi, -(double)n * r.de);
}

// FP32 copy of the kernel in the blocked, shifted layout the footprint
// kernel reads (see kernel_blocks in engine.h).
__global__ void k_kernel_blocks(KernelDev k, const double* K64, float* Kb)
{
    const int NB = kernel_blocks(k.KW);
    const long khp = (long)k.KH + 1;
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long total = 4L * NB * khp * 4;
    if (idx >= total) return;
    int j = (int)(idx % 4);
    long t = idx / 4;
    int n = (int)(t % khp);
    t /= khp;
    int b = (int)(t % NB);
    int sft = (int)(t / NB);
    int c = 4 * (b - kBlockPad) + sft + j;
    float v = 0.0f;
    if (n < k.KH && c >= 0 && c < k.KW) v = (float)K64[(long)n * k.KW + c];
    Kb[idx] = v;
}

// Per kernel row: FP64 sum, max, first/last non-zero column offset, and the
// prefix counts of non-zero cells (prefix[row][c] = non-zero cells in
// columns [0, c) of the row).  A wave per row, lanes over the columns in
// chunks of 64 (coalesced reads and writes; the counts from ballots); the
// lanes' FP64 partial sums are added by lane shuffles.
__global__ __launch_bounds__(256)
void k_kernel_rows(KernelDev k, const double* K64, double* rowsum, double* rowmax,
                   int2* rowrange, int32_t* prefix)
{
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (row >= k.KH) return;                             // the whole wave
    const double* kr = K64 + (long)row * k.KW;
    int32_t* pr = prefix + (long)row * (k.KW + 1);
    double s = 0.0, mx = 0.0;
    int lo = INT_MAX, hi = -1, cnt = 0;
    if (lane == 0) pr[0] = 0;
    for (int c0 = 0; c0 < k.KW; c0 += 64) {
        const int c = c0 + lane;
        const double v = c < k.KW ? kr[c] : 0.0;
        s += v;
        mx = fmax(mx, v);
        const unsigned long long nz = __ballot(v > 0.0);
        if (nz) {
            lo = min(lo, c0 + __builtin_ctzll(nz));
            hi = c0 + 63 - __builtin_clzll(nz);
        }
        const int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(nz >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((unsigned)nz, 0u));
        if (c < k.KW) pr[c + 1] = cnt + below + (v > 0.0 ? 1 : 0);
        cnt += __popcll(nz);
    }
    for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_xor(s, off);
        mx = fmax(mx, __shfl_xor(mx, off));
    }
    if (lane == 0) {
        rowsum[row] = s;
        rowmax[row] = mx;
        rowrange[row] = hi < 0 ? make_int2(INT_MAX, INT_MIN) : make_int2(lo - k.M, hi - k.M);
    }
}

// kinfo[0] = max K, kinfo[1] = sum K over the grid (one block).
__global__ void k_kernel_peak(KernelDev k, const double* rowsum, const double* rowmax,
                              double* kinfo)
{
    __shared__ double smax[256], ssum[256];
    double mx = 0.0, s = 0.0;
    for (int i = threadIdx.x; i < k.KH; i += blockDim.x) {
        mx = fmax(mx, rowmax[i]);
        s += rowsum[i];
    }
    smax[threadIdx.x] = mx;
    ssum[threadIdx.x] = s;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + off]);
            ssum[threadIdx.x] += ssum[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        kinfo[0] = smax[0];
        kinfo[1] = ssum[0];
    }
}

// Pixel-centre direction tables: colcs[u] = (cos az_u, sin az_u),
// rowtab[v] = (cos el_v, sin el_v, Omega_v, 0).  The solid angle is FP64
// (same integral as the normalisation) and stored in FP32.
__global__ void k_raster_tables(RasterDev r, float2* colcs, float4* rowtab)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    const float d2r = (float)(kPi / 180.0);
    if (i < r.W) {
        float a = (float)(r.az_min + ((double)i + 0.5) * r.dphi) * d2r;
        float sa, ca;
        sincosf(a, &sa, &ca);
        colcs[i] = make_float2(ca, sa);
    }
    if (i < r.H) {
        float e = (float)(r.el_max - ((double)i + 0.5) * r.de) * d2r;
        float se, ce;
        sincosf(e, &se, &ce);
        rowtab[i] = make_float4(ce, se, (float)row_omega(r, i), 0.0f);
    }
}

// omega[i] = Omega(v0 + i), the FP64 solid angle of a pixel of row v0 + i
// (rows above and below the image included).
__global__ void k_row_omega(RasterDev r, long v0, int n, double* omega)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) omega[i] = row_omega(r, v0 + i);
}

// FP64 cos and sin of the pixel-centre and edge angles of a raster (range
// modes): col[u] of az_min + (u + 1/2) dphi, row[v] of el_max - (v + 1/2) de,
// col_edge[u] of az_min + u dphi, row_edge[v] of el_max - v de.
__global__ void k_range_tables(RasterDev r, double2* col, double2* row, double2* col_edge,
                               double2* row_edge)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const double d2r = kPi / 180.0;
    if (i < r.W) {
        const double a = (r.az_min + ((double)i + 0.5) * r.dphi) * d2r;
        col[i] = make_double2(cos(a), sin(a));
    }
    if (i <= r.W) {
        const double a = (r.az_min + (double)i * r.dphi) * d2r;
        col_edge[i] = make_double2(cos(a), sin(a));
    }
    if (i < r.H) {
        const double e = (r.el_max - ((double)i + 0.5) * r.de) * d2r;
        row[i] = make_double2(cos(e), sin(e));
    }
    if (i <= r.H) {
        const double e = (r.el_max - (double)i * r.de) * d2r;
        row_edge[i] = make_double2(cos(e), sin(e));
    }
}

// Per beam: cos and sin of its azimuth and elevation offsets from the centre
// of its pixel (radians).  A kernel cell's true direction is then the
// direction of its pixel's centre turned by these offsets.
__global__ void k_beam_corr(RasterDev r, const double* az, const double* el, int B,
                            const lidar_beam_info* beams, double4* bcorr)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double d2r = kPi / 180.0;
    const double da = (az[b] - (r.az_min + ((double)beams[b].pixel_u + 0.5) * r.dphi)) * d2r;
    const double de = (el[b] - (r.el_max - ((double)beams[b].pixel_v + 0.5) * r.de)) * d2r;
    bcorr[b] = make_double4(cos(da), sin(da), cos(de), sin(de));
}

// Per beam (kSetupLanes lanes per beam, each over every kSetupLanes-th kernel
// row): containing pixel (floor rounding), FP64 normalisation over every
// kernel cell (on- and off-image rows), scale S_b = P_e / N_b, and the number
// of non-zero kernel cells inside the image.  Row solid angles come from the
// table omega (rows om_v0 .. om_v0 + om_n - 1, the same FP64 values) and are
// computed directly for beams beyond it; the lanes' partial sums are added by
// lane shuffles.  A beam not clipped at the image's left or right edge takes
// a row's whole count.
constexpr int kSetupLanes = 8;

__global__ __launch_bounds__(256)
void k_beam_setup(RasterDev r, KernelDev k, const double* az, const double* el,
                  int B, const double* rowsum, const int32_t* prefix,
                  const double* omega, long om_v0, int om_n,
                  double emit_power, lidar_beam_info* beams)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int sub = t % kSetupLanes;
    const int b = min(t / kSetupLanes, B - 1);           // the lanes past B repeat the last beam
    const bool own = t / kSetupLanes < B;
    double fu = floor((az[b] - r.az_min) / r.dphi);
    double fv = floor((r.el_max - el[b]) / r.de);
    // beams far outside the image keep an empty footprint
    const double lim = 1073741824.0;
    fu = fmin(fmax(fu, -lim), lim);
    fv = fmin(fmax(fv, -lim), lim);
    const long ub = (long)fu, vb = (long)fv;
    const bool tab = vb - k.N >= om_v0 && vb + k.N < om_v0 + om_n;
    const long c_lo = (long)-k.M > -ub ? (long)-k.M : -ub;
    const long c_hi = (long)k.M < (long)r.W - 1 - ub ? (long)k.M : (long)r.W - 1 - ub;
    const bool cols = c_lo <= c_hi, whole = c_lo == -k.M && c_hi == k.M;
    double nb = 0.0;
    uint32_t samples = 0;
    for (int n = sub; n < k.KH; n += kSetupLanes) {
        const long v = vb - k.N + n;
        nb += rowsum[n] * (tab ? omega[v - om_v0] : row_omega(r, v));
        if (cols && v >= 0 && v < r.H) {
            const int32_t* pr = prefix + (long)n * (k.KW + 1);
            samples += (uint32_t)(whole ? pr[k.KW] : pr[c_hi + k.M + 1] - pr[c_lo + k.M]);
        }
    }
    for (int off = kSetupLanes / 2; off > 0; off >>= 1) {
        nb += __shfl_xor(nb, off);
        samples += (uint32_t)__shfl_xor((int)samples, off);
    }
    if (sub != 0 || !own) return;
    lidar_beam_info bi;
    bi.pixel_u = (int32_t)ub;
    bi.pixel_v = (int32_t)vb;
    bi.scale = (float)(emit_power / nb);
    bi.floor = 0.0f;
    bi.samples = samples;
    bi.reserved = 0;
    beams[b] = bi;
}

// Centred Gaussian pulse sampled at the bin pitch, unit sum (FP32).
__global__ void k_pulse_taps(float sigma_ns, float bin_ns, int J, float* taps)
{
    __shared__ float w[kMaxTaps];
    int j = threadIdx.x;
    if (j <= 2 * J) {
        float t = (float)(j - J) * bin_ns;
        w[j] = expf(-(t * t) / (2.0f * sigma_ns * sigma_ns));
    }
    __syncthreads();
    if (j <= 2 * J) {
        float s = 0.0f;
        for (int i = 0; i <= 2 * J; ++i) s += w[i];
        taps[j] = w[j] / s;
    }
}

hipError_t launch_kernel_grid(hipStream_t s, PatternDev p, RasterDev r, KernelDev k,
                              double* K64)
{
    long total = (long)k.KW * k.KH;
    int blocks = (int)((total + 255) / 256);
    hipLaunchKernelGGL(k_kernel_grid, dim3(blocks), dim3(256), 0, s, p, r, k, K64);
    return hipGetLastError();
}

hipError_t launch_kernel_blocks(hipStream_t s, KernelDev k, const double* K64, float* Kb)
{
    long total = 4L * kernel_blocks(k.KW) * ((long)k.KH + 1) * 4;
    int blocks = (int)((total + 255) / 256);
    hipLaunchKernelGGL(k_kernel_blocks, dim3(blocks), dim3(256), 0, s, k, K64, Kb);
    return hipGetLastError();
}

hipError_t launch_kernel_rows(hipStream_t s, KernelDev k, const double* K64, double* rowsum,
                              double* rowmax, int2* rowrange, int32_t* prefix)
{
    hipLaunchKernelGGL(k_kernel_rows, dim3((k.KH + 3) / 4), dim3(256), 0, s, k, K64, rowsum,
                       rowmax, rowrange, prefix);
    return hipGetLastError();
}

hipError_t launch_kernel_peak(hipStream_t s, KernelDev k, const double* rowsum,
                              const double* rowmax, double* kinfo)
{
    hipLaunchKernelGGL(k_kernel_peak, dim3(1), dim3(256), 0, s, k, rowsum, rowmax, kinfo);
    return hipGetLastError();
}

hipError_t launch_raster_tables(hipStream_t s, RasterDev r, float2* colcs, float4* rowtab)
{
    int n = r.W > r.H ? r.W : r.H;
    hipLaunchKernelGGL(k_raster_tables, dim3((n + 255) / 256), dim3(256), 0, s, r, colcs, rowtab);
    return hipGetLastError();
}

hipError_t launch_beam_setup(hipStream_t s, RasterDev r, KernelDev k, const double* az,
                             const double* el, int B, const double* rowsum,
                             const int32_t* prefix, double* omega, double emit_power,
                             lidar_beam_info* beams)
{
    // rows -KH .. H + KH - 1: every beam whose footprint meets the image
    const long v0 = -(long)k.KH;
    const int n = r.H + 2 * k.KH;
    hipLaunchKernelGGL(k_row_omega, dim3((n + 255) / 256), dim3(256), 0, s, r, v0, n, omega);
    const long threads = (long)B * kSetupLanes;
    hipLaunchKernelGGL(k_beam_setup, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, r, k, az, el,
                       B, rowsum, prefix, (const double*)omega, v0, n, emit_power, beams);
    return hipGetLastError();
}

hipError_t launch_range_tables(hipStream_t s, RasterDev r, double2* col, double2* row,
                               double2* col_edge, double2* row_edge)
{
    const int n = (r.W > r.H ? r.W : r.H) + 1;
    hipLaunchKernelGGL(k_range_tables, dim3((n + 255) / 256), dim3(256), 0, s, r, col, row,
                       col_edge, row_edge);
    return hipGetLastError();
}

hipError_t launch_beam_corr(hipStream_t s, RasterDev r, const double* az, const double* el, int B,
                            const lidar_beam_info* beams, double4* bcorr)
{
    hipLaunchKernelGGL(k_beam_corr, dim3((B + 127) / 128), dim3(128), 0, s, r, az, el, B, beams,
                       bcorr);
    return hipGetLastError();
}

hipError_t launch_pulse_taps(hipStream_t s, float sigma_ns, float bin_ns, int J, float* taps)
{
    hipLaunchKernelGGL(k_pulse_taps, dim3(1), dim3(kMaxTaps), 0, s, sigma_ns, bin_ns, J, taps);
    return hipGetLastError();
}

}  // namespace lidar
