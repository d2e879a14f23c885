// Surrogate inputs, gate and fallback selection.
//
// Per frame: coarse cells (cw x ch pixels) hold the mean depth, gain and
// cos(theta) of their valid pixels, the reflectance summed over valid pixels
// per pixel of the cell and the summed sun shading; super-cells (sw x sh)
// hold the summed shade and sun shading of the pre-pass and the range of
// their time bins.  Per beam (one wave): the network input - 16 x 16 coarse
// cells around the beam's pixel in four channels, six beam parameters - a
// reference bin, an estimate of the sun floor and of the largest per-bin
// energy that the pattern's tails (outside the core box) can add.  After the
// network: the gate keeps a beam's predicted echoes when its confidence and
// tail checks pass, and lists the beam groups that hold any other beam for
// the plain path.  Validity, time bins and cos(theta) follow the pre-pass
// (Eqs. 3-4); the kernel is taken at each cell's centre.
#include <climits>
#include <type_traits>

#include "engine.h"

namespace lidar {

namespace {

__device__ inline int floordiv(int a, int b)
{
    const int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

__device__ inline uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Wave-wide reductions (all 64 lanes active) by DPP within quads, half-rows
// and rows, then row broadcasts; lane 63 holds the result, returned to every
// lane as a uniform value.
template <typename T, typename Op>
__device__ inline T wave_reduce(T v, T identity, Op op)
{
    auto step = [&](auto ctrl, auto row_mask) {
        const int o = __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, identity),
                                                  __builtin_bit_cast(int, v), decltype(ctrl)::value,
                                                  decltype(row_mask)::value, 0xf, false);
        v = op(v, __builtin_bit_cast(T, o));
    };
    using std::integral_constant;
    step(integral_constant<int, 0xb1>{}, integral_constant<int, 0xf>{});    // quad_perm [1,0,3,2]
    step(integral_constant<int, 0x4e>{}, integral_constant<int, 0xf>{});    // quad_perm [2,3,0,1]
    step(integral_constant<int, 0x141>{}, integral_constant<int, 0xf>{});   // row_half_mirror
    step(integral_constant<int, 0x140>{}, integral_constant<int, 0xf>{});   // row_mirror
    step(integral_constant<int, 0x142>{}, integral_constant<int, 0xa>{});   // row_bcast:15
    step(integral_constant<int, 0x143>{}, integral_constant<int, 0xc>{});   // row_bcast:31
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

__device__ inline float wave_sum(float v)
{
    return wave_reduce(v, 0.0f, [](float x, float y) { return x + y; });
}

__device__ inline float wave_maxf(float v)
{
    return wave_reduce(v, -INFINITY, [](float x, float y) { return fmaxf(x, y); });
}

__device__ inline float wave_minf(float v)
{
    return wave_reduce(v, INFINITY, [](float x, float y) { return fminf(x, y); });
}

__device__ inline int wave_mini(int v)
{
    return wave_reduce(v, INT_MAX, [](int x, int y) { return min(x, y); });
}

__device__ inline int wave_maxi(int v)
{
    return wave_reduce(v, INT_MIN, [](int x, int y) { return max(x, y); });
}

__device__ inline bool pixel_valid(float d, double to_bin, int R)
{
    return d > 0.0f && isfinite(d) && floor((double)d * to_bin) < (double)R;
}

// one thread per coarse cell
__global__ void k_coarse(CoarseArgs a)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.g.CW * a.g.CH) return;
    const int I = c % a.g.CW, J = c / a.g.CW;
    const int u0 = I * a.g.cw, v0 = J * a.g.ch;
    const int u1 = min(a.W, u0 + a.g.cw), v1 = min(a.H, v0 + a.g.ch);
    const float inv_pi = (float)(1.0 / kPi);
    float sd = 0.0f, sr = 0.0f, sg = 0.0f, sc = 0.0f, ss = 0.0f, sh = 0.0f;
    int nv = 0;
    for (int v = v0; v < v1; ++v) {
        const float4 rt = a.rowtab[v];
        for (int u = u0; u < u1; ++u) {
            const long px = (long)v * a.pitch + u;
            const float d = a.depth[px];
            if (!pixel_valid(d, a.to_bin, a.R)) continue;
            const float2 cs = a.colcs[u];
            const float vx = rt.x * cs.x, vy = rt.x * cs.y, vz = rt.y;
            const float nx = a.nx[px], ny = a.ny[px], nz = a.nz[px];
            const float rho = a.refl[px];
            const float gain = a.gain[px];
            const float ct = fmaxf(0.0f, -(nx * vx + ny * vy + nz * vz));
            sd += d;
            sr += rho;
            sg += gain;
            sc += ct;
            sh += rt.z * (gain * rho * inv_pi) * ct / (d * d);
            ss += rt.z * (rho * inv_pi) * fmaxf(0.0f, nx * a.sun_x + ny * a.sun_y + nz * a.sun_z);
            ++nv;
        }
    }
    const float nall = (float)((u1 - u0) * (v1 - v0));
    const float inv = nv > 0 ? 1.0f / (float)nv : 0.0f;
    a.cell[c] = make_float4(sd * inv, sr / nall, sg * inv, sc * inv);
    a.cell_sun[c] = ss;
    a.cell_shade[c] = sh;
}

// one wave per super-cell
__global__ void k_super(SuperArgs a)
{
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (c >= a.g.SW * a.g.SH) return;
    const int I = c % a.g.SW, J = c / a.g.SW;
    const int u0 = I * a.g.sw, v0 = J * a.g.sh;
    const int w = min(a.W, u0 + a.g.sw) - u0, h = min(a.H, v0 + a.g.sh) - v0;
    float shade = 0.0f, sun = 0.0f;
    int lo = INT_MAX, hi = INT_MIN;
    for (int q = lane; q < w * h; q += 64) {
        const int u = u0 + q % w, v = v0 + q / w;
        const long o = (((long)(u >> 2) * a.H + v) << 2) + (u & 3);
        const int2 r = a.pix[o];
        if (r.x < 0) continue;
        shade += __int_as_float(r.y);
        if (a.sun) sun += a.sun[o];
        lo = min(lo, r.x);
        hi = max(hi, r.x);
    }
    shade = wave_sum(shade);
    sun = wave_sum(sun);
    lo = wave_mini(lo);
    hi = wave_maxi(hi);
    if (lane == 0) {
        a.sup[c] = make_float2(shade, sun);
        a.range[c] = lo <= hi ? make_int2(lo, hi) : make_int2(0, -1);
    }
}

// one wave per beam
__global__ __launch_bounds__(256) void k_features(FeatArgs a)
{
    __shared__ float tail[4][kSurTailBins];
    __shared__ float refh[4][kSurRefWindow + 4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int b = blockIdx.x * 4 + wv;
    if (b >= a.B) return;                                  // whole wave
    float* th = tail[wv];
    th[lane] = 0.0f;                                       // kSurTailBins == 64
    const SurGeom g = a.g;
    const lidar_beam_info bi = a.beams[b];
    // the wave's beam: uniform, so the divisions below run on scalar registers
    const int u = __builtin_amdgcn_readfirstlane(bi.pixel_u), v = __builtin_amdgcn_readfirstlane(bi.pixel_v);
    const int Ib = floordiv(u, g.cw), Jb = floordiv(v, g.ch);
    uint16_t* x = a.X + (size_t)b * kSurIn;

    // the lane's 4 patch cells (lane + 64 s: 16 consecutive cells of a patch
    // row per quarter-wave, so that the loads coalesce)
    float4 rec[4];
    float csun[4];
    bool in[4];
    float kcore[4];                                        // K at the cell centre inside the core box
    int kc[4];                                             // candidate bins of the reference
    float wc[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int q = lane + 64 * s;
        const int I = Ib - kSurPatch / 2 + (q & 15), J = Jb - kSurPatch / 2 + (q >> 4);
        in[s] = I >= 0 && I < g.CW && J >= 0 && J < g.CH;
        rec[s] = in[s] ? a.cell[(long)J * g.CW + I] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        csun[s] = in[s] ? a.cell_sun[(long)J * g.CW + I] : 0.0f;
        const float cshade = in[s] ? a.cell_shade[(long)J * g.CW + I] : 0.0f;
        const int m = floordiv(2 * I * g.cw + g.cw - 2 * u, 2);
        const int n = floordiv(2 * J * g.ch + g.ch - 2 * v, 2);
        kcore[s] = (in[s] && abs(m) <= g.cm && abs(n) <= g.cn)
                       ? (float)a.K64[(long)(n + a.N) * a.KW + (m + a.M)] : 0.0f;
        kc[s] = INT_MAX;
        wc[s] = 0.0f;
        const float w = kcore[s] * cshade;
        if (rec[s].x > 0.0f && w > 0.0f) {
            kc[s] = (int)floor((double)rec[s].x * a.to_bin);
            wc[s] = w;
        }
    }
    // reference bin: first maximum of the (1, 2, 3, 2, 1)-smoothed histogram
    // of K * shade over the core cells' time bins, in a window from the
    // smallest; without core cells, the bin of the nearest cell mean depth
    int kmin = INT_MAX;
#pragma unroll
    for (int s = 0; s < 4; ++s) kmin = min(kmin, kc[s]);
    kmin = wave_mini(kmin);
    int k_ref = 0;
    if (kmin != INT_MAX) {
        float* hh = refh[wv];
        for (int j = lane; j < kSurRefWindow + 4; j += 64) hh[j] = 0.0f;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if (kc[s] != INT_MAX && kc[s] - kmin < kSurRefWindow) atomicAdd(&hh[kc[s] - kmin + 2], wc[s]);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        float best = -1.0f;
        int bj = INT_MAX;
        for (int q = 0; q < kSurRefWindow / 64; ++q) {
            const int j = lane * (kSurRefWindow / 64) + q;
            const float sm = hh[j] + 2.0f * hh[j + 1] + 3.0f * hh[j + 2] + 2.0f * hh[j + 3] + hh[j + 4];
            if (sm > best) {
                best = sm;
                bj = j;
            }
        }
        const float top = wave_maxf(best);
        const int jj = wave_mini(best == top ? bj : INT_MAX);
        k_ref = kmin + jj;
    } else {
        float m = INFINITY;
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if (rec[s].x > 0.0f) m = fminf(m, rec[s].x);
        m = wave_minf(m);
        k_ref = m < INFINITY ? (int)floor((double)m * a.to_bin) : 0;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int q = lane + 64 * s;
        const bool has = rec[s].x > 0.0f;
        // an input feature (stored as BF16): FP32 suffices
        const float dk = has ? (rec[s].x * (float)a.to_bin - ((float)k_ref + 0.5f)) * (1.0f / 64.0f) : 1.0f;
        x[q] = to_bf16(fminf(1.0f, fmaxf(-1.0f, dk)));
        x[256 + q] = to_bf16(in[s] ? rec[s].y : 0.0f);
        x[512 + q] = to_bf16(has ? log10f(rec[s].z) / 3.0f : 0.0f);
        x[768 + q] = to_bf16(has ? rec[s].w : 0.0f);
    }
    // sun floor of the core box from the coarse cells
    float asum = 0.0f;
#pragma unroll
    for (int s = 0; s < 4; ++s) asum += kcore[s] * csun[s];
    // super-cells outside the core box: sun floor and tail energy per bin
    const int I0 = max(0, floordiv(u - a.M, g.sw)), I1 = min(g.SW - 1, floordiv(u + a.M, g.sw));
    const int J0 = max(0, floordiv(v - a.N, g.sh)), J1 = min(g.SH - 1, floordiv(v + a.N, g.sh));
    const int nI = I1 - I0 + 1, nJ = J1 - J0 + 1;
    const int nb = (a.R + kSurTailBins - 1) / kSurTailBins;
    // (no super-cell lies outside a core box that spans the whole window)
    if (nI > 0 && nJ > 0 && (g.cm < a.M || g.cn < a.N)) {
        for (int q = lane; q < nI * nJ; q += 64) {
            const int Is = I0 + q % nI, Js = J0 + q / nI;
            const int m = floordiv(2 * Is * g.sw + g.sw - 2 * u, 2);
            const int n = floordiv(2 * Js * g.sh + g.sh - 2 * v, 2);
            if (abs(m) > a.M || abs(n) > a.N || (abs(m) <= g.cm && abs(n) <= g.cn)) continue;
            const float w = (float)a.K64[(long)(n + a.N) * a.KW + (m + a.M)];
            const long ci = (long)Js * g.SW + Is;
            const float2 sp = a.sup[ci];
            asum += w * sp.y;
            const int2 rg = a.range[ci];
            if (rg.y >= rg.x) {
                const float dens = w * sp.x / (float)(rg.y - rg.x + 1);
                for (int t = rg.x / nb; t <= rg.y / nb; ++t) atomicAdd(&th[t], dens);
            }
        }
    }
    asum = wave_sum(asum);
    const float e_tail = bi.scale * wave_maxf(th[lane]);
    const float a_est = a.ambient + a.sun_scale * asum;
    // the six beam parameters: uniform values, computed once per wave in
    // FP32 (they are stored as BF16) and picked by lanes 0..5
    if (lane < kSurIn - 1024) {
        const float p0 = ((float)(u - Ib * g.cw) + 0.5f) / (float)g.cw - 0.5f;
        const float p1 = ((float)(v - Jb * g.ch) + 0.5f) / (float)g.ch - 0.5f;
        const float p2 = (float)a.el[b] * (1.0f / 90.0f);
        const float p3 = (float)a.az[b] * (1.0f / 180.0f);
        const float p4 = a.threshold > 0.0f
                             ? fminf(2.0f, fmaxf(-4.0f, log10f(fmaxf(a_est, 1e-30f) / a.threshold))) / 4.0f
                             : 0.0f;
        const float p5 = (float)k_ref / (float)a.R;
        const float p = lane == 0 ? p0 : lane == 1 ? p1 : lane == 2 ? p2 : lane == 3 ? p3
                      : lane == 4 ? p4 : lane == 5 ? p5 : 0.0f;
        x[1024 + lane] = to_bf16(p);
    }
    if (lane == 0) {
        // the gate decision of the last surrogate frame (accepted) is left
        // as it is: only k_decode writes it
        SurAux* o = a.aux + b;
        o->k_ref = k_ref;
        o->e_tail = e_tail;
        o->a_est = a_est;
    }
}

// training targets from plain-path echoes
__global__ void k_labels(const lidar_echo* echoes, const int32_t* counts, const SurAux* aux, int B,
                         int E, float T, float* lab)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float* l = lab + (size_t)b * 16;
    for (int j = 0; j < 16; ++j) l[j] = 0.0f;
    const int n = counts[b];
    for (int e = 0; e < 3 && e < E; ++e) {
        if (n <= e) break;
        const lidar_echo ec = echoes[(size_t)b * E + e];
        l[e] = 1.0f;
        l[3 + e] = fminf(kSurDkClip, fmaxf(-kSurDkClip, (float)(ec.bin_peak - aux[b].k_ref) / kSurBinScale));
        l[6 + e] = log10f(fmaxf(ec.intensity, 1e-3f * T) / T);
        l[9 + e] = ec.pulse_width_ns / 4.0f;
    }
}

// gate and decode of the network outputs (one thread per beam)
__global__ void k_decode(DecodeArgs a)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B) return;
    const float* y = a.Y + (size_t)b * 16;
    SurAux aux = a.aux[b];
    const float T = a.threshold;
    // a tail contribution must stay well below what would change the
    // echoes: the distance of the floor to the threshold, or (floor above
    // the threshold: one run over every bin) the predicted peak
    const float margin = aux.a_est < T ? T - aux.a_est
                                       : (y[0] > 0.0f ? T * exp10f(y[6]) : 0.0f);
    const bool tail_ok = isinf(a.alpha) || aux.e_tail < a.alpha * margin;
    const bool accept = y[12] >= a.conf_logit && tail_ok;
    aux.accepted = accept ? 1 : 0;
    a.aux[b] = aux;
    if (!accept) return;
    lidar_echo* out = a.echoes + (size_t)b * a.E;
    int count = 0;
    for (int e = 0; e < 3; ++e) {
        if (!(y[e] > 0.0f)) continue;
        if (count < a.E) {
            const int k = min(a.R - 1, max(0, aux.k_ref + (int)rintf(kSurBinScale * y[3 + e])));
            const float epw = fmaxf(0.0f, 4.0f * y[9 + e]);
            const int half = (int)rintf(epw / (2.0f * (float)a.bin_ns));
            lidar_echo ec;
            ec.range_m = ((double)k + 0.5) * a.half_c_dt;
            ec.time_ns = ((double)k + 0.5) * a.bin_ns;
            ec.intensity = T * exp10f(y[6 + e]);
            ec.pulse_width_ns = epw;
            ec.bin_peak = k;
            ec.bin_first = max(0, k - half);
            ec.bin_last = min(a.R - 1, k + half);
            ec.flags = LIDAR_ECHO_SURROGATE;
            out[count] = ec;
        }
        ++count;
    }
    const lidar_echo z = {};
    for (int i = count; i < a.E; ++i) out[i] = z;
    a.counts[b] = count;
    a.beams[b].floor = aux.a_est;
}

// groups holding a beam that falls back: compacted for the plain path
__global__ void k_compact(CompactArgs a)
{
    const int gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= a.n_groups) return;
    int nfb = 0;
    for (int j = 0; j < a.G; ++j) {
        const int beam = a.groups[(size_t)gi * a.G + j];
        const bool fb = beam >= 0 && !a.aux[beam].accepted;
        a.groups_fb[(size_t)gi * a.G + j] = fb ? beam : -1;
        nfb += fb ? 1 : 0;
    }
    if (nfb > 0) {
        const int slot = atomicAdd(a.n_items, 1);
        a.items[slot] = make_int2(0, gi);
        atomicAdd(a.n_fallback, nfb);
    }
}

// Kept waveforms of the beams whose echoes the network predicted: no
// waveform is computed for them, so their rows are NaN (one workgroup per
// beam; the others' rows are written by the plain-path fallback).
__global__ void k_fill_accepted(const SurAux* aux, int B, int R, float* waves)
{
    const int b = blockIdx.x;
    if (b >= B || !aux[b].accepted) return;
    float* row = waves + (size_t)b * R;
    for (int k = threadIdx.x; k < R; k += blockDim.x) row[k] = __builtin_nanf("");
}

__global__ void k_aux_out(const SurAux* aux, int B, float* out)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    out[4 * b + 0] = (float)aux[b].k_ref;
    out[4 * b + 1] = aux[b].e_tail;
    out[4 * b + 2] = aux[b].a_est;
    out[4 * b + 3] = (float)aux[b].accepted;
}

inline unsigned blocks(long n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_coarse(hipStream_t s, const CoarseArgs& a)
{
    const long n = (long)a.g.CW * a.g.CH;
    hipLaunchKernelGGL(k_coarse, dim3(blocks(n, 128)), dim3(128), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_super(hipStream_t s, const SuperArgs& a)
{
    const long n = (long)a.g.SW * a.g.SH;
    hipLaunchKernelGGL(k_super, dim3(blocks(n, 4)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_features(hipStream_t s, const FeatArgs& a)
{
    hipLaunchKernelGGL(k_features, dim3(blocks(a.B, 4)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_labels(hipStream_t s, const lidar_echo* echoes, const int32_t* counts,
                         const SurAux* aux, int B, int E, float threshold, float* lab)
{
    hipLaunchKernelGGL(k_labels, dim3(blocks(B, 256)), dim3(256), 0, s, echoes, counts, aux, B, E,
                       threshold, lab);
    return hipGetLastError();
}

hipError_t launch_decode(hipStream_t s, const DecodeArgs& a)
{
    hipLaunchKernelGGL(k_decode, dim3(blocks(a.B, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_compact(hipStream_t s, const CompactArgs& a)
{
    hipLaunchKernelGGL(k_compact, dim3(blocks(a.n_groups, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_accepted(hipStream_t s, const SurAux* aux, int B, int R, float* waves)
{
    hipLaunchKernelGGL(k_fill_accepted, dim3(B), dim3(256), 0, s, aux, B, R, waves);
    return hipGetLastError();
}

hipError_t launch_aux_out(hipStream_t s, const SurAux* aux, int B, float* out)
{
    hipLaunchKernelGGL(k_aux_out, dim3(blocks(B, 256)), dim3(256), 0, s, aux, B, out);
    return hipGetLastError();
}

}  // namespace lidar
