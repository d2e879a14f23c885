// Fused per-beam kernel: footprint gather -> time-bin histogram in LDS ->
// ambient floor -> pulse convolution -> wavefront-ballot echo detection.
//
// One workgroup (4 waves of 64) per beam.  The beam's footprint (the kernel
// window of Eq. 5 / Alg. 1, clipped to the image) is cut into strips of 64
// kernel rows; in a strip every lane owns one row and the wave walks the
// strip's columns together, so each step reads 64 consecutive entries of the
// column-major kernel and pixel records (one coalesced load each).  A lane
// keeps a run accumulator (bin, sum) and only touches the LDS histogram when
// the time bin of its row changes: surfaces that are smooth along azimuth
// (road rows, box faces) collapse many samples into one LDS atomic, and the
// sky costs no atomics at all.
//
// The histogram holds sum K * shade; the beam scale S_b is applied once in
// the pulse convolution.  Echoes are maximal runs of xi_hat > T found with
// 64-bin ballots (section II-C, EPW paragraph).
#include <climits>

#include "engine.h"

namespace lidar {

namespace {

__device__ inline int wave_min(int x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o));
    return x;
}

__device__ inline int wave_max(int x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o));
    return x;
}

__device__ inline float wave_sum(float x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

constexpr int kWaves = kFootprintThreads / 64;

}  // namespace

template <bool SUN, bool KEEP>
__global__ __launch_bounds__(kFootprintThreads)
void k_footprint(FootprintArgs a)
{
    extern __shared__ float lds[];
    float* hist = lds;              // [R] sum K * shade per bin
    float* xh = lds + a.R;          // [R] xi_hat
    float* taps = lds + 2 * a.R;    // [2J+1]
    __shared__ float red[kWaves];

    // XCD-aware schedule: workgroups go round-robin over the 8 XCDs, so slot
    // s runs on XCD s % 8; each XCD takes one contiguous, spatially sorted
    // chunk of beams and the beams in flight on it share their pixels in L2.
    const int slot = blockIdx.x;
    const int idx = (slot % kXcds) * a.chunk + slot / kXcds;
    if (idx >= a.B) return;
    const int b = a.order[idx];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    for (int k = tid; k < a.R; k += kFootprintThreads) hist[k] = 0.0f;
    for (int j = tid; j <= 2 * a.J; j += kFootprintThreads) taps[j] = a.taps[j];
    __syncthreads();

    const lidar_beam_info bi = a.beams[b];
    const int ub = bi.pixel_u, vb = bi.pixel_v;
    const int n0 = max(-a.N, -vb), n1 = min(a.N, a.H - 1 - vb);
    const int c0 = max(-a.M, -ub), c1 = min(a.M, a.W - 1 - ub);
    float sacc = 0.0f;
    if (n0 <= n1 && c0 <= c1) {
        const int nrows = n1 - n0 + 1;
        const int nstrips = (nrows + 63) >> 6;
        const int ncols = c1 - c0 + 1;
        // at least 2 items per wave when the footprint is wide enough
        int nchunk = (2 * kWaves + nstrips - 1) / nstrips;
        nchunk = min(nchunk, max(1, ncols / 32));
        const int cw = (ncols + nchunk - 1) / nchunk;
        const int items = nstrips * nchunk;
        for (int it = wave; it < items; it += kWaves) {
            const int s = it / nchunk, ch = it - s * nchunk;
            const int n = n0 + s * 64 + lane;
            const bool rowok = n <= n1;
            const int nn = rowok ? n : n1;          // in-bounds row for idle lanes
            int2 rr = a.rowrange[nn + a.N];
            if (!rowok) rr = make_int2(INT_MAX, INT_MIN);
            const int mb = max(c0 + ch * cw, wave_min(rr.x));
            const int me = min(min(c1, c0 + ch * cw + cw - 1), wave_max(rr.y));
            if (mb > me) continue;
            const int koff = nn + a.N;
            const int poff = vb + nn;
            const float kmask = rowok ? 1.0f : 0.0f;
            const float* kcol = a.Kt + (long)(mb + a.M) * a.KH;
            const int2* pcol = a.pix + (long)(ub + mb) * a.H;
            const float* scol = SUN ? a.sun + (long)(ub + mb) * a.H : nullptr;
            int cur = -1;
            float acc = 0.0f;
            for (int m = mb; m <= me; ++m) {
                const float kv = kcol[koff] * kmask;
                const int2 rec = pcol[poff];
                const float t = kv * __int_as_float(rec.y);
                if (rec.x != cur && rec.x >= 0 && kv != 0.0f) {
                    if (acc != 0.0f) atomicAdd(&hist[cur], acc);
                    cur = rec.x;
                    acc = t;
                } else {
                    acc += t;
                }
                if (SUN) sacc += kv * scol[poff];
                kcol += a.KH;
                pcol += a.H;
                if (SUN) scol += a.H;
            }
            if (acc != 0.0f) atomicAdd(&hist[cur], acc);
        }
    }
    if (SUN) {
        const float w = wave_sum(sacc);
        if (lane == 0) red[wave] = w;
    }
    __syncthreads();
    float floor_b = a.ambient;
    if (SUN) {
        float tot = 0.0f;
#pragma unroll
        for (int i = 0; i < kWaves; ++i) tot += red[i];
        floor_b += a.sun_scale * tot;
    }

    // pulse convolution (zero outside [0, R)) plus the floor
    const float S = bi.scale;
    for (int k = tid; k < a.R; k += kFootprintThreads) {
        const int jlo = max(-a.J, k - (a.R - 1)), jhi = min(a.J, k);
        float s = 0.0f;
        for (int j = jlo; j <= jhi; ++j) s += taps[j + a.J] * hist[k - j];
        const float v = S * s + floor_b;
        xh[k] = v;
        if (KEEP) a.waves[(long)b * a.R + k] = v;
    }
    __syncthreads();
    if (wave != 0) return;

    // echo detection: runs of xi_hat > T, 64 bins per ballot
    const float T = a.threshold;
    const float dt = (float)a.bin_ns;
    lidar_echo* out = a.echoes + (long)b * a.E;
    int count = 0;
    int k0 = -1;                                    // first bin of the open run
    for (int base = 0; base < a.R; base += 64) {
        const int k = base + lane;
        const bool above = k < a.R && xh[k] > T;
        const unsigned long long mask = __ballot(above);
        const bool next_above = base + 64 < a.R && xh[base + 64] > T;
        const unsigned long long prev = (mask << 1) | (k0 >= 0 ? 1ull : 0ull);
        const unsigned long long nxt = (mask >> 1) | (next_above ? (1ull << 63) : 0ull);
        unsigned long long starts = mask & ~prev;
        unsigned long long ends = mask & ~nxt;
        while (starts | ends) {
            const int ps = starts ? __ffsll((long long)starts) - 1 : 64;
            const int pe = ends ? __ffsll((long long)ends) - 1 : 64;
            if (ps <= pe) {
                k0 = base + ps;
                starts &= starts - 1;
                continue;
            }
            ends &= ends - 1;
            const int k1 = base + pe;
            if (count < a.E) {
                // first maximum of the run
                float best = -INFINITY;
                int bk = INT_MAX;
                for (int s = k0; s <= k1; s += 64) {
                    const int kk = s + lane;
                    if (kk <= k1) {
                        const float x = xh[kk];
                        if (x > best) {
                            best = x;
                            bk = kk;
                        }
                    }
                }
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    const float ob = __shfl_xor(best, o);
                    const int oi = __shfl_xor(bk, o);
                    if (ob > best || (ob == best && oi < bk)) {
                        best = ob;
                        bk = oi;
                    }
                }
                if (lane == 0) {
                    // threshold crossings between bin centres, as fractions of
                    // a bin measured from the centre of the bin before the run
                    // and from the centre of its last bin
                    float f_up, f_dn;
                    uint32_t flags = 0;
                    if (k0 == 0) {
                        f_up = 0.5f;
                        flags |= LIDAR_ECHO_AT_FIRST_BIN;
                    } else {
                        const float xa = xh[k0 - 1], xb = xh[k0];
                        f_up = (T - xa) / (xb - xa);
                    }
                    if (k1 == a.R - 1) {
                        f_dn = 0.5f;
                        flags |= LIDAR_ECHO_AT_LAST_BIN;
                    } else {
                        const float xa = xh[k1], xb = xh[k1 + 1];
                        f_dn = (xa - T) / (xa - xb);
                    }
                    lidar_echo e;
                    e.range_m = ((double)bk + 0.5) * a.half_c_dt;
                    e.time_ns = ((double)bk + 0.5) * a.bin_ns;
                    e.intensity = best - floor_b;
                    e.pulse_width_ns = ((float)(k1 - k0 + 1) + f_dn - f_up) * dt;
                    e.bin_peak = bk;
                    e.bin_first = k0;
                    e.bin_last = k1;
                    e.flags = flags;
                    out[count] = e;
                }
            }
            ++count;
            k0 = -1;
        }
    }
    if (lane == 0) {
        a.counts[b] = count;
        a.beams[b].floor = floor_b;
        lidar_echo z = {};
        for (int i = count; i < a.E; ++i) out[i] = z;
    }
}

hipError_t launch_footprint(hipStream_t s, const FootprintArgs& a)
{
    const int grid = kXcds * a.chunk;
    const size_t lds = sizeof(float) * (2 * (size_t)a.R + 2 * (size_t)a.J + 1);
    const bool sun = a.sun != nullptr;
    const bool keep = a.waves != nullptr;
    if (sun && keep)
        hipLaunchKernelGGL((k_footprint<true, true>), dim3(grid), dim3(kFootprintThreads), lds, s, a);
    else if (sun)
        hipLaunchKernelGGL((k_footprint<true, false>), dim3(grid), dim3(kFootprintThreads), lds, s, a);
    else if (keep)
        hipLaunchKernelGGL((k_footprint<false, true>), dim3(grid), dim3(kFootprintThreads), lds, s, a);
    else
        hipLaunchKernelGGL((k_footprint<false, false>), dim3(grid), dim3(kFootprintThreads), lds, s, a);
    return hipGetLastError();
}

}  // namespace lidar
