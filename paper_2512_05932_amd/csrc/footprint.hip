// Fused processing of a group of G nearby beams: footprint gather -> per-beam
// time-bin histograms in LDS -> ambient floor -> pulse convolution ->
// wavefront-ballot echo detection.  Two kernels share the group body: one
// workgroup per group of one frame (`k_footprint`), and a persistent kernel
// that takes tickets of (frame, group) items of a whole batch from a work
// queue (`k_footprint_batch`).  A third, `k_footprint_batch_wave`, runs the
// same steps for one beam per wave (frames whose groups mostly hold a single
// beam), every wave taking its own tickets.  Tickets come from eight counters,
// one per XCD (next_ticket).
//
// Work decomposition.  A workgroup (4 waves of 64) takes a group of up to G
// beams formed by the host scheduler from beams close on the raster.  The
// union of their footprints (kernel windows of Eq. 5 / Alg. 1, clipped to the
// image) is cut into strips of `tile` image rows.  With tile = 64 every lane
// owns one row; with tile = 16 or 4 the 64 lanes are tile rows x 64/tile
// column phases, for small kernels.  A lane walks its row in aligned batches
// of 4 columns: pixel records, sun shading and the kernel are stored in
// 4-column blocks, so a batch is one 16-byte load per stream (per beam for the
// kernel).  A pixel's time bin does not depend on the beam, so the pixel
// record, the bin comparison and the sun shading are shared by the G beams;
// only the kernel value and two FMAs are per beam.
//
// Run accumulation.  A lane sums the weights of consecutive pixels of its row
// that fall into the same bin in registers (one sum per beam) and adds them to
// the LDS histograms when the bin changes.  Batches in which no lane's bin
// changes (most of them) take a branch-free fast path; otherwise the batch is
// replayed with the resets and the ended runs are flushed.  Rows that cross
// the same surface change bin together, so the flushing lanes usually share a
// bin: their G sums are reduced across the wave together (half and row lane
// swaps, then DPP), and one LDS atomic per bin and beam replaces one per lane,
// which would serialise on the shared address.
//
// The histograms hold sum K * shade; the beam scale S_b is applied in the
// pulse convolution (in place; 8 output bins per thread and blocks of 8 taps
// over zero-padded histograms, so the window lives in registers and no read
// needs a bounds check; with one pass per waveform all beams' outputs wait in
// registers for a single barrier).  The gather flags the chunks it writes (32 chunks of
// 64 or more bins, a register bit mask per lane, OR-reduced per wave):
// outputs whose inputs lie only in unflagged chunks are the floor without
// convolving, and the output pass flags the 64-bin chunks holding a bin above
// the threshold.  Echoes are maximal runs of xi_hat > T found with 64-bin
// ballots over the flagged chunks, one wave per beam (section II-C, EPW
// paragraph).
#include <climits>
#include <type_traits>

#include "engine.h"

namespace lidar {

namespace {

constexpr int kWaves = kFootprintThreads / 64;
static_assert(kPassBins == 8 * kFootprintThreads && kPassBins == 32 * 64,
              "a convolution pass is 8 bins per thread and one 32-bit word of 64-bin chunks");

template <int CTRL, int ROW_MASK>
__device__ inline int dpp_min(int v)
{
    return min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, CTRL, ROW_MASK, 0xf, false));
}

template <int CTRL, int ROW_MASK>
__device__ inline int dpp_max(int v)
{
    return max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, CTRL, ROW_MASK, 0xf, false));
}

// Minimum / maximum over the 64 lanes (all lanes active) by DPP: within
// quads, half-rows and rows, then row broadcasts; lane 63 holds the result,
// returned as a uniform value.
__device__ inline int wave_min(int x)
{
    x = dpp_min<0xb1, 0xf>(x);
    x = dpp_min<0x4e, 0xf>(x);
    x = dpp_min<0x141, 0xf>(x);
    x = dpp_min<0x140, 0xf>(x);
    x = dpp_min<0x142, 0xa>(x);
    x = dpp_min<0x143, 0xc>(x);
    return __builtin_amdgcn_readlane(x, 63);
}

template <int CTRL, int ROW_MASK>
__device__ inline float dpp_maxf(float v)
{
    return fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(
                        __float_as_int(-INFINITY), __float_as_int(v), CTRL, ROW_MASK, 0xf, false)));
}

__device__ inline float wave_maxf(float x)
{
    x = dpp_maxf<0xb1, 0xf>(x);
    x = dpp_maxf<0x4e, 0xf>(x);
    x = dpp_maxf<0x141, 0xf>(x);
    x = dpp_maxf<0x140, 0xf>(x);
    x = dpp_maxf<0x142, 0xa>(x);
    x = dpp_maxf<0x143, 0xc>(x);
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

__device__ inline unsigned long long wave_max_u64(unsigned long long x)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const unsigned long long y = __shfl_xor(x, m);
        x = y > x ? y : x;
    }
    return x;
}

__device__ inline int wave_max(int x)
{
    x = dpp_max<0xb1, 0xf>(x);
    x = dpp_max<0x4e, 0xf>(x);
    x = dpp_max<0x141, 0xf>(x);
    x = dpp_max<0x140, 0xf>(x);
    x = dpp_max<0x142, 0xa>(x);
    x = dpp_max<0x143, 0xc>(x);
    return __builtin_amdgcn_readlane(x, 63);
}

template <int CTRL, int ROW_MASK>
__device__ inline unsigned dpp_or(unsigned v)
{
    return v | (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, false);
}

// Bitwise OR over the 64 lanes (all active), returned as a uniform value.
__device__ inline unsigned wave_or(unsigned x)
{
    x = dpp_or<0xb1, 0xf>(x);
    x = dpp_or<0x4e, 0xf>(x);
    x = dpp_or<0x141, 0xf>(x);
    x = dpp_or<0x140, 0xf>(x);
    x = dpp_or<0x142, 0xa>(x);
    x = dpp_or<0x143, 0xc>(x);
    return (unsigned)__builtin_amdgcn_readlane((int)x, 63);
}

template <int CTRL, int ROW_MASK>
__device__ inline float dpp_add(float v)
{
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL,
                                                          ROW_MASK, 0xf, false));
}

// Sum over the 64 lanes (all lanes must be active); the total is returned in
// every lane as a uniform value.
__device__ inline float wave_total(float v)
{
    v = dpp_add<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
    v = dpp_add<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]
    v = dpp_add<0x141, 0xf>(v);   // row_half_mirror
    v = dpp_add<0x140, 0xf>(v);   // row_mirror: every lane holds its row's sum
    v = dpp_add<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Load of a read-only record at a uniform address through the scalar data
// cache (constant address space): the record lands in scalar registers.
template <typename T>
__device__ inline T load_uniform(const T* p)
{
    static_assert(sizeof(T) % 4 == 0, "whole dwords");
    struct Words { unsigned u[sizeof(T) / 4]; } w;
    const __attribute__((address_space(4))) unsigned* q =
        (const __attribute__((address_space(4))) unsigned*)p;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w.u[i] = q[i];
    return __builtin_bit_cast(T, w);
}

// An echo record stored field by field through a global-address-space
// pointer (a global store: a flat one would also count against the LDS
// counter, and the wave's next LDS wait would wait for it).
__device__ inline void store_echo(lidar_echo* dst, const lidar_echo& e)
{
    auto o = gptr(dst);
    o->range_m = e.range_m;
    o->time_ns = e.time_ns;
    o->intensity = e.intensity;
    o->pulse_width_ns = e.pulse_width_ns;
    o->bin_peak = e.bin_peak;
    o->bin_first = e.bin_first;
    o->bin_last = e.bin_last;
    o->flags = e.flags;
}

// Sum of two registers' 32-lane halves: lanes 0-31 get a(l) + a(l + 32),
// lanes 32-63 get b(l - 32) + b(l) (one v_permlane32_swap).
__device__ inline float swap_sum32(float a, float b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b),
                                                    false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// The same over 16-lane rows: rows 0 and 2 get a's row pairs (0+1, 2+3),
// rows 1 and 3 get b's (one v_permlane16_swap).
__device__ inline float swap_sum16(float a, float b)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b),
                                                    false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Totals over the 64 lanes of G per-beam values at once (G = 1, 2 or 4; all
// lanes active).  The half and row swaps fold the G registers into one so
// that every 16-lane row holds partial sums of a single beam, then a DPP sum
// within rows finishes: lane i * 64/G holds the total of beam i.
template <int G>
__device__ inline float group_totals(const float* v)
{
    float x;
    if constexpr (G == 4) {
        x = swap_sum16(swap_sum32(v[0], v[2]), swap_sum32(v[1], v[3]));
    } else if constexpr (G == 2) {
        const float y = swap_sum32(v[0], v[1]);
        x = swap_sum16(y, y);
    } else {
        const float y = swap_sum32(v[0], v[0]);
        x = swap_sum16(y, y);
    }
    x = dpp_add<0xb1, 0xf>(x);
    x = dpp_add<0x4e, 0xf>(x);
    x = dpp_add<0x141, 0xf>(x);
    return dpp_add<0x140, 0xf>(x);
}

// Fixed-point accumulation (batches): bin lo + j held as the 64-bit integer
// j at floats lo + 2j, lo + 2j + 1 of the histogram (lo even, so the
// integers are 8-byte aligned), in units of 2^-s, s chosen so that no bin
// can exceed 2^61 units; integer LDS atomics run at the full LDS rate, FP32
// ones do not (frames whose every pixel starts a run are bound by them).
// scale = 2^s.
struct IntAcc {
    float scale;
    int lo;
    bool each;      // every sample its own add (no run sums): frames whose runs are short
};

// t >= 0 in units of 2^-s, truncated (t * scale <= 2^61: exact scaling, then
// the integer part)
__device__ inline unsigned long long to_units(float t, float scale)
{
    return (unsigned long long)(t * scale);
}

// Add t into the bins of a pixel key: the bin itself, or with range keys
// (pixel range intervals) every bin first .. last of key = first | last << 16.
template <bool IACC = false>
__device__ inline void add_key(float* h, int key, float t, bool rng, IntAcc ia = IntAcc{})
{
    if constexpr (IACC) {
        atomicAdd((unsigned long long*)(h + ia.lo) + (key - ia.lo), to_units(t, ia.scale));
        return;
    }
    if (!rng) {
        atomicAdd(h + key, t);
        return;
    }
    const int k1 = key >> 16;
    for (int k = key & 0xffff; k <= k1; ++k) atomicAdd(h + k, t);
}

// Chunk flags (chunks of 1 << nzs bins) of the bins of a key.
__device__ inline unsigned key_chunks(int key, int nzs, bool rng)
{
    if (!rng) return 1u << (key >> nzs);
    const int c0 = (key & 0xffff) >> nzs, c1 = (key >> 16) >> nzs;
    return (c1 - c0 >= 31 ? ~0u : (2u << (c1 - c0)) - 1u) << c0;
}

// Flush the lanes in `fm` (lanes whose run ended) into the histograms.
// `stride` is the distance between the beams' histograms; bit c of the
// lane's nzb is set for every chunk c (bins c << nzs ..) that receives a sum.
// rng: the keys are bin ranges (first | last << 16).
template <int G, bool IACC = false>
__device__ inline void flush_runs(unsigned long long fm, bool fl, int cur, const float* acc,
                                  float* hist, int stride, unsigned& nzb, int nzs, int lane, bool rng,
                                  IntAcc ia = IntAcc{})
{
    unsigned long long m = fm;
    // lanes sharing a bin are reduced across the wave (a few bins per step)
#pragma unroll 1
    for (int peel = 0; peel < 4 && m; ++peel) {
        const int leader = __builtin_ctzll(m);
        const int key = __builtin_amdgcn_readlane(cur, leader);
        const unsigned long long same = __ballot(fl && cur == key) & m;
        if (__popcll(same) < 3) break;
        const bool in = (same >> lane) & 1ull;
        float v[G];
#pragma unroll
        for (int g = 0; g < G; ++g) v[g] = in ? acc[g] : 0.0f;
        const float t = group_totals<G>(v);
        constexpr int span = 64 / G;
        if (lane % span == 0 && t != 0.0f) add_key<IACC>(hist + (lane / span) * stride, key, t, rng, ia);
        nzb |= key_chunks(key, nzs, IACC ? false : rng);   // fixed point: centre bins
        m &= ~same;
    }
    if ((m >> lane) & 1ull) {
        nzb |= key_chunks(cur, nzs, IACC ? false : rng);
#pragma unroll
        for (int g = 0; g < G; ++g)
            if (acc[g] != 0.0f) add_key<IACC>(hist + g * stride, cur, acc[g], rng, ia);
    }
}

// 16-byte load at a uniform base plus a per-lane byte offset (the bases
// derive from kernel arguments, so these become global loads).
template <typename T>
__device__ inline T ld16(const char* base, unsigned byte_off)
{
    if constexpr (std::is_same_v<T, int4>) {
        const gint4 v = *gptr((const gint4*)(base + byte_off));
        return make_int4(v.x, v.y, v.z, v.w);
    } else {
        static_assert(std::is_same_v<T, float4>, "16-byte int4 or float4");
        const gfloat4 v = *gptr((const gfloat4*)(base + byte_off));
        return make_float4(v.x, v.y, v.z, v.w);
    }
}

// Time bin of one sample in LIDAR_RANGE_CORRECTED mode (FP64): the range on
// the pixel's plane along the kernel cell's true direction v, d (p.n)/(v.n)
// with the ratio limited to [1/2, 2] (2 where v misses the plane's facing
// side).  p is the pixel centre direction (cos/sin of its azimuth cs and
// elevation ce, se), v the same direction turned by the beam's offsets bc
// {cos daz, sin daz, cos del, sin del} from its pixel centre; -1 past R.
__device__ inline int corrected_bin(const float4& q, double2 cs, double ce, double se, const double4& bc,
                                    double to_bin, int R)
{
    const double nx = q.y, ny = q.z, nz = q.w;
    const double A = nx * cs.x + ny * cs.y;              // n along the azimuth direction
    const double Bp = ny * cs.x - nx * cs.y;              // n along the azimuth tangent
    const double pn = ce * A + se * nz;
    const double h = bc.x * A + bc.y * Bp;
    const double vn = bc.z * (ce * h + se * nz) + bc.w * (ce * nz - se * h);
    double r = pn / vn;
    if (!(r > 0.0)) r = 2.0;
    r = (double)q.x * fmin(2.0, fmax(0.5, r));
    const double k = floor(r * to_bin);
    return k < (double)R ? (int)k : -1;
}

// Gather of the union footprint of G beams into their histograms (strips of
// SH rows, 64/SH column phases) by nw waves, this one taking items it0,
// it0 + nw, ...; adds this lane's per-beam sun sums to sacc.  CORR (one
// beam): every sample's bin is its corrected range's (bc: the beam's
// offsets, R: bins); the pixel records still decide validity and shade.
// EACH (fixed point only): every sample is added on its own, with no run
// sums, for frames where neighbouring pixels mostly fall in different bins
// (there the run logic costs more than the adds it saves).
template <int G, int SH, bool SUN, bool CORR, bool IACC = false, bool EACH = false>
__device__ __attribute__((always_inline)) inline void gather_group(
    const FrameDev& f, const int* ub, const int* vb, const bool* have, int r0, int r1, int q0, int q1,
    float* hist, int stride, unsigned* nzmask, int nzs, int lane, int it0, int nw, float* sacc,
    const double4* bc = nullptr, int R = 0, IntAcc ia = IntAcc{})
{
    static_assert(!IACC || !CORR, "fixed point: centre bins");
    static_assert(!EACH || IACC, "per-sample adds: fixed point");
    static_assert(!CORR || G == 1, "corrected ranges differ per beam: one beam per group");
    const bool rng = f.span != 0;
    constexpr int P = 64 / SH;                      // column phases per strip
    const int row_in = lane % SH, phase = lane / SH;
    const int nrows = r1 - r0 + 1;
    const int nstrips = (nrows + SH - 1) / SH;
    const int q0a = q0 & ~3;                        // batches are aligned 4-column blocks
    const int ncols = q1 - q0a + 1;
    // column chunks give every wave work when a group has few strips (a
    // chunk spans at least 32 columns and two rounds of the column phases)
    int nchunk = nw > 1 ? (2 * nw + nstrips - 1) / nstrips : 1;
    nchunk = min(nchunk, max(1, ncols / max(32, 8 * P)));
    const int cw = (((ncols + nchunk - 1) / nchunk) + 3) & ~3;
    const int items = nstrips * nchunk;
    const size_t khp16 = (size_t)(f.KH + 1) * 16u;          // block stride in a copy
    const size_t copy_bytes = (size_t)f.NB * khp16;
    const size_t pstep = (size_t)f.H * 32u, sstep = (size_t)f.H * 16u;
    unsigned nzb = 0u;                                  // chunks this lane wrote
    for (int it = it0; it < items; it += nw) {
        const int s = it / nchunk, ch = it - s * nchunk;
        const int v = r0 + s * SH + row_in;
        const bool rowok = v <= r1;
        const int vv = rowok ? v : r1;                      // in-bounds row for idle lanes
        unsigned kvo[G];                                    // lane offset in a kernel block
        int lo[G], hi[G];
        int cb = INT_MAX, ce = INT_MIN;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int n = vv - vb[g];
            const bool ok = rowok && have[g] && n >= -f.N && n <= f.N;
            // lanes with nothing to add read the zero guard row
            kvo[g] = (unsigned)(ok ? n + f.N : f.KH) * 16u;
            int2 rr = make_int2(INT_MAX, INT_MIN);
            if (ok) {
                const gint2 t = *gptr((const gint2*)(f.rowrange + n + f.N));
                rr = make_int2(t.x, t.y);
            }
            const int wlo = wave_min(rr.x), whi = wave_max(rr.y);
            // absolute columns where this beam can have K > 0 in the strip
            lo[g] = __builtin_amdgcn_readfirstlane(wlo == INT_MAX ? INT_MAX : wlo + ub[g]);
            hi[g] = __builtin_amdgcn_readfirstlane(whi == INT_MIN ? INT_MIN : whi + ub[g]);
            cb = min(cb, lo[g]);
            ce = max(ce, hi[g]);
        }
        cb = max(cb, q0a + ch * cw);
        ce = min(ce, min(q1, q0a + ch * cw + cw - 1));
        if (cb > ce) continue;
        // whole 4-column blocks [cb/4, ce/4]; the extra columns lie outside
        // every beam's kernel support (or past the image: sky padding)
        const int blk0 = cb >> 2, nblk = (ce >> 2) - blk0 + 1;
        const int niter = (nblk + P - 1) / P;
        const char* pbase = (const char*)(f.pix + (size_t)blk0 * f.H * 4);
        const char* sbase = SUN ? (const char*)(f.sun + (size_t)blk0 * f.H * 4) : nullptr;
        const unsigned pvo = (unsigned)vv * 32u, svo = (unsigned)vv * 16u;
        const char* rbase = CORR ? (const char*)(f.rec4 + (size_t)blk0 * f.H * 4) : nullptr;
        double cel = 0.0, sel = 0.0;                     // CORR: the row's elevation cos, sin
        if (CORR) {
            const double2 rc = f.row64[vv];
            cel = rc.x;
            sel = rc.y;
        }
        // per beam: kernel copy (shift) and block of the first batch
        const char* kcopy[G];
        int kblk[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int c0 = 4 * blk0 - ub[g] + f.M;          // kernel column of column 4*blk0
            const int sft = c0 & 3;
            kcopy[g] = (const char*)f.Kb + (size_t)sft * copy_bytes;
            kblk[g] = ((c0 - sft) >> 2) + kBlockPad;
        }
        int cur = -1;
        float acc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = 0.0f;
        const char* pb = pbase + (size_t)phase * pstep;
        const char* sb = SUN ? sbase + (size_t)phase * sstep : nullptr;
        // loads of one batch; the next batch's loads are issued before the
        // current batch is processed, so their latency overlaps the work
        struct Loads {
            int4 ra, rb;
            float4 sq;
            float4 kq[G];
            float4 r4[CORR ? 4 : 1];
            int col;                                    // first column of the block read
        };
        auto fetch = [&](int i, Loads& L) {
            // this lane's block; with column phases the last round may run
            // past the span: such lanes re-read the last block with K = 0
            const int bi = i * P + phase;
            const bool act = P == 1 || bi < nblk;
            const size_t back = act ? 0 : (size_t)(bi - (nblk - 1));
            const char* pq = pb + (size_t)i * P * pstep - back * pstep;
            L.ra = ld16<int4>(pq, pvo);
            L.rb = ld16<int4>(pq, pvo + 16u);
            if (CORR) {
                const size_t rstep = (size_t)f.H * 64u;
                const char* rq = rbase + ((size_t)(act ? bi : nblk - 1)) * rstep;
#pragma unroll
                for (int j = 0; j < 4; ++j) L.r4[j] = ld16<float4>(rq, (unsigned)vv * 64u + 16u * j);
                L.col = 4 * (blk0 + (act ? bi : nblk - 1));
            }
            L.sq = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (SUN) L.sq = ld16<float4>(sb + (size_t)i * P * sstep - back * sstep, svo);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int b = min(max(kblk[g] + bi, 0), f.NB - 1);
                const unsigned ko = act ? kvo[g] : (unsigned)f.KH * 16u;
                L.kq[g] = ld16<float4>(kcopy[g] + (unsigned)(b * (int)khp16), ko);
            }
        };
        auto process = [&](const Loads& L) {
            const int4 ra = L.ra, rb = L.rb;
            const float sv[4] = {L.sq.x, L.sq.y, L.sq.z, L.sq.w};
            float kv[4][G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                kv[0][g] = L.kq[g].x;
                kv[1][g] = L.kq[g].y;
                kv[2][g] = L.kq[g].z;
                kv[3][g] = L.kq[g].w;
            }
            int bin[4] = {ra.x, ra.z, rb.x, rb.z};
            float sh[4] = {__int_as_float(ra.y), __int_as_float(ra.w),
                           __int_as_float(rb.y), __int_as_float(rb.w)};
            if (CORR) {
                // valid pixels (centre bin >= 0) take their corrected bin;
                // a sample past the last bin adds nothing
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (bin[j] >= 0) {
                        const double2 cs = f.col64[min(L.col + j, f.W - 1)];
                        bin[j] = corrected_bin(L.r4[j], cs, cel, sel, bc[0], f.to_bin, R);
                        if (bin[j] < 0) sh[j] = 0.0f;
                    }
                }
            }
            if constexpr (EACH) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const float t = kv[j][g] * sh[j];
                        if (t != 0.0f) {
                            add_key<true>(hist + g * stride, bin[j], t, rng, ia);
                            nzb |= key_chunks(bin[j], nzs, false);   // fixed point: centre bins
                        }
                        if (SUN) sacc[g] += kv[j][g] * sv[j];
                    }
                }
                return;
            }
            // fast path: accumulate without resets and detect breaks
            const int cur0 = cur;
            float acc0[G];
            unsigned long long nrm = 0;
#pragma unroll
            for (int g = 0; g < G; ++g) acc0[g] = acc[g];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                nrm |= __ballot(bin[j] != (j == 0 ? cur0 : bin[j - 1]));
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    acc[g] += kv[j][g] * sh[j];
                    if (SUN) sacc[g] += kv[j][g] * sv[j];
                }
            }
            cur = bin[3];
            if (nrm) {
                // some run ended: replay the batch from its start with the
                // resets, flushing every run that ends (same summation order
                // as the fast path where no run ends)
                float r[G];
                int c = cur0;
#pragma unroll
                for (int g = 0; g < G; ++g) r[g] = acc0[g];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const bool nr = bin[j] != c;
                    unsigned any = __builtin_bit_cast(unsigned, r[0]);
#pragma unroll
                    for (int g = 1; g < G; ++g) any |= __builtin_bit_cast(unsigned, r[g]);
                    const bool fl = nr && any != 0u;            // sums are >= 0
                    const unsigned long long fm = __ballot(fl);
                    if (fm) flush_runs<G, IACC>(fm, fl, c, r, hist, stride, nzb, nzs, lane, rng, ia);
#pragma unroll
                    for (int g = 0; g < G; ++g) r[g] = (nr ? 0.0f : r[g]) + kv[j][g] * sh[j];
                    c = bin[j];
                }
#pragma unroll
                for (int g = 0; g < G; ++g) acc[g] = r[g];
            }
        };
        // two load buffers in turn (no register copies between batches)
        Loads A, B;
        if (niter > 0) fetch(0, A);
        for (int i = 0; i < niter; i += 2) {
            // EACH: the next batch is fetched unconditionally (past the
            // strip it repeats the last batch, from the cache), so that the
            // wait before a batch's adds does not also wait for the next
            // batch's loads
            if (EACH || i + 1 < niter) fetch(min(i + 1, niter - 1), B);
            process(A);
            if (i + 1 >= niter) break;
            if (EACH || i + 2 < niter) fetch(min(i + 2, niter - 1), A);
            process(B);
        }
        unsigned any = __builtin_bit_cast(unsigned, acc[0]);
#pragma unroll
        for (int g = 1; g < G; ++g) any |= __builtin_bit_cast(unsigned, acc[g]);
        const bool fl = any != 0u;
        const unsigned long long fm = __ballot(fl);
        if (fm) flush_runs<G, IACC>(fm, fl, cur, acc, hist, stride, nzb, nzs, lane, rng, ia);
    }
    // the wave's chunk flags, one LDS atomic per wave
    nzb = wave_or(nzb);
    if (lane == 0 && nzb) atomicOr(nzmask, nzb);
}

// Direct gather of one beam for frames whose beams touch few of their pixels
// (the batch runs no pre-pass for them): the cells of the clipped footprint
// window are dealt round the lanes; a cell with K > 0 on a valid pixel takes
// the pixel's bin (FP64), shade and sun shading from the G-buffer planes with
// the pre-pass's formulas and adds K * shade into the histogram with an LDS
// atomic (such frames hold few samples; run sums would rarely pay).
template <bool SUN>
__device__ inline void gather_direct(const FrameDev& f, int R, int ub, int vb, int r0, int r1, int q0,
                                     int q1, float* hist, unsigned* nzmask, int nzs, int lane, float* sacc)
{
    const DirectDev d = load_uniform(f.direct);
    const int nc = q1 - q0 + 1, total = (r1 - r0 + 1) * nc;
    const size_t khp = (size_t)f.KH + 1;
    unsigned nzb = 0u;
    float sun = 0.0f;
    for (int i = lane; i < total; i += 64) {
        const int dv = i / nc;
        const int v = r0 + dv, u = q0 + (i - dv * nc);
        const int c = u - ub + f.M, n = v - vb + f.N;          // kernel column and row
        const float kv = gptr(f.Kb)[(((size_t)(c >> 2) + kBlockPad) * khp + n) * 4 + (c & 3)];
        if (!(kv > 0.0f)) continue;
        const long px = (long)v * d.pitch + u;
        const float dep = gptr(d.depth)[px];
        if (!(dep > 0.0f && isfinite(dep))) continue;
        const double kb = floor((double)dep * f.to_bin);
        if (!(kb < (double)R)) continue;
        const gfloat4 rt4 = *gptr((const gfloat4*)(d.rowtab + v));
        const float4 rt = make_float4(rt4.x, rt4.y, rt4.z, rt4.w);
        const float nx = gptr(d.nx)[px], ny = gptr(d.ny)[px], nz = gptr(d.nz)[px], rho = gptr(d.refl)[px];
        const gfloat2 cs2 = *gptr((const gfloat2*)(d.colcs + u));
        const float sh = pixel_shade(rt, make_float2(cs2.x, cs2.y), nx, ny, nz, rho, gptr(d.gain)[px], dep);
        const int bin = (int)kb;
        if (sh != 0.0f) {
            atomicAdd(hist + bin, kv * sh);
            nzb |= 1u << (bin >> nzs);
        }
        if (SUN) sun += kv * pixel_sun(d.sun_x, d.sun_y, d.sun_z, rt, nx, ny, nz, rho);
    }
    if (SUN) *sacc += sun;
    nzb = wave_or(nzb);
    if (lane == 0 && nzb) atomicOr(nzmask, nzb);
}

// Output bins k0 .. k0 + 7 of the pulse convolution, one block of 8 taps:
// o[q] += w[j] * x[q - j] for the window lo (x[-8 .. -1]) and hi (x[0 .. 7])
// relative to the block's first tap.
__device__ inline void conv_block(float* o, const float4& lo0, const float4& lo1,
                                  const float4& hi0, const float4& hi1, const float* w8)
{
    const float4 wa = *(const float4*)w8, wb = *(const float4*)(w8 + 4);
    const float w[8] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w};
    const float X[16] = {lo0.x, lo0.y, lo0.z, lo0.w, lo1.x, lo1.y, lo1.z, lo1.w,
                         hi0.x, hi0.y, hi0.z, hi0.w, hi1.x, hi1.y, hi1.z, hi1.w};
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int q = 0; q < 8; ++q) o[q] += w[j] * X[q - j + 8];
}

// o[q] = sum_t taps[t] * x[q - t] for q = 0..7 (x = histogram at k0 + J +
// conv_shift(J), the centre of the shifted taps), over nb blocks of 8 taps.
// Every read lies in the zero padding or the histogram; x is 16-byte aligned.
__device__ inline void conv8(float* o, const float* x, const float* taps, int nb)
{
    float4 h0 = *(const float4*)x, h1 = *(const float4*)(x + 4);
    float4 l0 = *(const float4*)(x - 8), l1 = *(const float4*)(x - 4);
#pragma unroll 1
    for (int b = 0; b < nb; b += 2) {
        conv_block(o, l0, l1, h0, h1, taps + 8 * b);
        if (b + 1 >= nb) break;
        // the next block's upper window is this block's lower one
        h0 = *(const float4*)(x - 8 * b - 16);
        h1 = *(const float4*)(x - 8 * b - 12);
        conv_block(o, h0, h1, l0, l1, taps + 8 * b + 8);
        if (b + 2 >= nb) break;
        l0 = *(const float4*)(x - 8 * b - 24);
        l1 = *(const float4*)(x - 8 * b - 20);
    }
}

// Bit i of the result is set when byte i of the 64-bit lane mask is non-zero.
__device__ inline unsigned bytes_any(unsigned long long b)
{
    b |= b >> 4;
    b |= b >> 2;
    b |= b >> 1;
    b &= 0x0101010101010101ull;
    return (unsigned)((b * 0x0102040810204080ull) >> 56);
}

// Pulse convolution outputs k0 .. k0 + 7 of histogram h (before the scale
// and the floor; zero from bin R on), skipped when the gather wrote none of
// the chunks holding their inputs (nzm, chunks of 1 << nzs bins).
__device__ inline void conv_out8(const float* h, const float* taps, const PathDev& p, int nb, int k0,
                                 unsigned nzm, int nzs, float* o8)
{
#pragma unroll
    for (int q = 0; q < 8; ++q) o8[q] = 0.0f;
    if (k0 >= p.R) return;
    const int c0 = max(0, k0 - p.J) >> nzs, c1 = min(p.R - 1, k0 + 7 + p.J) >> nzs;
    const unsigned span = c1 - c0 >= 31 ? ~0u : (2u << (c1 - c0)) - 1u;
    if ((nzm >> c0) & span) conv8(o8, h + k0 + p.J + conv_shift(p.J), taps, nb);
}

// xi_hat = scale * o8 + floor into bins k0 .. k0 + 7 (below R) of h, in place,
// of the kept waveform and of o8; bit q of the result: bin k0 + q is above T.
template <bool KEEP>
__device__ inline unsigned write_out8(float* h, float* kept, int k0, int R, float scale, float floor_b,
                                      float T, float* o8)
{
    float val[8];
    unsigned m8 = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        val[q] = scale * o8[q] + floor_b;
        m8 |= (k0 + q < R && val[q] > T ? 1u : 0u) << q;
    }
    if (k0 + 8 <= R) {
        *(float4*)(h + k0) = make_float4(val[0], val[1], val[2], val[3]);
        *(float4*)(h + k0 + 4) = make_float4(val[4], val[5], val[6], val[7]);
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (k0 + q < R) h[k0 + q] = val[q];
    }
    if (KEEP) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (k0 + q < R) gptr(kept)[k0 + q] = val[q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) o8[q] = val[q];
    return m8;
}

// Echoes of one waveform xh (xi_hat in LDS) by one wave: maximal runs above
// the threshold found with 64-bin ballots over the chunks flagged in am (bit
// c of word w: chunk 32 w + c of 64 bins holds a bin above T; a run cannot
// cross another chunk), their first maximum, crossings and pulse width
// (section II-C, EPW paragraph); writes the first E echoes (or, with an echo
// selection, the one selected run in slot 0), the count of all runs and the
// floor.
__device__ inline void detect_echoes(const FrameDev& f, const PathDev& p, int beam, const float* xh,
                                     const unsigned* am, float floor_b, int lane)
{
    const int R = p.R;
    const float T = p.threshold;
    const float dt = (float)p.bin_ns;
    const bool all = p.select == LIDAR_ECHO_ALL;
    lidar_echo* out = f.echoes + (size_t)beam * p.E;
    lidar_echo sel = {};                                 // selected run (lane 0)
    float sel_key = -INFINITY;
    int count = 0;
    int k0 = -1;                                         // first bin of the open run
    const int nw = (R + kPassBins - 1) / kPassBins;      // mask words of 32 chunks
    int w = 0;
    unsigned bits = __builtin_amdgcn_readfirstlane(am[0]);
    for (;;) {
        while (bits == 0u && ++w < nw) bits = __builtin_amdgcn_readfirstlane(am[w]);
        if (bits == 0u) break;
        const int base = (w * 32 + __builtin_ctz(bits)) * 64;
        bits &= bits - 1u;
        const int k = base + lane;
        const bool above = k < R && xh[k] > T;
        const unsigned long long mask = __ballot(above);
        const bool next_above = base + 64 < R && xh[base + 64] > T;
        const unsigned long long prev = (mask << 1) | (k0 >= 0 ? 1ull : 0ull);
        const unsigned long long nxt = (mask >> 1) | (next_above ? (1ull << 63) : 0ull);
        unsigned long long starts = mask & ~prev;
        unsigned long long ends = mask & ~nxt;
        while (starts | ends) {
            const int ps = starts ? __builtin_ctzll(starts) : 64;
            const int pe = ends ? __builtin_ctzll(ends) : 64;
            if (ps <= pe) {
                k0 = base + ps;
                starts &= starts - 1;
                continue;
            }
            ends &= ends - 1;
            const int k1 = base + pe;
            if (!all || count < p.E) {
                // first maximum of the run
                float lbest = -INFINITY;                 // this lane's first maximum
                int lbk = INT_MAX;
                for (int s = k0; s <= k1; s += 64) {
                    const int kk = s + lane;
                    if (kk <= k1) {
                        const float x = xh[kk];
                        if (x > lbest) {
                            lbest = x;
                            lbk = kk;
                        }
                    }
                }
                // the largest value, then the smallest bin holding it
                const float best = wave_maxf(lbest);
                const int bk = wave_min(lbest == best ? lbk : INT_MAX);
                if (lane == 0) {
                    // threshold crossings between bin centres, as fractions of
                    // a bin from the centre of the bin before the run and from
                    // the centre of its last bin
                    float f_up, f_dn;
                    uint32_t flags = 0;
                    if (k0 == 0) {
                        f_up = 0.5f;
                        flags |= LIDAR_ECHO_AT_FIRST_BIN;
                    } else {
                        const float xa = xh[k0 - 1], xb = xh[k0];
                        f_up = (T - xa) / (xb - xa);
                    }
                    if (k1 == R - 1) {
                        f_dn = 0.5f;
                        flags |= LIDAR_ECHO_AT_LAST_BIN;
                    } else {
                        const float xa = xh[k1], xb = xh[k1 + 1];
                        f_dn = (xa - T) / (xa - xb);
                    }
                    lidar_echo e;
                    e.range_m = ((double)bk + 0.5) * p.half_c_dt;
                    e.time_ns = ((double)bk + 0.5) * p.bin_ns;
                    e.intensity = best - floor_b;
                    e.pulse_width_ns = ((float)(k1 - k0 + 1) + f_dn - f_up) * dt;
                    e.bin_peak = bk;
                    e.bin_first = k0;
                    e.bin_last = k1;
                    e.flags = flags;
                    if (all) {
                        store_echo(out + count, e);
                    } else {
                        // strongest: largest peak; longest: widest pulse;
                        // nearest: the first run (the first wins every tie)
                        const float key = p.select == LIDAR_ECHO_STRONGEST ? best
                                        : p.select == LIDAR_ECHO_LONGEST ? e.pulse_width_ns : 0.0f;
                        if (count == 0 || key > sel_key) {
                            sel = e;
                            sel_key = key;
                        }
                    }
                }
            }
            ++count;
            k0 = -1;
        }
    }
    if (lane == 0) {
        if (!all && count > 0) store_echo(out, sel);
        gptr(f.counts)[beam] = count;
        gptr(f.beams)[beam].floor = floor_b;
    }
    const lidar_echo z = {};
    const int written = all ? count : min(count, 1);
    for (int i = written + lane; i < p.E; i += 64) store_echo(out + i, z);
}

// Echo selection on the raw signal (no pulse post-processing): the bin of
// S_b xi[k] with the largest value (RAW_STRONGEST; the first of equal
// maxima) or the first bin (RAW_NEAREST) at or above T, reported as a
// one-bin echo; one wave per beam over the chunks the gather wrote (nzm,
// chunks of 1 << nzs bins).  Also writes the count (1 or 0), the floor and,
// with KEEP, the raw signal as the kept waveform.
template <bool KEEP>
__device__ inline void detect_raw(const FrameDev& f, const PathDev& p, int beam, const float* h,
                                  unsigned nzm, int nzs, float scale, float floor_b, int lane)
{
    const int R = p.R;
    const float T = p.threshold;
    const bool nearest = p.select == LIDAR_ECHO_RAW_NEAREST;
    float lbest = -INFINITY;
    int lk = INT_MAX;
    int found = -1;
    for (unsigned bits = nzm; bits && found < 0;) {
        const int c = __builtin_ctz(bits);
        bits &= bits - 1u;
        const int end = min(R, (c + 1) << nzs);
        for (int base = c << nzs; base < end; base += 64) {
            const int k = base + lane;
            const float v = k < R ? scale * h[k] : -INFINITY;
            const bool above = v >= T;
            if (nearest) {
                const unsigned long long m = __ballot(above);
                if (m) {
                    found = base + __builtin_ctzll(m);
                    break;
                }
            } else if (above && v > lbest) {
                lbest = v;
                lk = k;
            }
        }
    }
    if (!nearest) {
        const float best = wave_maxf(lbest);
        if (best >= T) found = wave_min(lbest == best ? lk : INT_MAX);
    }
    lidar_echo* out = f.echoes + (size_t)beam * p.E;
    if (lane == 0) {
        if (found >= 0) {
            lidar_echo e;
            e.range_m = ((double)found + 0.5) * p.half_c_dt;
            e.time_ns = ((double)found + 0.5) * p.bin_ns;
            e.intensity = scale * h[found];
            e.pulse_width_ns = 0.0f;
            e.bin_peak = e.bin_first = e.bin_last = found;
            e.flags = 0;
            store_echo(out, e);
        }
        gptr(f.counts)[beam] = found >= 0 ? 1 : 0;
        gptr(f.beams)[beam].floor = floor_b;
    }
    const lidar_echo z = {};
    for (int i = (found >= 0 ? 1 : 0) + lane; i < p.E; i += 64) store_echo(out + i, z);
    if (KEEP) {
        auto w = gptr(f.waves + (size_t)beam * R);
        for (int k = lane; k < R; k += 64) w[k] = scale * h[k];
    }
}

// LDS written by some lanes of this wave is read by others after this point.
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// The wave schedule's convolution runs in passes of 512 bins (8 per lane).
constexpr int kWavePassBins = 512;
constexpr int kWavePasses = kWaveMaxBins / kWavePassBins;

// Lanes below this one with their bit set in m.
__device__ inline int lanes_below(unsigned long long m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// 64-bit key of a bin of a run: the value's bits in an order-preserving form,
// then the complement of the bin, so that the largest key is the run's
// largest value at its smallest bin (its first maximum).
__device__ inline unsigned long long peak_key(float v, int k)
{
    const unsigned u = __float_as_uint(v);
    const unsigned o = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return (unsigned long long)o << 32 | (0xffffffffu - (unsigned)k);
}

__device__ inline float peak_value(unsigned long long key)
{
    const unsigned o = (unsigned)(key >> 32);
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

// Echoes of the first runs of one waveform by one wave, for LIDAR_ECHO_ALL
// (the first E runs) and LIDAR_ECHO_NEAREST (the first run), found pass by
// pass as the convolution's outputs are written (runs_pass), then written out
// (runs_finish).  Bit q of lane l's above-threshold mask m8 in pass ps is bin
// ps * kWavePassBins + 8 l + q.  Run starts and ends come from the bits and
// a neighbour ballot (a run reaching the pass's last bin ends there until a
// later pass continues it and overwrites its end), a run's index from the
// starts before it (per-lane counts and a wave prefix), and each wanted run's
// first maximum from one 64-bit LDS max per bin (peak_key) into rk; rb
// receives its first and last bin.  Every run is counted.  The echoes, count
// and floor are those detect_echoes writes for the same waveform (section
// II-C, EPW paragraph).
struct RunScan {
    int want;           // runs that give echoes
    int base;           // runs started in earlier passes (uniform)
    unsigned carry;     // the bin before this pass is above T (uniform)
};

__device__ inline void runs_pass(RunScan& rs, int ps, unsigned m, const float* val, int lane,
                                 unsigned long long* rk, int2* rb)
{
    const unsigned long long b7 = __ballot((m >> 7) & 1u), b0 = __ballot(m & 1u);
    const unsigned prev = ((unsigned)((b7 << 1) >> lane) & 1u) | (lane == 0 ? rs.carry : 0u);
    const unsigned nxt = (unsigned)((b0 >> 1) >> lane) & 1u;
    const unsigned st = m & ~((m << 1) | prev);
    const unsigned en = m & ~((m >> 1) | (nxt << 7));
    const int ns = __popc(st);                           // at most 4
    const unsigned long long c0 = __ballot(ns & 1), c1 = __ballot(ns & 2), c2 = __ballot(ns & 4);
    // uniform: a wanted run starts here or continues from the last pass
    if (rs.base - (int)rs.carry < rs.want) {
        // bins before this lane's first start continue the previous run
        int id = rs.base + lanes_below(c0) + 2 * lanes_below(c1) + 4 * lanes_below(c2) - 1;
        // the lane's first bin, opaque to the optimiser: the keys' bin words
        // depend only on the lane, and hoisted out of the beam loop they
        // would hold 8 registers per pass for the kernel's lifetime
        int k8 = ps * kWavePassBins + lane * 8;
        asm volatile("" : "+v"(k8));
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            id += (st >> q) & 1u;
            if (((m >> q) & 1u) && id < rs.want) {
                const int k = k8 + q;
                atomicMax(rk + id, peak_key(val[q], k));
                if ((st >> q) & 1u) rb[id].x = k;
                if ((en >> q) & 1u) rb[id].y = k;
            }
        }
    }
    rs.base += __popcll(c0) + 2 * __popcll(c1) + 4 * __popcll(c2);
    rs.carry = (unsigned)(b7 >> 63);
}

// After every pass and a wave_sync: the echoes of the first runs from rk, rb
// and the crossings' bins in xh (xi_hat in LDS), the count, the floor.
__device__ inline void runs_finish(const RunScan& rs, const FrameDev& f, const PathDev& p, int beam,
                                   const float* xh, float floor_b, int lane, const unsigned long long* rk,
                                   const int2* rb)
{
    const int R = p.R;
    const float T = p.threshold;
    const int count = rs.base;
    const int nrun = min(count, rs.want);
    lidar_echo* out = f.echoes + (size_t)beam * p.E;
    if (lane < nrun) {
        const unsigned long long key = rk[lane];
        const int2 kk = rb[lane];
        const int k0 = kk.x, k1 = kk.y;
        const int bk = (int)(0xffffffffu - (unsigned)key);
        const float best = peak_value(key);
        const float dt = (float)p.bin_ns;
        // threshold crossings between bin centres, as fractions of a bin
        // from the centre of the bin before the run and from the centre of
        // its last bin
        float f_up, f_dn;
        uint32_t flags = 0;
        if (k0 == 0) {
            f_up = 0.5f;
            flags |= LIDAR_ECHO_AT_FIRST_BIN;
        } else {
            const float xa = xh[k0 - 1], xb = xh[k0];
            f_up = (T - xa) / (xb - xa);
        }
        if (k1 == R - 1) {
            f_dn = 0.5f;
            flags |= LIDAR_ECHO_AT_LAST_BIN;
        } else {
            const float xa = xh[k1], xb = xh[k1 + 1];
            f_dn = (xa - T) / (xa - xb);
        }
        lidar_echo e;
        e.range_m = ((double)bk + 0.5) * p.half_c_dt;
        e.time_ns = ((double)bk + 0.5) * p.bin_ns;
        e.intensity = best - floor_b;
        e.pulse_width_ns = ((float)(k1 - k0 + 1) + f_dn - f_up) * dt;
        e.bin_peak = bk;
        e.bin_first = k0;
        e.bin_last = k1;
        e.flags = flags;
        store_echo(out + lane, e);
    }
    if (lane == 0) {
        gptr(f.counts)[beam] = count;
        gptr(f.beams)[beam].floor = floor_b;
    }
    const lidar_echo z = {};
    for (int i = nrun + lane; i < p.E; i += 64) store_echo(out + i, z);
}

// One wave turns a fixed-point histogram of n integers into FP32 bins in
// place, in chunks of 64 integers: chunk c (integers 64c ..) writes floats
// lo + 64c .. lo + 64c + 63, which held integers 32c .. 32c + 31, already
// read by this chunk (before its writes) or an earlier one.  The floats past
// the bins, which held integers, are zeroed.  Returns the largest bin (every
// lane).
__device__ inline float fixed_to_float(float* h, int n, IntAcc ia, int lane)
{
    const float inv = 1.0f / ia.scale;                   // a power of two
    unsigned long long qmax = 0;
    for (int c = 0; c < n; c += 64) {                    // uniform
        const int j = c + lane;
        const unsigned long long q = j < n ? *(const unsigned long long*)(h + ia.lo + 2 * j) : 0ull;
        qmax = q > qmax ? q : qmax;
        wave_sync();
        if (j < n) h[ia.lo + j] = (float)q * inv;
        wave_sync();
    }
    for (int k = ia.lo + n + lane; k < ia.lo + 2 * n; k += 64) h[k] = 0.0f;
    wave_sync();
    return (float)wave_max_u64(qmax) * inv;
}

// The fixed-point unit of beams with at most `samples` cells each: no bin
// can exceed U = samples x max K x the frame's largest shade, so units of
// 2^-s with U < 2^(61 - s) cannot overflow.  Returns the number of integers
// (0: FP32 accumulation: no statistics, the integers would not fit the slot,
// or U out of range).
__device__ inline int fixed_unit(const FrameDev& f, float samples, int R, IntAcc* ia)
{
    if (!f.fstats) return 0;
    const int lo = f.fstats[1] & ~1, hi = f.fstats[2];
    const float U = samples * f.kmax * __int_as_float(f.fstats[0]);
    int e = 0;
    (void)frexpf(U, &e);                                 // U < 2^e
    // the integers of bins lo .. hi end inside the slot's R floats
    if (!(hi >= lo && lo + 2 * (hi - lo + 1) <= R && U > 0.0f && U < 1e30f && 61 - e <= 120)) return 0;
    ia->scale = ldexpf(1.0f, 61 - e);
    ia->lo = lo;
    ia->each = f.fstats[3] != 0;
    return hi - lo + 1;
}

// Whether the truncation error of a fixed-point histogram (under one unit per
// flush, at most `samples` flushes into a bin) exceeds 1e-6 of the least the
// waveform's maximum can be: the pulse's centre tap times the largest bin
// (S_b applied), or the floor.
__device__ inline bool fixed_too_coarse(float samples, IntAcc ia, float vmax, float tc, float scale,
                                        float floor_b)
{
    const float err = samples / ia.scale;
    return !(err * scale <= 1e-6f * (tc * vmax * scale + floor_b));
}

// The whole group after the histograms were zeroed: gather, floor, pulse,
// echoes.  All threads of the workgroup call it with the same group.  hist is
// beam 0's histogram, beam g's starts RS floats further (zero padding around
// each); bit c of *nzmask flags the chunks of 1 << nzs bins (chunk_shift) that
// the gather wrote, amask the 64-bin chunks of
// each waveform that hold a bin above the threshold.
template <int G, bool SUN, bool KEEP, bool CORR = false, bool DET = false, bool FX = false>
__device__ __attribute__((always_inline)) inline int2 process_group(const FrameDev& f, const PathDev& p, const int32_t* grp,
                              float* hist, const float* taps, float (*red)[kWaves],
                              unsigned* nzmask, unsigned (*amask)[kMaxBins / kPassBins + 1])
{
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int R = p.R;
    const int RS = conv_stride(R, p.J);
    const int nzs = chunk_shift(R);

    // group members (uniform over the workgroup: kept in scalar registers)
    int beam[G], ub[G], vb[G];
    float scale[G], given[G];
    bool have[G];
    float samples = 0.0f;                               // the most cells of a member (FX)
    int2 fxc = make_int2(0, 0);                          // this wave's counts {fixed point, redone} (FX)
    int umin = INT_MAX, umax = INT_MIN, vmin = INT_MAX, vmax = INT_MIN;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        beam[g] = load_uniform(grp + g);
        have[g] = beam[g] >= 0;
        ub[g] = vb[g] = 0;
        scale[g] = given[g] = 0.0f;
        if (have[g]) {
            // pixel and scale are not written by this kernel (only the floor is)
            const lidar_beam_info bi = load_uniform(f.beams + beam[g]);
            ub[g] = __builtin_amdgcn_readfirstlane(bi.pixel_u);
            vb[g] = __builtin_amdgcn_readfirstlane(bi.pixel_v);
            scale[g] = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(
                __builtin_bit_cast(int, bi.scale)));
            given[g] = bi.floor;                        // the floor when f.floor_given
            samples = fmaxf(samples, (float)bi.samples);
            umin = min(umin, ub[g]);
            umax = max(umax, ub[g]);
            vmin = min(vmin, vb[g]);
            vmax = max(vmax, vb[g]);
        }
    }
    // union window of the group's footprints, clipped to the image
    // (64-bit arithmetic: beams may lie far outside the image)
    const int r0 = (int)max(0L, (long)vmin - f.N), r1 = (int)min((long)f.H - 1, (long)vmax + f.N);
    const int q0 = (int)max(0L, (long)umin - f.M), q1 = (int)min((long)f.W - 1, (long)umax + f.M);
    float sacc[G];
#pragma unroll
    for (int g = 0; g < G; ++g) sacc[g] = 0.0f;
    double4 bc[1] = {make_double4(1.0, 0.0, 1.0, 0.0)};
    if (CORR && have[0]) bc[0] = load_uniform(f.bcorr + beam[0]);
    static_assert(!DET || G == 1, "deterministic groups hold one beam");
    static_assert(!FX || (!CORR && !DET && G <= kWaves), "fixed point: centre bins, a wave per member");
    // DET: every wave gathers into a histogram slot of its own
    float* ghist = DET ? hist + wave * RS : hist;
    // FX (batches): the members' histograms in fixed point with one unit
    IntAcc ia{0.0f, 0, false};
    const int span = FX && r0 <= r1 && q0 <= q1 ? fixed_unit(f, samples, R, &ia) : 0;
    // (run sums throughout: the per-sample adds are the wave schedule's)
    auto gather = [&](auto iacc, float* acc) {
        constexpr bool I = decltype(iacc)::value;
        if (f.tile == 64)
            gather_group<G, 64, SUN, CORR, I>(f, ub, vb, have, r0, r1, q0, q1, ghist, RS, nzmask, nzs, lane,
                                              wave, kWaves, acc, bc, R, ia);
        else if (f.tile == 16)
            gather_group<G, 16, SUN, CORR, I>(f, ub, vb, have, r0, r1, q0, q1, ghist, RS, nzmask, nzs, lane,
                                              wave, kWaves, acc, bc, R, ia);
        else
            gather_group<G, 4, SUN, CORR, I>(f, ub, vb, have, r0, r1, q0, q1, ghist, RS, nzmask, nzs, lane,
                                             wave, kWaves, acc, bc, R, ia);
    };
    if (r0 <= r1 && q0 <= q1) {
        bool done = false;
        if constexpr (FX) {
            if (span) {
                gather(std::true_type{}, sacc);
                done = true;
            }
        }
        if (!done) gather(std::false_type{}, sacc);
    }
    if (SUN) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const float w = wave_total(sacc[g]);
            if (lane == 0) red[g][wave] = w;
        }
    }
    __syncthreads();
    if constexpr (DET) {
        // the waves' slots summed into slot 0 in wave order: the waveform no
        // longer depends on which wave's LDS atomics came first
        for (int k = tid; k < R; k += kFootprintThreads) {
            float t = hist[k];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) t += hist[w * RS + k];
            hist[k] = t;
        }
        __syncthreads();
    }

    // pulse convolution in place, 8 consecutive bins per thread and pass with
    // a sliding register window: xi_hat = S_b (varpi * hist) + A_b
    float floor_b[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        float fl = p.ambient;
        if (SUN) {
            float t = 0.0f;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) t += red[g][w];
            fl += f.sun_scale * t;
        }
        floor_b[g] = f.floor_given ? given[g] : fl;
    }
    if constexpr (FX) {
        if (span) {
            // wave g turns member g's integers into FP32 bins; if any member's
            // truncation bound is too coarse, the group runs again with FP32
            // atomics
            __shared__ int fx_redo;
            if (tid == 0) fx_redo = 0;
            __syncthreads();
            float sc = 0.0f, fb = 0.0f;
            int mb = -1;                                 // this wave's member
#pragma unroll
            for (int g = 0; g < G; ++g)
                if (g == wave && have[g]) {
                    sc = scale[g];
                    fb = floor_b[g];
                    mb = beam[g];
                }
            if (mb >= 0) {
                const float ns = (float)load_uniform(f.beams + mb).samples;
                const float vm = fixed_to_float(hist + wave * RS, span, ia, lane);
                const bool bad = fixed_too_coarse(ns, ia, vm, taps[conv_shift(p.J) + p.J], sc, fb);
                fxc.x = 1;
                if (lane == 0 && bad) fx_redo = 1;
            }
            __syncthreads();
            if (fx_redo) {
                if (wave == 0) {
#pragma unroll
                    for (int g = 0; g < G; ++g) fxc.y += have[g] ? 1 : 0;
                }
                float4* h4 = (float4*)(hist - conv_pad(p.J));
                for (int k = tid; k < G * RS / 4; k += kFootprintThreads) h4[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (tid == 0) *nzmask = 0u;
                __syncthreads();
                float s2[G];
#pragma unroll
                for (int g = 0; g < G; ++g) s2[g] = 0.0f;
                if (r0 <= r1 && q0 <= q1) gather(std::false_type{}, s2);
                __syncthreads();
            }
        }
    }
    if (p.select >= LIDAR_ECHO_RAW_STRONGEST) {
        // single echo on the raw signal: no pulse convolution
        const unsigned nzr = __builtin_amdgcn_readfirstlane(*nzmask);
#pragma unroll 1
        for (int g = wave; g < G; g += kWaves)
            if (have[g]) detect_raw<KEEP>(f, p, beam[g], hist + g * RS, nzr, nzs, scale[g], floor_b[g], lane);
        return fxc;
    }
    constexpr int kPass = kPassBins;                    // 8 bins per thread and pass
    constexpr int kMaxPass = (kMaxBins + kPass - 1) / kPass;
    const float T = p.threshold;
    const int nb = conv_taps(p.J) / 8;
    const unsigned nzm = __builtin_amdgcn_readfirstlane(*nzmask);
    // outputs k0 .. k0 + 7 of pass ps for beam g into o8
    auto conv_pass = [&](int g, int ps, float* o8) {
        conv_out8(hist + g * RS, taps, p, nb, ps * kPass + tid * 8, nzm, nzs, o8);
    };
    // xi_hat of pass ps for beam g in place (after every read of it), the
    // kept waveform and the chunks above the threshold (this wave's 512 bins
    // are chunks 8 * wave .. 8 * wave + 7 of the pass)
    auto write_pass = [&](int g, int ps, float* o8) {
        if (ps * kPass >= R) return;                     // uniform
        const unsigned m8 = write_out8<KEEP>(hist + g * RS, KEEP ? f.waves + (size_t)beam[g] * R : nullptr,
                                             ps * kPass + tid * 8, R, scale[g], floor_b[g], T, o8);
        const unsigned byte = bytes_any(__ballot(m8 != 0u));
        if (lane == 0) ((unsigned char*)amask[g])[ps * 4 + wave] = (unsigned char)byte;
    };
    if (R <= kPass) {
        // one pass: every beam's outputs stay in registers, one barrier
        float o[G][8];
#pragma unroll
        for (int g = 0; g < G; ++g)
            if (have[g]) conv_pass(g, 0, o[g]);          // uniform
        __syncthreads();                                 // every read of the histograms is done
#pragma unroll
        for (int g = 0; g < G; ++g)
            if (have[g]) write_pass(g, 0, o[g]);
    } else {
#pragma unroll 1
        for (int g = 0; g < G; ++g) {
            if (!have[g]) continue;                      // uniform
            float o[kMaxPass][8];
#pragma unroll
            for (int ps = 0; ps < kMaxPass; ++ps) conv_pass(g, ps, o[ps]);
            __syncthreads();                             // every read of h is done
#pragma unroll
            for (int ps = 0; ps < kMaxPass; ++ps) write_pass(g, ps, o[ps]);
        }
    }
    __syncthreads();

    // echo detection: wave w takes beams w, w + 4, ...
#pragma unroll 1
    for (int g = wave; g < G; g += kWaves)
        if (have[g]) detect_echoes(f, p, beam[g], hist + g * RS, amask[g], floor_b[g], lane);
    return fxc;
}

// Whether pass ps (bins ps * kWavePassBins ..) of the wave schedule's
// convolution reads no chunk the gather wrote (nzm): every output of it is
// then zero (the union of conv_out8's per-lane chunk tests, widened).
__device__ inline bool pass_quiet(unsigned nzm, int nzs, int ps, int J, int R)
{
    const int k0 = ps * kWavePassBins;
    const int c0 = max(0, k0 - J) >> nzs, c1 = min(R - 1, k0 + kWavePassBins - 1 + J) >> nzs;
    const unsigned span = c1 - c0 >= 31 ? ~0u : (2u << (c1 - c0)) - 1u;
    return ((nzm >> c0) & span) == 0u;
}

// Zero what a beam of the wave schedule left in its histogram slot: the bins
// of the passes in `dirty` and the first and last bins of the passes in
// `edges` (process_beam_wave's return, bits 8 .. and 16 ..); the zero padding
// around the bins is never written.
template <int NP>
__device__ inline void clear_passes(float* hist, int R, unsigned dirty, unsigned edges, int lane)
{
#pragma unroll
    for (int ps = 0; ps < NP; ++ps) {
        const int k0 = ps * kWavePassBins, k1 = min(R, k0 + kWavePassBins);
        if ((dirty >> ps) & 1u)
            for (int k = k0 + lane; k < k1; k += 64) hist[k] = 0.0f;
        if (((edges >> ps) & 1u) && lane == 0) {
            hist[k0] = 0.0f;
            hist[k1 - 1] = 0.0f;
        }
    }
}

// One beam by one wave (the wave schedule of a batch), after the wave zeroed
// its histogram slot hist (zero padding around it) and its chunk flags nzw:
// the steps of process_group with wave-local ordering only, the convolution in
// NP passes of 512 bins (8 per lane; R <= kWavePassBins * NP).  Returns the
// fixed-point outcome (bit 0: fixed point, bit 1: run again in FP32) and what
// the beam left in its slot for clear_passes: bit 8 + ps for a pass whose bins
// were written, bit 16 + ps for a quiet pass of which only the first and last
// bins were (ALL and NEAREST with the floor at or below T: such a pass is the
// floor throughout, holds no run, and only its edge bins can be read, as the
// crossings of runs in the neighbouring passes).

template <int NP, bool SUN, bool KEEP>
__device__ __attribute__((always_inline)) inline int process_beam_wave(
    const FrameDev& f, const PathDev& p, int beam, float* hist, int RS, const float* taps, unsigned* nzw,
    unsigned* am, int lane, unsigned long long* rk, int2* rb)
{
    const int R = p.R;
    const int nzs = chunk_shift(R);
    const lidar_beam_info bi = load_uniform(f.beams + beam);
    const int u = __builtin_amdgcn_readfirstlane(bi.pixel_u);
    const int v = __builtin_amdgcn_readfirstlane(bi.pixel_v);
    const float scale = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(
        __builtin_bit_cast(int, bi.scale)));
    const int r0 = (int)max(0L, (long)v - f.N), r1 = (int)min((long)f.H - 1, (long)v + f.N);
    const int q0 = (int)max(0L, (long)u - f.M), q1 = (int)min((long)f.W - 1, (long)u + f.M);
    const bool one = true;
    const bool win = r0 <= r1 && q0 <= q1;
    // fixed point when the frame's bins fit the slot as 64-bit integers (not
    // in the instance for waveforms of up to 512 bins, whose registers are
    // budgeted for eight waves per SIMD)
    IntAcc ia{0.0f, 0, false};
    const int span = NP > 1 && win ? fixed_unit(f, (float)bi.samples, R, &ia) : 0;
    auto gather = [&](auto iacc, auto each, float* acc) {
        constexpr bool I = decltype(iacc)::value, E = decltype(each)::value;
        if (f.tile == 64)
            gather_group<1, 64, SUN, false, I, E>(f, &u, &v, &one, r0, r1, q0, q1, hist, RS, nzw, nzs, lane, 0,
                                                  1, acc, nullptr, 0, ia);
        else if (f.tile == 16)
            gather_group<1, 16, SUN, false, I, E>(f, &u, &v, &one, r0, r1, q0, q1, hist, RS, nzw, nzs, lane, 0,
                                                  1, acc, nullptr, 0, ia);
        else
            gather_group<1, 4, SUN, false, I, E>(f, &u, &v, &one, r0, r1, q0, q1, hist, RS, nzw, nzs, lane, 0,
                                                 1, acc, nullptr, 0, ia);
    };
    float sacc = 0.0f;
    if (win && f.direct)
        gather_direct<SUN>(f, R, u, v, r0, r1, q0, q1, hist, nzw, nzs, lane, &sacc);
    else if (win) {
        bool done = false;
        if constexpr (NP > 1) {
            if (span) {
                if (ia.each) gather(std::true_type{}, std::true_type{}, &sacc);
                else gather(std::true_type{}, std::false_type{}, &sacc);
                done = true;
            }
        }
        if (!done) gather(std::false_type{}, std::false_type{}, &sacc);
    }
    float floor_b = p.ambient;
    if (SUN) floor_b += f.sun_scale * wave_total(sacc);
    if (f.floor_given) floor_b = bi.floor;
    wave_sync();                                         // the histogram is complete
    int fx = 0;                                          // 1: fixed point, 3: fixed point run again
    if (NP > 1 && span) {
        // integers to FP32 bins in place; a beam whose truncation bound is
        // too coarse runs again with FP32 atomics
        const float vmax = fixed_to_float(hist, span, ia, lane);
        const bool redo = fixed_too_coarse((float)bi.samples, ia, vmax, taps[conv_shift(p.J) + p.J], scale,
                                           floor_b);
        fx = __builtin_amdgcn_readfirstlane(redo ? 3 : 1);
        if (redo) {
            for (int k = ia.lo + lane; k < ia.lo + 2 * span; k += 64) hist[k] = 0.0f;
            if (lane == 0) *nzw = 0u;
            wave_sync();
            float s2 = 0.0f;
            gather(std::false_type{}, std::false_type{}, &s2);
            wave_sync();
        }
    }
    const unsigned nzm = __builtin_amdgcn_readfirstlane(*nzw);
    const unsigned all_passes = ((1u << ((R + kWavePassBins - 1) / kWavePassBins)) - 1u) << 8;
    if (p.select >= LIDAR_ECHO_RAW_STRONGEST) {
        detect_raw<KEEP>(f, p, beam, hist, nzm, nzs, scale, floor_b, lane);
        return fx | (int)all_passes;
    }
    const int nb = conv_taps(p.J) / 8;
    float o[NP][8];
#pragma unroll
    for (int ps = 0; ps < NP; ++ps)
        conv_out8(hist, taps, p, nb, ps * kWavePassBins + lane * 8, nzm, nzs, o[ps]);
    // the first runs are found as the passes are written (ALL, NEAREST)
    const bool first = p.select == LIDAR_ECHO_ALL || p.select == LIDAR_ECHO_NEAREST;
    RunScan rs{p.select == LIDAR_ECHO_ALL ? p.E : 1, 0, 0u};
    if (first && lane < rs.want) rk[lane] = 0ull;
    wave_sync();                                         // every read of the histogram is done
    unsigned word = 0;                                   // chunks above the threshold
    unsigned slot = 0;                                   // what the beam leaves in its slot
    const bool quiet_ok = first && !(floor_b > p.threshold);
#pragma unroll
    for (int ps = 0; ps < NP; ++ps) {
        if (ps * kWavePassBins >= R) break;              // uniform
        if (quiet_ok && pass_quiet(nzm, nzs, ps, p.J, R)) {
            // xi_hat is the floor throughout: no run; the edge bins for the
            // crossings of runs in the neighbouring passes
            const int k0 = ps * kWavePassBins, k1 = min(R, k0 + kWavePassBins) - 1;
            if (lane == 0) {
                hist[k0] = floor_b;
                hist[k1] = floor_b;
            }
            if (KEEP) {
                auto w = gptr(f.waves + (size_t)beam * R);
                for (int k = k0 + lane; k <= k1; k += 64) w[k] = floor_b;
            }
            rs.carry = 0u;
            slot |= 1u << (16 + ps);
            continue;
        }
        slot |= 1u << (8 + ps);
        const unsigned m8 = write_out8<KEEP>(hist, KEEP ? f.waves + (size_t)beam * R : nullptr,
                                             ps * kWavePassBins + lane * 8, R, scale, floor_b,
                                             p.threshold, o[ps]);
        if (first) runs_pass(rs, ps, m8, o[ps], lane, rk, rb);
        else word |= bytes_any(__ballot(m8 != 0u)) << (8 * ps);
    }
    if (first) {
        wave_sync();
        runs_finish(rs, f, p, beam, hist, floor_b, lane, rk, rb);
        return fx | (int)slot;
    }
    if (lane == 0) am[0] = word;
    wave_sync();
    detect_echoes(f, p, beam, hist, am, floor_b, lane);
    return fx | (int)slot;
}

}  // namespace

// Zero the G padded histograms (float4 stores) and the chunk flags; load the
// taps with their zero padding.
__device__ inline void clear_group(float4* lds4, int n4, unsigned* nzmask, int tid)
{
    const float4 z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int k = tid; k < n4; k += kFootprintThreads) lds4[k] = z;
    if (tid == 0) *nzmask = 0u;
}

__device__ inline void load_taps(float* taps, const float* src, int J, int tid)
{
    const int d = conv_shift(J);
    for (int j = tid; j < conv_taps(J); j += kFootprintThreads)
        taps[j] = (j >= d && j - d <= 2 * J) ? src[j - d] : 0.0f;
}

template <int G, bool SUN, bool KEEP>
__global__ __launch_bounds__(kFootprintThreads)
void k_footprint(FootprintArgs a)
{
    extern __shared__ float4 lds4[];                // group_lds_bytes(G, R, J)
    const int RS = conv_stride(a.p.R, a.p.J);
    float* hist = (float*)lds4 + conv_pad(a.p.J);   // [G][RS]: sum K * shade, then xi_hat
    float* taps = (float*)lds4 + G * RS;            // [conv_taps(J)]
    __shared__ float red[G][kWaves];
    __shared__ unsigned nzmask;
    __shared__ unsigned amask[G][kMaxBins / kPassBins + 1];

    // XCD-aware schedule: workgroups go round-robin over the 8 XCDs, so slot
    // s runs on XCD s % 8; each XCD takes one contiguous run of the
    // spatially ordered groups, and the groups in flight on it share their
    // pixels in its L2.
    const int slot = blockIdx.x;
    const int gi = (slot % kXcds) * a.chunk + slot / kXcds;
    if (gi >= a.n_groups) return;
    const int tid = threadIdx.x;
    clear_group(lds4, G * RS / 4, &nzmask, tid);
    load_taps(taps, a.p.taps, a.p.J, tid);
    __syncthreads();
    process_group<G, SUN, KEEP>(a.f, a.p, a.groups + (size_t)gi * G, hist, taps, red, &nzmask,
                                amask);
}

// The single-frame kernel with groups of one beam: CORR gives every sample
// its corrected bin (LIDAR_RANGE_CORRECTED); DET (LIDAR_DETERMINISTIC) gives
// every wave its own histogram slot, the slots summed in a fixed order.
template <bool SUN, bool KEEP, bool CORR, bool DET>
__global__ __launch_bounds__(kFootprintThreads)
void k_footprint_one(FootprintArgs a)
{
    extern __shared__ float4 lds4[];
    constexpr int S = DET ? kWaves : 1;             // histogram slots
    const int RS = conv_stride(a.p.R, a.p.J);
    float* hist = (float*)lds4 + conv_pad(a.p.J);
    float* taps = (float*)lds4 + S * RS;
    __shared__ float red[1][kWaves];
    __shared__ unsigned nzmask;
    __shared__ unsigned amask[1][kMaxBins / kPassBins + 1];
    const int slot = blockIdx.x;
    const int gi = (slot % kXcds) * a.chunk + slot / kXcds;
    if (gi >= a.n_groups) return;
    const int tid = threadIdx.x;
    clear_group(lds4, S * RS / 4, &nzmask, tid);
    load_taps(taps, a.p.taps, a.p.J, tid);
    __syncthreads();
    process_group<1, SUN, KEEP, CORR, DET>(a.f, a.p, a.groups + gi, hist, taps, red, &nzmask, amask);
}

// Sun floor of every beam from a collector-sensitivity table: A_b = ambient
// + E_sun * sum over the kernel window (inside the image) of kappa(m, n) times
// the pixel's sun shading Omega (rho/pi) max(0, n.s) (zero for invalid
// pixels).  One workgroup per beam; lanes own rows, so the 16-byte loads of
// the 4-column blocks of sun shading and kappa coalesce as in the gather.
__global__ __launch_bounds__(256)
void k_sun_floor(SunFloorArgs a)
{
    __shared__ float part[256 / 64];
    const int b = blockIdx.x;
    if (b >= a.B) return;
    const lidar_beam_info bi = a.beams[b];
    const int u = bi.pixel_u, v = bi.pixel_v;
    const int r0 = (int)max(0L, (long)v - a.N), r1 = (int)min((long)a.H - 1, (long)v + a.N);
    const int q0 = (int)max(0L, (long)u - a.M), q1 = (int)min((long)a.W - 1, (long)u + a.M);
    float acc = 0.0f;
    if (r0 <= r1 && q0 <= q1) {
        const int nrows = r1 - r0 + 1, blk0 = q0 >> 2, nblk = (q1 >> 2) - blk0 + 1;
        const size_t khp16 = (size_t)(a.KH + 1) * 4;      // floats per kernel block
        for (int t = threadIdx.x; t < nrows * nblk; t += blockDim.x) {
            const int row = r0 + t % nrows, blk = blk0 + t / nrows;
            const float4 sv = *(const float4*)(a.sun + ((size_t)blk * a.H + row) * 4);
            const int c0 = 4 * blk - u + a.M;              // kernel column of the block's first column
            const int sft = c0 & 3;
            const int kb = min(max(((c0 - sft) >> 2) + kBlockPad, 0), a.NB - 1);
            const float4 kq = *(const float4*)(a.Kr + ((size_t)sft * a.NB + kb) * khp16 +
                                               (size_t)(row - v + a.N) * 4);
            acc += kq.x * sv.x + kq.y * sv.y + kq.z * sv.z + kq.w * sv.w;
        }
    }
    const float w = wave_total(acc);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) part[wv] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int i = 0; i < (int)(blockDim.x / 64); ++i) t += part[i];
        a.beams[b].floor = a.ambient + a.e_sun * t;
    }
}

// Next ticket from the dispenser of a batch: kXcds counters kQueueStride ints
// apart, counter c handing out tickets c, c + kXcds, ... (so the costliest
// tickets still go first).  A worker starts at its XCD's counter and moves to
// the next one when it runs dry; the atomics of the workers are spread over
// eight addresses instead of serialising on one, and a counter seen dry by a
// plain load is passed over without an atomic.  Returns n when every counter
// is exhausted.
__device__ inline int next_ticket(int* q, int& c, int n)
{
    for (int tried = 0; tried < kXcds; ++tried) {
        int* qc = q + c * kQueueStride;
        if (tried == 0 ||
            __hip_atomic_load(qc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) * kXcds + c < n) {
            const int t = atomicAdd(qc, 1) * kXcds + c;
            if (t < n) return t;
        }
        c = c + 1 == kXcds ? 0 : c + 1;
    }
    return n;
}

// Persistent kernel over the items of a batch: each workgroup repeatedly
// takes the next ticket (a run of items, costliest first) from the queue, so
// frames of very different sizes share the GPU without a tail of idle CUs,
// and cheap items cost a fraction of a queue atomic each.  Every workgroup
// exits once the queue is exhausted.
template <int G, bool SUN, bool KEEP>
__global__ __launch_bounds__(kFootprintThreads) __attribute__((amdgpu_waves_per_eu(KEEP || SUN ? 1 : 4)))
void k_footprint_batch(BatchArgs a)
{
    extern __shared__ float4 lds4[];
    const int RS = conv_stride(a.p.R, a.p.J);
    float* hist = (float*)lds4 + conv_pad(a.p.J);
    float* taps = (float*)lds4 + G * RS;
    __shared__ float red[G][kWaves];
    __shared__ unsigned nzmask;
    __shared__ unsigned amask[G][kMaxBins / kPassBins + 1];
    __shared__ int item_sh;
    const int tid = threadIdx.x;
    load_taps(taps, a.p.taps, a.p.J, tid);
    const int n_tickets = a.tickets ? a.n_tickets : (a.n_items_dev ? *a.n_items_dev : a.n_items);
    int qc = blockIdx.x % kXcds;                         // this workgroup's XCD (round-robin dispatch)
    // this wave's counts {beams in fixed point, beams run again}, added to the
    // batch's counters when the workgroup exits (one atomic per wave, not per
    // beam: contended atomics on one address cost more than small beams)
    __shared__ int fxn[kWaves][2];
    const int wave = tid >> 6;
    if ((tid & 63) < 2) fxn[wave][tid & 63] = 0;
    for (;;) {
        if (tid == 0) item_sh = a.tickets ? next_ticket(a.next_item, qc, n_tickets) : atomicAdd(a.next_item, 1);
        clear_group(lds4, G * RS / 4, &nzmask, tid);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(item_sh);
        if (t >= n_tickets) break;                       // uniform: every wave exits
        int i0 = t, i1 = t + 1;
        if (a.tickets) {
            i0 = load_uniform(a.tickets + t);
            i1 = load_uniform(a.tickets + t + 1);
        }
        // item_sh is rewritten only after the barrier that ends the first item
        for (int item = i0; item < i1; ++item) {
            if (item > i0) {
                clear_group(lds4, G * RS / 4, &nzmask, tid);
                __syncthreads();
            }
            const int2 it = load_uniform(a.items + item);       // read-only tables
            const FrameDev f = load_uniform(a.frames + it.x);
            const int2 c = process_group<G, SUN, KEEP, false, false, true>(f, a.p, a.groups + (size_t)it.y * G,
                                                                           hist, taps, red, &nzmask, amask);
            if ((tid & 63) == 0) {
                fxn[wave][0] += c.x;
                fxn[wave][1] += c.y;
            }
            __syncthreads();                             // histograms and item_sh reused
        }
    }
    if ((tid & 63) == 0 && a.fcount) {
        if (fxn[wave][0]) atomicAdd(a.fcount, fxn[wave][0]);
        if (fxn[wave][1]) atomicAdd(a.fcount + 1, fxn[wave][1]);
    }
}

// Wave schedule of a batch (frames whose groups are mostly single beams with
// small footprints, where three of the four waves of a group would idle):
// every wave of the persistent workgroups takes tickets from its own queue
// counter and processes the items' beams one by one in its own histogram slot,
// with no workgroup barrier after the taps are loaded; the workgroup's LDS is
// that of a group of kWaves beams.  Every wave exits once its queue is empty.
template <int NP, bool SUN, bool KEEP>
__global__ __launch_bounds__(kFootprintThreads) __attribute__((amdgpu_waves_per_eu(KEEP || SUN ? 1 : (NP == 1 ? 8 : 4))))
void k_footprint_batch_wave(BatchArgs a)
{
    constexpr int G = kWaves;
    extern __shared__ float4 lds4[];
    const int RS = conv_stride(a.p.R, a.p.J);
    float* taps = (float*)lds4 + G * RS;
    __shared__ unsigned nzw[kWaves];
    __shared__ unsigned amask[kWaves][kMaxBins / kPassBins + 1];
    __shared__ unsigned long long rkey[kWaves][kMaxEchoes];   // first runs: peak keys, bins
    __shared__ int2 rbin[kWaves][kMaxEchoes];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    load_taps(taps, a.p.taps, a.p.J, tid);
    clear_group(lds4, G * RS / 4, &nzw[0], tid);        // the zero paddings stay zero
    __syncthreads();
    float4* slot4 = lds4 + wave * (RS / 4);             // RS is a multiple of 4
    float* hist = (float*)slot4 + conv_pad(a.p.J);
    int qc = blockIdx.x % kXcds;                         // this workgroup's XCD (round-robin dispatch)
    // this wave's counts {beams in fixed point, beams run again}, added to the
    // batch's counters when the wave exits
    __shared__ int fxn[kWaves][2];
    if (lane < 2) fxn[wave][lane] = 0;
    int left = 0;                                        // what the last beam left in the slot
    for (;;) {
        int t = 0;
        if (lane == 0) t = next_ticket(a.next_item, qc, a.n_tickets);
        t = __builtin_amdgcn_readlane(t, 0);
        if (t >= a.n_tickets) break;                     // uniform over the wave
        const int i0 = load_uniform(a.tickets + t), i1 = load_uniform(a.tickets + t + 1);
        for (int item = i0; item < i1; ++item) {
            const int2 it = load_uniform(a.items + item);
            const FrameDev f = load_uniform(a.frames + it.x);
#pragma unroll 1
            for (int m = 0; m < G; ++m) {
                const int beam = load_uniform(a.groups + (size_t)it.y * G + m);
                if (beam < 0) continue;                  // uniform
                clear_passes<NP>(hist, a.p.R, (unsigned)left >> 8 & 0xffu, (unsigned)left >> 16 & 0xffu, lane);
                if (lane == 0) nzw[wave] = 0u;
                wave_sync();
                const int fx = process_beam_wave<NP, SUN, KEEP>(f, a.p, beam, hist, RS, taps, &nzw[wave],
                                                                amask[wave], lane, rkey[wave], rbin[wave]);
                left = fx;
                if (lane == 0 && (fx & 1)) {
                    fxn[wave][0] += 1;
                    fxn[wave][1] += (fx >> 1) & 1;
                }
                wave_sync();                             // the slot is reused
            }
        }
    }
    if (lane == 0 && a.fcount) {
        if (fxn[wave][0]) atomicAdd(a.fcount, fxn[wave][0]);
        if (fxn[wave][1]) atomicAdd(a.fcount + 1, fxn[wave][1]);
    }
}

__global__ void k_reset_queue(int* counter, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) counter[i] = 0;
}

template <int G>
static hipError_t launch_g(hipStream_t s, const FootprintArgs& a)
{
    const int grid = kXcds * a.chunk;
    const size_t lds = group_lds_bytes(G, a.p.R, a.p.J);
    const bool sun = a.f.sun != nullptr && !a.f.floor_given;   // a supplied floor needs no sun sum
    const bool keep = a.f.waves != nullptr;
    if (sun && keep)
        hipLaunchKernelGGL((k_footprint<G, true, true>), dim3(grid), dim3(kFootprintThreads), lds, s, a);
    else if (sun)
        hipLaunchKernelGGL((k_footprint<G, true, false>), dim3(grid), dim3(kFootprintThreads), lds, s, a);
    else if (keep)
        hipLaunchKernelGGL((k_footprint<G, false, true>), dim3(grid), dim3(kFootprintThreads), lds, s, a);
    else
        hipLaunchKernelGGL((k_footprint<G, false, false>), dim3(grid), dim3(kFootprintThreads), lds, s, a);
    return hipGetLastError();
}

template <int G>
static hipError_t launch_batch_g(hipStream_t s, const BatchArgs& a, int grid, bool sun, bool keep)
{
    const size_t lds = group_lds_bytes(G, a.p.R, a.p.J);
    if (sun && keep)
        hipLaunchKernelGGL((k_footprint_batch<G, true, true>), dim3(grid), dim3(kFootprintThreads), lds, s, a);
    else if (sun)
        hipLaunchKernelGGL((k_footprint_batch<G, true, false>), dim3(grid), dim3(kFootprintThreads), lds, s, a);
    else if (keep)
        hipLaunchKernelGGL((k_footprint_batch<G, false, true>), dim3(grid), dim3(kFootprintThreads), lds, s, a);
    else
        hipLaunchKernelGGL((k_footprint_batch<G, false, false>), dim3(grid), dim3(kFootprintThreads), lds, s, a);
    return hipGetLastError();
}

bool footprint_group_fits(int G, int R, int J, size_t lds_max)
{
    return group_lds_bytes(G, R, J) + 1024 <= lds_max;   // + static LDS of the kernels
}

hipError_t launch_footprint(hipStream_t s, const FootprintArgs& a)
{
    switch (a.G) {
    case 1: return launch_g<1>(s, a);
    case 2: return launch_g<2>(s, a);
    case 4: return launch_g<4>(s, a);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_footprint_batch(hipStream_t s, const BatchArgs& a, int grid, bool sun, bool keep)
{
    switch (a.G) {
    case 1: return launch_batch_g<1>(s, a, grid, sun, keep);
    case 2: return launch_batch_g<2>(s, a, grid, sun, keep);
    case 4: return launch_batch_g<4>(s, a, grid, sun, keep);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_footprint_batch_wave(hipStream_t s, const BatchArgs& a, int grid, bool sun, bool keep)
{
    if (a.G != kWaves || a.p.R > kWaveMaxBins || !a.tickets) return hipErrorInvalidValue;
    const size_t lds = group_lds_bytes(kWaves, a.p.R, a.p.J);
    const dim3 b(kFootprintThreads);
    // one output pass (fewer registers, more waves per SIMD) for short waveforms
    if (a.p.R <= kWavePassBins) {
        if (sun && keep)
            hipLaunchKernelGGL((k_footprint_batch_wave<1, true, true>), dim3(grid), b, lds, s, a);
        else if (sun)
            hipLaunchKernelGGL((k_footprint_batch_wave<1, true, false>), dim3(grid), b, lds, s, a);
        else if (keep)
            hipLaunchKernelGGL((k_footprint_batch_wave<1, false, true>), dim3(grid), b, lds, s, a);
        else
            hipLaunchKernelGGL((k_footprint_batch_wave<1, false, false>), dim3(grid), b, lds, s, a);
    } else {
        if (sun && keep)
            hipLaunchKernelGGL((k_footprint_batch_wave<kWavePasses, true, true>), dim3(grid), b, lds, s, a);
        else if (sun)
            hipLaunchKernelGGL((k_footprint_batch_wave<kWavePasses, true, false>), dim3(grid), b, lds, s, a);
        else if (keep)
            hipLaunchKernelGGL((k_footprint_batch_wave<kWavePasses, false, true>), dim3(grid), b, lds, s, a);
        else
            hipLaunchKernelGGL((k_footprint_batch_wave<kWavePasses, false, false>), dim3(grid), b, lds, s, a);
    }
    return hipGetLastError();
}

template <bool CORR, bool DET>
static hipError_t launch_one(hipStream_t s, const FootprintArgs& a)
{
    const int grid = kXcds * a.chunk;
    const size_t lds = group_lds_bytes(DET ? kWaves : 1, a.p.R, a.p.J);
    const bool sun = a.f.sun != nullptr && !a.f.floor_given, keep = a.f.waves != nullptr;
    if (sun && keep)
        hipLaunchKernelGGL((k_footprint_one<true, true, CORR, DET>), dim3(grid), dim3(kFootprintThreads), lds, s, a);
    else if (sun)
        hipLaunchKernelGGL((k_footprint_one<true, false, CORR, DET>), dim3(grid), dim3(kFootprintThreads), lds, s, a);
    else if (keep)
        hipLaunchKernelGGL((k_footprint_one<false, true, CORR, DET>), dim3(grid), dim3(kFootprintThreads), lds, s, a);
    else
        hipLaunchKernelGGL((k_footprint_one<false, false, CORR, DET>), dim3(grid), dim3(kFootprintThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_footprint_one(hipStream_t s, const FootprintArgs& a, bool corr, bool det)
{
    if (a.G != 1) return hipErrorInvalidValue;
    if (corr) return det ? launch_one<true, true>(s, a) : launch_one<true, false>(s, a);
    return det ? launch_one<false, true>(s, a) : launch_one<false, false>(s, a);
}

hipError_t launch_sun_floor(hipStream_t s, const SunFloorArgs& a)
{
    if (a.B <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sun_floor, dim3(a.B), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_reset_queue(hipStream_t s, int* counter, int n)
{
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(256), 0, s, counter, n);
    return hipGetLastError();
}

}  // namespace lidar
