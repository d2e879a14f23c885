// Internal declarations of the gfx950 LiDAR engine (kernels and launchers).
// Only the library's own translation units include this file.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/lidar_sim.h"

namespace lidar {

constexpr double kLight = 299792458.0;          // m/s
constexpr double kPi = 3.14159265358979323846;

constexpr int kMaxBins = 8000;                  // one padded waveform + taps fit the LDS of a group
constexpr int kMaxTaps = 257;
constexpr int kPassBins = 2048;                 // bins per convolution pass (8 per thread)
constexpr int kMaxEchoes = 8;                   // largest max_echoes
constexpr int kWaveMaxBins = 2048;              // longest waveform of the wave schedule (in registers)
// chunks of 1 << chunk_shift(R) bins (at least 64) cover R bins with at most 32
__host__ __device__ constexpr int chunk_shift(int R)
{
    int s = 6;
    while (((R + (1 << s) - 1) >> s) > 32) ++s;
    return s;
}

// LDS layout of a beam group in the footprint kernels: G waveforms of
// conv_stride(R, J) floats, each with conv_pad(J) zero bins before its R bins
// and at least J + 8 after them, every waveform 16-byte aligned; then the
// pulse taps, preceded by conv_shift(J) zeros (so that the tap centre falls on
// a multiple of 4) and padded with zeros to conv_taps(J) entries (whole
// blocks of 8).  The convolution reads and the output pass writes aligned
// 4-bin vectors without bounds checks.
__host__ __device__ constexpr int conv_shift(int J) { return ((J + 3) & ~3) - J; }
__host__ __device__ constexpr int conv_pad(int J) { return (J + 8 + 3) & ~3; }
__host__ __device__ constexpr int conv_stride(int R, int J)
{
    return conv_pad(J) + ((R + J + conv_shift(J) + 8 + 3) & ~3);
}
__host__ __device__ constexpr int conv_taps(int J) { return (2 * J + 1 + conv_shift(J) + 7) & ~7; }
inline size_t group_lds_bytes(int G, int R, int J)
{
    return sizeof(float) * ((size_t)G * conv_stride(R, J) + conv_taps(J));
}
constexpr int kFootprintThreads = 256;          // 4 waves of 64
constexpr int kWavesPerGroup = kFootprintThreads / 64;
constexpr int kXcds = 8;                        // MI355X: 8 XCDs, round-robin dispatch
constexpr int kQueueStride = 32;                // ints between ticket counters (128 bytes)
constexpr int kQueueInts = kXcds * kQueueStride;  // one ticket dispenser

// Pattern as the set-up kernels see it (device copy of the table).
struct PatternDev {
    int kind;                   // LIDAR_PATTERN_GAUSS / LIDAR_PATTERN_TABLE
    double sx, sy, trunc;       // Gaussian sigma (deg), cut radius (sigmas)
    const float* table;         // [ny][nx]
    int nx, ny;
    double hx, hy;              // table half extents (deg)
};

// Raster geometry in FP64 (degrees).
struct RasterDev {
    int W, H;
    double az_min, el_max;
    double dphi, de;
};

// Kernel grid geometry: offsets m in [-M, M] (columns), n in [-N, N] (rows).
struct KernelDev {
    int M, N, KW, KH;
};

// ---- set-up (FP64 resample of the pattern and per-beam normalisation) ----
hipError_t launch_kernel_grid(hipStream_t s, PatternDev p, RasterDev r, KernelDev k,
                              double* K64);
hipError_t launch_kernel_blocks(hipStream_t s, KernelDev k, const double* K64, float* Kb);
hipError_t launch_kernel_rows(hipStream_t s, KernelDev k, const double* K64, double* rowsum,
                              double* rowmax, int2* rowrange, int32_t* prefix);
hipError_t launch_kernel_peak(hipStream_t s, KernelDev k, const double* rowsum,
                              const double* rowmax, double* kinfo);
hipError_t launch_raster_tables(hipStream_t s, RasterDev r, float2* colcs, float4* rowtab);
// omega: scratch of H + 2 KH doubles (per-row solid angles)
hipError_t launch_beam_setup(hipStream_t s, RasterDev r, KernelDev k, const double* az,
                             const double* el, int B, const double* rowsum,
                             const int32_t* prefix, double* omega, double emit_power,
                             lidar_beam_info* beams);
hipError_t launch_pulse_taps(hipStream_t s, float sigma_ns, float bin_ns, int J, float* taps);

// FP64 direction tables of a raster for the range modes: cos and sin of the
// pixel-centre azimuth of every column / elevation of every row, and of the
// column and row edges (W + 1 and H + 1 entries; edge u is az_min + u dphi,
// edge v is el_max - v de).
struct RangeTables {
    const double2* col;         // [W]
    const double2* row;         // [H]
    const double2* col_edge;    // [W + 1]
    const double2* row_edge;    // [H + 1]
};
hipError_t launch_range_tables(hipStream_t s, RasterDev r, double2* col, double2* row,
                               double2* col_edge, double2* row_edge);

// A generic pointer into device memory as a global-address-space pointer:
// its accesses become global loads and stores.  Pointers read from a table
// (a batch's frames) are generic, and flat accesses also count against the
// LDS counter, so that every wait for a load would wait for the LDS
// atomics too (and the reverse).
// (HIP's vector and record types have no constructor or assignment from an
// object in another address space: vectors are read as builtin vectors and
// converted, records are written field by field.)
typedef int gint2 __attribute__((ext_vector_type(2)));
typedef int gint4 __attribute__((ext_vector_type(4)));
typedef float gfloat2 __attribute__((ext_vector_type(2)));
typedef float gfloat4 __attribute__((ext_vector_type(4)));
template <typename T>
__device__ inline const __attribute__((address_space(1))) T* gptr(const T* p)
{
    return (const __attribute__((address_space(1))) T*)p;
}

template <typename T>
__device__ inline __attribute__((address_space(1))) T* gptr(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}

// ---- per frame ----
struct PrepassArgs {
    const float *depth, *refl, *gain, *nx, *ny, *nz;
    long pitch;
    int W, H;
    const float2* colcs;        // [W] (cos az, sin az) of pixel centres
    const float4* rowtab;       // [H] (cos el, sin el, Omega, 0) of pixel rows
    double to_bin;              // 2 / (c dt), FP64
    int R;
    float sun_x, sun_y, sun_z;
    int2* pix;                  // [W4/4][H][4] {bin, shade bits}, 4-column blocks
    float* sun;                 // [W4/4][H][4] sun shading, 4-column blocks (or null)
    int W4;                     // W rounded up to a multiple of 4 (padding: sky)
    int range_mode;             // LIDAR_RANGE_*: INTERVAL packs {first | last << 16} bins
                                // and the shade per bin; CORRECTED also writes rec4
    RangeTables rt;             // range modes: FP64 direction tables
    float4* rec4;               // CORRECTED: [W4/4][H][4] {depth, nx, ny, nz} (or null)
    // CENTRE batches: per tile (row-major over the frame's tiles) the
    // statistics {largest shade (FP32 bits), first bin, last bin, 0} of its
    // valid pixels (or null)
    int* stats;
};
// The per-pixel factors of the footprint weight, shared by the pre-pass and
// the direct gather so that both give the same bits: shade Omega beta
// cos(theta) / d^2 with beta = g rho / pi and cos(theta) = max(0, -n.v)
// (rt: cos el, sin el, Omega of the row; cs: cos az, sin az of the column),
// and the sun shading Omega (rho / pi) max(0, n.s).
__device__ inline float pixel_shade(float4 rt, float2 cs, float nx, float ny, float nz, float rho,
                                    float g, float d)
{
    const float inv_pi = (float)(1.0 / kPi);
    const float vx = rt.x * cs.x, vy = rt.x * cs.y, vz = rt.y;
    const float ct = fmaxf(0.0f, -(nx * vx + ny * vy + nz * vz));
    return rt.z * (g * rho * inv_pi) * ct / (d * d);
}
__device__ inline float pixel_sun(float sx, float sy, float sz, float4 rt, float nx, float ny, float nz,
                                  float rho)
{
    const float inv_pi = (float)(1.0 / kPi);
    const float ns = fmaxf(0.0f, nx * sx + ny * sy + nz * sz);
    return rt.z * (rho * inv_pi) * ns;
}

// A frame's G-buffer planes for the direct gather (the pre-pass inputs).
struct DirectDev {
    const float *depth, *refl, *gain, *nx, *ny, *nz;
    long pitch;
    const float2* colcs;        // [W] (cos az, sin az) of pixel centres
    const float4* rowtab;       // [H] (cos el, sin el, Omega, 0) of pixel rows
    float sun_x, sun_y, sun_z;
    int pad;
};
hipError_t launch_prepass(hipStream_t s, const PrepassArgs& a, bool with_sun);
// all frames of a batch in one launch (tile_off: [n + 1] prefix of prepass_tiles)
int prepass_tiles(const PrepassArgs& a);
hipError_t launch_prepass_batch(hipStream_t s, const PrepassArgs* frames, const int* tile_off,
                                int n, int total_tiles, bool with_sun, int range_mode);
// frame statistics of n frames ({largest shade bits, first bin, last bin, 0}
// each) from the tiles' records, then four zero counters
hipError_t launch_reduce_stats(hipStream_t s, const int* tiles, const int* tile_off, int* stats, int n);

// Kernel table in 4-column blocks, in four copies shifted by one column:
// copy s, block b, row n holds K(c, n) for the kernel columns
// c = 4(b - 2) + s + j, j = 0..3 (zero outside [0, KW) and in the guard row
// n = KH).  Block 0 and block NB-1 of every copy are all zero.
constexpr int kBlockPad = 2;
__host__ __device__ inline int kernel_blocks(int KW) { return (KW + 12) / 4 + 1; }

// One frame as the footprint kernels see it.  Beam indices in groups are
// local to the frame; the output pointers are already offset to the frame.
struct FrameDev {
    const int2* pix;            // [W4/4][H][4] {bin, shade bits}
    const float* sun;           // [W4/4][H][4] or null
    int W, H;
    const float* Kb;            // [4][NB][KH+1][4], see kernel_blocks
    const int2* rowrange;       // [KH] first/last m with K > 0 (empty row: INT_MAX, INT_MIN)
    int M, N, KW, KH, NB;
    int tile;                   // strip height: 64, 16 or 4 rows (64/tile column phases)
    float sun_scale;            // E_sun / max K (0: no sun term)
    int wave;                   // batches: 1 = the frame's items go to the wave schedule
    int span;                   // 1: pixel keys are {first | last << 16} bin ranges
    int floor_given;            // 1: the floor A_b is in beams[].floor (kappa table)
    // batches, wave schedule: frames whose beams touch few of their pixels
    // gather straight from the planes (no pre-pass, pix and sun unused)
    const DirectDev* direct;    // or null
    // batches, wave schedule: the pre-pass statistics of the frame (see
    // PrepassArgs::stats; null: FP32 accumulation) and the kernel's maximum
    const int* fstats;
    float kmax;
    // LIDAR_RANGE_CORRECTED (one beam per group): records, FP64 tables, and
    // per beam (cos, sin) of the beam's azimuth and elevation offsets from its
    // pixel centre (radians)
    const float4* rec4;         // [W4/4][H][4] {depth, nx, ny, nz}
    const double2* col64;       // [W] pixel-centre azimuth cos, sin
    const double2* row64;       // [H] pixel-centre elevation cos, sin
    const double4* bcorr;       // [B] {cos daz, sin daz, cos del, sin del}
    double to_bin;              // 2 / (c dt)
    lidar_beam_info* beams;     // [B] in: pixel, scale; out: floor
    lidar_echo* echoes;         // [B][E]
    int32_t* counts;            // [B]
    float* waves;               // [B][R] or null
};

// Parameters shared by every frame of a handle.
struct PathDev {
    const float* taps;          // [2J+1]
    int J, R, E;
    int select;                 // LIDAR_ECHO_*
    float threshold;
    float ambient;
    double half_c_dt;           // (c/2) dt in metres, FP64
    double bin_ns;
};

struct FootprintArgs {
    FrameDev f;
    PathDev p;
    const int32_t* groups;      // [n_groups][G] beam indices, -1 = empty slot
    int n_groups, G, chunk;     // chunk = ceil(n_groups / kXcds)
};
hipError_t launch_footprint(hipStream_t s, const FootprintArgs& a);

// Persistent launch over the (frame, group) items of a batch.
struct BatchArgs {
    const FrameDev* frames;     // [n_frames]
    PathDev p;
    const int32_t* groups;      // [total groups][G]: each frame's groups, concatenated
    const int2* items;          // [n_items] {frame, global group index}, costliest first
    int n_items, G;
    int* next_item;             // work-queue counter(s), zeroed by k_reset_queue: with tickets
                                // kXcds counters kQueueStride ints apart, else one
    const int* n_items_dev;     // if set: the item count, read on the device
    // if set: the queue hands out tickets, ticket t = items [tickets[t],
    // tickets[t + 1]) (non-empty); else one item per queue step
    const int* tickets;         // [n_tickets + 1]
    int n_tickets;
    int* fcount;                // {beams in fixed point, beams run again in FP32} (or null)
};
hipError_t launch_footprint_batch(hipStream_t s, const BatchArgs& a, int grid, bool sun,
                                  bool keep);
// the wave schedule over the tickets of a (kWavesPerGroup beams per group,
// R <= kWaveMaxBins); each wave takes tickets from *next_item
hipError_t launch_footprint_batch_wave(hipStream_t s, const BatchArgs& a, int grid, bool sun,
                                       bool keep);
hipError_t launch_reset_queue(hipStream_t s, int* counter, int n = 1);
// single frame with groups of one beam: corr = LIDAR_RANGE_CORRECTED bins,
// det = a histogram slot per wave summed in wave order (LIDAR_DETERMINISTIC)
hipError_t launch_footprint_one(hipStream_t s, const FootprintArgs& a, bool corr, bool det);
// per-beam offsets of the beams from their pixel centres (corrected range)
hipError_t launch_beam_corr(hipStream_t s, RasterDev r, const double* az, const double* el, int B,
                            const lidar_beam_info* beams, double4* bcorr);
// sun floor from a kappa table: beams[b].floor = ambient + E_sun sum over the
// kernel window of kappa * sun shading (kappa in the blocked layout of Kb)
struct SunFloorArgs {
    const float* sun;           // [W4/4][H][4]
    int W, H;
    const float* Kr;            // [4][NB][KH+1][4] kappa blocks
    int M, N, KW, KH, NB;
    float ambient, e_sun;
    lidar_beam_info* beams;
    int B;
};
hipError_t launch_sun_floor(hipStream_t s, const SunFloorArgs& a);
// whether G histograms of R bins plus the pulse taps fit the LDS budget
bool footprint_group_fits(int G, int R, int J, size_t lds_max = 65536);

// ---- range stacking (Alg. 2) with a separable kernel --------------------
constexpr int kRsMaxHalf = 127;         // half extents M, N of the separable kernel
struct RangeStackArgs {
    const int2* pix;            // pre-pass records [W4/4][H][4]
    int W, H, W4, R;
    const float* hk;            // [2M + 1] along the rows (columns m = -M..M)
    const float* vk;            // [2N + 1] along the columns (rows n = -N..N)
    int M, N;
    float rho_min;
    float bound;                // sum H * sum V (slice skipping)
    const int* smax;            // [R] largest shade per slice (FP32 bits)
    int32_t* s_nearest;         // [H][W]
    float* xi_nearest;          // [H][W]
};
// smax_scratch: [R] ints
hipError_t launch_range_stacking(hipStream_t s, const RangeStackArgs& a, int* smax_scratch);

// ---- reprojection of a pinhole rendering ---------------------------------
struct ReprojectArgs {
    int W, H;                   // output raster
    double az_min, el_max, dphi, de;
    int SW, SH;                 // pinhole image
    long spitch;                // elements between pinhole rows
    double fx, fy, cx, cy;
    double rot[9];              // camera -> sensor, row-major
    int fmt;                    // LIDAR_DEPTH_*
    int correct;                // normal-based range correction to the output direction
    double z_near, z_far;
    const void* depth;
    const float *refl, *gain, *nx, *ny, *nz;
    float* out;                 // [6][H][W]: depth, reflectance, gain, normal x, y, z
};
hipError_t launch_reproject(hipStream_t s, const ReprojectArgs& a);

// ---- host utility: a growable device buffer -----------------------------
template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    hipError_t ensure(size_t count)
    {
        if (count <= n && p) return hipSuccess;
        release();
        if (count == 0) return hipSuccess;
        hipError_t e = hipMalloc(&p, sizeof(T) * count);
        if (e == hipSuccess) n = count;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

// ---- surrogate network ---------------------------------------------------
// 1056 -> 256 -> 256 -> 256 -> 16; flat FP32 parameters [W1 (row-major
// in x out), b1, W2, b2, W3, b3, W4, b4].
constexpr int kSurIn = 1056, kSurInUsed = 1030, kSurHid = 256, kSurOut = 16, kSurOutUsed = 13;
constexpr long kSurOffW1 = 0;
constexpr long kSurOffB1 = kSurOffW1 + (long)kSurIn * kSurHid;
constexpr long kSurOffW2 = kSurOffB1 + kSurHid;
constexpr long kSurOffB2 = kSurOffW2 + (long)kSurHid * kSurHid;
constexpr long kSurOffW3 = kSurOffB2 + kSurHid;
constexpr long kSurOffB3 = kSurOffW3 + (long)kSurHid * kSurHid;
constexpr long kSurOffW4 = kSurOffB3 + kSurHid;
constexpr long kSurOffB4 = kSurOffW4 + (long)kSurHid * kSurOut;
constexpr long kSurParams = kSurOffB4 + kSurOut;
// loss: peak-bin outputs in units of 16 bins, squared-error weights
constexpr float kSurBinScale = 16.0f, kSurWBin = 64.0f, kSurWInt = 1.0f, kSurWEpw = 1.0f;

__host__ __device__ inline bool sur_is_weight(long i)
{
    return i < kSurOffB1 || (i >= kSurOffW2 && i < kSurOffB2) ||
           (i >= kSurOffW3 && i < kSurOffB3) || (i >= kSurOffW4 && i < kSurOffB4);
}

// C[M][N] (FP32, row stride ldc) = sum_k A(i, k) B(k, j), BF16 operands with
// A(i, k) = A[i sam + k sak] and B(k, j) = B[k sbk + j sbn].
struct GemmArgs {
    const uint16_t* A;
    long sam, sak;
    const uint16_t* B;
    long sbk, sbn;
    float* C;
    long ldc;
    int M, N, K;
    int ksplit;                 // > 1: K split over grid.z, added into a zeroed C
};
struct AdamArgs {
    float lr, beta1, beta2, eps;
    float decay_factor;         // 1 - lr * weight_decay
    float inv_bc1, inv_bc2;     // 1 / (1 - beta^t)
};
// det: no split of K (atomic adds in any order), so the result has a fixed order
hipError_t launch_gemm_bf16(hipStream_t s, const GemmArgs& g, bool det = false);
// Library GEMMs (hipBLASLt) for the training products; blas_gemm returns
// hipErrorNotSupported for layouts without a unit stride or when the library
// has no algorithm (the caller then runs launch_gemm_bf16)
struct BlasCtx;
BlasCtx* blas_create();                 // null when the library cannot start
void blas_destroy(BlasCtx* c);
hipError_t blas_gemm(BlasCtx* c, hipStream_t s, const GemmArgs& g);
hipError_t launch_bias_gelu(hipStream_t s, float* Z, const float* bias, uint16_t* H, long n, int C);
hipError_t launch_bias(hipStream_t s, float* Y, const float* bias, long n, int C);
hipError_t launch_loss(hipStream_t s, const float* Y, const float* lab, long n, uint16_t* dYb,
                       float* loss_sum);
hipError_t launch_gelu_back(hipStream_t s, const float* dH, const float* Z, uint16_t* dZb, long count);
hipError_t launch_colsum(hipStream_t s, const uint16_t* D, long n, int C, float* out, bool det = false);
hipError_t launch_zero_f32(hipStream_t s, float* p, long n);
// minibatch rows perm_e(pos0 + i), i < b, of X [n][1056] BF16 and lab [n][16]
// (perm_e: the seeded Feistel permutation of epoch e on values of 2 half bits)
hipError_t launch_gather_rows(hipStream_t s, const uint16_t* X, const float* lab, long n, int half,
                              unsigned long long seed, unsigned long long epoch, long pos0, int b,
                              uint16_t* Xb, float* Lb);
hipError_t launch_adamw(hipStream_t s, float* theta, const float* grad, float* m, float* v,
                        uint16_t* theta_b, long n, const AdamArgs& a);
hipError_t launch_to_bf16(hipStream_t s, const float* x, uint16_t* y, long n);

// ---- surrogate inputs, gate and fallback ----------------------------------
constexpr int kSurPatch = 16;           // patch of 16 x 16 coarse cells
constexpr int kSurTailBins = 64;        // coarse time bins of the tail estimate
constexpr double kSurCoreFraction = 2e-4;
constexpr int kSurRefWindow = 512;      // time bins of the reference-bin histogram
constexpr float kSurDkClip = 4.0f;      // offset labels clipped to +-64 bins

// Cell sizes: coarse cells (cw x ch pixels) tile the kernel's core box
// (cells with K >= 2e-4 max K, half extents cm, cn) 16 x 16 times;
// super-cells (sw x sh) tile the kernel window 16 x 16 times.
struct SurGeom {
    int cm, cn, cw, ch, sw, sh, CW, CH, SW, SH;
};

struct CoarseArgs {
    const float *depth, *refl, *gain, *nx, *ny, *nz;
    long pitch;
    int W, H;
    const float2* colcs;
    const float4* rowtab;
    double to_bin;
    int R;
    float sun_x, sun_y, sun_z;
    SurGeom g;
    float4* cell;               // [CH][CW] {mean depth, reflectance cover, mean gain, mean cos}
    float* cell_sun;            // [CH][CW] sum of sun shading
    float* cell_shade;          // [CH][CW] sum of shade
};
struct SuperArgs {
    const int2* pix;            // pre-pass records [W4/4][H][4]
    const float* sun;           // or null
    int W, H;
    SurGeom g;
    float2* sup;                // [SH][SW] {shade sum, sun sum}
    int2* range;                // [SH][SW] {first, last} time bin (0, -1: none)
};
struct SurAux {
    int k_ref;
    float e_tail, a_est;
    int accepted;
};
struct FeatArgs {
    const lidar_beam_info* beams;
    const double *az, *el;
    int B;
    const float* depth;
    long pitch;
    int W, H;
    double to_bin;
    int R;
    const float4* cell;
    const float* cell_sun;
    const float* cell_shade;
    const float2* sup;
    const int2* range;
    const double* K64;
    int M, N, KW;
    SurGeom g;
    float ambient, sun_scale, threshold;
    uint16_t* X;                // [B][1056] BF16
    SurAux* aux;                // [B]
};
struct DecodeArgs {
    const float* Y;             // [B][16]
    SurAux* aux;
    int B, R, E;
    float threshold;
    float conf_logit;           // accept when y[12] >= conf_logit
    float alpha;                // and E_tail < alpha * margin
    double half_c_dt, bin_ns;
    lidar_beam_info* beams;
    lidar_echo* echoes;
    int32_t* counts;
};
struct CompactArgs {
    const int32_t* groups;      // [n_groups][G]
    int n_groups, G;
    const SurAux* aux;
    int32_t* groups_fb;         // [n_groups][G]: fallback beams, -1 elsewhere
    int2* items;                // [n_groups] {0, group}
    int* n_items;               // compacted item count
    int* n_fallback;            // fallback beams (accumulated)
};
hipError_t launch_coarse(hipStream_t s, const CoarseArgs& a);
hipError_t launch_super(hipStream_t s, const SuperArgs& a);
hipError_t launch_features(hipStream_t s, const FeatArgs& a);
hipError_t launch_labels(hipStream_t s, const lidar_echo* echoes, const int32_t* counts,
                         const SurAux* aux, int B, int E, float threshold, float* lab);
hipError_t launch_decode(hipStream_t s, const DecodeArgs& a);
hipError_t launch_compact(hipStream_t s, const CompactArgs& a);
hipError_t launch_aux_out(hipStream_t s, const SurAux* aux, int B, float* out);
// NaN rows of the kept waveforms [B][R] of accepted beams
hipError_t launch_fill_accepted(hipStream_t s, const SurAux* aux, int B, int R, float* waves);

// fused inference: X [n][1056] BF16 -> Y [n][16] FP32, transposed BF16
// weights Wt1 [256][1056], Wt2, Wt3 [256][256], Wt4 [16][256]
struct InferArgs {
    const uint16_t* X;
    long n;
    const uint16_t *Wt1, *Wt2, *Wt3, *Wt4;
    const float *b1, *b2, *b3, *b4;
    float* Y;
};
constexpr long kSurWtSize = (long)kSurIn * kSurHid + 2L * kSurHid * kSurHid + (long)kSurHid * kSurOut;
hipError_t launch_transpose_weights(hipStream_t s, const uint16_t* theta_b, uint16_t* wt);
hipError_t launch_mlp_infer(hipStream_t s, const InferArgs& a);

struct SurNet {
    DevBuf<float> theta, m, v, grad;    // FP32 [kSurParams]
    DevBuf<uint16_t> theta_b;           // BF16 operand copy
    DevBuf<uint16_t> theta_t;           // transposed BF16 weights [kSurWtSize]
    bool t_stale = true;
    long step = 0;
    bool ready = false;
    bool det = false;                   // LIDAR_DETERMINISTIC: gradients in a fixed order
};
struct SurWork {                        // activations of up to `cap` rows
    long cap = 0;
    DevBuf<float> Z1, Z2, Z3, Y, dH, loss;
    DevBuf<uint16_t> H1, H2, H3, dYb, dZb;
    BlasCtx* blas = nullptr;            // library GEMMs of the training products (or null)
    bool blas_tried = false;
    hipError_t ensure(long n);
    SurWork() = default;
    SurWork(const SurWork&) = delete;
    SurWork& operator=(const SurWork&) = delete;
    ~SurWork() { blas_destroy(blas); }
};
// Y (w.Y, [n][16] FP32) of the rows X ([n][1056] BF16), keeping the
// activations for the backward pass
hipError_t sur_forward(hipStream_t s, const SurNet& net, const uint16_t* X, long n, SurWork& w);
// Y ([n][16] FP32) of the rows X by the fused kernel (activations in LDS)
hipError_t sur_infer(hipStream_t s, SurNet& net, const uint16_t* X, long n, float* Y);
// loss (added into w.loss[0]) and parameter gradient (net.grad) of rows X
// with labels lab ([n][16]); runs the forward pass first
hipError_t sur_gradients(hipStream_t s, SurNet& net, const uint16_t* X, const float* lab, long n,
                         SurWork& w);

}  // namespace lidar
