// Engine and C-ABI of the gfx950 LiDAR library (declared in
// include/lidar_sim.h).  The host side validates arguments, owns device
// buffers, decides sizes, forms and orders the beam groups, captures batches
// into HIP graphs and autotunes them, and enqueues kernels on the caller's
// stream; every step of the model itself runs in the kernels.
//
// Floating-point contraction is off in this file so that the host's FP64
// decisions (kernel extent M, N and pulse half-width J) use plain IEEE
// operations in the order written.
#pragma clang fp contract(off)

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "engine.h"

using namespace lidar;

namespace {

thread_local std::string g_create_error;

struct EventPair {
    hipEvent_t a, b;
};

// Host copy of a pattern and its beams.
struct PatternHost {
    uint32_t kind = 0;
    double sigma[2] = {0, 0}, trunc = 0, half[2] = {0, 0};
    uint32_t nx = 0, ny = 0;
    std::vector<float> table;
    std::vector<float> rx;             // optional kappa table (sun term), same grid as table
    std::vector<double> az, el;
};

// One frame's device state: pattern copy, kernel set-up for its raster,
// pixel records and beam groups.  The per-beam outputs live with the caller
// of setup_frame (the handle in single-frame mode, the batch otherwise).
struct FrameState {
    PatternHost pat;
    lidar_gbuffer_desc gb{};
    DevBuf<float> d_table;
    DevBuf<double> d_az, d_el;
    KernelDev k{};
    double kmax = 0.0;
    uint64_t samples = 0;
    DevBuf<double> d_K64, d_rowsum, d_rowmax, d_kinfo, d_omega;
    DevBuf<float> d_Kb;
    DevBuf<int2> d_rowrange;
    DevBuf<int32_t> d_prefix;
    DevBuf<float2> d_colcs;
    DevBuf<float4> d_rowtab;
    DevBuf<int2> d_pix;
    DevBuf<float> d_sun;
    // kappa table of the sun term: device copy, resampled grid, blocks
    DevBuf<float> d_rx, d_Kr;
    DevBuf<double> d_K64rx;
    // range modes: FP64 direction tables, beam offsets, depth/normal records
    DevBuf<double2> d_col64, d_row64, d_cole, d_rowe;
    DevBuf<double4> d_bcorr;
    DevBuf<float4> d_rec4;
    std::vector<int32_t> groups;       // [n_groups][G], -1 = empty slot
    std::vector<uint64_t> group_cost;  // samples of the group's beams
    int n_groups = 0;
    int tile = 64;
    int wave = 0;                      // batches: wave schedule (one wave per group, see footprint.hip)
    int direct = 0;                    // batches: gathered from the planes without a pre-pass
    // surrogate inputs
    SurGeom geom{};
    bool geom_ok = false;
    DevBuf<float4> d_cell;
    DevBuf<float> d_cell_sun, d_cell_shade;
    DevBuf<float2> d_sup;
    DevBuf<int2> d_range;
};

}  // namespace

struct lidar_sim {
    lidar_sim_params prm{};
    hipStream_t stream = nullptr;
    std::string err;
    int J = 0;
    int G = 4;                         // beams per group (LDS budget)
    DevBuf<float> d_taps;

    int cus = 256;                     // compute units of the device (queried at create)
    size_t lds_max = 65536;            // LDS of a workgroup on the device (queried at create)

    // single-frame mode
    bool have_pattern = false, have_gbuffer = false, setup_ok = false, have_result = false;
    uint64_t pattern_gen = 0;          // incremented by every set_pattern
    FrameState single;
    DevBuf<lidar_beam_info> d_beams;
    DevBuf<lidar_echo> d_echoes;
    DevBuf<int32_t> d_counts, d_groups;
    DevBuf<float> d_waves;

    // batch mode
    bool batch_ok = false, batch_result = false;
    std::vector<lidar_gbuffer_desc> batch_gb;
    std::vector<lidar_pattern_desc> batch_pd;
    std::vector<std::unique_ptr<FrameState>> frames;
    std::vector<uint64_t> beam_off;    // [n_frames + 1]
    DevBuf<lidar_beam_info> b_beams;
    DevBuf<lidar_echo> b_echoes;
    DevBuf<int32_t> b_counts, b_groups, b_queue;
    DevBuf<float> b_waves;
    DevBuf<FrameDev> b_frames;
    DevBuf<int2> b_items;
    uint64_t b_items_n = 0, b_samples = 0;
    DevBuf<int32_t> b_tickets;         // [b_tickets_n + 1] item runs handed out by the queues
    int b_tickets_n = 0;
    int b_tickets_g = 0;               // tickets 0 .. b_tickets_g - 1: group schedule; the rest: wave
    uint64_t b_wave_items = 0;
    DevBuf<PrepassArgs> b_prep;        // [n_frames] pre-pass arguments of the batch's frames
    DevBuf<DirectDev> b_direct;        // [n_frames] planes of the frames gathered directly
    DevBuf<int> b_fstats;              // [n_frames][4] pre-pass statistics (fixed-point accumulation)
    DevBuf<int> b_tstats;              // [pre-pass tiles][4] the tiles' statistics
    DevBuf<int32_t> b_prep_off;        // [n_frames + 1] first pre-pass tile of each frame
    int b_prep_tiles = 0;
    int b_grid = 0;
    bool b_autotuned = false;
    double b_autotune_ms = 0.0;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::map<int, std::pair<int, int>> tuned;  // kernel-height class -> strip height, wave schedule

    // surrogate network, inputs, gate and fallback
    SurNet net;
    SurWork work;
    DevBuf<uint16_t> mb_x;             // minibatch of surrogate_train: inputs [b][1056]
    DevBuf<float> mb_l;                //   and labels [b][16]
    DevBuf<uint16_t> s_X;
    DevBuf<SurAux> s_aux;
    DevBuf<int32_t> s_groups_fb;
    DevBuf<int2> s_items;
    DevBuf<int> s_cnt;                 // [0] fallback items, [1] queue, [2] fallback beams (running)
    DevBuf<FrameDev> s_frame;
    FrameDev s_frame_host{};
    uint64_t s_aux_gen = ~0ull;        // pattern generation whose gate decisions s_aux holds
    const SurAux* s_aux_ptr = nullptr; // allocation those decisions were written to
    float gate_conf_logit = 0.0f;      // logit of c_min = 0.5
    float gate_alpha = 0.5f;
    bool plain_result = false;

    // reprojected G-buffer (set_gbuffer_pinhole): [6][H][W]
    DevBuf<float> rp_planes;
    bool gb_owned = false;

    // range stacking: separable kernel factors (device, host copy), slice maxima
    DevBuf<float> rs_k;
    std::vector<float> rs_host;
    uint32_t rs_M = ~0u, rs_N = ~0u;
    DevBuf<int> rs_smax;

    // stats
    lidar_stats st{};
    std::vector<EventPair> pending_fp, pending_pp, pending_bt, pending_sur, pool;
};

// ---- scratch of the allocation-free entry point -----------------------------
// lidar_sim_simulate_static works entirely in this file-scope device array:
// every GPU the library runs on holds its own copy at its own address (taken
// once per device with hipGetSymbolAddress), kept until the process ends.  In
// host code the name is not a device address; host code uses only the
// address recorded per device.
namespace lidar {
constexpr size_t kStaticScratchBytes = LIDAR_STATIC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
}  // namespace lidar

namespace {

constexpr int kMaxStaticDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxStaticDevices] = {};

// Device address of the current device's scratch array, recorded at the first
// call on that device (with the device current).
hipError_t static_scratch_addr(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxStaticDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(lidar::scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

}  // namespace

namespace {

// Record an error on the handle (or, without one, as the thread's last
// handle-less error: failed create or simulate_static).
lidar_status fail(lidar_sim* h, lidar_status code, const std::string& msg)
{
    if (h) h->err = msg;
    else g_create_error = msg;
    return code;
}

lidar_status hip_fail(lidar_sim* h, hipError_t e, const char* what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory) return fail(h, LIDAR_E_NOMEM, m);
    return fail(h, LIDAR_E_HIP, m);
}

#define HIP_TRY(h, expr, what)                                        \
    do {                                                              \
        hipError_t e_ = (expr);                                       \
        if (e_ != hipSuccess) return hip_fail((h), e_, (what));       \
    } while (0)

#define LIDAR_TRY(expr)                                               \
    do {                                                              \
        lidar_status s_ = (expr);                                     \
        if (s_ != LIDAR_OK) return s_;                                \
    } while (0)

bool is_fin(double x) { return std::isfinite(x); }

EventPair take_pair(lidar_sim* h, hipError_t* e)
{
    EventPair p{};
    if (!h->pool.empty()) {
        p = h->pool.back();
        h->pool.pop_back();
        *e = hipSuccess;
        return p;
    }
    *e = hipEventCreate(&p.a);
    if (*e == hipSuccess) *e = hipEventCreate(&p.b);
    return p;
}

lidar_status drain_events(lidar_sim* h)
{
    auto drain = [&](std::vector<EventPair>& v, double& ms, uint64_t& n) -> hipError_t {
        for (auto& p : v) {
            hipError_t e = hipEventSynchronize(p.b);
            if (e != hipSuccess) return e;
            float t = 0.0f;
            e = hipEventElapsedTime(&t, p.a, p.b);
            if (e != hipSuccess) return e;
            ms += t;
            ++n;
            h->pool.push_back(p);
        }
        v.clear();
        return hipSuccess;
    };
    HIP_TRY(h, drain(h->pending_fp, h->st.footprint_ms, h->st.footprint_launches), "event timing");
    HIP_TRY(h, drain(h->pending_pp, h->st.prepass_ms, h->st.prepass_launches), "event timing");
    HIP_TRY(h, drain(h->pending_bt, h->st.batch_ms, h->st.batch_launches), "event timing");
    uint64_t n_sur = 0;
    HIP_TRY(h, drain(h->pending_sur, h->st.surrogate_ms, n_sur), "event timing");
    return LIDAR_OK;
}

RasterDev raster_of(const lidar_gbuffer_desc& g)
{
    RasterDev r;
    r.W = (int)g.width;
    r.H = (int)g.height;
    r.az_min = g.az_min_deg;
    r.el_max = g.el_max_deg;
    r.dphi = (g.az_max_deg - g.az_min_deg) / (double)g.width;
    r.de = (g.el_max_deg - g.el_min_deg) / (double)g.height;
    return r;
}

bool same_raster(const lidar_gbuffer_desc& a, const lidar_gbuffer_desc& b)
{
    return a.width == b.width && a.height == b.height && a.az_min_deg == b.az_min_deg &&
           a.az_max_deg == b.az_max_deg && a.el_min_deg == b.el_min_deg &&
           a.el_max_deg == b.el_max_deg;
}

bool same_gbuffer(const lidar_gbuffer_desc& a, const lidar_gbuffer_desc& b)
{
    return same_raster(a, b) && a.pitch == b.pitch && a.depth == b.depth &&
           a.reflectance == b.reflectance && a.retro_gain == b.retro_gain &&
           a.normal_x == b.normal_x && a.normal_y == b.normal_y && a.normal_z == b.normal_z;
}

bool same_pattern(const lidar_pattern_desc& a, const lidar_pattern_desc& b)
{
    return a.kind == b.kind && a.n_beams == b.n_beams && a.sigma_deg[0] == b.sigma_deg[0] &&
           a.sigma_deg[1] == b.sigma_deg[1] && a.trunc_sigmas == b.trunc_sigmas &&
           a.table == b.table && a.nx == b.nx && a.ny == b.ny &&
           a.half_deg[0] == b.half_deg[0] && a.half_deg[1] == b.half_deg[1] &&
           a.beam_az_deg == b.beam_az_deg && a.beam_el_deg == b.beam_el_deg;
}

// ---- validation --------------------------------------------------------

lidar_status check_pattern(lidar_sim* h, const lidar_pattern_desc* pd, const std::string& w)
{
    if (!pd) return fail(h, LIDAR_E_INVALID, w + "pattern is NULL");
    if (pd->n_beams == 0 || !pd->beam_az_deg || !pd->beam_el_deg)
        return fail(h, LIDAR_E_INVALID, w + "pattern needs n_beams >= 1 and beam angle arrays");
    if (pd->n_beams > (1u << 26)) return fail(h, LIDAR_E_INVALID, w + "too many beams (max 2^26)");
    for (uint32_t i = 0; i < pd->n_beams; ++i)
        if (!is_fin(pd->beam_az_deg[i]) || !is_fin(pd->beam_el_deg[i]))
            return fail(h, LIDAR_E_INVALID, w + "non-finite beam angle");
    if (pd->kind == LIDAR_PATTERN_GAUSS) {
        if (pd->rx_table)
            return fail(h, LIDAR_E_INVALID, w + "rx_table needs a table pattern (its grid)");
        if (!(pd->sigma_deg[0] > 0) || !(pd->sigma_deg[1] > 0) || !is_fin(pd->sigma_deg[0]) ||
            !is_fin(pd->sigma_deg[1]) || !(pd->trunc_sigmas > 0) || !is_fin(pd->trunc_sigmas))
            return fail(h, LIDAR_E_INVALID, w + "Gaussian pattern needs sigma > 0 and trunc_sigmas > 0");
    } else if (pd->kind == LIDAR_PATTERN_TABLE) {
        if (!pd->table || pd->nx < 2 || pd->ny < 2 || (uint64_t)pd->nx * pd->ny > (1u << 24))
            return fail(h, LIDAR_E_INVALID, w + "table pattern needs a table of at least 2x2 (max 16M cells)");
        if (!(pd->half_deg[0] > 0) || !(pd->half_deg[1] > 0) || !is_fin(pd->half_deg[0]) ||
            !is_fin(pd->half_deg[1]))
            return fail(h, LIDAR_E_INVALID, w + "table pattern needs half extents > 0");
        bool any = false;
        for (uint64_t i = 0; i < (uint64_t)pd->nx * pd->ny; ++i) {
            float v = pd->table[i];
            if (!std::isfinite(v) || v < 0.0f)
                return fail(h, LIDAR_E_INVALID, w + "table values must be finite and >= 0");
            any |= v > 0.0f;
        }
        if (!any) return fail(h, LIDAR_E_INVALID, w + "table is all zero (pattern integral is 0)");
        if (pd->rx_table)
            for (uint64_t i = 0; i < (uint64_t)pd->nx * pd->ny; ++i) {
                const float v = pd->rx_table[i];
                if (!std::isfinite(v) || v < 0.0f)
                    return fail(h, LIDAR_E_INVALID, w + "rx_table values must be finite and >= 0");
            }
    } else {
        return fail(h, LIDAR_E_INVALID, w + "unknown pattern kind");
    }
    return LIDAR_OK;
}

lidar_status check_gbuffer(lidar_sim* h, const lidar_gbuffer_desc* g, const std::string& w)
{
    if (!g) return fail(h, LIDAR_E_INVALID, w + "gbuffer is NULL");
    if (g->width == 0 || g->height == 0 || g->pitch < g->width)
        return fail(h, LIDAR_E_INVALID, w + "gbuffer needs width, height >= 1 and pitch >= width");
    if ((uint64_t)g->width * g->height > (1ull << 31))
        return fail(h, LIDAR_E_INVALID, w + "gbuffer larger than 2^31 pixels");
    if (!g->depth || !g->reflectance || !g->retro_gain || !g->normal_x || !g->normal_y || !g->normal_z)
        return fail(h, LIDAR_E_INVALID, w + "gbuffer plane pointer is NULL");
    if (!is_fin(g->az_min_deg) || !is_fin(g->az_max_deg) || !is_fin(g->el_min_deg) ||
        !is_fin(g->el_max_deg) || !(g->az_min_deg < g->az_max_deg) || !(g->el_min_deg < g->el_max_deg))
        return fail(h, LIDAR_E_INVALID, w + "gbuffer angle ranges must be finite with min < max");
    if (g->el_min_deg < -90.0 || g->el_max_deg > 90.0)
        return fail(h, LIDAR_E_INVALID, w + "gbuffer elevations must lie in [-90, 90]");
    return LIDAR_OK;
}

lidar_status check_params(const lidar_sim_params* p, std::string& why)
{
    if (!p) { why = "params is NULL"; return LIDAR_E_INVALID; }
    if (p->n_bins < 1 || p->n_bins > (uint32_t)kMaxBins) {
        why = "n_bins must be in [1, 8000]";
        return LIDAR_E_INVALID;
    }
    if (p->max_echoes < 1 || p->max_echoes > (uint32_t)kMaxEchoes) {
        why = "max_echoes must be in [1, 8]";
        return LIDAR_E_INVALID;
    }
    if (!(p->bin_ns > 0.0) || !is_fin(p->bin_ns)) { why = "bin_ns must be > 0"; return LIDAR_E_INVALID; }
    if (!is_fin(p->threshold)) { why = "threshold must be finite"; return LIDAR_E_INVALID; }
    if (!(p->emit_power >= 0.0) || !is_fin(p->emit_power)) { why = "emit_power must be >= 0"; return LIDAR_E_INVALID; }
    if (p->pulse_taps) {
        if (p->n_pulse_taps < 1 || p->n_pulse_taps > (uint32_t)kMaxTaps || p->n_pulse_taps % 2 == 0) {
            why = "n_pulse_taps must be odd, 1..257";
            return LIDAR_E_INVALID;
        }
        double sum = 0.0;
        for (uint32_t i = 0; i < p->n_pulse_taps; ++i) {
            const float t = p->pulse_taps[i];
            if (!std::isfinite(t) || t < 0.0f) { why = "pulse_taps must be finite and >= 0"; return LIDAR_E_INVALID; }
            sum += t;
        }
        if (!(sum > 0.0)) { why = "pulse_taps must have a positive sum"; return LIDAR_E_INVALID; }
    } else {
        if (!(p->pulse_fwhm_ns > 0.0) || !is_fin(p->pulse_fwhm_ns)) { why = "pulse_fwhm_ns must be > 0"; return LIDAR_E_INVALID; }
        if (!(p->pulse_trunc_sigmas > 0.0) || !is_fin(p->pulse_trunc_sigmas)) { why = "pulse_trunc_sigmas must be > 0"; return LIDAR_E_INVALID; }
    }
    if (p->echo_select > (uint32_t)LIDAR_ECHO_RAW_NEAREST) { why = "unknown echo_select"; return LIDAR_E_INVALID; }
    if (p->range_mode > (uint32_t)LIDAR_RANGE_INTERVAL) { why = "unknown range_mode"; return LIDAR_E_INVALID; }
    if (!is_fin(p->ambient_const) || !(p->sun_irradiance >= 0.0) || !is_fin(p->sun_irradiance)) {
        why = "ambient_const must be finite and sun_irradiance >= 0";
        return LIDAR_E_INVALID;
    }
    for (double c : p->sun_dir)
        if (!is_fin(c)) { why = "sun_dir must be finite"; return LIDAR_E_INVALID; }
    if (p->flags & ~(uint32_t)(LIDAR_KEEP_WAVEFORMS | LIDAR_PROFILE | LIDAR_AUTOTUNE | LIDAR_DETERMINISTIC)) {
        why = "unknown flags";
        return LIDAR_E_INVALID;
    }
    if (!p->pulse_taps) {
        double sigma = p->pulse_fwhm_ns / (2.0 * std::sqrt(2.0 * std::log(2.0)));
        double J = std::ceil(p->pulse_trunc_sigmas * sigma / p->bin_ns);
        if (!(2.0 * J + 1.0 <= kMaxTaps)) { why = "pulse longer than 257 taps"; return LIDAR_E_INVALID; }
    }
    return LIDAR_OK;
}

// Half-width J of the pulse and, for a tabulated pulse, its taps at unit sum
// (FP64 sum, rounded to FP32).
int pulse_half_width(const lidar_sim_params* p)
{
    if (p->pulse_taps) return (int)(p->n_pulse_taps - 1) / 2;
    double sigma = p->pulse_fwhm_ns / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    return (int)std::ceil(p->pulse_trunc_sigmas * sigma / p->bin_ns);
}

std::vector<float> tabulated_taps(const lidar_sim_params* p)
{
    double sum = 0.0;
    for (uint32_t i = 0; i < p->n_pulse_taps; ++i) sum += (double)p->pulse_taps[i];
    std::vector<float> t(p->n_pulse_taps);
    for (uint32_t i = 0; i < p->n_pulse_taps; ++i) t[i] = (float)((double)p->pulse_taps[i] / sum);
    return t;
}

// ---- pattern copies and kernel set-up -----------------------------------

lidar_status copy_pattern(lidar_sim* h, FrameState& fs, const lidar_pattern_desc* pd)
{
    PatternHost& p = fs.pat;
    const size_t B = pd->n_beams;
    p.kind = pd->kind;
    p.az.assign(pd->beam_az_deg, pd->beam_az_deg + B);
    p.el.assign(pd->beam_el_deg, pd->beam_el_deg + B);
    if (pd->kind == LIDAR_PATTERN_GAUSS) {
        p.sigma[0] = pd->sigma_deg[0];
        p.sigma[1] = pd->sigma_deg[1];
        p.trunc = pd->trunc_sigmas;
        p.nx = p.ny = 0;
        p.table.clear();
    } else {
        p.nx = pd->nx;
        p.ny = pd->ny;
        p.half[0] = pd->half_deg[0];
        p.half[1] = pd->half_deg[1];
        p.table.assign(pd->table, pd->table + (size_t)pd->nx * pd->ny);
    }
    if (pd->kind == LIDAR_PATTERN_TABLE && pd->rx_table)
        p.rx.assign(pd->rx_table, pd->rx_table + (size_t)pd->nx * pd->ny);
    else
        p.rx.clear();
    hipStream_t s = h->stream;
    HIP_TRY(h, fs.d_az.ensure(B), "allocate beams");
    HIP_TRY(h, fs.d_el.ensure(B), "allocate beams");
    HIP_TRY(h, hipMemcpyAsync(fs.d_az.p, p.az.data(), B * sizeof(double), hipMemcpyHostToDevice, s), "copy beams");
    HIP_TRY(h, hipMemcpyAsync(fs.d_el.p, p.el.data(), B * sizeof(double), hipMemcpyHostToDevice, s), "copy beams");
    if (p.kind == LIDAR_PATTERN_TABLE) {
        HIP_TRY(h, fs.d_table.ensure(p.table.size()), "allocate table");
        HIP_TRY(h, hipMemcpyAsync(fs.d_table.p, p.table.data(), p.table.size() * sizeof(float),
                                  hipMemcpyHostToDevice, s), "copy table");
    }
    if (!p.rx.empty()) {
        HIP_TRY(h, fs.d_rx.ensure(p.rx.size()), "allocate rx table");
        HIP_TRY(h, hipMemcpyAsync(fs.d_rx.p, p.rx.data(), p.rx.size() * sizeof(float),
                                  hipMemcpyHostToDevice, s), "copy rx table");
    }
    HIP_TRY(h, hipStreamSynchronize(s), "pattern copy synchronise");
    return LIDAR_OK;
}

// Kernel extent on the pixel-offset grid: M = floor(extent_az / dphi),
// N = floor(extent_el / de), extent = trunc * sigma (Gaussian) or the table's
// half extent.
void kernel_extent(const PatternHost& p, const RasterDev& r, double* M, double* N)
{
    if (p.kind == LIDAR_PATTERN_GAUSS) {
        *M = std::floor(p.trunc * p.sigma[0] / r.dphi);
        *N = std::floor(p.trunc * p.sigma[1] / r.de);
    } else {
        *M = std::floor(p.half[0] / r.dphi);
        *N = std::floor(p.half[1] / r.de);
    }
}

// Strip height for a kernel of KH rows when no tuned value exists: 64-row
// strips for tall kernels, 16 or 4 rows (with 4 or 16 column phases) for
// short ones.
int default_tile(int KH) { return KH >= 40 ? 64 : (KH >= 10 ? 16 : 4); }

// Kernel-height class of the autotuner (next power of two).
int height_class(int KH)
{
    int c = 1;
    while (c < KH && c < (1 << 14)) c <<= 1;
    return c;
}

// Beam scheduler.  Beams are grouped G at a time so that one workgroup can
// share the pixel reads of nearby footprints: beams are sorted by their
// (approximate) pixel row band, then column, and a group takes consecutive
// beams of one band whose columns lie within one kernel width.  The groups
// are then ordered by column so that the groups in flight on one XCD cover a
// narrow band of the image.  Scheduling only: the exact pixel of each beam is
// computed on the GPU.
void build_groups(FrameState& fs, const RasterDev& r, int G,
                  const std::vector<lidar_beam_info>& bi)
{
    const PatternHost& p = fs.pat;
    const KernelDev& k = fs.k;
    const size_t B = p.az.size();
    std::vector<double> uf(B), vf(B);
    for (size_t i = 0; i < B; ++i) {
        uf[i] = std::floor((p.az[i] - r.az_min) / r.dphi);
        vf[i] = std::floor((r.el_max - p.el[i]) / r.de);
    }
    auto make = [&](double band, std::vector<std::vector<int32_t>>& groups) {
        std::vector<int32_t> idx(B);
        std::iota(idx.begin(), idx.end(), 0);
        std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) {
            double bx = std::floor(vf[x] / band), by = std::floor(vf[y] / band);
            if (bx != by) return bx < by;
            return uf[x] < uf[y];
        });
        groups.clear();
        std::vector<int32_t> cur;
        double cur_band = 0, cur_u0 = 0;
        for (int32_t i : idx) {
            double b = std::floor(vf[i] / band);
            bool fits = !cur.empty() && (int)cur.size() < G && b == cur_band &&
                        uf[i] - cur_u0 <= (double)k.KW;
            if (!fits && !cur.empty()) {
                groups.push_back(cur);
                cur.clear();
            }
            if (cur.empty()) {
                cur_band = b;
                cur_u0 = uf[i];
            }
            cur.push_back(i);
        }
        if (!cur.empty()) groups.push_back(cur);
    };
    std::vector<std::vector<int32_t>> groups;
    make(1.0, groups);
    if (G > 1 && groups.size() * 2 > B) {
        // few beams share a pixel row: group across a band of rows
        make(std::max(1.0, std::floor(k.KH / 8.0)), groups);
    }
    std::stable_sort(groups.begin(), groups.end(), [&](const std::vector<int32_t>& x,
                                                       const std::vector<int32_t>& y) {
        if (uf[x[0]] != uf[y[0]]) return uf[x[0]] < uf[y[0]];
        return vf[x[0]] < vf[y[0]];
    });
    fs.groups.assign(groups.size() * G, -1);
    fs.group_cost.assign(groups.size(), 0);
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        uint64_t cost = 0;
        for (size_t j = 0; j < groups[gi].size(); ++j) {
            fs.groups[gi * G + j] = groups[gi][j];
            cost += bi[groups[gi][j]].samples;
        }
        fs.group_cost[gi] = cost;
    }
    fs.n_groups = (int)groups.size();
}

// Resample the frame's kernel on its raster, per-row data, raster tables and
// per-beam set-up (pixel, scale, sample count) into `beams`; synchronises
// once to check the pattern integral and to form the beam groups.
lidar_status setup_frame(lidar_sim* h, FrameState& fs, lidar_beam_info* beams, const std::string& w)
{
    const lidar_gbuffer_desc& g = fs.gb;
    RasterDev r = raster_of(g);
    double Mf, Nf;
    kernel_extent(fs.pat, r, &Mf, &Nf);
    if (!(Mf >= 0 && Nf >= 0) || Mf > 4096 || Nf > 4096 || (2 * Mf + 1) * (2 * Nf + 1) > 16.0e6)
        return fail(h, LIDAR_E_INVALID, w + "kernel grid too large for this raster (more than 16M "
                                            "cells or 8193 columns/rows)");
    // the footprint kernel addresses one group window of pixel records with
    // 32-bit byte offsets
    if ((4.0 * Mf + 8.0) * (double)g.height * 8.0 >= 2147483648.0)
        return fail(h, LIDAR_E_INVALID, w + "kernel window times image height too large "
                                            "(4*M+8)*height*8 must stay below 2^31 bytes");
    KernelDev k;
    k.M = (int)Mf;
    k.N = (int)Nf;
    k.KW = 2 * k.M + 1;
    k.KH = 2 * k.N + 1;
    const size_t cells = (size_t)k.KW * k.KH;
    const size_t B = fs.pat.az.size();
    HIP_TRY(h, fs.d_K64.ensure(cells), "allocate kernel");
    HIP_TRY(h, fs.d_Kb.ensure((size_t)4 * kernel_blocks(k.KW) * (k.KH + 1) * 4),
            "allocate kernel blocks");
    HIP_TRY(h, fs.d_rowsum.ensure(k.KH), "allocate kernel rows");
    HIP_TRY(h, fs.d_rowmax.ensure(k.KH), "allocate kernel rows");
    HIP_TRY(h, fs.d_rowrange.ensure(k.KH), "allocate kernel rows");
    HIP_TRY(h, fs.d_prefix.ensure((size_t)k.KH * (k.KW + 1)), "allocate kernel rows");
    HIP_TRY(h, fs.d_kinfo.ensure(2), "allocate kernel info");
    HIP_TRY(h, fs.d_colcs.ensure(g.width), "allocate raster tables");
    HIP_TRY(h, fs.d_rowtab.ensure(g.height), "allocate raster tables");
    HIP_TRY(h, fs.d_omega.ensure((size_t)g.height + 2 * (size_t)k.KH), "allocate raster tables");

    PatternDev p;
    p.kind = (int)fs.pat.kind;
    p.sx = fs.pat.sigma[0];
    p.sy = fs.pat.sigma[1];
    p.trunc = fs.pat.trunc;
    p.table = fs.d_table.p;
    p.nx = (int)fs.pat.nx;
    p.ny = (int)fs.pat.ny;
    p.hx = fs.pat.half[0];
    p.hy = fs.pat.half[1];
    hipStream_t s = h->stream;
    HIP_TRY(h, launch_kernel_grid(s, p, r, k, fs.d_K64.p), "kernel grid launch");
    HIP_TRY(h, launch_kernel_blocks(s, k, fs.d_K64.p, fs.d_Kb.p), "kernel blocks launch");
    HIP_TRY(h, launch_kernel_rows(s, k, fs.d_K64.p, fs.d_rowsum.p, fs.d_rowmax.p,
                                  fs.d_rowrange.p, fs.d_prefix.p), "kernel rows launch");
    HIP_TRY(h, launch_kernel_peak(s, k, fs.d_rowsum.p, fs.d_rowmax.p, fs.d_kinfo.p),
            "kernel peak launch");
    HIP_TRY(h, launch_raster_tables(s, r, fs.d_colcs.p, fs.d_rowtab.p), "raster tables launch");
    HIP_TRY(h, launch_beam_setup(s, r, k, fs.d_az.p, fs.d_el.p, (int)B, fs.d_rowsum.p,
                                 fs.d_prefix.p, fs.d_omega.p, h->prm.emit_power, beams),
            "beam setup launch");
    if (!fs.pat.rx.empty()) {
        // kappa on the same pixel-offset grid and in the same blocks as K
        PatternDev prx = p;
        prx.table = fs.d_rx.p;
        HIP_TRY(h, fs.d_K64rx.ensure(cells), "allocate kappa grid");
        HIP_TRY(h, fs.d_Kr.ensure((size_t)4 * kernel_blocks(k.KW) * (k.KH + 1) * 4), "allocate kappa blocks");
        HIP_TRY(h, launch_kernel_grid(s, prx, r, k, fs.d_K64rx.p), "kappa grid launch");
        HIP_TRY(h, launch_kernel_blocks(s, k, fs.d_K64rx.p, fs.d_Kr.p), "kappa blocks launch");
    }
    if (h->prm.range_mode != LIDAR_RANGE_CENTRE) {
        HIP_TRY(h, fs.d_col64.ensure(g.width), "allocate range tables");
        HIP_TRY(h, fs.d_row64.ensure(g.height), "allocate range tables");
        HIP_TRY(h, fs.d_cole.ensure((size_t)g.width + 1), "allocate range tables");
        HIP_TRY(h, fs.d_rowe.ensure((size_t)g.height + 1), "allocate range tables");
        HIP_TRY(h, launch_range_tables(s, r, fs.d_col64.p, fs.d_row64.p, fs.d_cole.p, fs.d_rowe.p),
                "range tables launch");
    }
    if (h->prm.range_mode == LIDAR_RANGE_CORRECTED) {
        HIP_TRY(h, fs.d_bcorr.ensure(B), "allocate beam offsets");
        HIP_TRY(h, launch_beam_corr(s, r, fs.d_az.p, fs.d_el.p, (int)B, beams, fs.d_bcorr.p),
                "beam offsets launch");
    }
    // the pattern's integral over the grid must be positive: checked once per
    // (pattern, raster), which synchronises the stream
    double kinfo[2];
    HIP_TRY(h, hipMemcpyAsync(kinfo, fs.d_kinfo.p, sizeof(kinfo), hipMemcpyDeviceToHost, s),
            "copy kernel info");
    std::vector<lidar_beam_info> bi(B);
    HIP_TRY(h, hipMemcpyAsync(bi.data(), beams, sizeof(lidar_beam_info) * B,
                              hipMemcpyDeviceToHost, s), "copy beam info");
    HIP_TRY(h, hipStreamSynchronize(s), "set-up synchronise");
    if (!(kinfo[1] > 0.0) || !is_fin(kinfo[1]) || !(kinfo[0] > 0.0))
        return fail(h, LIDAR_E_INVALID, w + "pattern integral over the kernel grid is not positive "
                                            "(kernel narrower than one pixel or all-zero table)");
    uint64_t total = 0;
    for (auto& x : bi) total += x.samples;
    fs.k = k;
    fs.geom_ok = false;
    fs.kmax = kinfo[0];
    fs.samples = total;
    fs.tile = default_tile(k.KH);
    build_groups(fs, r, h->G, bi);
    return LIDAR_OK;
}

lidar_status alloc_pixels(lidar_sim* h, FrameState& fs)
{
    const size_t W4 = (fs.gb.width + 3) & ~3u;
    const size_t npix = W4 * fs.gb.height;
    HIP_TRY(h, fs.d_pix.ensure(npix), "allocate pixel records");
    if (h->prm.sun_irradiance != 0.0) HIP_TRY(h, fs.d_sun.ensure(npix), "allocate sun shading");
    if (h->prm.range_mode == LIDAR_RANGE_CORRECTED) HIP_TRY(h, fs.d_rec4.ensure(npix), "allocate depth records");
    return LIDAR_OK;
}

PrepassArgs prepass_args(const lidar_sim* h, FrameState& fs)
{
    const lidar_gbuffer_desc& g = fs.gb;
    const bool sun = h->prm.sun_irradiance != 0.0;
    PrepassArgs pa{};
    pa.depth = g.depth;
    pa.refl = g.reflectance;
    pa.gain = g.retro_gain;
    pa.nx = g.normal_x;
    pa.ny = g.normal_y;
    pa.nz = g.normal_z;
    pa.pitch = (long)g.pitch;
    pa.W = (int)g.width;
    pa.H = (int)g.height;
    pa.W4 = (int)((g.width + 3) & ~3u);
    pa.colcs = fs.d_colcs.p;
    pa.rowtab = fs.d_rowtab.p;
    pa.to_bin = 2.0 / (kLight * (h->prm.bin_ns * 1e-9));
    pa.R = (int)h->prm.n_bins;
    pa.sun_x = (float)h->prm.sun_dir[0];
    pa.sun_y = (float)h->prm.sun_dir[1];
    pa.sun_z = (float)h->prm.sun_dir[2];
    pa.pix = fs.d_pix.p;
    pa.sun = sun ? fs.d_sun.p : nullptr;
    pa.range_mode = (int)h->prm.range_mode;
    pa.rt.col = fs.d_col64.p;
    pa.rt.row = fs.d_row64.p;
    pa.rt.col_edge = fs.d_cole.p;
    pa.rt.row_edge = fs.d_rowe.p;
    pa.rec4 = h->prm.range_mode == LIDAR_RANGE_CORRECTED ? fs.d_rec4.p : nullptr;
    pa.stats = nullptr;
    return pa;
}

// Sun floor from the frame's kappa table into beams[].floor (frames with
// one; the footprint kernel then reads the floor instead of summing it).
lidar_status enqueue_sun_floor(lidar_sim* h, FrameState& fs, lidar_beam_info* beams, hipStream_t s)
{
    const bool sun = h->prm.sun_irradiance != 0.0;
    if (fs.pat.rx.empty() || !sun) return LIDAR_OK;
    SunFloorArgs a;
    a.sun = sun ? fs.d_sun.p : nullptr;
    a.W = (int)fs.gb.width;
    a.H = (int)fs.gb.height;
    a.Kr = fs.d_Kr.p;
    a.M = fs.k.M;
    a.N = fs.k.N;
    a.KW = fs.k.KW;
    a.KH = fs.k.KH;
    a.NB = kernel_blocks(fs.k.KW);
    a.ambient = (float)h->prm.ambient_const;
    a.e_sun = (float)h->prm.sun_irradiance;
    a.beams = beams;
    a.B = (int)fs.pat.az.size();
    HIP_TRY(h, launch_sun_floor(s, a), "sun floor launch");
    return LIDAR_OK;
}

lidar_status enqueue_prepass(lidar_sim* h, FrameState& fs, hipStream_t s)
{
    HIP_TRY(h, launch_prepass(s, prepass_args(h, fs), h->prm.sun_irradiance != 0.0),
            "pre-pass launch");
    return LIDAR_OK;
}

bool fixed_point_ok(const lidar_sim* h);

// The pre-pass of every frame of the batch in one launch (tables built by
// setup_batch), then the frames' statistics for fixed-point accumulation.
lidar_status enqueue_batch_prepass(lidar_sim* h, hipStream_t s)
{
    HIP_TRY(h, launch_prepass_batch(s, h->b_prep.p, h->b_prep_off.p, (int)h->frames.size(),
                                    h->b_prep_tiles, h->prm.sun_irradiance != 0.0,
                                    (int)h->prm.range_mode),
            "batch pre-pass launch");
    // floors of the frames with a kappa table
    for (size_t i = 0; i < h->frames.size(); ++i)
        LIDAR_TRY(enqueue_sun_floor(h, *h->frames[i], h->b_beams.p + h->beam_off[i], s));
    if (h->b_fstats.p && fixed_point_ok(h))
        HIP_TRY(h, launch_reduce_stats(s, h->b_tstats.p, h->b_prep_off.p, h->b_fstats.p, (int)h->frames.size()),
                "statistics launch");
    return LIDAR_OK;
}

FrameDev frame_view(const lidar_sim* h, const FrameState& fs, lidar_beam_info* beams,
                    lidar_echo* echoes, int32_t* counts, float* waves)
{
    const bool sun = h->prm.sun_irradiance != 0.0;
    const bool given = !fs.pat.rx.empty() && sun;    // floor from the kappa kernel
    FrameDev f{};
    f.pix = fs.d_pix.p;
    // the sun records stay addressable with a supplied floor: batch kernels
    // run one SUN instantiation for all frames (the sum is then discarded)
    f.sun = sun ? fs.d_sun.p : nullptr;
    f.span = h->prm.range_mode == LIDAR_RANGE_INTERVAL ? 1 : 0;
    f.floor_given = given ? 1 : 0;
    f.rec4 = fs.d_rec4.p;
    f.col64 = fs.d_col64.p;
    f.row64 = fs.d_row64.p;
    f.bcorr = fs.d_bcorr.p;
    f.to_bin = 2.0 / (kLight * (h->prm.bin_ns * 1e-9));
    f.W = (int)fs.gb.width;
    f.H = (int)fs.gb.height;
    f.Kb = fs.d_Kb.p;
    f.rowrange = fs.d_rowrange.p;
    f.M = fs.k.M;
    f.N = fs.k.N;
    f.KW = fs.k.KW;
    f.KH = fs.k.KH;
    f.NB = kernel_blocks(fs.k.KW);
    f.tile = fs.tile;
    f.sun_scale = sun ? (float)(h->prm.sun_irradiance / fs.kmax) : 0.0f;
    f.beams = beams;
    f.echoes = echoes;
    f.counts = counts;
    f.waves = waves;
    return f;
}

PathDev path_view(const lidar_sim* h)
{
    PathDev p;
    p.taps = h->d_taps.p;
    p.J = h->J;
    p.R = (int)h->prm.n_bins;
    p.E = (int)h->prm.max_echoes;
    p.select = (int)h->prm.echo_select;
    p.threshold = (float)h->prm.threshold;
    p.ambient = (float)h->prm.ambient_const;
    p.half_c_dt = 0.5 * kLight * (h->prm.bin_ns * 1e-9);
    p.bin_ns = h->prm.bin_ns;
    return p;
}

// ---- surrogate inputs, gate, fallback ---------------------------------------

// Cell sizes of the surrogate's inputs from the frame's kernel grid (host
// copy; once per pattern and raster).
lidar_status sur_geometry(lidar_sim* h, FrameState& fs)
{
    if (fs.geom_ok) return LIDAR_OK;
    const KernelDev& k = fs.k;
    std::vector<double> K((size_t)k.KW * k.KH);
    HIP_TRY(h, hipMemcpyAsync(K.data(), fs.d_K64.p, K.size() * sizeof(double), hipMemcpyDeviceToHost,
                              h->stream), "copy kernel grid");
    HIP_TRY(h, hipStreamSynchronize(h->stream), "kernel grid synchronise");
    int cm = 0, cn = 0;
    for (int n = 0; n < k.KH; ++n)
        for (int m = 0; m < k.KW; ++m)
            if (K[(size_t)n * k.KW + m] >= kSurCoreFraction * fs.kmax) {
                cm = std::max(cm, std::abs(m - k.M));
                cn = std::max(cn, std::abs(n - k.N));
            }
    SurGeom g;
    g.cm = cm;
    g.cn = cn;
    g.cw = std::max(1, (2 * cm + 1 + kSurPatch - 1) / kSurPatch);
    g.ch = std::max(1, (2 * cn + 1 + kSurPatch - 1) / kSurPatch);
    g.sw = std::max(1, (k.KW + kSurPatch - 1) / kSurPatch);
    g.sh = std::max(1, (k.KH + kSurPatch - 1) / kSurPatch);
    const int W = (int)fs.gb.width, H = (int)fs.gb.height;
    g.CW = (W + g.cw - 1) / g.cw;
    g.CH = (H + g.ch - 1) / g.ch;
    g.SW = (W + g.sw - 1) / g.sw;
    g.SH = (H + g.sh - 1) / g.sh;
    HIP_TRY(h, fs.d_cell.ensure((size_t)g.CW * g.CH), "allocate coarse cells");
    HIP_TRY(h, fs.d_cell_sun.ensure((size_t)g.CW * g.CH), "allocate coarse cells");
    HIP_TRY(h, fs.d_cell_shade.ensure((size_t)g.CW * g.CH), "allocate coarse cells");
    HIP_TRY(h, fs.d_sup.ensure((size_t)g.SW * g.SH), "allocate super-cells");
    HIP_TRY(h, fs.d_range.ensure((size_t)g.SW * g.SH), "allocate super-cells");
    fs.geom = g;
    fs.geom_ok = true;
    return LIDAR_OK;
}

// Enqueue the pre-pass, the coarse and super-cell maps and the per-beam
// network inputs (into X) of the single frame.
lidar_status sur_inputs(lidar_sim* h, FrameState& fs, uint16_t* X)
{
    hipStream_t s = h->stream;
    const lidar_gbuffer_desc& g = fs.gb;
    const int B = (int)fs.pat.az.size();
    HIP_TRY(h, h->s_aux.ensure(B), "allocate surrogate beam data");
    if (h->s_aux_gen != h->pattern_gen || h->s_aux_ptr != h->s_aux.p) {
        // no gate decision yet for these beams
        HIP_TRY(h, launch_zero_f32(s, (float*)h->s_aux.p, (long)B * (long)(sizeof(SurAux) / 4)),
                "clear surrogate beam data");
        h->s_aux_gen = h->pattern_gen;
        h->s_aux_ptr = h->s_aux.p;
    }
    LIDAR_TRY(enqueue_prepass(h, fs, s));
    const bool sun = h->prm.sun_irradiance != 0.0;
    const double to_bin = 2.0 / (kLight * (h->prm.bin_ns * 1e-9));
    CoarseArgs ca;
    ca.depth = g.depth;
    ca.refl = g.reflectance;
    ca.gain = g.retro_gain;
    ca.nx = g.normal_x;
    ca.ny = g.normal_y;
    ca.nz = g.normal_z;
    ca.pitch = (long)g.pitch;
    ca.W = (int)g.width;
    ca.H = (int)g.height;
    ca.colcs = fs.d_colcs.p;
    ca.rowtab = fs.d_rowtab.p;
    ca.to_bin = to_bin;
    ca.R = (int)h->prm.n_bins;
    ca.sun_x = (float)h->prm.sun_dir[0];
    ca.sun_y = (float)h->prm.sun_dir[1];
    ca.sun_z = (float)h->prm.sun_dir[2];
    ca.g = fs.geom;
    ca.cell = fs.d_cell.p;
    ca.cell_sun = fs.d_cell_sun.p;
    ca.cell_shade = fs.d_cell_shade.p;
    HIP_TRY(h, launch_coarse(s, ca), "coarse cells launch");
    SuperArgs sa;
    sa.pix = fs.d_pix.p;
    sa.sun = sun ? fs.d_sun.p : nullptr;
    sa.W = ca.W;
    sa.H = ca.H;
    sa.g = fs.geom;
    sa.sup = fs.d_sup.p;
    sa.range = fs.d_range.p;
    // super-cells feed only the sun floor and tail energy outside the core box:
    // none when the core box spans the kernel window (as for truncated Gaussians)
    if (fs.geom.cm < fs.k.M || fs.geom.cn < fs.k.N)
        HIP_TRY(h, launch_super(s, sa), "super-cells launch");
    FeatArgs fa;
    fa.beams = h->d_beams.p;
    fa.az = fs.d_az.p;
    fa.el = fs.d_el.p;
    fa.B = B;
    fa.depth = g.depth;
    fa.pitch = (long)g.pitch;
    fa.W = ca.W;
    fa.H = ca.H;
    fa.to_bin = to_bin;
    fa.R = ca.R;
    fa.cell = fs.d_cell.p;
    fa.cell_sun = fs.d_cell_sun.p;
    fa.cell_shade = fs.d_cell_shade.p;
    fa.sup = fs.d_sup.p;
    fa.range = fs.d_range.p;
    fa.K64 = fs.d_K64.p;
    fa.M = fs.k.M;
    fa.N = fs.k.N;
    fa.KW = fs.k.KW;
    fa.g = fs.geom;
    fa.ambient = (float)h->prm.ambient_const;
    fa.sun_scale = sun ? (float)(h->prm.sun_irradiance / fs.kmax) : 0.0f;
    fa.threshold = (float)h->prm.threshold;
    fa.X = X;
    fa.aux = h->s_aux.p;
    HIP_TRY(h, launch_features(s, fa), "features launch");
    return LIDAR_OK;
}

// ---- batches ---------------------------------------------------------------

void free_graph(lidar_sim* h)
{
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->graph_exec = nullptr;
    h->graph = nullptr;
}

// Enqueue the batch on s: the pre-pass of every frame (optional), the queue
// reset and the persistent footprint launches over `items`: handed out in the
// runs `tickets` if given (the first n_group of them to the group schedule,
// the rest to the wave schedule), else one by one to the group schedule.
lidar_status enqueue_batch(lidar_sim* h, hipStream_t s, const int2* items, uint64_t n_items,
                           bool with_prepass, const int32_t* tickets = nullptr, int n_tickets = 0,
                           int n_group = -1)
{
    if (n_group < 0) n_group = n_tickets;
    if (with_prepass) LIDAR_TRY(enqueue_batch_prepass(h, s));
    HIP_TRY(h, launch_reset_queue(s, h->b_queue.p, 2 * kQueueInts), "queue reset launch");
    BatchArgs ba{};
    ba.frames = h->b_frames.p;
    ba.p = path_view(h);
    ba.groups = h->b_groups.p;
    ba.items = items;
    ba.n_items = (int)n_items;
    ba.G = h->G;
    ba.next_item = h->b_queue.p;
    ba.n_items_dev = nullptr;
    ba.tickets = tickets;
    ba.n_tickets = n_group;
    ba.fcount = fixed_point_ok(h) && h->b_fstats.p ? h->b_fstats.p + 4 * h->frames.size() : nullptr;
    const bool sun = h->prm.sun_irradiance != 0.0;
    const bool keep = (h->prm.flags & LIDAR_KEEP_WAVEFORMS) != 0;
    if (!tickets || n_group > 0)
        HIP_TRY(h, launch_footprint_batch(s, ba, h->b_grid, sun, keep), "batch footprint launch");
    if (tickets && n_tickets > n_group) {
        ba.tickets = tickets + n_group;
        ba.n_tickets = n_tickets - n_group;
        ba.next_item = h->b_queue.p + kQueueInts;
        HIP_TRY(h, launch_footprint_batch_wave(s, ba, h->b_grid, sun, keep), "batch wave-schedule launch");
    }
    return LIDAR_OK;
}

// Device table of the frames (pointers into the batch outputs, current tiles).
lidar_status upload_frame_table(lidar_sim* h)
{
    const bool keep = (h->prm.flags & LIDAR_KEEP_WAVEFORMS) != 0;
    const size_t E = h->prm.max_echoes, R = h->prm.n_bins;
    std::vector<FrameDev> fd(h->frames.size());
    for (size_t i = 0; i < h->frames.size(); ++i) {
        const uint64_t o = h->beam_off[i];
        fd[i] = frame_view(h, *h->frames[i], h->b_beams.p + o, h->b_echoes.p + o * E,
                           h->b_counts.p + o, keep ? h->b_waves.p + o * R : nullptr);
        fd[i].wave = h->frames[i]->wave;
        fd[i].direct = h->frames[i]->direct ? h->b_direct.p + i : nullptr;
        fd[i].fstats = !h->frames[i]->direct && fixed_point_ok(h) ? h->b_fstats.p + 4 * i : nullptr;
        fd[i].kmax = (float)h->frames[i]->kmax;
    }
    HIP_TRY(h, h->b_frames.ensure(fd.size()), "allocate frame table");
    HIP_TRY(h, hipMemcpyAsync(h->b_frames.p, fd.data(), fd.size() * sizeof(FrameDev),
                              hipMemcpyHostToDevice, h->stream), "copy frame table");
    HIP_TRY(h, hipStreamSynchronize(h->stream), "frame table synchronise");
    return LIDAR_OK;
}

// Tickets over items in queue order: runs of consecutive items whose cost
// reaches a target that shrinks with the work left (guided self-scheduling: a
// quarter of an even share per worker), at most kMaxTicket items; the costly
// head goes one item per ticket, the cheap tail in runs, and the last tickets
// are small again so that the workers finish together.  The workers are the
// workgroups of the group schedule or the waves of the wave schedule; a
// ticket costs at least min_cost where items allow (each ticket is a queue
// atomic, which matters when the items are tiny).
std::vector<int32_t> build_tickets(const uint64_t* cost, size_t n, uint64_t workers, int32_t first,
                                   uint64_t min_cost = 0)
{
    constexpr size_t kMaxTicket = 256;
    std::vector<int32_t> tickets;
    uint64_t remaining = 0;
    for (size_t j = 0; j < n; ++j) remaining += cost[j];
    for (size_t j = 0; j < n;) {
        const uint64_t target = remaining / (4 * workers);
        uint64_t acc = 0;
        size_t k = j;
        do acc += cost[k++];
        while (k < n && k - j < kMaxTicket && (acc < target || acc < min_cost));
        tickets.push_back(first + (int32_t)k);
        remaining -= acc;
        j = k;
    }
    return tickets;
}

// Smallest ticket of the wave schedule: the convolution and detection cost
// of four single-beam items (see the item cost in setup_batch).
uint64_t wave_ticket_cost(const lidar_sim* h)
{
    return 4 * (uint64_t)h->G * h->prm.n_bins * (2 * h->J + 1) / 8;
}

// Whether the batch may use the wave schedule: one histogram slot per wave
// (groups of kWavesPerGroup) and waveforms short enough for registers.
bool wave_schedule_ok(const lidar_sim* h)
{
    return h->G == kWavesPerGroup && (int)h->prm.n_bins <= kWaveMaxBins;
}

// Whether the wave schedule may accumulate in fixed point (pixel keys are
// single bins: centre ranges).
bool fixed_point_ok(const lidar_sim* h)
{
    return wave_schedule_ok(h) && h->prm.range_mode == LIDAR_RANGE_CENTRE;
}

// Autotuner: for every kernel-height class of the batch, time the persistent
// launch over that class's items alone (in tickets, as the batch runs them)
// with each candidate strip height, in the group and in the wave schedule,
// and keep the fastest.  The pixel records are computed once first; the
// results are remembered by the handle for later batches.
lidar_status autotune_batch(lidar_sim* h, const std::vector<int2>& items, const std::vector<uint64_t>& cost)
{
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = h->stream;
    LIDAR_TRY(enqueue_batch_prepass(h, s));
    std::map<int, std::vector<size_t>> by_class;
    for (size_t j = 0; j < items.size(); ++j) {
        const FrameState& fs = *h->frames[items[j].x];
        if (!fs.direct) by_class[height_class(fs.k.KH)].push_back(j);   // direct frames: wave, no strips
    }
    DevBuf<int2> d_trial;
    DevBuf<int32_t> d_tickets;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    lidar_status st = he == hipSuccess ? LIDAR_OK : hip_fail(h, he, "autotune events");
    const int n_modes = wave_schedule_ok(h) ? 2 : 1;
    for (auto& kv : by_class) {
        if (st != LIDAR_OK) break;
        const int cls = kv.first;
        std::vector<int2> its;
        std::vector<uint64_t> cs;
        for (size_t j : kv.second) {
            its.push_back(items[j]);
            cs.push_back(cost[j]);
        }
        he = d_trial.ensure(its.size());
        if (he == hipSuccess)
            he = hipMemcpyAsync(d_trial.p, its.data(), its.size() * sizeof(int2),
                                hipMemcpyHostToDevice, s);
        if (he != hipSuccess) {
            st = hip_fail(h, he, "autotune items");
            break;
        }
        float best = 1e30f;
        int best_tile = default_tile(cls), best_wave = 0;
        for (int mode = 0; mode < n_modes && st == LIDAR_OK; ++mode) {
            std::vector<int32_t> tk(1, 0);
            const std::vector<int32_t> runs =
                build_tickets(cs.data(), cs.size(), (uint64_t)h->b_grid * (mode ? kWavesPerGroup : 1), 0,
                              mode ? wave_ticket_cost(h) : 0);
            tk.insert(tk.end(), runs.begin(), runs.end());
            he = d_tickets.ensure(tk.size());
            if (he == hipSuccess)
                he = hipMemcpyAsync(d_tickets.p, tk.data(), tk.size() * sizeof(int32_t),
                                    hipMemcpyHostToDevice, s);
            if (he != hipSuccess) {
                st = hip_fail(h, he, "autotune tickets");
                break;
            }
            for (int tile : {64, 16, 4}) {
                if (tile == 64 && cls < 16) continue;   // strips 4x taller than the kernel
                for (auto& fs : h->frames)
                    if (height_class(fs->k.KH) == cls && !fs->direct) {
                        fs->tile = tile;
                        fs->wave = mode;
                    }
                if ((st = upload_frame_table(h)) != LIDAR_OK) break;
                float ms = 0.0f;
                for (int rep = 0; rep < 2 && st == LIDAR_OK; ++rep) {
                    he = hipEventRecord(e0, s);
                    if (he != hipSuccess) { st = hip_fail(h, he, "autotune event"); break; }
                    const int nt = (int)tk.size() - 1;
                    if ((st = enqueue_batch(h, s, d_trial.p, its.size(), false, d_tickets.p, nt,
                                            mode ? 0 : nt)) != LIDAR_OK)
                        break;
                    he = hipEventRecord(e1, s);
                    if (he == hipSuccess) he = hipEventSynchronize(e1);
                    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
                    if (he != hipSuccess) { st = hip_fail(h, he, "autotune timing"); break; }
                }
                if (st != LIDAR_OK) break;
                if (ms < best) {
                    best = ms;
                    best_tile = tile;
                    best_wave = mode;
                }
            }
        }
        if (st != LIDAR_OK) break;
        h->tuned[cls] = {best_tile, best_wave};
        for (auto& fs : h->frames)
            if (height_class(fs->k.KH) == cls && !fs->direct) {
                fs->tile = best_tile;
                fs->wave = best_wave;
            }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    LIDAR_TRY(st);
    LIDAR_TRY(upload_frame_table(h));
    h->b_autotuned = true;
    h->b_autotune_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return LIDAR_OK;
}

lidar_status setup_batch(lidar_sim* h, const lidar_gbuffer_desc* gbs, const lidar_pattern_desc* pds,
                         uint32_t n)
{
    // a previous batch may still run on the stream with these buffers
    HIP_TRY(h, hipStreamSynchronize(h->stream), "batch synchronise");
    h->batch_ok = false;
    h->batch_result = false;
    free_graph(h);
    for (uint32_t i = 0; i < n; ++i) {
        const std::string who = "frame " + std::to_string(i) + ": ";
        LIDAR_TRY(check_pattern(h, &pds[i], who));
        LIDAR_TRY(check_gbuffer(h, &gbs[i], who));
    }
    h->frames.resize(n);
    h->beam_off.assign(n + 1, 0);
    for (uint32_t i = 0; i < n; ++i) {
        if (!h->frames[i]) h->frames[i].reset(new (std::nothrow) FrameState());
        if (!h->frames[i]) return fail(h, LIDAR_E_NOMEM, "out of host memory");
        h->beam_off[i + 1] = h->beam_off[i] + pds[i].n_beams;
    }
    const uint64_t B = h->beam_off[n];
    const size_t E = h->prm.max_echoes, R = h->prm.n_bins;
    HIP_TRY(h, h->b_beams.ensure(B), "allocate batch beams");
    HIP_TRY(h, h->b_echoes.ensure(B * E), "allocate batch echoes");
    HIP_TRY(h, h->b_counts.ensure(B), "allocate batch counts");
    if (h->prm.flags & LIDAR_KEEP_WAVEFORMS) HIP_TRY(h, h->b_waves.ensure(B * R), "allocate batch waveforms");
    HIP_TRY(h, h->b_queue.ensure(2 * kQueueInts), "allocate work queues");
    std::vector<uint64_t> group_off(n + 1, 0);
    uint64_t samples = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const std::string who = "frame " + std::to_string(i) + ": ";
        FrameState& fs = *h->frames[i];
        fs.gb = gbs[i];
        LIDAR_TRY(copy_pattern(h, fs, &pds[i]));
        LIDAR_TRY(setup_frame(h, fs, h->b_beams.p + h->beam_off[i], who));
        auto it = h->tuned.find(height_class(fs.k.KH));
        if (it != h->tuned.end()) std::tie(fs.tile, fs.wave) = it->second;
        LIDAR_TRY(alloc_pixels(h, fs));
        group_off[i + 1] = group_off[i] + fs.n_groups;
        samples += fs.samples;
    }
    const uint64_t total_groups = group_off[n];
    if (total_groups >= (1ull << 31)) return fail(h, LIDAR_E_INVALID, "batch has more than 2^31 beam groups");
    // pre-pass tables: every frame's arguments and tile offsets (the host
    // vectors outlive the copies: the frame-table upload below synchronises)
    std::vector<PrepassArgs> pa(n);
    std::vector<int32_t> off(n + 1, 0);
    {
        uint64_t tiles = 0;
        std::vector<DirectDev> dd(n);
        if (fixed_point_ok(h)) HIP_TRY(h, h->b_fstats.ensure(4 * (size_t)n + 4), "allocate frame statistics");
        for (uint32_t i = 0; i < n; ++i) {
            FrameState& fs = *h->frames[i];
            pa[i] = prepass_args(h, fs);
            off[i] = (int32_t)tiles;
            // frames whose beams touch few of their pixels (at most one
            // sample per two pixels) with small footprints (at most 256
            // samples per beam: one wave walks a beam's cells, with an
            // atomic per cell) skip the pre-pass: the wave schedule gathers
            // them from the planes
            const uint64_t nb = fs.pat.az.size();
            fs.direct = wave_schedule_ok(h) && h->prm.range_mode == LIDAR_RANGE_CENTRE &&
                        fs.pat.rx.empty() && 2 * fs.samples <= (uint64_t)fs.gb.width * fs.gb.height &&
                        fs.samples <= 256 * nb;
            if (!fs.direct) tiles += (uint64_t)prepass_tiles(pa[i]);
            dd[i] = DirectDev{pa[i].depth, pa[i].refl, pa[i].gain, pa[i].nx, pa[i].ny, pa[i].nz,
                              pa[i].pitch, pa[i].colcs, pa[i].rowtab, pa[i].sun_x, pa[i].sun_y,
                              pa[i].sun_z, 0};
        }
        HIP_TRY(h, h->b_direct.ensure(n), "allocate direct-gather table");
        HIP_TRY(h, hipMemcpyAsync(h->b_direct.p, dd.data(), n * sizeof(DirectDev), hipMemcpyHostToDevice,
                                  h->stream), "copy direct-gather table");
        HIP_TRY(h, hipStreamSynchronize(h->stream), "direct-gather table synchronise");
        if (tiles >= (1ull << 31)) return fail(h, LIDAR_E_INVALID, "batch has more than 2^31 pre-pass tiles");
        // the tiles' statistics records, frame i's from its first tile on
        if (fixed_point_ok(h)) {
            HIP_TRY(h, h->b_tstats.ensure(4 * std::max<uint64_t>(tiles, 1)), "allocate tile statistics");
            for (uint32_t i = 0; i < n; ++i)
                if (!h->frames[i]->direct) pa[i].stats = h->b_tstats.p + 4 * (size_t)off[i];
        }
        off[n] = (int32_t)tiles;
        h->b_prep_tiles = (int)tiles;
        HIP_TRY(h, h->b_prep.ensure(n), "allocate pre-pass table");
        HIP_TRY(h, h->b_prep_off.ensure(n + 1), "allocate pre-pass offsets");
        HIP_TRY(h, hipMemcpyAsync(h->b_prep.p, pa.data(), n * sizeof(PrepassArgs),
                                  hipMemcpyHostToDevice, h->stream), "copy pre-pass table");
        HIP_TRY(h, hipMemcpyAsync(h->b_prep_off.p, off.data(), (n + 1) * sizeof(int32_t),
                                  hipMemcpyHostToDevice, h->stream), "copy pre-pass offsets");
    }
    // every frame's groups in one table; work items ordered by estimated
    // cost, costliest first (gather samples plus the convolution and
    // detection work of the group's R bins)
    const int G = h->G;
    std::vector<int32_t> groups(total_groups * G);
    std::vector<int2> items(total_groups);
    std::vector<uint64_t> cost(total_groups);
    const uint64_t bin_cost = (uint64_t)G * R * (2 * h->J + 1) / 8;
    for (uint32_t i = 0; i < n; ++i) {
        FrameState& fs = *h->frames[i];
        std::copy(fs.groups.begin(), fs.groups.end(), groups.begin() + group_off[i] * G);
        for (int gi = 0; gi < fs.n_groups; ++gi) {
            const uint64_t gidx = group_off[i] + gi;
            items[gidx] = make_int2((int)i, (int)gidx);
            cost[gidx] = fs.group_cost[gi] + bin_cost;
        }
    }
    HIP_TRY(h, h->b_groups.ensure(groups.size()), "allocate batch groups");
    HIP_TRY(h, hipMemcpyAsync(h->b_groups.p, groups.data(), groups.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, h->stream), "copy batch groups");
    h->b_items_n = total_groups;
    h->b_samples = samples;
    // persistent grid: as many workgroups as the CUs hold at the LDS-bound
    // occupancy (extra workgroups would find the queue empty and exit)
    const size_t lds = group_lds_bytes(G, R, h->J) + 2048;   // + static LDS
    const size_t per_cu = std::max<size_t>(1, std::min<size_t>(8, (160 * 1024) / lds));
    h->b_grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)h->cus * per_cu, total_groups));
    // schedule per frame: remembered from an earlier autotuning of the class,
    // else the wave schedule where most groups hold a single beam (three of
    // the four waves of a group would idle), then the autotuner if asked
    for (uint32_t i = 0; i < n; ++i) {
        FrameState& fs = *h->frames[i];
        auto it = h->tuned.find(height_class(fs.k.KH));
        if (it != h->tuned.end()) continue;
        uint64_t members = 0;
        for (int32_t b : fs.groups) members += b >= 0 ? 1 : 0;
        fs.wave = wave_schedule_ok(h) && members < 2 * (uint64_t)fs.n_groups ? 1 : 0;
    }
    if (!wave_schedule_ok(h))
        for (auto& fs : h->frames) fs->wave = 0;
    for (auto& fs : h->frames)
        if (fs->direct) fs->wave = 1;            // the direct gather runs in the wave schedule
    LIDAR_TRY(upload_frame_table(h));
    h->b_autotuned = false;
    h->b_autotune_ms = 0.0;
    if (h->prm.flags & LIDAR_AUTOTUNE) {
        std::vector<size_t> order(total_groups);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
        std::vector<int2> by_cost(total_groups);
        std::vector<uint64_t> c_by_cost(total_groups);
        for (size_t j = 0; j < total_groups; ++j) {
            by_cost[j] = items[order[j]];
            c_by_cost[j] = cost[order[j]];
        }
        LIDAR_TRY(autotune_batch(h, by_cost, c_by_cost));
    }
    // queue order: the group schedule's items, then the wave schedule's, each
    // costliest first; tickets never mix the two
    std::vector<size_t> order(total_groups);
    std::iota(order.begin(), order.end(), 0);
    auto wave_of = [&](size_t j) { return h->frames[items[j].x]->wave; };
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
        const int wx = wave_of(x), wy = wave_of(y);
        return wx != wy ? wx < wy : cost[x] > cost[y];
    });
    std::vector<int2> sorted(total_groups);
    std::vector<uint64_t> sorted_cost(total_groups);
    std::vector<char> sorted_wave(total_groups);
    for (size_t j = 0; j < total_groups; ++j) {
        sorted[j] = items[order[j]];
        sorted_cost[j] = cost[order[j]];
        sorted_wave[j] = (char)wave_of(order[j]);
    }
    HIP_TRY(h, h->b_items.ensure(sorted.size()), "allocate batch items");
    HIP_TRY(h, hipMemcpyAsync(h->b_items.p, sorted.data(), sorted.size() * sizeof(int2),
                              hipMemcpyHostToDevice, h->stream), "copy batch items");
    size_t n_group_items = 0;
    while (n_group_items < total_groups && !sorted_wave[n_group_items]) ++n_group_items;
    std::vector<int32_t> tickets(1, 0);
    const std::vector<int32_t> tg = build_tickets(sorted_cost.data(), n_group_items, h->b_grid, 0);
    const std::vector<int32_t> tw =
        build_tickets(sorted_cost.data() + n_group_items, total_groups - n_group_items,
                      (uint64_t)h->b_grid * kWavesPerGroup, (int32_t)n_group_items, wave_ticket_cost(h));
    tickets.insert(tickets.end(), tg.begin(), tg.end());
    tickets.insert(tickets.end(), tw.begin(), tw.end());
    h->b_tickets_n = (int)tickets.size() - 1;
    h->b_tickets_g = (int)tg.size();
    h->b_wave_items = total_groups - n_group_items;
    HIP_TRY(h, h->b_tickets.ensure(tickets.size()), "allocate batch tickets");
    HIP_TRY(h, hipMemcpyAsync(h->b_tickets.p, tickets.data(), tickets.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, h->stream), "copy batch tickets");
    HIP_TRY(h, hipStreamSynchronize(h->stream), "batch tables synchronise");
    // capture the batch into a graph on a private stream; it is launched on
    // the handle's stream
    if (!h->capture_stream)
        HIP_TRY(h, hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking),
                "create capture stream");
    HIP_TRY(h, hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal),
            "begin graph capture");
    lidar_status st = enqueue_batch(h, h->capture_stream, h->b_items.p, h->b_items_n, true,
                                    h->b_tickets.p, h->b_tickets_n, h->b_tickets_g);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(h->capture_stream, &graph);
    if (st != LIDAR_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    HIP_TRY(h, e, "end graph capture");
    h->graph = graph;
    HIP_TRY(h, hipGraphInstantiate(&h->graph_exec, graph, nullptr, nullptr, 0), "instantiate graph");
    h->batch_gb.assign(gbs, gbs + n);
    h->batch_pd.assign(pds, pds + n);
    h->batch_ok = true;
    return LIDAR_OK;
}


// ---- allocation-free frame ---------------------------------------------------

// Byte offsets of the static path's buffers in the scratch array (256-byte
// aligned), in the order they are taken.
struct ScratchPlan {
    size_t off = 0;
    template <typename T>
    size_t take(size_t count)
    {
        const size_t o = off;
        off = (off + count * sizeof(T) + 255) & ~(size_t)255;
        return o;
    }
};

// The plain path of one frame (set-up, pre-pass, fused footprint kernel) with
// every device buffer carved from the static scratch array; errors go to the
// thread's handle-less error text.
lidar_status simulate_static(const lidar_sim_params* prm, const lidar_pattern_desc* pd,
                             const lidar_gbuffer_desc* gb, hipStream_t s, lidar_echo* echoes,
                             int32_t* counts, lidar_beam_info* beams)
{
    lidar_sim* const h = nullptr;          // errors: g_create_error
    std::string why;
    if (check_params(prm, why) != LIDAR_OK) return fail(h, LIDAR_E_INVALID, why);
    if (prm->flags != 0)
        return fail(h, LIDAR_E_INVALID, "simulate_static takes no flags (no kept waveforms, "
                                        "profiling or autotuning)");
    LIDAR_TRY(check_pattern(h, pd, ""));
    LIDAR_TRY(check_gbuffer(h, gb, ""));
    if (!echoes || !counts || !beams)
        return fail(h, LIDAR_E_INVALID, "simulate_static needs the device outputs echoes, "
                                        "n_echoes and beams");
    if (prm->range_mode != LIDAR_RANGE_CENTRE || (pd->kind == LIDAR_PATTERN_TABLE && pd->rx_table))
        return fail(h, LIDAR_E_UNSUPPORTED, "simulate_static runs centre ranges without an rx_table");
    // host copy of the pattern (as copy_pattern, without device buffers)
    FrameState fs;
    PatternHost& pat = fs.pat;
    const size_t B = pd->n_beams;
    pat.kind = pd->kind;
    pat.az.assign(pd->beam_az_deg, pd->beam_az_deg + B);
    pat.el.assign(pd->beam_el_deg, pd->beam_el_deg + B);
    if (pd->kind == LIDAR_PATTERN_GAUSS) {
        pat.sigma[0] = pd->sigma_deg[0];
        pat.sigma[1] = pd->sigma_deg[1];
        pat.trunc = pd->trunc_sigmas;
    } else {
        pat.nx = pd->nx;
        pat.ny = pd->ny;
        pat.half[0] = pd->half_deg[0];
        pat.half[1] = pd->half_deg[1];
        pat.table.assign(pd->table, pd->table + (size_t)pd->nx * pd->ny);
    }
    fs.gb = *gb;
    const RasterDev r = raster_of(*gb);
    double Mf, Nf;
    kernel_extent(pat, r, &Mf, &Nf);
    if (!(Mf >= 0 && Nf >= 0) || Mf > 4096 || Nf > 4096 || (2 * Mf + 1) * (2 * Nf + 1) > 16.0e6)
        return fail(h, LIDAR_E_INVALID, "kernel grid too large for this raster (more than 16M "
                                        "cells or 8193 columns/rows)");
    if ((4.0 * Mf + 8.0) * (double)gb->height * 8.0 >= 2147483648.0)
        return fail(h, LIDAR_E_INVALID, "kernel window times image height too large "
                                        "(4*M+8)*height*8 must stay below 2^31 bytes");
    KernelDev k;
    k.M = (int)Mf;
    k.N = (int)Nf;
    k.KW = 2 * k.M + 1;
    k.KH = 2 * k.N + 1;
    fs.k = k;
    const double sigma = prm->pulse_fwhm_ns / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    const int J = pulse_half_width(prm);
    const std::vector<float> tab = prm->pulse_taps ? tabulated_taps(prm) : std::vector<float>();
    int G = 4;
    while (G > 1 && !footprint_group_fits(G, (int)prm->n_bins, J)) G /= 2;
    const bool sun = prm->sun_irradiance != 0.0;
    const size_t W = gb->width, H = gb->height, W4 = (W + 3) & ~(size_t)3;
    const size_t NB = (size_t)kernel_blocks(k.KW), KW = (size_t)k.KW, KH = (size_t)k.KH;
    // the beam groups (host scheduling from the beams' pixels; costs unused)
    build_groups(fs, r, G, std::vector<lidar_beam_info>(B));
    // scratch layout; checked against the array's size before any device call
    ScratchPlan plan;
    const size_t o_taps = plan.take<float>(2 * (size_t)J + 1);
    const size_t o_table = plan.take<float>(pat.table.size());
    const size_t o_az = plan.take<double>(B), o_el = plan.take<double>(B);
    const size_t o_K64 = plan.take<double>(KW * KH);
    const size_t o_Kb = plan.take<float>(4 * NB * (KH + 1) * 4);
    const size_t o_rowsum = plan.take<double>(KH), o_rowmax = plan.take<double>(KH);
    const size_t o_rowrange = plan.take<int2>(KH);
    const size_t o_prefix = plan.take<int32_t>(KH * (KW + 1));
    const size_t o_kinfo = plan.take<double>(2);
    const size_t o_omega = plan.take<double>(H + 2 * KH);
    const size_t o_colcs = plan.take<float2>(W), o_rowtab = plan.take<float4>(H);
    const size_t o_pix = plan.take<int2>(W4 * H);
    const size_t o_sun = plan.take<float>(sun ? W4 * H : 0);
    const size_t o_groups = plan.take<int32_t>(fs.groups.size());
    if (plan.off > kStaticScratchBytes)
        return fail(h, LIDAR_E_INVALID,
                    "simulate_static: this frame needs " + std::to_string(plan.off) +
                        " bytes of scratch, the static area holds " +
                        std::to_string(kStaticScratchBytes) + " (about 8 bytes per pixel, 12 with "
                        "the sun term, 16 per beam, and the kernel tables)");
    char* base = nullptr;
    HIP_TRY(h, static_scratch_addr((void**)&base), "static scratch address");
    float* taps = (float*)(base + o_taps);
    float* table = (float*)(base + o_table);
    double* az = (double*)(base + o_az);
    double* el = (double*)(base + o_el);
    double* K64 = (double*)(base + o_K64);
    float* Kb = (float*)(base + o_Kb);
    double* rowsum = (double*)(base + o_rowsum);
    double* rowmax = (double*)(base + o_rowmax);
    int2* rowrange = (int2*)(base + o_rowrange);
    int32_t* prefix = (int32_t*)(base + o_prefix);
    double* kinfo_d = (double*)(base + o_kinfo);
    double* omega = (double*)(base + o_omega);
    float2* colcs = (float2*)(base + o_colcs);
    float4* rowtab = (float4*)(base + o_rowtab);
    int2* pix = (int2*)(base + o_pix);
    float* sunb = sun ? (float*)(base + o_sun) : nullptr;
    int32_t* groups = (int32_t*)(base + o_groups);
    // host inputs into the scratch (the host copies stay alive until the
    // synchronisation below)
    HIP_TRY(h, hipMemcpyAsync(az, pat.az.data(), B * sizeof(double), hipMemcpyHostToDevice, s), "copy beams");
    HIP_TRY(h, hipMemcpyAsync(el, pat.el.data(), B * sizeof(double), hipMemcpyHostToDevice, s), "copy beams");
    if (!pat.table.empty())
        HIP_TRY(h, hipMemcpyAsync(table, pat.table.data(), pat.table.size() * sizeof(float),
                                  hipMemcpyHostToDevice, s), "copy table");
    HIP_TRY(h, hipMemcpyAsync(groups, fs.groups.data(), fs.groups.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, s), "copy beam groups");
    if (!tab.empty())
        HIP_TRY(h, hipMemcpyAsync(taps, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice, s),
                "copy pulse taps");
    else
        HIP_TRY(h, launch_pulse_taps(s, (float)sigma, (float)prm->bin_ns, J, taps), "pulse taps launch");
    PatternDev pdev;
    pdev.kind = (int)pat.kind;
    pdev.sx = pat.sigma[0];
    pdev.sy = pat.sigma[1];
    pdev.trunc = pat.trunc;
    pdev.table = pat.table.empty() ? nullptr : table;
    pdev.nx = (int)pat.nx;
    pdev.ny = (int)pat.ny;
    pdev.hx = pat.half[0];
    pdev.hy = pat.half[1];
    HIP_TRY(h, launch_kernel_grid(s, pdev, r, k, K64), "kernel grid launch");
    HIP_TRY(h, launch_kernel_blocks(s, k, K64, Kb), "kernel blocks launch");
    HIP_TRY(h, launch_kernel_rows(s, k, K64, rowsum, rowmax, rowrange, prefix), "kernel rows launch");
    HIP_TRY(h, launch_kernel_peak(s, k, rowsum, rowmax, kinfo_d), "kernel peak launch");
    HIP_TRY(h, launch_raster_tables(s, r, colcs, rowtab), "raster tables launch");
    HIP_TRY(h, launch_beam_setup(s, r, k, az, el, (int)B, rowsum, prefix, omega, prm->emit_power, beams),
            "beam setup launch");
    double kinfo[2];
    HIP_TRY(h, hipMemcpyAsync(kinfo, kinfo_d, sizeof(kinfo), hipMemcpyDeviceToHost, s), "copy kernel info");
    HIP_TRY(h, hipStreamSynchronize(s), "set-up synchronise");
    if (!(kinfo[1] > 0.0) || !is_fin(kinfo[1]) || !(kinfo[0] > 0.0))
        return fail(h, LIDAR_E_INVALID, "pattern integral over the kernel grid is not positive "
                                        "(kernel narrower than one pixel or all-zero table)");
    // the frame: pre-pass, then the fused footprint kernel (asynchronous);
    // value-initialised, so the pointers it does not set (statistics,
    // range tables) are null
    PrepassArgs pa{};
    pa.depth = gb->depth;
    pa.refl = gb->reflectance;
    pa.gain = gb->retro_gain;
    pa.nx = gb->normal_x;
    pa.ny = gb->normal_y;
    pa.nz = gb->normal_z;
    pa.pitch = (long)gb->pitch;
    pa.W = (int)W;
    pa.H = (int)H;
    pa.W4 = (int)W4;
    pa.colcs = colcs;
    pa.rowtab = rowtab;
    pa.to_bin = 2.0 / (kLight * (prm->bin_ns * 1e-9));
    pa.R = (int)prm->n_bins;
    pa.sun_x = (float)prm->sun_dir[0];
    pa.sun_y = (float)prm->sun_dir[1];
    pa.sun_z = (float)prm->sun_dir[2];
    pa.pix = pix;
    pa.sun = sunb;
    pa.range_mode = LIDAR_RANGE_CENTRE;
    pa.rt = RangeTables{};
    pa.rec4 = nullptr;
    pa.stats = nullptr;
    HIP_TRY(h, launch_prepass(s, pa, sun), "pre-pass launch");
    FootprintArgs fa;
    FrameDev& f = fa.f;
    f = FrameDev{};
    f.pix = pix;
    f.sun = sunb;
    f.W = (int)W;
    f.H = (int)H;
    f.Kb = Kb;
    f.rowrange = rowrange;
    f.M = k.M;
    f.N = k.N;
    f.KW = k.KW;
    f.KH = k.KH;
    f.NB = (int)NB;
    f.tile = default_tile(k.KH);
    f.sun_scale = sun ? (float)(prm->sun_irradiance / kinfo[0]) : 0.0f;
    f.beams = beams;
    f.echoes = echoes;
    f.counts = counts;
    f.waves = nullptr;
    PathDev& pp = fa.p;
    pp.taps = taps;
    pp.J = J;
    pp.R = (int)prm->n_bins;
    pp.E = (int)prm->max_echoes;
    pp.select = (int)prm->echo_select;
    pp.threshold = (float)prm->threshold;
    pp.ambient = (float)prm->ambient_const;
    pp.half_c_dt = 0.5 * kLight * (prm->bin_ns * 1e-9);
    pp.bin_ns = prm->bin_ns;
    fa.groups = groups;
    fa.n_groups = fs.n_groups;
    fa.G = G;
    fa.chunk = (fs.n_groups + kXcds - 1) / kXcds;
    HIP_TRY(h, launch_footprint(s, fa), "footprint launch");
    return LIDAR_OK;
}

}  // namespace

extern "C" {

lidar_status lidar_sim_create(const lidar_sim_params* params, void* hip_stream, lidar_sim** out)
{
    g_create_error.clear();
    if (!out) {
        g_create_error = "out is NULL";
        return LIDAR_E_INVALID;
    }
    *out = nullptr;
    std::string why;
    lidar_status st = check_params(params, why);
    if (st != LIDAR_OK) {
        g_create_error = why;
        return st;
    }
    lidar_sim* h = new (std::nothrow) lidar_sim();
    if (!h) {
        g_create_error = "out of host memory";
        return LIDAR_E_NOMEM;
    }
    h->prm = *params;
    h->stream = (hipStream_t)hip_stream;
    {
        int dev = 0, n = 0, l = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            h->cus = n;
        if (hipDeviceGetAttribute(&l, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            l >= 65536)
            h->lds_max = (size_t)l;
    }
    // the handle keeps no pointer into the caller's table
    h->prm.pulse_taps = nullptr;
    double sigma = params->pulse_fwhm_ns / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    h->J = pulse_half_width(params);
    const bool det = (params->flags & LIDAR_DETERMINISTIC) != 0;
    // groups of one beam for corrected ranges (per-beam bins) and for the
    // deterministic mode (a histogram slot per wave); otherwise the largest
    // group whose workgroup leaves room for two per CU in the LDS
    h->G = params->range_mode == LIDAR_RANGE_CORRECTED || det ? 1 : 4;
    while (h->G > 1 && !footprint_group_fits(h->G, (int)params->n_bins, h->J, h->lds_max / 2)) h->G /= 2;
    if (det && !footprint_group_fits(kWavesPerGroup, (int)params->n_bins, h->J, h->lds_max)) {
        g_create_error = "LIDAR_DETERMINISTIC: four histograms of n_bins do not fit the LDS";
        lidar_sim_destroy(h);
        return LIDAR_E_UNSUPPORTED;
    }
    h->net.det = det;
    hipError_t e = h->d_taps.ensure(2 * h->J + 1);
    if (e == hipSuccess) {
        if (params->pulse_taps) {
            const std::vector<float> t = tabulated_taps(params);
            e = hipMemcpyAsync(h->d_taps.p, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice,
                               h->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        } else {
            e = launch_pulse_taps(h->stream, (float)sigma, (float)params->bin_ns, h->J, h->d_taps.p);
        }
    }
    if (e != hipSuccess) {
        g_create_error = std::string("pulse taps: ") + hipGetErrorString(e);
        lidar_sim_destroy(h);
        return e == hipErrorOutOfMemory ? LIDAR_E_NOMEM : LIDAR_E_HIP;
    }
    h->st.n_taps = (uint32_t)(2 * h->J + 1);
    *out = h;
    return LIDAR_OK;
}

lidar_status lidar_sim_destroy(lidar_sim* h)
{
    if (!h) return LIDAR_OK;
    (void)hipStreamSynchronize(h->stream);
    for (auto* v : {&h->pending_fp, &h->pending_pp, &h->pending_bt, &h->pending_sur, &h->pool})
        for (auto& p : *v) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
    free_graph(h);
    if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
    delete h;   // the device buffers free themselves
    return LIDAR_OK;
}

lidar_status lidar_sim_set_pattern(lidar_sim* h, const lidar_pattern_desc* pd)
{
    if (!h) return LIDAR_E_INVALID;
    LIDAR_TRY(check_pattern(h, pd, ""));
    LIDAR_TRY(copy_pattern(h, h->single, pd));
    ++h->pattern_gen;
    h->have_pattern = true;
    h->setup_ok = false;
    h->have_result = false;
    return LIDAR_OK;
}

lidar_status lidar_sim_set_gbuffer(lidar_sim* h, const lidar_gbuffer_desc* g)
{
    if (!h) return LIDAR_E_INVALID;
    LIDAR_TRY(check_gbuffer(h, g, ""));
    if (h->setup_ok && !same_raster(h->single.gb, *g)) h->setup_ok = false;
    h->single.gb = *g;
    h->have_gbuffer = true;
    h->gb_owned = false;
    return LIDAR_OK;
}

lidar_status lidar_sim_set_gbuffer_pinhole(lidar_sim* h, const lidar_pinhole_desc* src,
                                           uint32_t width, uint32_t height, double az_min_deg,
                                           double az_max_deg, double el_min_deg, double el_max_deg)
{
    if (!h) return LIDAR_E_INVALID;
    if (!src) return fail(h, LIDAR_E_INVALID, "pinhole descriptor is NULL");
    if (src->width == 0 || src->height == 0 || src->pitch < src->width ||
        src->width > (1u << 20) || src->height > (1u << 20) || src->pitch > (1ull << 30))
        return fail(h, LIDAR_E_INVALID, "pinhole image needs width, height >= 1 and pitch >= width");
    if (!src->depth || !src->reflectance || !src->retro_gain || !src->normal_x || !src->normal_y ||
        !src->normal_z)
        return fail(h, LIDAR_E_INVALID, "pinhole plane pointer is NULL");
    if (!(src->fx > 0) || !(src->fy > 0) || !is_fin(src->fx) || !is_fin(src->fy) || !is_fin(src->cx) ||
        !is_fin(src->cy))
        return fail(h, LIDAR_E_INVALID, "pinhole intrinsics need finite fx, fy > 0, cx, cy");
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double dot = 0.0;
            for (int k = 0; k < 3; ++k) dot += src->rot[3 * k + r] * src->rot[3 * k + c];
            if (!(std::fabs(dot - (r == c ? 1.0 : 0.0)) < 1e-6))
                return fail(h, LIDAR_E_INVALID, "pinhole rotation must be orthonormal");
        }
    if (src->depth_format > (uint32_t)LIDAR_DEPTH_WINDOW_U24 || src->normal_correct > 1)
        return fail(h, LIDAR_E_INVALID, "unknown pinhole depth format or correction flag");
    if (src->depth_format >= (uint32_t)LIDAR_DEPTH_WINDOW_F32 &&
        !(src->z_near > 0 && src->z_far > src->z_near && is_fin(src->z_far)))
        return fail(h, LIDAR_E_INVALID, "window depth needs clip planes 0 < near < far");
    lidar_gbuffer_desc g{};
    g.width = width;
    g.height = height;
    g.pitch = width;
    g.az_min_deg = az_min_deg;
    g.az_max_deg = az_max_deg;
    g.el_min_deg = el_min_deg;
    g.el_max_deg = el_max_deg;
    // placeholders for the plane check; the real pointers follow the allocation
    const float* ph = (const float*)src->reflectance;
    g.depth = g.reflectance = g.retro_gain = g.normal_x = g.normal_y = g.normal_z = ph;
    LIDAR_TRY(check_gbuffer(h, &g, "output raster: "));
    HIP_TRY(h, h->rp_planes.ensure((size_t)6 * width * height), "allocate reprojected planes");
    float* out = h->rp_planes.p;
    const size_t plane = (size_t)width * height;
    g.depth = out;
    g.reflectance = out + plane;
    g.retro_gain = out + 2 * plane;
    g.normal_x = out + 3 * plane;
    g.normal_y = out + 4 * plane;
    g.normal_z = out + 5 * plane;
    const RasterDev r = raster_of(g);
    ReprojectArgs a;
    a.W = (int)width;
    a.H = (int)height;
    a.az_min = r.az_min;
    a.el_max = r.el_max;
    a.dphi = r.dphi;
    a.de = r.de;
    a.SW = (int)src->width;
    a.SH = (int)src->height;
    a.spitch = (long)src->pitch;
    a.fx = src->fx;
    a.fy = src->fy;
    a.cx = src->cx;
    a.cy = src->cy;
    for (int i = 0; i < 9; ++i) a.rot[i] = src->rot[i];
    a.fmt = (int)src->depth_format;
    a.correct = (int)src->normal_correct;
    a.z_near = src->z_near;
    a.z_far = src->z_far;
    a.depth = src->depth;
    a.refl = src->reflectance;
    a.gain = src->retro_gain;
    a.nx = src->normal_x;
    a.ny = src->normal_y;
    a.nz = src->normal_z;
    a.out = out;
    HIP_TRY(h, launch_reproject(h->stream, a), "reprojection launch");
    if (h->setup_ok && !same_raster(h->single.gb, g)) h->setup_ok = false;
    h->single.gb = g;
    h->have_gbuffer = true;
    h->gb_owned = true;
    return LIDAR_OK;
}

lidar_status lidar_sim_range_stacking(lidar_sim* h, const float* row_kernel, uint32_t M,
                                      const float* col_kernel, uint32_t N, double rho_min,
                                      int32_t* s_nearest, float* xi_nearest)
{
    if (!h) return LIDAR_E_INVALID;
    if (!h->have_gbuffer) return fail(h, LIDAR_E_STATE, "range_stacking before set_gbuffer");
    if (!row_kernel || !col_kernel || !s_nearest || !xi_nearest)
        return fail(h, LIDAR_E_INVALID, "range_stacking needs both kernel factors and both outputs");
    if (M > (uint32_t)kRsMaxHalf || N > (uint32_t)kRsMaxHalf)
        return fail(h, LIDAR_E_INVALID, "range_stacking kernel half extents must be <= 127");
    if (!(rho_min > 0.0) || !is_fin(rho_min)) return fail(h, LIDAR_E_INVALID, "rho_min must be > 0");
    if (h->prm.range_mode != LIDAR_RANGE_CENTRE)
        return fail(h, LIDAR_E_UNSUPPORTED, "range_stacking slices the pixels' centre ranges");
    const size_t KW = 2 * (size_t)M + 1, KH = 2 * (size_t)N + 1;
    double sh = 0.0, sv = 0.0;
    std::vector<float> k(KW + KH);
    for (size_t i = 0; i < KW; ++i) {
        if (!std::isfinite(row_kernel[i]) || row_kernel[i] < 0.0f)
            return fail(h, LIDAR_E_INVALID, "kernel factors must be finite and >= 0");
        k[i] = row_kernel[i];
        sh += row_kernel[i];
    }
    for (size_t i = 0; i < KH; ++i) {
        if (!std::isfinite(col_kernel[i]) || col_kernel[i] < 0.0f)
            return fail(h, LIDAR_E_INVALID, "kernel factors must be finite and >= 0");
        k[KW + i] = col_kernel[i];
        sv += col_kernel[i];
    }
    hipStream_t s = h->stream;
    FrameState& fs = h->single;
    const lidar_gbuffer_desc& g = fs.gb;
    if (M != h->rs_M || N != h->rs_N || k != h->rs_host) {
        // new factors: copied once (the stream is synchronised so that the
        // host copy may change afterwards)
        HIP_TRY(h, h->rs_k.ensure(k.size()), "allocate kernel factors");
        h->rs_host = k;
        h->rs_M = M;
        h->rs_N = N;
        HIP_TRY(h, hipMemcpyAsync(h->rs_k.p, h->rs_host.data(), k.size() * sizeof(float),
                                  hipMemcpyHostToDevice, s), "copy kernel factors");
        HIP_TRY(h, hipStreamSynchronize(s), "kernel factors synchronise");
    }
    // pixel records of the current G-buffer (raster tables, pre-pass)
    HIP_TRY(h, fs.d_colcs.ensure(g.width), "allocate raster tables");
    HIP_TRY(h, fs.d_rowtab.ensure(g.height), "allocate raster tables");
    HIP_TRY(h, launch_raster_tables(s, raster_of(g), fs.d_colcs.p, fs.d_rowtab.p), "raster tables launch");
    LIDAR_TRY(alloc_pixels(h, fs));
    LIDAR_TRY(enqueue_prepass(h, fs, s));
    HIP_TRY(h, h->rs_smax.ensure(h->prm.n_bins), "allocate slice maxima");
    RangeStackArgs a;
    a.pix = fs.d_pix.p;
    a.W = (int)g.width;
    a.H = (int)g.height;
    a.W4 = (int)((g.width + 3) & ~3u);
    a.R = (int)h->prm.n_bins;
    a.hk = h->rs_k.p;
    a.vk = h->rs_k.p + KW;
    a.M = (int)M;
    a.N = (int)N;
    a.rho_min = (float)rho_min;
    a.bound = (float)(sh * sv);
    a.smax = nullptr;
    a.s_nearest = s_nearest;
    a.xi_nearest = xi_nearest;
    HIP_TRY(h, launch_range_stacking(s, a, h->rs_smax.p), "range stacking launch");
    return LIDAR_OK;
}

lidar_status lidar_sim_read_gbuffer(lidar_sim* h, float* planes, int dst_is_device)
{
    if (!h) return LIDAR_E_INVALID;
    if (!planes) return fail(h, LIDAR_E_INVALID, "planes is NULL");
    if (!h->gb_owned) return fail(h, LIDAR_E_STATE, "the current G-buffer is not a reprojected one");
    const size_t n = (size_t)6 * h->single.gb.width * h->single.gb.height;
    HIP_TRY(h, hipMemcpyAsync(planes, h->rp_planes.p, n * sizeof(float),
                              dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream),
            "copy G-buffer");
    if (!dst_is_device) HIP_TRY(h, hipStreamSynchronize(h->stream), "read synchronise");
    return LIDAR_OK;
}

static lidar_status ensure_setup(lidar_sim* h, const char* who)
{
    if (!h->have_pattern) return fail(h, LIDAR_E_STATE, std::string(who) + " before set_pattern");
    if (!h->have_gbuffer) return fail(h, LIDAR_E_STATE, std::string(who) + " before set_gbuffer");
    FrameState& fs = h->single;
    const size_t B = fs.pat.az.size();
    if (!h->setup_ok) {
        HIP_TRY(h, h->d_beams.ensure(B), "allocate beams");
        LIDAR_TRY(setup_frame(h, fs, h->d_beams.p, ""));
        HIP_TRY(h, h->d_groups.ensure(fs.groups.size()), "allocate beam groups");
        HIP_TRY(h, hipMemcpyAsync(h->d_groups.p, fs.groups.data(), fs.groups.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, h->stream), "copy beam groups");
        HIP_TRY(h, hipStreamSynchronize(h->stream), "set-up synchronise");
        auto it = h->tuned.find(height_class(fs.k.KH));
        if (it != h->tuned.end()) fs.tile = it->second.first;
        h->setup_ok = true;
    }
    LIDAR_TRY(alloc_pixels(h, fs));
    return LIDAR_OK;
}

static lidar_status simulate_surrogate(lidar_sim* h);

lidar_status lidar_sim_simulate_frame(lidar_sim* h, uint32_t mode)
{
    if (!h) return LIDAR_E_INVALID;
    if (mode != LIDAR_MODE_PLAIN && mode != LIDAR_MODE_SURROGATE)
        return fail(h, LIDAR_E_UNSUPPORTED, "unknown simulate_frame mode");
    LIDAR_TRY(ensure_setup(h, "simulate_frame"));
    if (mode == LIDAR_MODE_SURROGATE) return simulate_surrogate(h);
    FrameState& fs = h->single;
    const size_t B = fs.pat.az.size();
    const uint32_t R = h->prm.n_bins, E = h->prm.max_echoes;
    const bool keep = (h->prm.flags & LIDAR_KEEP_WAVEFORMS) != 0;
    const bool prof = (h->prm.flags & LIDAR_PROFILE) != 0;
    HIP_TRY(h, h->d_echoes.ensure(B * E), "allocate echoes");
    HIP_TRY(h, h->d_counts.ensure(B), "allocate counts");
    if (keep) HIP_TRY(h, h->d_waves.ensure(B * (size_t)R), "allocate waveforms");

    hipStream_t s = h->stream;
    FootprintArgs fa;
    fa.f = frame_view(h, fs, h->d_beams.p, h->d_echoes.p, h->d_counts.p, keep ? h->d_waves.p : nullptr);
    fa.p = path_view(h);
    fa.groups = h->d_groups.p;
    fa.n_groups = fs.n_groups;
    fa.G = h->G;
    fa.chunk = (fs.n_groups + kXcds - 1) / kXcds;

    EventPair pp{}, fp{};
    if (prof) {
        hipError_t e;
        pp = take_pair(h, &e);
        HIP_TRY(h, e, "create events");
        fp = take_pair(h, &e);
        HIP_TRY(h, e, "create events");
        HIP_TRY(h, hipEventRecord(pp.a, s), "record event");
    }
    LIDAR_TRY(enqueue_prepass(h, fs, s));
    LIDAR_TRY(enqueue_sun_floor(h, fs, h->d_beams.p, s));
    if (prof) {
        HIP_TRY(h, hipEventRecord(pp.b, s), "record event");
        HIP_TRY(h, hipEventRecord(fp.a, s), "record event");
    }
    const bool corr = h->prm.range_mode == LIDAR_RANGE_CORRECTED;
    const bool det = (h->prm.flags & LIDAR_DETERMINISTIC) != 0;
    if (corr || det)
        HIP_TRY(h, launch_footprint_one(s, fa, corr, det), "footprint launch");
    else
        HIP_TRY(h, launch_footprint(s, fa), "footprint launch");
    if (prof) {
        HIP_TRY(h, hipEventRecord(fp.b, s), "record event");
        h->pending_pp.push_back(pp);
        h->pending_fp.push_back(fp);
    }
    h->have_result = true;
    h->plain_result = true;
    ++h->st.frames;
    return LIDAR_OK;
}

// The network on every beam, the gate, and the plain path on the groups of
// the beams that fall back - all enqueued, no host round trip.
// The surrogate's inputs and decoding assume the default path: every run
// reported, centre ranges, kappa = K / max K.
static lidar_status surrogate_supported(lidar_sim* h, const char* who)
{
    if (h->prm.echo_select != LIDAR_ECHO_ALL || h->prm.range_mode != LIDAR_RANGE_CENTRE ||
        !h->single.pat.rx.empty())
        return fail(h, LIDAR_E_UNSUPPORTED, std::string(who) + " needs echo_select ALL, range_mode "
                                            "CENTRE and no rx_table");
    return LIDAR_OK;
}

static lidar_status simulate_surrogate(lidar_sim* h)
{
    if (!h->net.ready) return fail(h, LIDAR_E_STATE, "surrogate mode without surrogate weights");
    LIDAR_TRY(surrogate_supported(h, "surrogate mode"));
    if (h->prm.flags & LIDAR_DETERMINISTIC)
        return fail(h, LIDAR_E_UNSUPPORTED, "LIDAR_DETERMINISTIC covers simulate_frame (plain) only");
    FrameState& fs = h->single;
    const int B = (int)fs.pat.az.size();
    const uint32_t R = h->prm.n_bins, E = h->prm.max_echoes;
    const bool keep = (h->prm.flags & LIDAR_KEEP_WAVEFORMS) != 0;
    const bool prof = (h->prm.flags & LIDAR_PROFILE) != 0;
    hipStream_t s = h->stream;
    LIDAR_TRY(sur_geometry(h, fs));
    HIP_TRY(h, h->d_echoes.ensure((size_t)B * E), "allocate echoes");
    HIP_TRY(h, h->d_counts.ensure(B), "allocate counts");
    if (keep) HIP_TRY(h, h->d_waves.ensure((size_t)B * R), "allocate waveforms");
    HIP_TRY(h, h->s_X.ensure((size_t)B * kSurIn), "allocate surrogate inputs");
    HIP_TRY(h, h->work.ensure(B), "allocate surrogate workspace");
    HIP_TRY(h, h->s_groups_fb.ensure((size_t)fs.n_groups * h->G), "allocate fallback groups");
    HIP_TRY(h, h->s_items.ensure(fs.n_groups), "allocate fallback items");
    if (!h->s_cnt.p) {
        HIP_TRY(h, h->s_cnt.ensure(4), "allocate counters");
        HIP_TRY(h, launch_reset_queue(s, h->s_cnt.p, 4), "counter reset");
    }
    HIP_TRY(h, h->s_frame.ensure(1), "allocate frame table");
    EventPair ev{};
    if (prof) {
        hipError_t e;
        ev = take_pair(h, &e);
        HIP_TRY(h, e, "create events");
        HIP_TRY(h, hipEventRecord(ev.a, s), "record event");
    }
    LIDAR_TRY(sur_inputs(h, fs, h->s_X.p));
    HIP_TRY(h, sur_infer(s, h->net, h->s_X.p, B, h->work.Y.p), "surrogate forward");
    HIP_TRY(h, launch_reset_queue(s, h->s_cnt.p, 2), "counter reset");
    DecodeArgs da;
    da.Y = h->work.Y.p;
    da.aux = h->s_aux.p;
    da.B = B;
    da.R = (int)R;
    da.E = (int)E;
    da.threshold = (float)h->prm.threshold;
    da.conf_logit = h->gate_conf_logit;
    da.alpha = h->gate_alpha;
    da.half_c_dt = 0.5 * kLight * (h->prm.bin_ns * 1e-9);
    da.bin_ns = h->prm.bin_ns;
    da.beams = h->d_beams.p;
    da.echoes = h->d_echoes.p;
    da.counts = h->d_counts.p;
    HIP_TRY(h, launch_decode(s, da), "gate launch");
    CompactArgs cp;
    cp.groups = h->d_groups.p;
    cp.n_groups = fs.n_groups;
    cp.G = h->G;
    cp.aux = h->s_aux.p;
    cp.groups_fb = h->s_groups_fb.p;
    cp.items = h->s_items.p;
    cp.n_items = h->s_cnt.p;
    cp.n_fallback = h->s_cnt.p + 2;
    HIP_TRY(h, launch_compact(s, cp), "fallback selection launch");
    // the plain path over the selected groups (count read on the device)
    const FrameDev fd = frame_view(h, fs, h->d_beams.p, h->d_echoes.p, h->d_counts.p,
                                   keep ? h->d_waves.p : nullptr);
    if (std::memcmp(&fd, &h->s_frame_host, sizeof(FrameDev)) != 0) {
        h->s_frame_host = fd;
        HIP_TRY(h, hipMemcpyAsync(h->s_frame.p, &h->s_frame_host, sizeof(FrameDev),
                                  hipMemcpyHostToDevice, s), "copy frame table");
        HIP_TRY(h, hipStreamSynchronize(s), "frame table synchronise");
    }
    BatchArgs ba{};
    ba.frames = h->s_frame.p;
    ba.p = path_view(h);
    ba.groups = h->s_groups_fb.p;
    ba.items = h->s_items.p;
    ba.n_items = fs.n_groups;
    ba.G = h->G;
    ba.next_item = h->s_cnt.p + 1;
    ba.n_items_dev = h->s_cnt.p;
    ba.tickets = nullptr;
    ba.n_tickets = 0;
    const size_t lds = group_lds_bytes(h->G, (int)R, h->J) + 2048;   // + static LDS
    const size_t per_cu = std::max<size_t>(1, std::min<size_t>(8, (160 * 1024) / lds));
    const int grid = (int)std::max<size_t>(1, std::min<size_t>((size_t)h->cus * per_cu, (size_t)fs.n_groups));
    HIP_TRY(h, launch_footprint_batch(s, ba, grid, h->prm.sun_irradiance != 0.0, keep),
            "fallback footprint launch");
    // no waveform is computed for the beams the network answered
    if (keep) HIP_TRY(h, launch_fill_accepted(s, h->s_aux.p, B, (int)R, h->d_waves.p), "waveform fill launch");
    if (prof) {
        HIP_TRY(h, hipEventRecord(ev.b, s), "record event");
        h->pending_sur.push_back(ev);
    }
    h->have_result = true;
    h->plain_result = false;
    ++h->st.frames;
    ++h->st.surrogate_frames;
    h->st.surrogate_beams += (uint64_t)B;
    return LIDAR_OK;
}

lidar_status lidar_sim_read_echoes(lidar_sim* h, lidar_echo* echoes, int32_t* n_echoes,
                                   float* waveforms, lidar_beam_info* beams, int dst_is_device)
{
    if (!h) return LIDAR_E_INVALID;
    if (!h->have_result) return fail(h, LIDAR_E_STATE, "read_echoes before simulate_frame");
    if (waveforms && !(h->prm.flags & LIDAR_KEEP_WAVEFORMS))
        return fail(h, LIDAR_E_INVALID, "waveforms requested without LIDAR_KEEP_WAVEFORMS");
    const size_t B = h->single.pat.az.size();
    const hipMemcpyKind kind = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    hipStream_t s = h->stream;
    if (echoes)
        HIP_TRY(h, hipMemcpyAsync(echoes, h->d_echoes.p, B * h->prm.max_echoes * sizeof(lidar_echo),
                                  kind, s), "copy echoes");
    if (n_echoes)
        HIP_TRY(h, hipMemcpyAsync(n_echoes, h->d_counts.p, B * sizeof(int32_t), kind, s), "copy counts");
    if (waveforms)
        HIP_TRY(h, hipMemcpyAsync(waveforms, h->d_waves.p, B * (size_t)h->prm.n_bins * sizeof(float),
                                  kind, s), "copy waveforms");
    if (beams)
        HIP_TRY(h, hipMemcpyAsync(beams, h->d_beams.p, B * sizeof(lidar_beam_info), kind, s),
                "copy beam info");
    if (!dst_is_device) HIP_TRY(h, hipStreamSynchronize(s), "read synchronise");
    return LIDAR_OK;
}

lidar_status lidar_sim_simulate_batch(lidar_sim* h, const lidar_gbuffer_desc* frames,
                                      const lidar_pattern_desc* patterns, uint32_t n_frames)
{
    if (!h) return LIDAR_E_INVALID;
    if (!frames || !patterns || n_frames == 0)
        return fail(h, LIDAR_E_INVALID, "simulate_batch needs n_frames >= 1 and both arrays");
    if (n_frames > 65536) return fail(h, LIDAR_E_INVALID, "too many frames (max 65536)");
    if (h->prm.range_mode == LIDAR_RANGE_CORRECTED)
        return fail(h, LIDAR_E_UNSUPPORTED, "range_mode CORRECTED runs in simulate_frame only");
    if (h->prm.flags & LIDAR_DETERMINISTIC)
        return fail(h, LIDAR_E_UNSUPPORTED, "LIDAR_DETERMINISTIC covers simulate_frame (plain) only");
    bool same = h->batch_ok && h->batch_gb.size() == n_frames;
    for (uint32_t i = 0; same && i < n_frames; ++i)
        same = same_gbuffer(h->batch_gb[i], frames[i]) && same_pattern(h->batch_pd[i], patterns[i]);
    if (!same) LIDAR_TRY(setup_batch(h, frames, patterns, n_frames));
    const bool prof = (h->prm.flags & LIDAR_PROFILE) != 0;
    EventPair bt{};
    if (prof) {
        hipError_t e;
        bt = take_pair(h, &e);
        HIP_TRY(h, e, "create events");
        HIP_TRY(h, hipEventRecord(bt.a, h->stream), "record event");
    }
    HIP_TRY(h, hipGraphLaunch(h->graph_exec, h->stream), "graph launch");
    if (prof) {
        HIP_TRY(h, hipEventRecord(bt.b, h->stream), "record event");
        h->pending_bt.push_back(bt);
    }
    h->batch_result = true;
    h->st.frames += n_frames;
    return LIDAR_OK;
}

lidar_status lidar_sim_read_batch(lidar_sim* h, uint32_t frame, lidar_echo* echoes,
                                  int32_t* n_echoes, float* waveforms, lidar_beam_info* beams,
                                  int dst_is_device)
{
    if (!h) return LIDAR_E_INVALID;
    if (!h->batch_result) return fail(h, LIDAR_E_STATE, "read_batch before simulate_batch");
    if (frame >= h->frames.size()) return fail(h, LIDAR_E_INVALID, "frame index out of range");
    if (waveforms && !(h->prm.flags & LIDAR_KEEP_WAVEFORMS))
        return fail(h, LIDAR_E_INVALID, "waveforms requested without LIDAR_KEEP_WAVEFORMS");
    const uint64_t o = h->beam_off[frame], B = h->beam_off[frame + 1] - o;
    const size_t E = h->prm.max_echoes, R = h->prm.n_bins;
    const hipMemcpyKind kind = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    hipStream_t s = h->stream;
    if (echoes)
        HIP_TRY(h, hipMemcpyAsync(echoes, h->b_echoes.p + o * E, B * E * sizeof(lidar_echo), kind, s),
                "copy echoes");
    if (n_echoes)
        HIP_TRY(h, hipMemcpyAsync(n_echoes, h->b_counts.p + o, B * sizeof(int32_t), kind, s), "copy counts");
    if (waveforms)
        HIP_TRY(h, hipMemcpyAsync(waveforms, h->b_waves.p + o * R, B * R * sizeof(float), kind, s),
                "copy waveforms");
    if (beams)
        HIP_TRY(h, hipMemcpyAsync(beams, h->b_beams.p + o, B * sizeof(lidar_beam_info), kind, s),
                "copy beam info");
    if (!dst_is_device) HIP_TRY(h, hipStreamSynchronize(s), "read synchronise");
    return LIDAR_OK;
}

lidar_status lidar_sim_batch_info(lidar_sim* h, lidar_batch_info* out)
{
    if (!h) return LIDAR_E_INVALID;
    if (!out) return fail(h, LIDAR_E_INVALID, "out is NULL");
    if (!h->batch_ok) return fail(h, LIDAR_E_STATE, "no batch has been set up");
    lidar_batch_info bi{};
    bi.n_frames = (uint32_t)h->frames.size();
    bi.group_size = (uint32_t)h->G;
    bi.n_beams = h->beam_off.back();
    bi.n_items = h->b_items_n;
    bi.samples = h->b_samples;
    bi.grid = (uint32_t)h->b_grid;
    bi.graph = h->graph_exec ? 1u : 0u;
    bi.autotuned = h->b_autotuned ? 1u : 0u;
    bi.wave_items = (uint32_t)h->b_wave_items;
    bi.autotune_ms = h->b_autotune_ms;
    for (const auto& fs : h->frames) bi.direct_frames += fs->direct ? 1u : 0u;
    if (h->b_fstats.p && fixed_point_ok(h)) {
        // the frames' statistics {shade, first bin, last bin, short runs},
        // then the counters {fixed-point beams, redone}
        const size_t n = h->frames.size();
        std::vector<int> c(4 * n + 2);
        HIP_TRY(h, hipMemcpyAsync(c.data(), h->b_fstats.p, c.size() * sizeof(int), hipMemcpyDeviceToHost,
                                  h->stream), "copy fixed-point counters");
        HIP_TRY(h, hipStreamSynchronize(h->stream), "batch info synchronise");
        bi.fixed_point_beams = (uint32_t)c[4 * n];
        bi.fixed_point_redone = (uint32_t)c[4 * n + 1];
        for (size_t i = 0; i < n; ++i)
            bi.short_run_frames += !h->frames[i]->direct && c[4 * i + 3] ? 1u : 0u;
    }
    *out = bi;
    return LIDAR_OK;
}

lidar_status lidar_sim_reset_batch(lidar_sim* h)
{
    if (!h) return LIDAR_E_INVALID;
    HIP_TRY(h, hipStreamSynchronize(h->stream), "reset synchronise");
    free_graph(h);
    h->batch_ok = false;
    h->batch_result = false;
    h->batch_gb.clear();
    h->batch_pd.clear();
    return LIDAR_OK;
}

lidar_status lidar_sim_surrogate_set_weights(lidar_sim* h, const float* params, uint64_t n_params)
{
    if (!h) return LIDAR_E_INVALID;
    if (!params || n_params != (uint64_t)kSurParams)
        return fail(h, LIDAR_E_INVALID, "surrogate weights need LIDAR_SUR_PARAMS values");
    for (uint64_t i = 0; i < n_params; ++i)
        if (!std::isfinite(params[i])) return fail(h, LIDAR_E_INVALID, "non-finite surrogate weight");
    SurNet& n = h->net;
    const size_t P = (size_t)kSurParams;
    HIP_TRY(h, n.theta.ensure(P), "allocate surrogate weights");
    HIP_TRY(h, n.m.ensure(P), "allocate surrogate weights");
    HIP_TRY(h, n.v.ensure(P), "allocate surrogate weights");
    HIP_TRY(h, n.grad.ensure(P), "allocate surrogate weights");
    HIP_TRY(h, n.theta_b.ensure(P), "allocate surrogate weights");
    hipStream_t s = h->stream;
    HIP_TRY(h, hipMemcpyAsync(n.theta.p, params, P * sizeof(float), hipMemcpyHostToDevice, s),
            "copy surrogate weights");
    HIP_TRY(h, launch_zero_f32(s, n.m.p, (long)P), "zero moments");
    HIP_TRY(h, launch_zero_f32(s, n.v.p, (long)P), "zero moments");
    HIP_TRY(h, launch_to_bf16(s, n.theta.p, n.theta_b.p, (long)P), "weight copy");
    HIP_TRY(h, hipStreamSynchronize(s), "weights synchronise");
    n.step = 0;
    n.t_stale = true;
    n.ready = true;
    return LIDAR_OK;
}

lidar_status lidar_sim_surrogate_get_weights(lidar_sim* h, float* params, uint64_t n_params)
{
    if (!h) return LIDAR_E_INVALID;
    if (!params || n_params != (uint64_t)kSurParams)
        return fail(h, LIDAR_E_INVALID, "surrogate weights need LIDAR_SUR_PARAMS values");
    if (!h->net.ready) return fail(h, LIDAR_E_STATE, "no surrogate weights set");
    HIP_TRY(h, hipMemcpyAsync(params, h->net.theta.p, (size_t)kSurParams * sizeof(float),
                              hipMemcpyDeviceToHost, h->stream), "copy surrogate weights");
    HIP_TRY(h, hipStreamSynchronize(h->stream), "weights synchronise");
    return LIDAR_OK;
}

static lidar_status sur_check(lidar_sim* h, const void* x, const void* y, uint32_t n)
{
    if (!x || !y || n == 0) return fail(h, LIDAR_E_INVALID, "surrogate call needs x, outputs and n >= 1");
    if (!h->net.ready) return fail(h, LIDAR_E_STATE, "no surrogate weights set");
    HIP_TRY(h, h->work.ensure((long)n), "allocate surrogate workspace");
    if (!h->work.blas_tried && !h->net.det) {
        // the library GEMMs of the training products (the own kernel runs
        // where the library cannot start)
        h->work.blas = blas_create();
        h->work.blas_tried = true;
    }
    return LIDAR_OK;
}

lidar_status lidar_sim_surrogate_forward(lidar_sim* h, const void* x, float* y, uint32_t n)
{
    if (!h) return LIDAR_E_INVALID;
    LIDAR_TRY(sur_check(h, x, y, n));
    HIP_TRY(h, sur_infer(h->stream, h->net, (const uint16_t*)x, (long)n, y), "surrogate forward");
    return LIDAR_OK;
}

static lidar_status sur_grads(lidar_sim* h, const void* x, const float* labels, uint32_t n)
{
    LIDAR_TRY(sur_check(h, x, labels, n));
    HIP_TRY(h, launch_zero_f32(h->stream, h->work.loss.p, 1), "zero loss");
    HIP_TRY(h, sur_gradients(h->stream, h->net, (const uint16_t*)x, labels, (long)n, h->work),
            "surrogate gradients");
    return LIDAR_OK;
}

lidar_status lidar_sim_surrogate_gradients(lidar_sim* h, const void* x, const float* labels,
                                           uint32_t n, float* grads, float* loss)
{
    if (!h) return LIDAR_E_INVALID;
    LIDAR_TRY(sur_grads(h, x, labels, n));
    if (grads)
        HIP_TRY(h, hipMemcpyAsync(grads, h->net.grad.p, (size_t)kSurParams * sizeof(float),
                                  hipMemcpyDeviceToDevice, h->stream), "copy gradients");
    if (loss)
        HIP_TRY(h, hipMemcpyAsync(loss, h->work.loss.p, sizeof(float), hipMemcpyDeviceToDevice,
                                  h->stream), "copy loss");
    return LIDAR_OK;
}

static bool hparams_ok(const lidar_train_hparams* hp)
{
    return hp && hp->lr > 0 && hp->beta1 >= 0 && hp->beta1 < 1 && hp->beta2 >= 0 && hp->beta2 < 1 &&
           hp->eps > 0 && hp->weight_decay >= 0 && is_fin(hp->lr) && is_fin(hp->eps) &&
           is_fin(hp->weight_decay);
}

// One AdamW step with learning rate lr on the rows (x, labels); the loss
// before the step into *loss (device, nullable).
static lidar_status adam_step(lidar_sim* h, const void* x, const float* labels, uint32_t n,
                              const lidar_train_hparams* hp, double lr, float* loss)
{
    LIDAR_TRY(sur_grads(h, x, labels, n));
    SurNet& net = h->net;
    const long t = ++net.step;
    AdamArgs a;
    a.lr = (float)lr;
    a.beta1 = (float)hp->beta1;
    a.beta2 = (float)hp->beta2;
    a.eps = (float)hp->eps;
    a.decay_factor = (float)(1.0 - lr * hp->weight_decay);
    a.inv_bc1 = (float)(1.0 / (1.0 - std::pow(hp->beta1, (double)t)));
    a.inv_bc2 = (float)(1.0 / (1.0 - std::pow(hp->beta2, (double)t)));
    HIP_TRY(h, launch_adamw(h->stream, net.theta.p, net.grad.p, net.m.p, net.v.p, net.theta_b.p,
                            kSurParams, a), "AdamW launch");
    net.t_stale = true;
    if (loss)
        HIP_TRY(h, hipMemcpyAsync(loss, h->work.loss.p, sizeof(float), hipMemcpyDeviceToDevice,
                                  h->stream), "copy loss");
    return LIDAR_OK;
}

lidar_status lidar_sim_surrogate_train_step(lidar_sim* h, const void* x, const float* labels,
                                            uint32_t n, const lidar_train_hparams* hp, float* loss)
{
    if (!h) return LIDAR_E_INVALID;
    if (!hparams_ok(hp)) return fail(h, LIDAR_E_INVALID, "hyper-parameters out of range");
    return adam_step(h, x, labels, n, hp, hp->lr, loss);
}

lidar_status lidar_sim_surrogate_train(lidar_sim* h, const void* x, const float* labels, uint64_t n,
                                       uint32_t batch, uint32_t steps, const lidar_train_hparams* hp,
                                       double lr_final, uint64_t seed, float* losses,
                                       uint32_t log_every)
{
    if (!h) return LIDAR_E_INVALID;
    if (!x || !labels || n == 0 || batch == 0)
        return fail(h, LIDAR_E_INVALID, "surrogate_train needs x, labels, n >= 1 and batch >= 1");
    if (n >= (1ull << 62)) return fail(h, LIDAR_E_INVALID, "surrogate_train: too many rows");
    if (!hparams_ok(hp)) return fail(h, LIDAR_E_INVALID, "hyper-parameters out of range");
    if (!(lr_final >= 0.0) || !is_fin(lr_final))
        return fail(h, LIDAR_E_INVALID, "lr_final must be finite and >= 0");
    if (losses && log_every == 0) return fail(h, LIDAR_E_INVALID, "losses need log_every >= 1");
    if (!h->net.ready) return fail(h, LIDAR_E_STATE, "no surrogate weights set");
    const uint32_t b = (uint32_t)std::min<uint64_t>(batch, n);
    HIP_TRY(h, h->mb_x.ensure((size_t)b * kSurIn), "allocate minibatch");
    HIP_TRY(h, h->mb_l.ensure((size_t)b * kSurOut), "allocate minibatch");
    int half = 1;                                    // 2^(2 half) >= n
    while ((1ull << (2 * half)) < n) ++half;
    uint64_t epoch = 0, pos = 0;
    for (uint32_t t = 0; t < steps; ++t) {
        if (pos + b > n) {
            ++epoch;
            pos = 0;
        }
        HIP_TRY(h, launch_gather_rows(h->stream, (const uint16_t*)x, labels, (long)n, half, seed, epoch,
                                      (long)pos, (int)b, h->mb_x.p, h->mb_l.p), "minibatch launch");
        pos += b;
        // linear decay, one rounding per operation (no fused multiply-add)
        const double f = (double)t / (double)std::max<uint32_t>(1u, steps - 1);
        const double span = lr_final - hp->lr;
        const double step_lr = span * f;
        const double lr = hp->lr + step_lr;
        float* out = losses && t % log_every == 0 ? losses + t / log_every : nullptr;
        LIDAR_TRY(adam_step(h, h->mb_x.p, h->mb_l.p, b, hp, lr, out));
    }
    return LIDAR_OK;
}

lidar_status lidar_sim_surrogate_set_gate(lidar_sim* h, double c_min, double alpha)
{
    if (!h) return LIDAR_E_INVALID;
    if (!(c_min >= 0.0 && c_min <= 1.0) || !(alpha >= 0.0))
        return fail(h, LIDAR_E_INVALID, "gate needs c_min in [0, 1] and alpha >= 0");
    h->gate_conf_logit = c_min >= 1.0 ? INFINITY
                         : c_min <= 0.0 ? -INFINITY
                                        : (float)std::log(c_min / (1.0 - c_min));
    h->gate_alpha = alpha >= 1e30 ? INFINITY : (float)alpha;
    return LIDAR_OK;
}

lidar_status lidar_sim_surrogate_features(lidar_sim* h, void* x, float* labels, float* aux)
{
    if (!h) return LIDAR_E_INVALID;
    if (!x) return fail(h, LIDAR_E_INVALID, "surrogate_features needs x");
    LIDAR_TRY(ensure_setup(h, "surrogate_features"));
    if (labels && !(h->have_result && h->plain_result))
        return fail(h, LIDAR_E_STATE, "labels need a plain simulate_frame on these inputs");
    if (labels && h->prm.max_echoes < 3) return fail(h, LIDAR_E_INVALID, "labels need max_echoes >= 3");
    LIDAR_TRY(surrogate_supported(h, "surrogate_features"));
    FrameState& fs = h->single;
    const int B = (int)fs.pat.az.size();
    LIDAR_TRY(sur_geometry(h, fs));
    LIDAR_TRY(sur_inputs(h, fs, (uint16_t*)x));
    if (labels)
        HIP_TRY(h, launch_labels(h->stream, h->d_echoes.p, h->d_counts.p, h->s_aux.p, B,
                                 (int)h->prm.max_echoes, (float)h->prm.threshold, labels),
                "labels launch");
    if (aux) HIP_TRY(h, launch_aux_out(h->stream, h->s_aux.p, B, aux), "aux launch");
    return LIDAR_OK;
}

lidar_status lidar_sim_get_stats(lidar_sim* h, lidar_stats* out)
{
    if (!h) return LIDAR_E_INVALID;
    if (!out) return fail(h, LIDAR_E_INVALID, "out is NULL");
    LIDAR_TRY(drain_events(h));
    h->st.n_beams = h->single.pat.az.size();
    h->st.samples_per_frame = h->setup_ok ? h->single.samples : 0;
    h->st.kernel_w = h->setup_ok ? (uint32_t)h->single.k.KW : 0;
    h->st.kernel_h = h->setup_ok ? (uint32_t)h->single.k.KH : 0;
    if (h->s_cnt.p) {
        int fb = 0;
        HIP_TRY(h, hipMemcpyAsync(&fb, h->s_cnt.p + 2, sizeof(int), hipMemcpyDeviceToHost, h->stream),
                "copy fallback count");
        HIP_TRY(h, hipStreamSynchronize(h->stream), "stats synchronise");
        h->st.fallback_beams = (uint64_t)fb;
    }
    *out = h->st;
    return LIDAR_OK;
}

lidar_status lidar_sim_reset_stats(lidar_sim* h)
{
    if (!h) return LIDAR_E_INVALID;
    LIDAR_TRY(drain_events(h));
    h->st.frames = 0;
    h->st.footprint_ms = 0.0;
    h->st.footprint_launches = 0;
    h->st.prepass_ms = 0.0;
    h->st.prepass_launches = 0;
    h->st.batch_ms = 0.0;
    h->st.batch_launches = 0;
    h->st.surrogate_beams = 0;
    h->st.fallback_beams = 0;
    h->st.surrogate_ms = 0.0;
    h->st.surrogate_frames = 0;
    if (h->s_cnt.p) HIP_TRY(h, launch_reset_queue(h->stream, h->s_cnt.p + 2, 1), "counter reset");
    return LIDAR_OK;
}

lidar_status lidar_sim_simulate_static(const lidar_sim_params* params, const lidar_pattern_desc* pattern,
                                       const lidar_gbuffer_desc* gbuffer, void* hip_stream,
                                       lidar_echo* echoes, int32_t* n_echoes, lidar_beam_info* beams)
{
    g_create_error.clear();
    return simulate_static(params, pattern, gbuffer, (hipStream_t)hip_stream, echoes, n_echoes, beams);
}

const char* lidar_sim_last_error(const lidar_sim* h)
{
    if (!h) return g_create_error.c_str();
    return h->err.c_str();
}

}  // extern "C"
