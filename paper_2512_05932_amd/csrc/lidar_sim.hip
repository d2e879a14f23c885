// Engine and C-ABI of the gfx950 LiDAR library (declared in
// include/lidar_sim.h).  The host side validates arguments, owns device
// buffers, decides sizes and the beam schedule, and enqueues kernels on the
// caller's stream; every step of the model itself runs in the kernels.
//
// Floating-point contraction is off in this file so that the host's FP64
// decisions (kernel extent M, N and pulse half-width J) use plain IEEE
// operations in the order written.
#pragma clang fp contract(off)

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "engine.h"

using namespace lidar;

namespace {

thread_local std::string g_create_error;

template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t count)
    {
        if (count <= n && p) return hipSuccess;
        if (p) {
            (void)hipFree(p);
            p = nullptr;
            n = 0;
        }
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

struct EventPair {
    hipEvent_t a, b;
};

}  // namespace

struct lidar_sim {
    lidar_sim_params prm{};
    hipStream_t stream = nullptr;
    std::string err;

    // pattern (host copies + device copies)
    bool have_pattern = false;
    uint64_t pattern_version = 0;
    uint32_t kind = 0;
    double sigma[2] = {0, 0}, trunc = 0, half[2] = {0, 0};
    uint32_t nx = 0, ny = 0;
    std::vector<double> az, el;
    DevBuf<float> d_table;
    DevBuf<double> d_az, d_el;
    DevBuf<int32_t> d_groups;
    int G = 1, n_groups = 0;

    // raster of the current G-buffer
    bool have_gbuffer = false;
    lidar_gbuffer_desc gb{};

    // derived set-up, valid for (pattern_version, raster)
    bool setup_ok = false;
    uint64_t setup_version = ~0ull;
    lidar_gbuffer_desc setup_gb{};
    KernelDev kgeom{};
    double kmax = 0.0;
    uint64_t samples = 0;
    DevBuf<double> d_K64, d_rowsum, d_rowmax, d_kinfo;
    DevBuf<float> d_Kb;
    DevBuf<int2> d_rowrange;
    DevBuf<int32_t> d_prefix;
    DevBuf<float2> d_colcs;
    DevBuf<float4> d_rowtab;
    DevBuf<lidar_beam_info> d_beams;

    // pulse
    int J = 0;
    DevBuf<float> d_taps;

    // per frame
    DevBuf<int2> d_pix;
    DevBuf<float> d_sun;
    DevBuf<lidar_echo> d_echoes;
    DevBuf<int32_t> d_counts;
    DevBuf<float> d_waves;
    bool have_result = false;

    // stats
    lidar_stats st{};
    std::vector<EventPair> pending_fp, pending_pp, pool;
};

namespace {

lidar_status fail(lidar_sim* h, lidar_status code, const std::string& msg)
{
    if (h) h->err = msg;
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

// Kernel extent on the pixel-offset grid: M = floor(extent_az / dphi),
// N = floor(extent_el / de), extent = trunc * sigma (Gaussian) or the table's
// half extent.
void kernel_extent(const lidar_sim* h, const RasterDev& r, double* M, double* N)
{
    if (h->kind == LIDAR_PATTERN_GAUSS) {
        *M = std::floor(h->trunc * h->sigma[0] / r.dphi);
        *N = std::floor(h->trunc * h->sigma[1] / r.de);
    } else {
        *M = std::floor(h->half[0] / r.dphi);
        *N = std::floor(h->half[1] / r.de);
    }
}

// Beam scheduler.  Beams are grouped G at a time so that one workgroup can
// share the pixel reads of nearby footprints: beams are sorted by their
// (approximate) pixel row band, then column, and a group takes consecutive
// beams of one band whose columns lie within one kernel width.  The groups
// are then ordered by column so that the groups in flight on one XCD cover a
// narrow band of the image.  Scheduling only: the exact pixel of each beam is
// computed on the GPU.
void build_groups(const std::vector<double>& az, const std::vector<double>& el,
                  const RasterDev& r, const KernelDev& k, int G, std::vector<int32_t>& out,
                  int* n_groups)
{
    const size_t B = az.size();
    std::vector<double> uf(B), vf(B);
    for (size_t i = 0; i < B; ++i) {
        uf[i] = std::floor((az[i] - r.az_min) / r.dphi);
        vf[i] = std::floor((r.el_max - el[i]) / r.de);
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
            double bi = std::floor(vf[i] / band);
            bool fits = !cur.empty() && (int)cur.size() < G && bi == cur_band &&
                        uf[i] - cur_u0 <= (double)k.KW;
            if (!fits && !cur.empty()) {
                groups.push_back(cur);
                cur.clear();
            }
            if (cur.empty()) {
                cur_band = bi;
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
    out.assign(groups.size() * G, -1);
    for (size_t gi = 0; gi < groups.size(); ++gi)
        for (size_t j = 0; j < groups[gi].size(); ++j) out[gi * G + j] = groups[gi][j];
    *n_groups = (int)groups.size();
}

lidar_status run_setup(lidar_sim* h)
{
    const lidar_gbuffer_desc& g = h->gb;
    RasterDev r = raster_of(g);
    double Mf, Nf;
    kernel_extent(h, r, &Mf, &Nf);
    if (!(Mf >= 0 && Nf >= 0) || Mf > 4096 || Nf > 4096 || (2 * Mf + 1) * (2 * Nf + 1) > 16.0e6)
        return fail(h, LIDAR_E_INVALID, "kernel grid too large for this raster (more than 16M "
                                        "cells or 8193 columns/rows)");
    // the footprint kernel addresses one group window of pixel records with
    // 32-bit byte offsets
    if ((4.0 * Mf + 8.0) * (double)g.height * 8.0 >= 2147483648.0)
        return fail(h, LIDAR_E_INVALID, "kernel window times image height too large "
                                        "(4*M+8)*height*8 must stay below 2^31 bytes");
    KernelDev k;
    k.M = (int)Mf;
    k.N = (int)Nf;
    k.KW = 2 * k.M + 1;
    k.KH = 2 * k.N + 1;
    const size_t cells = (size_t)k.KW * k.KH;
    HIP_TRY(h, h->d_K64.ensure(cells), "allocate kernel");
    HIP_TRY(h, h->d_Kb.ensure((size_t)4 * kernel_blocks(k.KW) * (k.KH + 1) * 4),
            "allocate kernel blocks");
    HIP_TRY(h, h->d_rowsum.ensure(k.KH), "allocate kernel rows");
    HIP_TRY(h, h->d_rowmax.ensure(k.KH), "allocate kernel rows");
    HIP_TRY(h, h->d_rowrange.ensure(k.KH), "allocate kernel rows");
    HIP_TRY(h, h->d_prefix.ensure((size_t)k.KH * (k.KW + 1)), "allocate kernel rows");
    HIP_TRY(h, h->d_kinfo.ensure(2), "allocate kernel info");
    HIP_TRY(h, h->d_colcs.ensure(g.width), "allocate raster tables");
    HIP_TRY(h, h->d_rowtab.ensure(g.height), "allocate raster tables");
    HIP_TRY(h, h->d_beams.ensure(h->az.size()), "allocate beams");

    PatternDev p;
    p.kind = (int)h->kind;
    p.sx = h->sigma[0];
    p.sy = h->sigma[1];
    p.trunc = h->trunc;
    p.table = h->d_table.p;
    p.nx = (int)h->nx;
    p.ny = (int)h->ny;
    p.hx = h->half[0];
    p.hy = h->half[1];
    hipStream_t s = h->stream;
    HIP_TRY(h, launch_kernel_grid(s, p, r, k, h->d_K64.p), "kernel grid launch");
    HIP_TRY(h, launch_kernel_blocks(s, k, h->d_K64.p, h->d_Kb.p), "kernel blocks launch");
    HIP_TRY(h, launch_kernel_rows(s, k, h->d_K64.p, h->d_rowsum.p, h->d_rowmax.p,
                                  h->d_rowrange.p, h->d_prefix.p), "kernel rows launch");
    HIP_TRY(h, launch_kernel_peak(s, k, h->d_rowsum.p, h->d_rowmax.p, h->d_kinfo.p),
            "kernel peak launch");
    HIP_TRY(h, launch_raster_tables(s, r, h->d_colcs.p, h->d_rowtab.p), "raster tables launch");
    HIP_TRY(h, launch_beam_setup(s, r, k, h->d_az.p, h->d_el.p, (int)h->az.size(),
                                 h->d_rowsum.p, h->d_prefix.p, h->prm.emit_power,
                                 h->d_beams.p), "beam setup launch");
    // the pattern's integral over the grid must be positive: checked once per
    // (pattern, raster), which synchronises the stream
    double kinfo[2];
    HIP_TRY(h, hipMemcpyAsync(kinfo, h->d_kinfo.p, sizeof(kinfo), hipMemcpyDeviceToHost, s),
            "copy kernel info");
    std::vector<lidar_beam_info> bi(h->az.size());
    HIP_TRY(h, hipMemcpyAsync(bi.data(), h->d_beams.p, sizeof(lidar_beam_info) * bi.size(),
                              hipMemcpyDeviceToHost, s), "copy beam info");
    HIP_TRY(h, hipStreamSynchronize(s), "set-up synchronise");
    if (!(kinfo[1] > 0.0) || !is_fin(kinfo[1]) || !(kinfo[0] > 0.0))
        return fail(h, LIDAR_E_INVALID, "pattern integral over the kernel grid is not positive "
                                        "(kernel narrower than one pixel or all-zero table)");
    uint64_t total = 0;
    for (auto& x : bi) total += x.samples;
    // beam groups for the footprint kernel
    int G = 4;
    while (G > 1 && !footprint_group_fits(G, (int)h->prm.n_bins, h->J)) G /= 2;
    std::vector<int32_t> groups;
    int n_groups = 0;
    build_groups(h->az, h->el, r, k, G, groups, &n_groups);
    HIP_TRY(h, h->d_groups.ensure(groups.size()), "allocate beam groups");
    HIP_TRY(h, hipMemcpyAsync(h->d_groups.p, groups.data(), groups.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, s), "copy beam groups");
    HIP_TRY(h, hipStreamSynchronize(s), "set-up synchronise");
    h->G = G;
    h->n_groups = n_groups;
    h->kgeom = k;
    h->kmax = kinfo[0];
    h->samples = total;
    h->setup_gb = g;
    h->setup_version = h->pattern_version;
    h->setup_ok = true;
    return LIDAR_OK;
}

lidar_status check_params(const lidar_sim_params* p, std::string& why)
{
    if (!p) { why = "params is NULL"; return LIDAR_E_INVALID; }
    if (p->n_bins < 1 || p->n_bins > (uint32_t)kMaxBins) {
        why = "n_bins must be in [1, 8000]";
        return LIDAR_E_INVALID;
    }
    if (p->max_echoes < 1 || p->max_echoes > 8) { why = "max_echoes must be in [1, 8]"; return LIDAR_E_INVALID; }
    if (!(p->bin_ns > 0.0) || !is_fin(p->bin_ns)) { why = "bin_ns must be > 0"; return LIDAR_E_INVALID; }
    if (!is_fin(p->threshold)) { why = "threshold must be finite"; return LIDAR_E_INVALID; }
    if (!(p->emit_power >= 0.0) || !is_fin(p->emit_power)) { why = "emit_power must be >= 0"; return LIDAR_E_INVALID; }
    if (!(p->pulse_fwhm_ns > 0.0) || !is_fin(p->pulse_fwhm_ns)) { why = "pulse_fwhm_ns must be > 0"; return LIDAR_E_INVALID; }
    if (!(p->pulse_trunc_sigmas > 0.0) || !is_fin(p->pulse_trunc_sigmas)) { why = "pulse_trunc_sigmas must be > 0"; return LIDAR_E_INVALID; }
    if (!is_fin(p->ambient_const) || !(p->sun_irradiance >= 0.0) || !is_fin(p->sun_irradiance)) {
        why = "ambient_const must be finite and sun_irradiance >= 0";
        return LIDAR_E_INVALID;
    }
    for (double c : p->sun_dir)
        if (!is_fin(c)) { why = "sun_dir must be finite"; return LIDAR_E_INVALID; }
    if (p->flags & ~(uint32_t)(LIDAR_KEEP_WAVEFORMS | LIDAR_PROFILE)) { why = "unknown flags"; return LIDAR_E_INVALID; }
    if (p->reserved != 0) { why = "reserved must be 0"; return LIDAR_E_INVALID; }
    double sigma = p->pulse_fwhm_ns / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    double J = std::ceil(p->pulse_trunc_sigmas * sigma / p->bin_ns);
    if (!(2.0 * J + 1.0 <= kMaxTaps)) { why = "pulse longer than 257 taps"; return LIDAR_E_INVALID; }
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
    double sigma = params->pulse_fwhm_ns / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    h->J = (int)std::ceil(params->pulse_trunc_sigmas * sigma / params->bin_ns);
    hipError_t e = h->d_taps.ensure(2 * h->J + 1);
    if (e == hipSuccess)
        e = launch_pulse_taps(h->stream, (float)sigma, (float)params->bin_ns, h->J, h->d_taps.p);
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
    for (auto* v : {&h->pending_fp, &h->pending_pp, &h->pool})
        for (auto& p : *v) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
    h->d_table.release(); h->d_az.release(); h->d_el.release(); h->d_groups.release();
    h->d_K64.release(); h->d_rowsum.release(); h->d_rowmax.release(); h->d_kinfo.release();
    h->d_Kb.release(); h->d_rowrange.release(); h->d_prefix.release();
    h->d_colcs.release(); h->d_rowtab.release(); h->d_beams.release(); h->d_taps.release();
    h->d_pix.release(); h->d_sun.release(); h->d_echoes.release(); h->d_counts.release();
    h->d_waves.release();
    delete h;
    return LIDAR_OK;
}

lidar_status lidar_sim_set_pattern(lidar_sim* h, const lidar_pattern_desc* pd)
{
    if (!h) return LIDAR_E_INVALID;
    if (!pd) return fail(h, LIDAR_E_INVALID, "pattern is NULL");
    if (pd->n_beams == 0 || !pd->beam_az_deg || !pd->beam_el_deg)
        return fail(h, LIDAR_E_INVALID, "pattern needs n_beams >= 1 and beam angle arrays");
    if (pd->n_beams > (1u << 26)) return fail(h, LIDAR_E_INVALID, "too many beams (max 2^26)");
    for (uint32_t i = 0; i < pd->n_beams; ++i)
        if (!is_fin(pd->beam_az_deg[i]) || !is_fin(pd->beam_el_deg[i]))
            return fail(h, LIDAR_E_INVALID, "non-finite beam angle");
    if (pd->kind == LIDAR_PATTERN_GAUSS) {
        if (!(pd->sigma_deg[0] > 0) || !(pd->sigma_deg[1] > 0) || !is_fin(pd->sigma_deg[0]) ||
            !is_fin(pd->sigma_deg[1]) || !(pd->trunc_sigmas > 0) || !is_fin(pd->trunc_sigmas))
            return fail(h, LIDAR_E_INVALID, "Gaussian pattern needs sigma > 0 and trunc_sigmas > 0");
    } else if (pd->kind == LIDAR_PATTERN_TABLE) {
        if (!pd->table || pd->nx < 2 || pd->ny < 2 || (uint64_t)pd->nx * pd->ny > (1u << 24))
            return fail(h, LIDAR_E_INVALID, "table pattern needs a table of at least 2x2 (max 16M cells)");
        if (!(pd->half_deg[0] > 0) || !(pd->half_deg[1] > 0) || !is_fin(pd->half_deg[0]) ||
            !is_fin(pd->half_deg[1]))
            return fail(h, LIDAR_E_INVALID, "table pattern needs half extents > 0");
        bool any = false;
        for (uint64_t i = 0; i < (uint64_t)pd->nx * pd->ny; ++i) {
            float v = pd->table[i];
            if (!std::isfinite(v) || v < 0.0f)
                return fail(h, LIDAR_E_INVALID, "table values must be finite and >= 0");
            any |= v > 0.0f;
        }
        if (!any) return fail(h, LIDAR_E_INVALID, "table is all zero (pattern integral is 0)");
    } else {
        return fail(h, LIDAR_E_INVALID, "unknown pattern kind");
    }
    const size_t B = pd->n_beams;
    h->az.assign(pd->beam_az_deg, pd->beam_az_deg + B);
    h->el.assign(pd->beam_el_deg, pd->beam_el_deg + B);
    HIP_TRY(h, h->d_az.ensure(B), "allocate beams");
    HIP_TRY(h, h->d_el.ensure(B), "allocate beams");
    hipStream_t s = h->stream;
    // pageable sources: these copies complete before the call returns
    HIP_TRY(h, hipMemcpyAsync(h->d_az.p, h->az.data(), B * sizeof(double), hipMemcpyHostToDevice, s), "copy beams");
    HIP_TRY(h, hipMemcpyAsync(h->d_el.p, h->el.data(), B * sizeof(double), hipMemcpyHostToDevice, s), "copy beams");
    h->kind = pd->kind;
    if (pd->kind == LIDAR_PATTERN_GAUSS) {
        h->sigma[0] = pd->sigma_deg[0];
        h->sigma[1] = pd->sigma_deg[1];
        h->trunc = pd->trunc_sigmas;
        h->nx = h->ny = 0;
    } else {
        const size_t cells = (size_t)pd->nx * pd->ny;
        HIP_TRY(h, h->d_table.ensure(cells), "allocate table");
        HIP_TRY(h, hipMemcpyAsync(h->d_table.p, pd->table, cells * sizeof(float),
                                  hipMemcpyHostToDevice, s), "copy table");
        h->nx = pd->nx;
        h->ny = pd->ny;
        h->half[0] = pd->half_deg[0];
        h->half[1] = pd->half_deg[1];
    }
    HIP_TRY(h, hipStreamSynchronize(s), "set_pattern synchronise");
    h->have_pattern = true;
    ++h->pattern_version;
    h->setup_ok = false;
    h->have_result = false;
    return LIDAR_OK;
}

lidar_status lidar_sim_set_gbuffer(lidar_sim* h, const lidar_gbuffer_desc* g)
{
    if (!h) return LIDAR_E_INVALID;
    if (!g) return fail(h, LIDAR_E_INVALID, "gbuffer is NULL");
    if (g->width == 0 || g->height == 0 || g->pitch < g->width)
        return fail(h, LIDAR_E_INVALID, "gbuffer needs width, height >= 1 and pitch >= width");
    if ((uint64_t)g->width * g->height > (1ull << 31))
        return fail(h, LIDAR_E_INVALID, "gbuffer larger than 2^31 pixels");
    if (!g->depth || !g->reflectance || !g->retro_gain || !g->normal_x || !g->normal_y || !g->normal_z)
        return fail(h, LIDAR_E_INVALID, "gbuffer plane pointer is NULL");
    if (!is_fin(g->az_min_deg) || !is_fin(g->az_max_deg) || !is_fin(g->el_min_deg) ||
        !is_fin(g->el_max_deg) || !(g->az_min_deg < g->az_max_deg) || !(g->el_min_deg < g->el_max_deg))
        return fail(h, LIDAR_E_INVALID, "gbuffer angle ranges must be finite with min < max");
    if (g->el_min_deg < -90.0 || g->el_max_deg > 90.0)
        return fail(h, LIDAR_E_INVALID, "gbuffer elevations must lie in [-90, 90]");
    h->gb = *g;
    h->have_gbuffer = true;
    if (h->setup_ok && !same_raster(h->setup_gb, *g)) h->setup_ok = false;
    return LIDAR_OK;
}

lidar_status lidar_sim_simulate_frame(lidar_sim* h, uint32_t mode)
{
    if (!h) return LIDAR_E_INVALID;
    if (mode != LIDAR_MODE_PLAIN) return fail(h, LIDAR_E_UNSUPPORTED, "only LIDAR_MODE_PLAIN is implemented");
    if (!h->have_pattern) return fail(h, LIDAR_E_STATE, "simulate_frame before set_pattern");
    if (!h->have_gbuffer) return fail(h, LIDAR_E_STATE, "simulate_frame before set_gbuffer");
    if (!h->setup_ok || h->setup_version != h->pattern_version) {
        lidar_status st = run_setup(h);
        if (st != LIDAR_OK) return st;
    }
    const lidar_gbuffer_desc& g = h->gb;
    const int W4 = (int)((g.width + 3) & ~3u);
    const size_t npix = (size_t)W4 * g.height;
    const size_t B = h->az.size();
    const uint32_t R = h->prm.n_bins, E = h->prm.max_echoes;
    const bool sun = h->prm.sun_irradiance != 0.0;
    const bool keep = (h->prm.flags & LIDAR_KEEP_WAVEFORMS) != 0;
    const bool prof = (h->prm.flags & LIDAR_PROFILE) != 0;
    HIP_TRY(h, h->d_pix.ensure(npix), "allocate pixel records");
    if (sun) HIP_TRY(h, h->d_sun.ensure(npix), "allocate sun shading");
    HIP_TRY(h, h->d_echoes.ensure(B * E), "allocate echoes");
    HIP_TRY(h, h->d_counts.ensure(B), "allocate counts");
    if (keep) HIP_TRY(h, h->d_waves.ensure(B * (size_t)R), "allocate waveforms");

    hipStream_t s = h->stream;
    RasterDev r = raster_of(g);
    PrepassArgs pa;
    pa.depth = g.depth;
    pa.refl = g.reflectance;
    pa.gain = g.retro_gain;
    pa.nx = g.normal_x;
    pa.ny = g.normal_y;
    pa.nz = g.normal_z;
    pa.pitch = (long)g.pitch;
    pa.W = r.W;
    pa.H = r.H;
    pa.colcs = h->d_colcs.p;
    pa.rowtab = h->d_rowtab.p;
    pa.to_bin = 2.0 / (kLight * (h->prm.bin_ns * 1e-9));
    pa.R = (int)R;
    pa.sun_x = (float)h->prm.sun_dir[0];
    pa.sun_y = (float)h->prm.sun_dir[1];
    pa.sun_z = (float)h->prm.sun_dir[2];
    pa.pix = h->d_pix.p;
    pa.sun = sun ? h->d_sun.p : nullptr;
    pa.W4 = W4;

    FootprintArgs fa;
    fa.pix = h->d_pix.p;
    fa.sun = sun ? h->d_sun.p : nullptr;
    fa.W = r.W;
    fa.H = r.H;
    fa.Kb = h->d_Kb.p;
    fa.NB = kernel_blocks(h->kgeom.KW);
    fa.rowrange = h->d_rowrange.p;
    fa.M = h->kgeom.M;
    fa.N = h->kgeom.N;
    fa.KW = h->kgeom.KW;
    fa.KH = h->kgeom.KH;
    fa.groups = h->d_groups.p;
    fa.n_groups = h->n_groups;
    fa.G = h->G;
    fa.chunk = (h->n_groups + kXcds - 1) / kXcds;
    fa.beams = h->d_beams.p;
    fa.taps = h->d_taps.p;
    fa.J = h->J;
    fa.R = (int)R;
    fa.threshold = (float)h->prm.threshold;
    fa.ambient = (float)h->prm.ambient_const;
    fa.sun_scale = sun ? (float)(h->prm.sun_irradiance / h->kmax) : 0.0f;
    fa.E = (int)E;
    fa.echoes = h->d_echoes.p;
    fa.counts = h->d_counts.p;
    fa.waves = keep ? h->d_waves.p : nullptr;
    fa.half_c_dt = 0.5 * kLight * (h->prm.bin_ns * 1e-9);
    fa.bin_ns = h->prm.bin_ns;

    EventPair pp{}, fp{};
    if (prof) {
        hipError_t e;
        pp = take_pair(h, &e);
        HIP_TRY(h, e, "create events");
        fp = take_pair(h, &e);
        HIP_TRY(h, e, "create events");
        HIP_TRY(h, hipEventRecord(pp.a, s), "record event");
    }
    HIP_TRY(h, launch_prepass(s, pa, sun), "pre-pass launch");
    if (prof) {
        HIP_TRY(h, hipEventRecord(pp.b, s), "record event");
        HIP_TRY(h, hipEventRecord(fp.a, s), "record event");
    }
    HIP_TRY(h, launch_footprint(s, fa), "footprint launch");
    if (prof) {
        HIP_TRY(h, hipEventRecord(fp.b, s), "record event");
        h->pending_pp.push_back(pp);
        h->pending_fp.push_back(fp);
    }
    h->have_result = true;
    ++h->st.frames;
    return LIDAR_OK;
}

lidar_status lidar_sim_read_echoes(lidar_sim* h, lidar_echo* echoes, int32_t* n_echoes,
                                   float* waveforms, lidar_beam_info* beams, int dst_is_device)
{
    if (!h) return LIDAR_E_INVALID;
    if (!h->have_result) return fail(h, LIDAR_E_STATE, "read_echoes before simulate_frame");
    if (waveforms && !(h->prm.flags & LIDAR_KEEP_WAVEFORMS))
        return fail(h, LIDAR_E_INVALID, "waveforms requested without LIDAR_KEEP_WAVEFORMS");
    const size_t B = h->az.size();
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

lidar_status lidar_sim_get_stats(lidar_sim* h, lidar_stats* out)
{
    if (!h || !out) return h ? fail(h, LIDAR_E_INVALID, "out is NULL") : LIDAR_E_INVALID;
    lidar_status st = drain_events(h);
    if (st != LIDAR_OK) return st;
    h->st.n_beams = h->az.size();
    h->st.samples_per_frame = h->setup_ok ? h->samples : 0;
    h->st.kernel_w = h->setup_ok ? (uint32_t)h->kgeom.KW : 0;
    h->st.kernel_h = h->setup_ok ? (uint32_t)h->kgeom.KH : 0;
    *out = h->st;
    return LIDAR_OK;
}

lidar_status lidar_sim_reset_stats(lidar_sim* h)
{
    if (!h) return LIDAR_E_INVALID;
    lidar_status st = drain_events(h);
    if (st != LIDAR_OK) return st;
    h->st.frames = 0;
    h->st.footprint_ms = 0.0;
    h->st.footprint_launches = 0;
    h->st.prepass_ms = 0.0;
    h->st.prepass_launches = 0;
    return LIDAR_OK;
}

const char* lidar_sim_last_error(const lidar_sim* h)
{
    if (!h) return g_create_error.c_str();
    return h->err.c_str();
}

}  // extern "C"
