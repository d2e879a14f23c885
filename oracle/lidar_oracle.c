/*
 * FP64 CPU oracle of the single-bounce beam-iteration LiDAR model.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the HIP path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it; the product
 * path never does.  It shares no code, header, table or constant with the HIP
 * library.
 *
 * What it computes (paper section II, Eq. 2-5, Alg. 1, and the echo
 * post-processing of section II-C), for every beam b:
 *   1. the pixel (u_b, v_b) that contains the beam centre Psi_b
 *      (Alg. 1, roundToPixels);
 *   2. the centred kernel K[m][n] = (kappa*eta)(m*dphi, -n*de) on the
 *      pixel-offset grid, m in [-M, M], n in [-N, N] (Eq. 5, Alg. 1 input
 *      kappa*eta[2M+1][2N+1]);
 *   3. the normalisation N_b = sum over all kernel cells of K * Omega(v_b + n),
 *      Omega the exact solid angle of an equiangular pixel row from
 *      d(omega) = sin(theta) d(theta) d(phi) (Eq. 2), and S_b = P_e / N_b;
 *   4. the footprint sum of Eq. 5 with rho_hat = beta cos(theta) / d^2
 *      (unit isotropic source at the sensor, Eq. 4), beta = g * rho / pi,
 *      each pixel placed in the single time bin k = floor(2 d / (c dt))
 *      (the Dirac delta of Eq. 3), accumulated (+=) over the kernel cells;
 *   5. the ambient floor A_b: a constant plus sunlight received through the
 *      collector sensitivity kappa = K / max K from Lambertian surfaces
 *      (section II-A: stray light is computed like the laser term with the
 *      source substituted);
 *   6. the pulse convolution xi_hat = varpi * xi + A_b with a centred, unit-sum
 *      Gaussian pulse of the given FWHM (section II-C, EPW paragraph);
 *   7. the echoes: maximal runs of bins with xi_hat > T (strict), each with
 *      its first peak bin, peak intensity above the floor, FP64 range of the
 *      peak bin centre and the echo pulse width from linearly interpolated
 *      threshold crossings (section II-C, EPW paragraph).
 *
 * Options of the same path:
 *   - a tabulated pulse varpi (samples at the bin pitch, centred), used
 *     normalised to unit sum like the Gaussian (section II-C, EPW paragraph);
 *   - a collector sensitivity table kappa for the sun term, measured apart
 *     from the combined pattern (section III-B); without it kappa = K/max K;
 *   - range modes (section II-D, rasterization; Alg. 1, pixelRangeInterval):
 *     the pixel's centre range (default); the range corrected to the true
 *     direction v of each kernel cell, r = d (p.n) / (v.n) with p the pixel
 *     centre direction; or the pixel's range interval, the plane through
 *     the pixel's centre point with normal n met by the four corner rays,
 *     the pixel's weight shared evenly by the bins of that interval;
 *   - echo selection (section II-C, after Alg. 1): the strongest, nearest or
 *     longest (widest EPW) run of xi_hat, or, without the pulse
 *     post-processing, the strongest or nearest bin of the raw signal at or
 *     above T (the single echo comparable to range stacking, Alg. 2).
 *
 * Readings where the paper is silent (each one is listed in the design doc):
 * accumulate rather than assign in Alg. 1; a single bin per pixel;
 * floor rounding to the containing pixel; correlation orientation
 * (kernel indexed by pixel minus beam); equiangular raster; per-beam
 * normalisation of the combined kernel; beta = g*rho/pi; cos(theta) kept for
 * retroreflectors; radial depth; invalid pixels skipped; ambient added after
 * the pulse convolution; kappa = K / max K; strict threshold; range at the
 * peak bin centre; intensity = peak minus floor.
 *
 * Built with -O2 -ffp-contract=off so that every floating-point decision that
 * selects an integer (pixel index, kernel support, time bin, tap count) is
 * taken with plain IEEE double operations in the order written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_C_LIGHT 299792458.0
#define ORC_PI 3.14159265358979323846

typedef struct {
    int32_t width, height;
    double az_min, az_max, el_min, el_max; /* degrees */
} orc_raster;

typedef struct {
    int32_t kind;           /* 1 = Gaussian, 2 = table */
    double sigma_az, sigma_el, trunc_sigmas;
    const float* table;     /* [ny][nx], row 0 = +elevation */
    int32_t nx, ny;
    double half_az, half_el;
    const float* rx_table;  /* optional kappa [ny][nx] on the table's grid (kind 2) */
} orc_pattern;

enum { ORC_ALL = 0, ORC_STRONGEST = 1, ORC_NEAREST = 2, ORC_LONGEST = 3,
       ORC_RAW_STRONGEST = 4, ORC_RAW_NEAREST = 5 };
enum { ORC_RANGE_CENTRE = 0, ORC_RANGE_CORRECTED = 1, ORC_RANGE_INTERVAL = 2 };

typedef struct {
    int32_t n_bins, max_echoes;
    double bin_ns, threshold, emit_power;
    double pulse_fwhm_ns, pulse_trunc_sigmas;
    double ambient_const, sun_irradiance;
    double sun_dir[3];
    const double* pulse_taps;   /* optional tabulated pulse, n_pulse_taps samples */
    int32_t n_pulse_taps;
    int32_t echo_select;        /* ORC_ALL .. ORC_RAW_NEAREST */
    int32_t range_mode;         /* ORC_RANGE_* */
} orc_params;

typedef struct {
    double range_m, time_ns;
    double intensity, pulse_width_ns;
    int32_t bin_peak, bin_first, bin_last, flags;
} orc_echo;

static double deg2rad(double d) { return d * (ORC_PI / 180.0); }

/* ---- raster geometry -------------------------------------------------- */

double orc_dphi(const orc_raster* r) { return (r->az_max - r->az_min) / (double)r->width; }
double orc_de(const orc_raster* r) { return (r->el_max - r->el_min) / (double)r->height; }

/* Solid angle (sr) of one pixel of row v of an equiangular raster: the
 * integral of cos(e) de dphi over the pixel, i.e. dphi * (sin e_top - sin e_bot).
 * Defined for any integer v, including rows outside the image. */
double orc_row_solid_angle(const orc_raster* r, int64_t v)
{
    double de = orc_de(r);
    double e_top = r->el_max - (double)v * de;
    double e_bot = r->el_max - (double)(v + 1) * de;
    return deg2rad(orc_dphi(r)) * (sin(deg2rad(e_top)) - sin(deg2rad(e_bot)));
}

/* Pixel containing the direction (az, el): floor rounding, section II-C. */
void orc_beam_pixel(const orc_raster* r, double az, double el, int64_t* u, int64_t* v)
{
    *u = (int64_t)floor((az - r->az_min) / orc_dphi(r));
    *v = (int64_t)floor((r->el_max - el) / orc_de(r));
}

/* ---- centred kernel ---------------------------------------------------- */

void orc_kernel_extent(const orc_raster* r, const orc_pattern* p, int32_t* M, int32_t* N)
{
    double dphi = orc_dphi(r), de = orc_de(r);
    if (p->kind == 1) {
        *M = (int32_t)floor(p->trunc_sigmas * p->sigma_az / dphi);
        *N = (int32_t)floor(p->trunc_sigmas * p->sigma_el / de);
    } else {
        *M = (int32_t)floor(p->half_az / dphi);
        *N = (int32_t)floor(p->half_el / de);
    }
}

static double table_at(const orc_pattern* p, int64_t i, int64_t j)
{
    if (i < 0 || j < 0 || i >= p->nx || j >= p->ny) return 0.0;
    return (double)p->table[j * (int64_t)p->nx + i];
}

/* Pattern value at an angular offset (x along azimuth, y along elevation, in
 * degrees) from the beam centre. */
double orc_pattern_value(const orc_pattern* p, double x, double y)
{
    if (p->kind == 1) {
        double qx = x / p->sigma_az, qy = y / p->sigma_el;
        double q = qx * qx + qy * qy;
        if (q > p->trunc_sigmas * p->trunc_sigmas) return 0.0;
        return exp(-0.5 * q);
    }
    /* the table covers [-half, half] on both axes and the pattern is zero
     * outside it; inside, bilinear interpolation between cell centres, with
     * zero beyond the outermost centres */
    if (fabs(x) > p->half_az || fabs(y) > p->half_el) return 0.0;
    double cx = 2.0 * p->half_az / (double)p->nx;
    double cy = 2.0 * p->half_el / (double)p->ny;
    double fx = (x + p->half_az) / cx - 0.5;
    double fy = (p->half_el - y) / cy - 0.5;
    double i0 = floor(fx), j0 = floor(fy);
    double tx = fx - i0, ty = fy - j0;
    int64_t i = (int64_t)i0, j = (int64_t)j0;
    double v00 = table_at(p, i, j), v10 = table_at(p, i + 1, j);
    double v01 = table_at(p, i, j + 1), v11 = table_at(p, i + 1, j + 1);
    double top = (1.0 - tx) * v00 + tx * v10;
    double bot = (1.0 - tx) * v01 + tx * v11;
    return (1.0 - ty) * top + ty * bot;
}

/* K[n + N][m + M] for pixel offsets (m, n): column offset m along azimuth,
 * row offset n downwards (towards lower elevation). */
void orc_kernel_grid(const orc_raster* r, const orc_pattern* p, double* K)
{
    int32_t M, N;
    orc_kernel_extent(r, p, &M, &N);
    double dphi = orc_dphi(r), de = orc_de(r);
    for (int32_t n = -N; n <= N; ++n)
        for (int32_t m = -M; m <= M; ++m)
            K[(int64_t)(n + N) * (2 * M + 1) + (m + M)] =
                orc_pattern_value(p, (double)m * dphi, -(double)n * de);
}

/* ---- pulse ------------------------------------------------------------- */

int32_t orc_pulse_half_taps(const orc_params* q)
{
    if (q->pulse_taps) return (q->n_pulse_taps - 1) / 2;
    double sigma = q->pulse_fwhm_ns / (2.0 * sqrt(2.0 * log(2.0)));
    return (int32_t)ceil(q->pulse_trunc_sigmas * sigma / q->bin_ns);
}

/* Centred pulse sampled at the bin pitch, normalised to unit sum; taps[j + J]
 * for j in [-J, J]: the given table, or a Gaussian of the given FWHM. */
void orc_pulse_taps(const orc_params* q, double* taps)
{
    int32_t J = orc_pulse_half_taps(q);
    double s = 0.0;
    if (q->pulse_taps) {
        for (int32_t j = -J; j <= J; ++j) {
            taps[j + J] = q->pulse_taps[j + J];
            s += taps[j + J];
        }
    } else {
        double sigma = q->pulse_fwhm_ns / (2.0 * sqrt(2.0 * log(2.0)));
        for (int32_t j = -J; j <= J; ++j) {
            double t = (double)j * q->bin_ns;
            taps[j + J] = exp(-(t * t) / (2.0 * sigma * sigma));
            s += taps[j + J];
        }
    }
    for (int32_t j = -J; j <= J; ++j) taps[j + J] /= s;
}

/* ---- echoes ------------------------------------------------------------ */

/* Maximal runs of xi_hat > T; returns the number of runs, stores the first
 * max_echoes of them. */
int32_t orc_detect(const double* xh, int32_t R, double T, double floor_b, double bin_ns,
                   int32_t max_echoes, orc_echo* out)
{
    double half_c_dt = 0.5 * ORC_C_LIGHT * (bin_ns * 1e-9);
    int32_t count = 0;
    int32_t k = 0;
    while (k < R) {
        if (!(xh[k] > T)) { ++k; continue; }
        int32_t k0 = k;
        while (k + 1 < R && xh[k + 1] > T) ++k;
        int32_t k1 = k;
        if (count < max_echoes) {
            int32_t kp = k0;
            for (int32_t i = k0 + 1; i <= k1; ++i)
                if (xh[i] > xh[kp]) kp = i;
            double t_up, t_dn;
            int32_t flags = 0;
            if (k0 == 0) { t_up = 0.0; flags |= 1; }
            else t_up = ((double)(k0 - 1) + 0.5) * bin_ns +
                        bin_ns * (T - xh[k0 - 1]) / (xh[k0] - xh[k0 - 1]);
            if (k1 == R - 1) { t_dn = (double)R * bin_ns; flags |= 2; }
            else t_dn = ((double)k1 + 0.5) * bin_ns +
                        bin_ns * (xh[k1] - T) / (xh[k1] - xh[k1 + 1]);
            orc_echo* e = &out[count];
            e->bin_peak = kp;
            e->bin_first = k0;
            e->bin_last = k1;
            e->flags = flags;
            e->time_ns = ((double)kp + 0.5) * bin_ns;
            e->range_m = ((double)kp + 0.5) * half_c_dt;
            e->intensity = xh[kp] - floor_b;
            e->pulse_width_ns = t_dn - t_up;
        }
        ++count;
        ++k;
    }
    return count;
}

/* Pick one of the runs of xi_hat (echo selection): the strongest (largest
 * peak), the nearest (first) or the longest (widest pulse width); the first
 * such run wins a tie.  runs[0..n) hold every run in time order. */
static int32_t orc_pick(const orc_echo* runs, int32_t n, int32_t mode)
{
    int32_t best = 0;
    for (int32_t i = 1; i < n; ++i) {
        if (mode == ORC_STRONGEST) {
            double a = runs[i].intensity, b = runs[best].intensity;
            if (a > b) best = i;
        } else if (mode == ORC_LONGEST) {
            if (runs[i].pulse_width_ns > runs[best].pulse_width_ns) best = i;
        }
    }
    return best;
}

/* Echoes of one beam under the selection mode: xh is xi_hat, xi the raw
 * binned signal (scaled by S_b); writes max_echoes slots (zeroed beyond the
 * echoes kept) and returns the count (all runs, or 0/1 for the raw modes). */
int32_t orc_select(const double* xi, const double* xh, int32_t R, double T, double floor_b,
                   double bin_ns, int32_t max_echoes, int32_t mode, orc_echo* out)
{
    memset(out, 0, sizeof(orc_echo) * (size_t)max_echoes);
    if (mode == ORC_ALL) return orc_detect(xh, R, T, floor_b, bin_ns, max_echoes, out);
    if (mode == ORC_RAW_STRONGEST || mode == ORC_RAW_NEAREST) {
        int32_t k = -1;
        for (int32_t i = 0; i < R; ++i) {
            if (!(xi[i] >= T)) continue;
            if (k < 0) k = i;
            if (mode == ORC_RAW_NEAREST) break;
            if (xi[i] > xi[k]) k = i;
        }
        if (k < 0) return 0;
        double half_c_dt = 0.5 * ORC_C_LIGHT * (bin_ns * 1e-9);
        out[0].bin_peak = out[0].bin_first = out[0].bin_last = k;
        out[0].time_ns = ((double)k + 0.5) * bin_ns;
        out[0].range_m = ((double)k + 0.5) * half_c_dt;
        out[0].intensity = xi[k];
        out[0].pulse_width_ns = 0.0;
        out[0].flags = 0;
        return 1;
    }
    orc_echo* runs = (orc_echo*)malloc(sizeof(orc_echo) * (size_t)(R / 2 + 1));
    int32_t n = orc_detect(xh, R, T, floor_b, bin_ns, R / 2 + 1, runs);
    if (n > 0) out[0] = runs[mode == ORC_NEAREST ? 0 : orc_pick(runs, n, mode)];
    free(runs);
    return n;
}

/* ---- range of a sample ----------------------------------------------------- */

static void orc_dir(double az_deg, double el_deg, double* d)
{
    double a = deg2rad(az_deg), e = deg2rad(el_deg);
    d[0] = cos(e) * cos(a);
    d[1] = cos(e) * sin(a);
    d[2] = sin(e);
}

/* Range at which the plane through the point d*p (p: unit pixel-centre
 * direction) with normal n meets the ray along w: d (p.n) / (w.n), the
 * ratio (p.n)/(w.n) limited to [1/2, 2] (and 2 when the ray misses the
 * plane's side facing the sensor). */
double orc_plane_range(double d, const double* p, const double* w, const double* n)
{
    double pn = p[0] * n[0] + p[1] * n[1] + p[2] * n[2];
    double wn = w[0] * n[0] + w[1] * n[1] + w[2] * n[2];
    double q = pn / wn;
    if (!(q > 0.0)) q = 2.0;
    if (q < 0.5) q = 0.5;
    if (q > 2.0) q = 2.0;
    return d * q;
}

/* The pixel's range interval (Alg. 1, pixelRangeInterval): the centre range
 * and the ranges of the four corner rays on the pixel's plane; *r0, *r1 are
 * their minimum and maximum. */
void orc_pixel_interval(const orc_raster* r, int64_t u, int64_t v, double d, const double* n,
                        double* r0, double* r1)
{
    double dphi = orc_dphi(r), de = orc_de(r), p[3], w[3];
    orc_dir(r->az_min + ((double)u + 0.5) * dphi, r->el_max - ((double)v + 0.5) * de, p);
    double lo = d, hi = d;
    for (int c = 0; c < 4; ++c) {
        double az = r->az_min + (double)(u + (c & 1)) * dphi;
        double el = r->el_max - (double)(v + (c >> 1)) * de;
        orc_dir(az, el, w);
        double rc = orc_plane_range(d, p, w, n);
        if (rc < lo) lo = rc;
        if (rc > hi) hi = rc;
    }
    *r0 = lo;
    *r1 = hi;
}

/* ---- the whole per-beam path -------------------------------------------- */

/*
 * Planes are host float32 [H][W] row-major.  Outputs (all per beam, any may
 * be NULL): xi [B][R] raw binned signal, xi_hat [B][R] pulse-convolved signal
 * plus floor, floor [B], echoes [B][max_echoes], n_echoes [B],
 * samples [B] (kernel cells with K > 0 inside the image), scale [B] (S_b),
 * pix [B][2] (u_b, v_b).
 */
int orc_simulate(const orc_raster* r, const float* depth, const float* refl,
                 const float* gain, const float* nxp, const float* nyp, const float* nzp,
                 const orc_pattern* p, int32_t B, const double* beam_az,
                 const double* beam_el, const orc_params* q, double* xi_out,
                 double* xh_out, double* floor_out, orc_echo* echoes,
                 int32_t* n_echoes, int64_t* samples, double* scale_out,
                 int64_t* pix_out, int n_threads)
{
    const int32_t W = r->width, H = r->height, R = q->n_bins;
    int32_t M, N;
    orc_kernel_extent(r, p, &M, &N);
    const int64_t KW = 2 * M + 1, KH = 2 * N + 1;
    double* K = (double*)malloc(sizeof(double) * KW * KH);
    if (!K) return -1;
    orc_kernel_grid(r, p, K);
    double kmax = 0.0;
    for (int64_t i = 0; i < KW * KH; ++i) if (K[i] > kmax) kmax = K[i];
    /* collector sensitivity of the sun term: the kappa table resampled like
     * K, or K / max K */
    double* kap = (double*)malloc(sizeof(double) * KW * KH);
    if (!kap) { free(K); return -1; }
    if (p->kind == 2 && p->rx_table) {
        orc_pattern rx = *p;
        rx.table = p->rx_table;
        orc_kernel_grid(r, &rx, kap);
    } else {
        for (int64_t i = 0; i < KW * KH; ++i) kap[i] = K[i] / kmax;
    }

    int32_t J = orc_pulse_half_taps(q);
    double* taps = (double*)malloc(sizeof(double) * (2 * J + 1));
    orc_pulse_taps(q, taps);

    /* pixel-centre direction tables (FP64) */
    double dphi = orc_dphi(r), de = orc_de(r);
    double* cphi = (double*)malloc(sizeof(double) * W);
    double* sphi = (double*)malloc(sizeof(double) * W);
    double* cel = (double*)malloc(sizeof(double) * H);
    double* sel = (double*)malloc(sizeof(double) * H);
    for (int32_t u = 0; u < W; ++u) {
        double a = deg2rad(r->az_min + ((double)u + 0.5) * dphi);
        cphi[u] = cos(a); sphi[u] = sin(a);
    }
    for (int32_t v = 0; v < H; ++v) {
        double e = deg2rad(r->el_max - ((double)v + 0.5) * de);
        cel[v] = cos(e); sel[v] = sin(e);
    }
    const double to_bin = 2.0 / (ORC_C_LIGHT * (q->bin_ns * 1e-9));

#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (int32_t b = 0; b < B; ++b) {
        double* xi = (double*)calloc((size_t)R, sizeof(double));
        double* xh = (double*)malloc(sizeof(double) * R);
        int64_t ub, vb;
        orc_beam_pixel(r, beam_az[b], beam_el[b], &ub, &vb);
        double true_dir[3];

        /* normalisation over the whole kernel, on- and off-image rows */
        double nb = 0.0;
        for (int64_t n = -N; n <= N; ++n) {
            double om = orc_row_solid_angle(r, vb + n);
            for (int64_t m = -M; m <= M; ++m) nb += K[(n + N) * KW + (m + M)] * om;
        }
        double Sb = q->emit_power / nb;

        double sun_acc = 0.0;
        int64_t nsamp = 0;
        for (int64_t n = -N; n <= N; ++n) {
            int64_t v = vb + n;
            if (v < 0 || v >= H) continue;
            double om = orc_row_solid_angle(r, v);
            for (int64_t m = -M; m <= M; ++m) {
                /* the laser term covers the cells with K > 0, the sun term
                 * the cells with kappa > 0 (the same cells without a kappa
                 * table) */
                double kv = K[(n + N) * KW + (m + M)];
                double ka = kap[(n + N) * KW + (m + M)];
                if (!(kv > 0.0) && !(ka > 0.0)) continue;
                int64_t u = ub + m;
                if (u < 0 || u >= W) continue;
                if (kv > 0.0) ++nsamp;
                int64_t px = v * W + u;
                double d = (double)depth[px];
                if (!(isfinite(d) && d > 0.0)) continue;
                double nrm[3] = {(double)nxp[px], (double)nyp[px], (double)nzp[px]};
                /* the pixel's bins: its centre bin, the bin of the range
                 * corrected to this kernel cell's true direction, or the bins
                 * of its range interval */
                double kb = floor(d * to_bin), k0 = kb, k1 = kb;
                int pixel_ok = kb >= 0.0 && kb < (double)R;
                if (q->range_mode == ORC_RANGE_INTERVAL) {
                    double r0, r1;
                    orc_pixel_interval(r, u, v, d, nrm, &r0, &r1);
                    k0 = floor(r0 * to_bin);
                    k1 = floor(r1 * to_bin);
                    pixel_ok = k0 < (double)R;
                }
                if (!pixel_ok) continue;
                double vx = cel[v] * cphi[u], vy = cel[v] * sphi[u], vz = sel[v];
                double nx = nrm[0], ny = nrm[1], nz = nrm[2];
                double cos_t = -(nx * vx + ny * vy + nz * vz);
                if (cos_t < 0.0) cos_t = 0.0;
                double rho = (double)refl[px];
                double beta = (double)gain[px] * rho / ORC_PI;
                double w = Sb * kv * om * beta * cos_t / (d * d);
                if (q->range_mode == ORC_RANGE_CORRECTED) {
                    double pd[3] = {vx, vy, vz};
                    orc_dir(beam_az[b] + (double)m * dphi, beam_el[b] - (double)n * de, true_dir);
                    double kc = floor(orc_plane_range(d, pd, true_dir, nrm) * to_bin);
                    if (kc >= 0.0 && kc < (double)R) xi[(int64_t)kc] += w;
                } else if (q->range_mode == ORC_RANGE_INTERVAL) {
                    double share = w / (k1 - k0 + 1.0);
                    for (double k = k0; k <= k1 && k < (double)R; k += 1.0) xi[(int64_t)k] += share;
                } else {
                    xi[(int64_t)kb] += w;
                }
                if (q->sun_irradiance != 0.0) {
                    double ns = nx * q->sun_dir[0] + ny * q->sun_dir[1] + nz * q->sun_dir[2];
                    if (ns < 0.0) ns = 0.0;
                    sun_acc += ka * om * (rho / ORC_PI) * ns;
                }
            }
        }
        double fl = q->ambient_const + q->sun_irradiance * sun_acc;

        for (int32_t k = 0; k < R; ++k) {
            double s = 0.0;
            for (int32_t j = -J; j <= J; ++j) {
                int32_t i = k - j;
                if (i < 0 || i >= R) continue;
                s += taps[j + J] * xi[i];
            }
            xh[k] = s + fl;
        }
        orc_echo tmp[8];
        orc_echo* eo = echoes ? &echoes[(int64_t)b * q->max_echoes] : tmp;
        int32_t ne = orc_select(xi, xh, R, q->threshold, fl, q->bin_ns, q->max_echoes,
                                q->echo_select, eo);
        if (n_echoes) n_echoes[b] = ne;
        if (xi_out) memcpy(&xi_out[(int64_t)b * R], xi, sizeof(double) * R);
        if (xh_out) memcpy(&xh_out[(int64_t)b * R], xh, sizeof(double) * R);
        if (floor_out) floor_out[b] = fl;
        if (samples) samples[b] = nsamp;
        if (scale_out) scale_out[b] = Sb;
        if (pix_out) { pix_out[2 * b] = ub; pix_out[2 * b + 1] = vb; }
        free(xi);
        free(xh);
    }
    free(K); free(kap); free(taps); free(cphi); free(sphi); free(cel); free(sel);
    return 0;
}
