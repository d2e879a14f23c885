/*
 * lidar_sim.h -- C-ABI of the MI355X (gfx950) single-bounce LiDAR engine.
 *
 * The engine evaluates the beam-iteration form of the single-bounce LiDAR
 * model ("Physically-Based Simulation of Automotive LiDAR", section II,
 * Eq. 2-5, Alg. 1): for every beam of a steering pattern it integrates a
 * rasterised NIR G-buffer over the beam's footprint, bins the weighted returns
 * by round-trip time, adds the ambient floor, convolves the laser pulse and
 * thresholds the waveform into echoes with range, intensity and echo pulse
 * width (section II-C, EPW paragraph).
 *
 * Conventions shared by every entry point
 *   - Every call returns a lidar_status; nothing aborts or throws across the
 *     ABI.  After a failure lidar_sim_last_error() describes it.
 *   - A handle is not thread-safe; use one handle per stream.  All GPU work is
 *     enqueued on the hipStream_t given to lidar_sim_create (passed as void*;
 *     NULL = the default stream).
 *   - Host inputs (pattern table, beam list) are copied at the call.  Device
 *     G-buffer planes are borrowed: the caller keeps them alive and unchanged
 *     until the lidar_sim_simulate_frame that reads them has completed on the
 *     stream.
 *   - Results live in library-owned device memory until
 *     lidar_sim_read_echoes copies them out.
 *
 * Raster: an equiangular azimuth/elevation image of width W and height H
 * (the reprojected spherical raster of section II-C).  Column u covers
 * azimuth [az_min + u*dphi, az_min + (u+1)*dphi), dphi = (az_max-az_min)/W;
 * row v covers elevation [el_max - (v+1)*de, el_max - v*de),
 * de = (el_max-el_min)/H; row 0 is the top.  Angles are in degrees.  The unit
 * direction of (az, el) in the sensor frame (x forward, y left, z up) is
 * (cos el cos az, cos el sin az, sin el).
 */
#ifndef LIDAR_SIM_H
#define LIDAR_SIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lidar_sim lidar_sim;   /* opaque, library-owned */

typedef int32_t lidar_status;
enum {
    LIDAR_OK = 0,
    LIDAR_E_INVALID = -1,      /* bad argument (null, out of range, non-finite) */
    LIDAR_E_STATE = -2,        /* call out of order (e.g. simulate before set_pattern) */
    LIDAR_E_HIP = -3,          /* a HIP runtime call failed; last_error has its text */
    LIDAR_E_NOMEM = -4,        /* device or host allocation failed */
    LIDAR_E_UNSUPPORTED = -5   /* valid request this build does not implement */
};

/* lidar_sim_params.flags */
enum {
    LIDAR_KEEP_WAVEFORMS = 1u,  /* keep xi_hat [n_beams][n_bins] for read_echoes */
    LIDAR_PROFILE = 2u,         /* time the footprint kernel with HIP events */
    LIDAR_AUTOTUNE = 4u,        /* batches: time the tile candidates per kernel-size
                                   class when a batch is set up, keep the fastest */
    LIDAR_DETERMINISTIC = 8u    /* bit-identical results when the same inputs are
                                   simulated again on the same device: simulate_frame
                                   (plain) runs groups of one beam whose four waves
                                   gather into histograms of their own, summed in a
                                   fixed order (about twice the frame time); the
                                   surrogate's forward, gradients and AdamW steps run
                                   without split-K atomics (the reported loss may
                                   still differ in its last bits).  simulate_batch and
                                   surrogate-mode frames return LIDAR_E_UNSUPPORTED;
                                   create does when four histograms of n_bins do not
                                   fit a workgroup's LDS. */
};

/* lidar_pattern_desc.kind */
enum { LIDAR_PATTERN_GAUSS = 1, LIDAR_PATTERN_TABLE = 2 };

/* lidar_sim_params.echo_select: which echoes a beam reports (section II-C,
 * after Alg. 1: a single echo per beam, searched for the strongest, nearest
 * or longest one).  ALL: the first max_echoes runs of xi_hat > T in time
 * order.  STRONGEST / NEAREST / LONGEST: the one run with the largest peak,
 * the first run, or the run with the largest pulse width (the first such run
 * on a tie) in slot 0; n_echoes still counts every run.  RAW_STRONGEST /
 * RAW_NEAREST: without the pulse post-processing, the bin of the raw binned
 * signal S_b xi[k] with the largest value, or the first bin, at or above T
 * (the single echo comparable to range stacking, Alg. 2): slot 0 holds it
 * as a one-bin echo (bin_first = bin_peak = bin_last, pulse width 0,
 * intensity S_b xi[k], no floor) and n_echoes is 1 or 0; kept waveforms are
 * then the raw S_b xi. */
enum { LIDAR_ECHO_ALL = 0, LIDAR_ECHO_STRONGEST = 1, LIDAR_ECHO_NEAREST = 2,
       LIDAR_ECHO_LONGEST = 3, LIDAR_ECHO_RAW_STRONGEST = 4, LIDAR_ECHO_RAW_NEAREST = 5 };

/* lidar_sim_params.range_mode: the range a pixel contributes at (section
 * II-D, rasterization; Alg. 1, pixelRangeInterval).  CENTRE: its depth, one
 * time bin.  CORRECTED: for every beam and kernel cell, the range on the
 * pixel's plane (centre point d p, normal n) along the cell's true direction
 * v = dir(az_b + m dphi, el_b - n de): d (p.n) / (v.n), the ratio limited to
 * [1/2, 2] (2 where v misses the plane's facing side); one bin per sample.
 * INTERVAL: the range interval [r0, r1] of the pixel's plane over its
 * centre and four corner rays (same ratio limit); the pixel's weight is
 * shared evenly by the bins of that interval (bins past the last one are
 * dropped), and the pixel counts (also for the sun term) when its depth is
 * valid and r0 is inside the bin window.  CORRECTED runs one beam per
 * workgroup and only in lidar_sim_simulate_frame (LIDAR_MODE_PLAIN);
 * INTERVAL also in batches. */
enum { LIDAR_RANGE_CENTRE = 0, LIDAR_RANGE_CORRECTED = 1, LIDAR_RANGE_INTERVAL = 2 };

/* lidar_sim_simulate_frame mode: the plain method, or the learned surrogate
 * with the plain method as fallback (extension) */
enum { LIDAR_MODE_PLAIN = 0, LIDAR_MODE_SURROGATE = 1 };

/* lidar_echo.flags; LIDAR_ECHO_SURROGATE marks echoes predicted by the
 * surrogate network (bin_first / bin_last then follow from the predicted
 * width) */
enum { LIDAR_ECHO_AT_FIRST_BIN = 1u, LIDAR_ECHO_AT_LAST_BIN = 2u, LIDAR_ECHO_SURROGATE = 4u };

/* Sensor and receiver parameters of one handle (copied at create). */
typedef struct {
    uint32_t n_bins;           /* R: time bins of the waveform, 1..8000 */
    uint32_t max_echoes;       /* echoes kept per beam, 1..8 (all are counted) */
    double bin_ns;             /* bin width dt (ns), > 0 */
    double threshold;          /* detection threshold T in waveform units; an echo
                                  is a maximal run of bins with xi_hat > T */
    double emit_power;         /* P_e: the footprint weights of a beam sum to P_e
                                  times the shading over its whole kernel */
    double pulse_fwhm_ns;      /* FWHM of the Gaussian pulse varpi (ns), > 0; unused
                                  with pulse_taps */
    double pulse_trunc_sigmas; /* pulse taps j with |j| <= ceil(this*sigma/dt) */
    double ambient_const;      /* constant floor added to every bin */
    double sun_irradiance;     /* E_sun, 0 = no sun term */
    double sun_dir[3];         /* unit vector towards the sun, sensor frame */
    uint32_t flags;            /* LIDAR_KEEP_WAVEFORMS | LIDAR_PROFILE | LIDAR_AUTOTUNE |
                                  LIDAR_DETERMINISTIC */
    uint32_t echo_select;      /* LIDAR_ECHO_ALL .. LIDAR_ECHO_RAW_NEAREST */
    uint32_t range_mode;       /* LIDAR_RANGE_CENTRE | _CORRECTED | _INTERVAL */
    uint32_t n_pulse_taps;     /* with pulse_taps: odd, 1..257 */
    const float* pulse_taps;   /* optional tabulated pulse varpi (host, copied at
                                  create): n_pulse_taps samples at the bin pitch,
                                  centred on the middle one, finite, >= 0, positive
                                  sum; used normalised to unit sum like the Gaussian
                                  (section II-C, EPW paragraph: varpi is the emitted
                                  pulse, in general a measured shape); NULL: the
                                  Gaussian of pulse_fwhm_ns */
} lidar_sim_params;

/* Combined emitter x collector pattern (kappa*eta, Eq. 5) and the beams. */
typedef struct {
    uint32_t kind;             /* LIDAR_PATTERN_GAUSS or LIDAR_PATTERN_TABLE */
    uint32_t n_beams;          /* >= 1 */
    double sigma_deg[2];       /* GAUSS: sigma along azimuth, elevation (deg) */
    double trunc_sigmas;       /* GAUSS: zero outside the ellipse of this radius */
    const float* table;        /* TABLE: host [ny][nx] row-major, finite, >= 0; row 0
                                  is +elevation; cell centres span +-half_deg; the
                                  pattern is bilinear between cell centres and zero
                                  outside [-half, half] */
    uint32_t nx, ny;           /* TABLE: table size, >= 2 each */
    double half_deg[2];        /* TABLE: half extent along azimuth, elevation */
    const double* beam_az_deg; /* host [n_beams] beam-centre azimuths */
    const double* beam_el_deg; /* host [n_beams] beam-centre elevations */
    const float* rx_table;     /* TABLE, optional: collector sensitivity kappa (section
                                  III-B: measured apart from the emitter) on the
                                  table's grid, finite, >= 0, copied; the sun term
                                  sums kappa Omega (rho/pi) max(0, n.s) over the
                                  kernel-window cells with kappa > 0.  NULL: kappa =
                                  K / max K over the cells with K > 0.  Not with
                                  LIDAR_MODE_SURROGATE (its floor estimate uses
                                  K / max K) */
} lidar_pattern_desc;

/* One rendered frame: six float32 device planes [height][pitch] (borrowed). */
typedef struct {
    uint32_t width, height;    /* >= 1 */
    uint64_t pitch;            /* elements between rows, >= width */
    double az_min_deg, az_max_deg, el_min_deg, el_max_deg;   /* min < max */
    const float* depth;        /* radial range (m) of the pixel-centre ray; a pixel
                                  with non-finite or <= 0 depth, or beyond the last
                                  bin, returns nothing (sky) */
    const float* reflectance;  /* Lambertian albedo rho */
    const float* retro_gain;   /* g: the BRDF is g*rho/pi (g = 1: diffuse) */
    const float* normal_x;     /* unit surface normal, sensor frame */
    const float* normal_y;
    const float* normal_z;
} lidar_gbuffer_desc;

/* One echo (section II-C, EPW paragraph). */
typedef struct {
    double range_m;            /* (c/2) (bin_peak + 1/2) dt, computed in FP64 */
    double time_ns;            /* (bin_peak + 1/2) dt */
    float intensity;           /* xi_hat at the peak minus the floor A_b */
    float pulse_width_ns;      /* t_down - t_up from linearly interpolated crossings
                                  of T between bin centres (edge time at bin 0/R-1) */
    int32_t bin_peak;          /* first bin of the run holding its maximum */
    int32_t bin_first;         /* first bin of the run (xi_hat > T) */
    int32_t bin_last;          /* last bin of the run */
    uint32_t flags;            /* LIDAR_ECHO_AT_FIRST_BIN | LIDAR_ECHO_AT_LAST_BIN */
} lidar_echo;

/* Per-beam by-products of the last frame. */
typedef struct {
    int32_t pixel_u, pixel_v;  /* pixel containing the beam centre (floor rounding;
                                  may lie outside the image) */
    float scale;               /* S_b = P_e / sum_kernel K * Omega (FP64, rounded) */
    float floor;               /* A_b = ambient_const + E_sun * sum kappa Omega
                                  (rho/pi) max(0, n.s) over the footprint */
    uint32_t samples;          /* kernel cells with K > 0 inside the image */
    uint32_t reserved;
} lidar_beam_info;

/* How a batch is scheduled (lidar_sim_batch_info). */
typedef struct {
    uint32_t n_frames;
    uint32_t group_size;       /* G: beams per workgroup item */
    uint64_t n_beams;          /* sum over frames */
    uint64_t n_items;          /* (frame, beam group) work items */
    uint64_t samples;          /* sum over frames of beam-pixel samples */
    uint32_t grid;             /* workgroups of the persistent launch */
    uint32_t graph;            /* 1 when the batch replays a captured HIP graph */
    uint32_t autotuned;        /* 1 when the tiles came from timed trials */
    uint32_t wave_items;       /* items of frames on the wave schedule (one wave per
                                  item instead of one workgroup; see the frames'
                                  schedule in lidar_sim_simulate_batch) */
    double autotune_ms;        /* time spent in the trials */
    uint32_t direct_frames;    /* frames gathered straight from their G-buffer planes
                                  without a pre-pass: those on the wave schedule
                                  whose beams hold at most one sample per two pixels
                                  (range_mode CENTRE, no kappa table) */
    uint32_t fixed_point_beams;    /* last run (synchronises): beams accumulated as
                                      64-bit fixed-point integers (range_mode CENTRE,
                                      the frame's bins spanning at most n_bins / 2) */
    uint32_t fixed_point_redone;   /* of those, beams run again with FP32 atomics
                                      because the fixed-point truncation bound
                                      exceeded 1e-6 of their waveform's maximum */
    uint32_t short_run_frames;     /* last run (synchronises): frames flagged as short-run
                                      because more than half of their valid pixels fall
                                      in another bin than their left neighbour; on the
                                      wave schedule their fixed-point gathers add every
                                      sample on its own instead of summing runs of equal
                                      bins (the group schedule keeps run sums) */
} lidar_batch_info;

/* Counters of a handle since create or the last reset_stats. */
typedef struct {
    uint64_t frames;           /* frames enqueued (simulate_frame calls plus batch frames) */
    uint64_t n_beams;          /* beams of the current pattern */
    uint64_t samples_per_frame;/* sum over beams of lidar_beam_info.samples */
    uint32_t kernel_w, kernel_h;   /* 2M+1, 2N+1 of the current kernel grid */
    uint32_t n_taps;           /* pulse taps 2J+1 */
    uint32_t reserved;
    double footprint_ms;       /* LIDAR_PROFILE: summed footprint kernel time */
    uint64_t footprint_launches;
    double prepass_ms;         /* LIDAR_PROFILE: summed G-buffer pre-pass time */
    uint64_t prepass_launches;
    double batch_ms;           /* LIDAR_PROFILE: summed batch graph time (pre-passes included) */
    uint64_t batch_launches;
    uint64_t surrogate_beams;  /* beams of LIDAR_MODE_SURROGATE frames */
    uint64_t fallback_beams;   /* of those, beams simulated by the plain path */
    double surrogate_ms;       /* LIDAR_PROFILE: summed surrogate frame time (all kernels) */
    uint64_t surrogate_frames;
} lidar_stats;

/* Create a handle with the given parameters on a HIP stream (void* =
 * hipStream_t, NULL = default stream).  *out receives the handle.  The
 * parameters are the receiver's: time bins and bin width (the range
 * resolution dr of Alg. 1), detection threshold T and pulse varpi of the EPW
 * post-processing (section II-C), emitted power, ambient and sun terms
 * (section II-A).
 * Errors: LIDAR_E_INVALID for null pointers or parameters out of range,
 * LIDAR_E_HIP, LIDAR_E_NOMEM.  No handle is returned on error. */
lidar_status lidar_sim_create(const lidar_sim_params* params, void* hip_stream,
                              lidar_sim** out);

/* Synchronise the stream and free every resource of the handle (NULL is a
 * no-op). */
lidar_status lidar_sim_destroy(lidar_sim* h);

/* Copy a pattern and beam list (host memory) into the handle.  The centred
 * kernel K = (kappa*eta)(Phi - Psi_b) of Eq. 5 is resampled on the pixel-offset
 * grid of the current raster at the next simulate_frame.
 * Errors: LIDAR_E_INVALID (null, n_beams = 0, unknown kind, sigma or half
 * extent <= 0, non-finite or negative table values, all-zero table,
 * non-finite beam angles), LIDAR_E_NOMEM, LIDAR_E_HIP. */
lidar_status lidar_sim_set_pattern(lidar_sim* h, const lidar_pattern_desc* pattern);

/* Record the device planes and raster of the next frame (borrowed): the
 * rendered ranges, BRDF terms and normals that Alg. 1 takes as input
 * (rho_hat, varrho, nu), on the equiangular raster of section II-C.
 * Errors: LIDAR_E_INVALID (null planes, zero size, pitch < width, inverted or
 * non-finite angle ranges), LIDAR_E_NOMEM, LIDAR_E_HIP. */
lidar_status lidar_sim_set_gbuffer(lidar_sim* h, const lidar_gbuffer_desc* gbuffer);

/* Enqueue one frame on the handle's stream: kernel/normalisation set-up when
 * the pattern or raster changed, the G-buffer pre-pass, then the fused
 * footprint gather / time binning / ambient / pulse / echo kernel: for
 * every beam the sum of Eq. 5 over its kernel cells (Alg. 1), the ambient
 * floor (section II-A), xi_hat = varpi * xi and the echoes (section II-C, EPW
 * paragraph).
 * mode LIDAR_MODE_SURROGATE (extension; needs surrogate weights): the
 * network predicts every beam's echoes from its inputs (see
 * lidar_sim_surrogate_features), the gate (lidar_sim_surrogate_set_gate)
 * keeps the confident ones and the plain kernel runs on the groups of the
 * others, on the device without a host round trip.  Asynchronous.
 * Errors: LIDAR_E_STATE (no pattern or G-buffer yet), LIDAR_E_INVALID (kernel
 * grid too large, pattern integral <= 0 over the kernel),
 * LIDAR_E_UNSUPPORTED (other modes), LIDAR_E_STATE (surrogate mode without
 * weights), LIDAR_E_HIP. */
lidar_status lidar_sim_simulate_frame(lidar_sim* h, uint32_t mode);

/* Copy the last frame's results out: the echoes (range, intensity, pulse
 * width; section II-C) and, on request, the waveforms xi_hat[B][R] (Alg. 1's
 * result, pulse-convolved).  echoes: [n_beams][max_echoes] (unused
 * slots zeroed), n_echoes: [n_beams] runs found (may exceed max_echoes),
 * waveforms: [n_beams][n_bins] xi_hat (needs LIDAR_KEEP_WAVEFORMS), beams:
 * [n_beams].  After a LIDAR_MODE_SURROGATE frame the waveform rows of the
 * beams whose echoes the network predicted (flag LIDAR_ECHO_SURROGATE) are
 * NaN: no waveform is computed for them.  Any output may be NULL.
 * dst_is_device != 0: the destinations
 * are device pointers and the copies are enqueued on the stream; else they are
 * host pointers and the call synchronises the stream.
 * Errors: LIDAR_E_STATE (no frame simulated), LIDAR_E_INVALID (waveforms
 * without LIDAR_KEEP_WAVEFORMS), LIDAR_E_HIP. */
lidar_status lidar_sim_read_echoes(lidar_sim* h, lidar_echo* echoes, int32_t* n_echoes,
                                   float* waveforms, lidar_beam_info* beams,
                                   int dst_is_device);

/* Extension: many frames in one launch.  frames[i] and patterns[i] describe
 * frame i (its own raster, device G-buffer planes, pattern and beams); every
 * frame uses the handle's sensor parameters.  The first call with a set of
 * descriptors copies the patterns, resamples every frame's kernel, forms the
 * beam groups of all frames into one work list ordered by estimated cost
 * (costliest first), picks each frame's schedule - the group schedule (a
 * workgroup per beam group) or, for frames whose groups mostly hold one beam,
 * the wave schedule (each wave of a workgroup takes its own groups; only with
 * 4-beam groups and n_bins <= 2048) - optionally autotunes the strip height
 * and the schedule of each kernel-size class (LIDAR_AUTOTUNE), and captures
 * the whole batch - per-frame pre-passes plus one persistent footprint launch
 * per schedule, each taking work items from a queue - into a HIP graph.  Later calls with identical descriptors (same
 * pointers, sizes and values) only replay the graph; the caller may change the
 * contents of the G-buffer planes between calls, but not the host pattern or
 * beam arrays (call lidar_sim_reset_batch after changing those in place).
 * Results of frame i are read with lidar_sim_read_batch.  Asynchronous except
 * for the first call of a new batch.
 * Errors: as set_pattern / set_gbuffer for any frame (the message names it),
 * LIDAR_E_INVALID (n_frames = 0 or a null array), LIDAR_E_HIP, LIDAR_E_NOMEM. */
lidar_status lidar_sim_simulate_batch(lidar_sim* h, const lidar_gbuffer_desc* frames,
                                      const lidar_pattern_desc* patterns, uint32_t n_frames);

/* Results of frame `frame` of the last batch, laid out as in
 * lidar_sim_read_echoes for that frame's beams.
 * Errors: LIDAR_E_STATE (no batch simulated), LIDAR_E_INVALID (frame out of
 * range, waveforms without LIDAR_KEEP_WAVEFORMS), LIDAR_E_HIP. */
lidar_status lidar_sim_read_batch(lidar_sim* h, uint32_t frame, lidar_echo* echoes,
                                  int32_t* n_echoes, float* waveforms, lidar_beam_info* beams,
                                  int dst_is_device);

/* Schedule of the current batch.  Errors: LIDAR_E_INVALID (null),
 * LIDAR_E_STATE (no batch). */
lidar_status lidar_sim_batch_info(lidar_sim* h, lidar_batch_info* out);

/* Forget the cached batch (set-up, schedule, graph); the next
 * simulate_batch sets it up again.  Errors: LIDAR_E_INVALID (null). */
lidar_status lidar_sim_reset_batch(lidar_sim* h);

/* ---- Extension: learned surrogate ----------------------------------------
 * A multilayer perceptron 1056 -> 256 -> 256 -> 256 -> 16 with GELU
 * activations (inputs 1030..1055 and outputs 13..15 are zero padding),
 * trained with AdamW on echoes that the plain path produced.  Products run
 * in BF16 on the matrix cores with FP32 accumulation; the optimiser keeps
 * FP32 weights.  Parameters are one flat FP32 vector of LIDAR_SUR_PARAMS
 * values: W1 [1056][256] (row-major, input x output), b1 [256], W2 [256][256],
 * b2, W3 [256][256], b3, W4 [256][16], b4 [16].
 * Outputs y[0..2]: existence logits of echoes 1..3 (in time order);
 * y[3..5]: peak bin minus the beam's reference bin, in units of 16 bins;
 * y[6..8]: log10(intensity / T); y[9..11]: pulse width / 4 ns; y[12]:
 * confidence logit.  Label rows use the same layout (existence as 0 / 1,
 * y[12..15] unused). */
#define LIDAR_SUR_IN 1056u
#define LIDAR_SUR_OUT 16u
#define LIDAR_SUR_PARAMS 406288u

typedef struct {
    double lr, beta1, beta2, eps;
    double weight_decay;       /* decoupled, applied to W1..W4 only */
} lidar_train_hparams;

/* Load parameters (host, n_params = LIDAR_SUR_PARAMS values, finite) and
 * reset the optimiser state (moments and step count).
 * Errors: LIDAR_E_INVALID (null, wrong count, non-finite value), LIDAR_E_HIP,
 * LIDAR_E_NOMEM. */
lidar_status lidar_sim_surrogate_set_weights(lidar_sim* h, const float* params, uint64_t n_params);

/* Copy the current FP32 parameters to the host (synchronises).
 * Errors: LIDAR_E_INVALID, LIDAR_E_STATE (no weights), LIDAR_E_HIP. */
lidar_status lidar_sim_surrogate_get_weights(lidar_sim* h, float* params, uint64_t n_params);

/* Network outputs for n input rows.  x: device, [n][1056] bfloat16 bit
 * patterns (uint16); y: device, [n][16] FP32.  Asynchronous.
 * Errors: LIDAR_E_INVALID (null, n = 0), LIDAR_E_STATE (no weights),
 * LIDAR_E_HIP, LIDAR_E_NOMEM. */
lidar_status lidar_sim_surrogate_forward(lidar_sim* h, const void* x, float* y, uint32_t n);

/* Mean loss over the n rows (the sum over echoes of the existence
 * cross-entropy and, for existing echoes, 64 (dk' - dk)^2 + (li' - li)^2 +
 * (w' - w)^2, plus the confidence cross-entropy against "every existence
 * right and every existing peak in its bin") and its gradient with respect
 * to the parameters, without an update.  labels: device [n][16]; grads:
 * device [LIDAR_SUR_PARAMS] (nullable); loss: device [1] (nullable).
 * Errors: as lidar_sim_surrogate_forward. */
lidar_status lidar_sim_surrogate_gradients(lidar_sim* h, const void* x, const float* labels,
                                           uint32_t n, float* grads, float* loss);

/* One AdamW step on the mean loss of the n rows (bias-corrected moments;
 * theta <- theta (1 - lr wd) for weights, then theta -= lr m_hat /
 * (sqrt(v_hat) + eps)).  loss: device [1] (nullable), the loss before the
 * step.  Errors: as lidar_sim_surrogate_forward, LIDAR_E_INVALID for
 * hyper-parameters out of range. */
lidar_status lidar_sim_surrogate_train_step(lidar_sim* h, const void* x, const float* labels,
                                            uint32_t n, const lidar_train_hparams* hp,
                                            float* loss);

/* The whole training loop inside the library: `steps` AdamW steps (the
 * update of surrogate_train_step) over minibatches of b = min(batch, n) of
 * the n rows (x: device [n][1056] bfloat16, labels: device [n][16]).  Rows
 * are visited in epochs e = 0, 1, ...: step t takes the next b positions p of
 * the current epoch, row P_e(p) each, and an epoch with fewer than b
 * positions left ends there (its remainder is skipped).  P_e is a
 * permutation of 0 .. n-1 computed on the device: with k = 2 h the smallest
 * even number >= 2 with 2^k >= n, a four-round Feistel network on k-bit
 * values (left and right halves of h bits; round r = 0..3 maps (L, R) to
 * (R, L xor (mix(key_r xor R) and (2^h - 1))), key_r = seed xor ((4 e + r + 1)
 * * 0x9e3779b97f4a7c15 mod 2^64), mix the SplitMix64 output function),
 * applied again while the value is >= n (cycle walking).  The learning rate
 * of step t is hp->lr + (lr_final - hp->lr) t / max(1, steps - 1).
 * losses: device [ceil(steps / log_every)] (nullable; log_every >= 1 then):
 * the loss of steps 0, log_every, 2 log_every, ... before their update.
 * Enqueued on the stream (asynchronous); the minibatch buffers are the
 * handle's.  Extension of the method (a learned surrogate).
 * Errors: LIDAR_E_INVALID (null x or labels, n = 0 or >= 2^62, batch = 0,
 * hyper-parameters as train_step, lr_final < 0 or non-finite, losses with
 * log_every = 0), LIDAR_E_STATE (no weights), LIDAR_E_NOMEM, LIDAR_E_HIP. */
lidar_status lidar_sim_surrogate_train(lidar_sim* h, const void* x, const float* labels, uint64_t n,
                                       uint32_t batch, uint32_t steps, const lidar_train_hparams* hp,
                                       double lr_final, uint64_t seed, float* losses,
                                       uint32_t log_every);

/* Gate of LIDAR_MODE_SURROGATE: a beam keeps the network's echoes when its
 * confidence sigmoid(y[12]) >= c_min and its tail estimate E_tail (the
 * largest per-bin energy the pattern outside its core box can add, from
 * super-cells of the frame) is below alpha times the margin (T - A_b, or,
 * with the floor A_b above T, the predicted peak above the floor); every
 * other beam runs the plain path.  c_min = 1 sends every beam to the plain
 * path; alpha >= 1e30 (or infinity) switches the tail check off, so c_min = 0
 * with such an alpha keeps every prediction.  Defaults: 0.5, 0.5.
 * Errors: LIDAR_E_INVALID (c_min outside [0, 1], alpha < 0 or NaN). */
lidar_status lidar_sim_surrogate_set_gate(lidar_sim* h, double c_min, double alpha);

/* Network inputs of the current frame (pattern and G-buffer as set): x,
 * device [n_beams][1056] bfloat16; aux (nullable), device [n_beams][4] FP32
 * {reference bin, E_tail, estimated floor A_b, 1 if the last surrogate
 * frame on the current pattern kept the network's echoes, else 0 (0 before
 * any surrogate frame)}; labels (nullable), device [n_beams][16] FP32 training
 * targets from the echoes of the last simulate_frame, which must have run
 * in LIDAR_MODE_PLAIN on the same inputs (existence, (peak bin - reference
 * bin) / 16, log10(max(intensity, 1e-3 T) / T), pulse width / 4 ns).
 * Asynchronous.  Errors: LIDAR_E_STATE (no pattern, G-buffer, or - for
 * labels - plain frame), LIDAR_E_INVALID, LIDAR_E_HIP, LIDAR_E_NOMEM. */
lidar_status lidar_sim_surrogate_features(lidar_sim* h, void* x, float* labels, float* aux);

/* ---- Pinhole renderings (section II-C: reprojection; section II-D: z buffer)
 * A rasterising renderer gives a pinhole image; the beams need an
 * equiangular raster.  Depth formats of lidar_pinhole_desc.depth: */
enum { LIDAR_DEPTH_RANGE = 0,        /* float radial range along the pixel's centre ray */
       LIDAR_DEPTH_EYE_Z = 1,        /* float eye-space z (along the optical axis) */
       LIDAR_DEPTH_WINDOW_F32 = 2,   /* float window depth w in [0, 1): z = n f / (f - w (f - n)) */
       LIDAR_DEPTH_WINDOW_U16 = 3,   /* uint16 window depth, w = q / 65535 */
       LIDAR_DEPTH_WINDOW_U24 = 4 }; /* uint32 holding a 24-bit window depth, w = q / (2^24 - 1) */

typedef struct {
    uint32_t width, height;    /* pinhole image, >= 1 */
    uint64_t pitch;            /* elements between rows of every plane, >= width */
    double fx, fy, cx, cy;     /* intrinsics: image x = fx X/Z + cx, y = fy Y/Z + cy in the
                                  camera frame (x right, y down, z forward); pixel (i, j)
                                  covers [i, i+1) x [j, j+1); fx, fy > 0 */
    double rot[9];             /* camera-to-sensor rotation, row-major (v_sensor = rot v_camera),
                                  orthonormal */
    uint32_t depth_format;     /* LIDAR_DEPTH_* */
    uint32_t normal_correct;   /* 1: each output range is corrected from the pinhole pixel's
                                  centre ray to the output direction with the normal,
                                  r (p.n)/(v.n), ratio limited to [1/2, 2] (section II-D) */
    double z_near, z_far;      /* clip planes of the window formats, 0 < near < far */
    const void* depth;         /* device [height][pitch], float / uint16 / uint32 by format;
                                  non-finite or <= 0 (range, z), w >= 1 or < 0: sky */
    const float* reflectance;  /* device [height][pitch] planes (borrowed until the */
    const float* retro_gain;   /*   reprojection has run on the stream) */
    const float* normal_x;     /* unit normals in the camera frame */
    const float* normal_y;
    const float* normal_z;
} lidar_pinhole_desc;

/* Reproject a pinhole rendering onto an equiangular raster (width x height
 * over [az_min, az_max] x [el_min, el_max], degrees) in library-owned device
 * planes and make them the handle's G-buffer, as lidar_sim_set_gbuffer does.
 * Every output pixel takes the pinhole pixel containing the projection of its
 * centre direction as it is (no depth interpolation, which would put ranges
 * between targets; section II-D); its depth is decoded to the radial range
 * along that pixel's centre ray (optionally corrected to the output
 * direction), reflectance and gain are copied, the normal is turned into the
 * sensor frame; pixels that see no pinhole pixel are sky.  Index and range
 * decisions in FP64.  Enqueued on the stream (asynchronous).
 * Errors: LIDAR_E_INVALID (null planes, sizes, non-positive focal lengths,
 * non-orthonormal rotation, unknown format, clip planes, raster as in
 * set_gbuffer), LIDAR_E_NOMEM, LIDAR_E_HIP. */
lidar_status lidar_sim_set_gbuffer_pinhole(lidar_sim* h, const lidar_pinhole_desc* src,
                                           uint32_t width, uint32_t height, double az_min_deg,
                                           double az_max_deg, double el_min_deg, double el_max_deg);

/* Copy the library-owned G-buffer of the last set_gbuffer_pinhole out:
 * planes [6][height][width] float32 (depth, reflectance, retro gain, normal
 * x, y, z), host (synchronises) or device (dst_is_device != 0, enqueued).
 * Errors: LIDAR_E_INVALID (null), LIDAR_E_STATE (the current G-buffer is the
 * caller's), LIDAR_E_HIP. */
lidar_status lidar_sim_read_gbuffer(lidar_sim* h, float* planes, int dst_is_device);

/* ---- Range stacking (section II-C, Alg. 2) ---------------------------------
 * The paper's second algorithm on the current G-buffer: the rendered
 * intensities rho_hat Omega (as in the footprint weights, without S_b) are
 * split into depth slices of one time bin; each slice is correlated with the
 * separable kernel K[n][m] = V[n] H[m] (kappa*eta ~ H * V, the paper's
 * speed-up for separable kernels; m along the columns, n along the rows, the
 * kernel indexed by pixel minus centre as in Eq. 5); every pixel keeps the
 * nearest slice whose correlation is >= rho_min and that value.  Slices that
 * cannot reach rho_min anywhere (largest shade of the slice times sum H
 * times sum V below rho_min) are skipped; a tile stops once every pixel has
 * its slice.  Equivalent to the beam-iteration's raw nearest echo of a beam
 * centred on the pixel with threshold rho_min S_b.
 * row_kernel: host [2M+1] H, col_kernel: host [2N+1] V (finite, >= 0;
 * M, N <= 127).  s_nearest: device [height][width] int32 slice (n_bins when no
 * slice reaches rho_min); xi_nearest: device [height][width] float (0 there).
 * Needs a G-buffer (set_gbuffer or set_gbuffer_pinhole), range_mode CENTRE.
 * Enqueued on the stream (synchronises only when the kernel factors change).
 * Errors: LIDAR_E_STATE (no G-buffer), LIDAR_E_INVALID, LIDAR_E_UNSUPPORTED
 * (other range modes), LIDAR_E_NOMEM, LIDAR_E_HIP. */
lidar_status lidar_sim_range_stacking(lidar_sim* h, const float* row_kernel, uint32_t M,
                                      const float* col_kernel, uint32_t N, double rho_min,
                                      int32_t* s_nearest, float* xi_nearest);

/* Counters since create or the last reset (synchronises profiling events).
 * Errors: LIDAR_E_INVALID (null), LIDAR_E_HIP. */
lidar_status lidar_sim_get_stats(lidar_sim* h, lidar_stats* out);

/* Zero the frame and timing counters.  Errors: LIDAR_E_INVALID (null). */
lidar_status lidar_sim_reset_stats(lidar_sim* h);

/* ---- Allocation-free frame ------------------------------------------------
 * For callers that cannot allocate device memory (serving loops and
 * harnesses that forbid hipMalloc): set_pattern + set_gbuffer +
 * simulate_frame(LIDAR_MODE_PLAIN) + read_echoes(dst_is_device = 1) in one
 * stateless call that allocates nothing.  Every device buffer of the frame
 * (pulse taps, pattern and beam copies, kernel tables, beam groups, pixel
 * records) is carved from a static device array of LIDAR_STATIC_SCRATCH_BYTES
 * that each GPU holds from the library's first use on it until the process
 * ends; frames whose buffers do not fit (about 8 bytes per pixel of the
 * width rounded up to 4, 12 with the sun term, 16 per beam, plus the kernel
 * tables: 55 MB for an 8192x512 frame with a 225x641 kernel) are rejected
 * with LIDAR_E_INVALID.  params->flags must be 0 (no kept waveforms,
 * profiling or autotuning); range modes other than LIDAR_RANGE_CENTRE and
 * an rx_table give LIDAR_E_UNSUPPORTED.  Outputs, all device pointers owned by the
 * caller: echoes [n_beams][max_echoes], n_echoes [n_beams], beams
 * [n_beams] (laid out as in lidar_sim_read_echoes).  Host inputs are copied;
 * the G-buffer planes are read on the stream.  The call synchronises the
 * stream once, after the kernel set-up (the pattern-integral check), and
 * returns with the frame's pre-pass and footprint kernel enqueued.  Every
 * call on a GPU uses that GPU's one array: calls whose work overlaps on one
 * GPU (different streams or threads) race; calls one after another on the
 * same stream do not.  Errors: as create, set_pattern, set_gbuffer and
 * simulate_frame, LIDAR_E_INVALID for null outputs or a frame too large
 * for the array; lidar_sim_last_error(NULL) describes them. */
#define LIDAR_STATIC_SCRATCH_BYTES (64u << 20)
lidar_status lidar_sim_simulate_static(const lidar_sim_params* params,
                                       const lidar_pattern_desc* pattern,
                                       const lidar_gbuffer_desc* gbuffer, void* hip_stream,
                                       lidar_echo* echoes, int32_t* n_echoes,
                                       lidar_beam_info* beams);

/* Text of the last error of the handle (handle-owned; "" if none).  With a
 * NULL handle: the last error of a failed lidar_sim_create or
 * lidar_sim_simulate_static in this thread. */
const char* lidar_sim_last_error(const lidar_sim* h);

#ifdef __cplusplus
}
#endif

#endif /* LIDAR_SIM_H */
