"""Benchmark of the plain beam-iteration hot path on one MI355X.

One step = one frame of the scanning-sensor workload (8192x512 G-buffer over
145 x 3.2 deg, road plus 24 boxes, 1 % retroreflective patches of gain 500,
16 x 1800 beams with the tabulated 256x256 elliptic pattern whose 1e-4 tails
reach 2 deg, 2048 bins of 0.5 ns, sun floor, up to 3 echoes): the G-buffer
pre-pass plus the fused footprint / time-bin / floor / pulse / echo kernel,
with the G-buffer already resident in HBM.

Prints one JSON line.  ``value`` is beam-pixel samples per second (in-image
kernel cells with K > 0, summed over beams, per frame, times frames / time).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "beam-pixel samples/s + beams/s (1 GPU), surrogate vs plain at ≤1-bin range err"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3          # vector FP32 with packed FMA (256 CU x 2.4 GHz x 256)
FP32_UNPACKED_TFLOPS = 78.6       # one FMA per lane and clock (the build does not pack)
FP64_PEAK_TFLOPS = 78.6
LDS_PEAK_GBS = 256 * 2.4 * 128.0  # 128 B per clock per CU
TA_PEAK_GBS = 256 * 2.4 * 64.0    # vector-memory data path: 64 B per clock per CU
# algorithmic FP32 operations per beam-pixel sample: the weight
# S_b * K * Omega * beta * cos(theta) / d^2 (5 multiplies) and its add into the
# time bin; with the sun term one more multiply-add (kappa times the pixel's
# sun shading Omega (rho/pi) max(0, n.s), added into the floor)
FLOPS_PER_SAMPLE = 6
FLOPS_PER_SAMPLE_SUN = 2
# FP64 operations of a sample's corrected range (range_mode CORRECTED): the
# normal's azimuth components (2 x 3), p.n (3), the turned direction's v.n
# (3 + 3 + 3 + 3), the ratio and its limits (3), range and bin (3)
FP64_PER_CORRECTED_SAMPLE = 27


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle timing (for profiler runs)")
    ap.add_argument("--traffic", type=str,
                    default=os.path.join(ROOT, "profiles", "k_footprint_scan8192x512_traffic.json"),
                    help="JSON file with per-dispatch HBM bytes of the footprint kernel "
                         "(ignored when it was taken with another kernel source)")
    ap.add_argument("--counters", type=str,
                    default=os.path.join(ROOT, "profiles", "k_footprint_scan8192x512_counters.json"),
                    help="JSON file with per-dispatch SQ/TA counters of the footprint kernel "
                         "(ignored when taken with another kernel source)")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the measurements of the options and of range stacking")
    ap.add_argument("--rows-only", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-frame batch measurement")
    ap.add_argument("--batch-only", action="store_true",
                    help="only measure the 64-frame batch (for profiler runs)")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--batch-scene", choices=("all", "iid", "road"), default="all",
                    help="restrict the batch to its i.i.d.-surface or its road frames (profiling)")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the surrogate training and inference measurement")
    ap.add_argument("--surrogate-only", action="store_true")
    ap.add_argument("--sur-train-frames", type=int, default=16)
    ap.add_argument("--sur-steps", type=int, default=3000)
    ap.add_argument("--sur-eval-frames", type=int, default=32)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times) and exit: the "
                         "reference for scaling the HBM byte counters")
    return ap.parse_args()


def copy_calibration(mib: int):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4}), flush=True)


def _profile_record(path):
    """A profiles/ JSON record, or None when it was taken with a different
    kernel source (its sha256 is stored with it)."""
    import hashlib
    if not path or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, rec.get("source", ""))
    if not os.path.exists(src):
        return None
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec.get("source_sha256"):
            return None
    return rec


def measured_traffic(path):
    """HBM bytes per launch of the footprint kernel from rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes (scaled by a plain-copy calibration), or None when the
    counters were taken with a different kernel source."""
    rec = _profile_record(path)
    return rec.get("bytes_per_launch") if rec else None


VMEM_BYTES_PER_SAMPLE = 7.0       # 8 B pixel record + 4 B sun shading per 4 beams, 4 B kernel per beam


def unit_figures(path, ms, samples):
    """LDS and vector-memory figures of the footprint kernel at the measured
    launch time, from its counter record (per dispatch, one rocprofv3 --pmc
    pass of the same command): LDS bytes, at least 4 per lane of every LDS
    instruction (SQ_INSTS_LDS x 64 x 4), against 128 B per clock and CU, with
    the LDS busy and bank-conflict fractions; algorithmic bytes through the
    vector-memory path (VMEM_BYTES_PER_SAMPLE per sample) against 64 B per
    clock and CU, with the texture-address unit's busy fraction
    (GRBM_TA_BUSY / GRBM_GUI_ACTIVE); VALU busy (SQ_INSTS_VALU x 4 cycles per
    wave64 instruction over 1024 SIMDs)."""
    rec = _profile_record(path)
    if not rec or not ms:
        return None
    c = rec["counters"]
    cycles = c["GRBM_GUI_ACTIVE"] / 8.0            # summed over the 8 XCDs
    lds_bytes = c["SQ_INSTS_LDS"] * 64 * 4
    vmem_bytes = samples * VMEM_BYTES_PER_SAMPLE
    t = ms * 1e-3
    return {
        "lds": {"min_bytes_per_launch": lds_bytes, "achieved": lds_bytes / t / 1e9,
                "peak": LDS_PEAK_GBS, "unit": "GB/s", "frac": lds_bytes / t / 1e9 / LDS_PEAK_GBS,
                "busy_frac": c["SQ_LDS_IDX_ACTIVE"] / (cycles * 256),
                "bank_conflict_frac_of_active": c["SQ_LDS_BANK_CONFLICT"] / max(1.0, c["SQ_LDS_IDX_ACTIVE"])},
        "vmem": {"bytes_per_launch": vmem_bytes, "achieved": vmem_bytes / t / 1e9,
                 "peak": TA_PEAK_GBS, "unit": "GB/s", "frac": vmem_bytes / t / 1e9 / TA_PEAK_GBS,
                 "ta_busy_frac": c["GRBM_TA_BUSY"] / c["GRBM_GUI_ACTIVE"]},
        "valu_busy_frac": c["SQ_INSTS_VALU"] * 4 / (cycles * 1024),
        "counter_source": "profiles/" + os.path.basename(path)}


def precision_report(w, planes, n_sample=240, seed=7):
    """Error of every output field against the FP64 oracle on a seeded sample
    of the frame's beams (the GPU runs the whole frame with waveforms kept)."""
    import numpy as np
    import torch
    import oracle
    import scenes
    import paper_2512_05932_amd as lidar
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(w.pattern.n_beams, size=min(n_sample, w.pattern.n_beams),
                             replace=False))
    sim = lidar.LidarSim(w.params, stream=torch.cuda.current_stream(), keep_waveforms=True)
    sim.set_pattern(w.pattern)
    sim.set_gbuffer(w.gbuffer.raster, planes)
    sim.simulate_frame()
    got = sim.read(waveforms=True)
    sim.close()
    sub = scenes.subset_beams(w, idx)
    ref = oracle.simulate(w.gbuffer, sub.pattern, sub.params, want_xi=False)
    T, E = w.params.threshold, w.params.max_echoes
    peak = ref.xi_hat.max(axis=1)
    wav = got["waveforms"][idx].astype(np.float64)
    wave_err = np.abs(wav - ref.xi_hat).max(axis=1) / peak
    amb = (np.abs(ref.xi_hat - T) <= 1e-5 * peak[:, None]).any(axis=1)
    cnt = got["n_echoes"][idx]
    bi = got["beams"][idx]
    rng_bins, int_err, epw_err, n_e = [], [], [], 0
    for k in np.nonzero(~amb)[0]:
        for i in range(min(int(ref.n_echoes[k]), E)):
            ge, re = got["echoes"][idx[k], i], ref.echoes[k, i]
            n_e += 1
            rng_bins.append(abs(int(ge["bin_peak"]) - int(re["bin_peak"])))
            int_err.append(abs(float(ge["intensity"]) - re["intensity"]) / peak[k])
            epw_err.append(abs(float(ge["pulse_width_ns"]) - re["pulse_width_ns"]))
    return {"beams": int(len(idx)), "threshold_ambiguous_beams": int(amb.sum()),
            "waveform_max_rel_err": float(wave_err.max()),
            "waveform_mean_rel_err": float(wave_err.mean()),
            "echo_count_exact_frac": float((cnt[~amb] == ref.n_echoes[~amb]).mean()),
            "echoes_compared": n_e,
            "range_max_bin_err": int(max(rng_bins) if rng_bins else 0),
            "range_exact_frac": float(np.mean(np.array(rng_bins) == 0) if rng_bins else 1.0),
            "intensity_max_rel_err": float(max(int_err) if int_err else 0.0),
            "epw_max_abs_err_ns": float(max(epw_err) if epw_err else 0.0),
            "floor_max_rel_err": float((np.abs(bi["floor"] - ref.floor) /
                                        np.maximum(ref.floor, 1e-300)).max()),
            "scale_max_rel_err": float((np.abs(bi["scale"] - ref.scale) / ref.scale).max()),
            "pixel_exact": bool(np.array_equal(bi["pixel_u"], ref.pixel[:, 0]) and
                                np.array_equal(bi["pixel_v"], ref.pixel[:, 1])),
            "samples_exact": bool(np.array_equal(bi["samples"], ref.samples)),
            "reference": "FP64 CPU oracle"}


def cpu_baseline(w):
    """The FP64 oracle as it stands, on the host cores: one full frame with
    every core, plus a 1-core rate on a beam sample."""
    import numpy as np
    import oracle
    cores = os.cpu_count() or 1
    env_threads = os.environ.get("OMP_NUM_THREADS")
    threads = int(env_threads) if env_threads and env_threads.isdigit() else cores
    t0 = time.perf_counter()
    res = oracle.simulate(w.gbuffer, w.pattern, w.params, want_xi=False, want_xi_hat=False,
                          n_threads=threads)
    dt = time.perf_counter() - t0
    samples = float(res.samples.sum())
    import scenes
    sub = scenes.subset_beams(w, np.arange(0, w.pattern.n_beams, 97))
    t1 = time.perf_counter()
    r1 = oracle.simulate(w.gbuffer, sub.pattern, sub.params, want_xi=False, want_xi_hat=False,
                         n_threads=1)
    d1 = time.perf_counter() - t1
    return {"value": samples / dt, "unit": "beam-pixel samples/s", "cores": threads,
            "kind": "oracle",
            "sample": f"one full frame ({w.pattern.n_beams} beams, {samples:.3e} samples, "
                      f"{dt:.2f} s) on {threads} threads",
            "beams_per_s": w.pattern.n_beams / dt,
            "one_core_samples_per_s": float(r1.samples.sum()) / d1,
            "one_core_sample": f"{sub.pattern.n_beams} beams (every 97th), {d1:.2f} s"}


def batch_report(args):
    """The 64-frame uneven batch (512x256 to 4096x2048 G-buffers, grid /
    Lissajous / jittered steering, 5k-100k beams and 20-20,000 pixel
    footprints per frame) as one replayed HIP graph: pre-passes, queue reset
    and the persistent footprint launch.  Set-up and autotuning happen in the
    first call and are reported apart; the timed replays start with the
    G-buffers resident in HBM."""
    import torch
    import scenes
    import paper_2512_05932_amd as lidar
    t0 = time.perf_counter()
    bw = scenes.frame_batch(args.seed)
    if args.batch_scene != "all":
        bw = scenes.BatchWorkload(f"{bw.name}-{args.batch_scene}",
                                  [f for f in bw.frames if f.meta["scene"] == args.batch_scene], bw.params)
    gen_s = time.perf_counter() - t0
    planes = [lidar.upload_gbuffer(f.gbuffer, "cuda:0") for f in bw.frames]
    stream = torch.cuda.current_stream()
    sim = lidar.LidarSim(bw.params, stream=stream, profile=True, autotune=True)
    batch = lidar.Batch([(f.gbuffer.raster, p) for f, p in zip(bw.frames, planes)],
                        [f.pattern for f in bw.frames])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.simulate_batch(batch)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t1
    info = sim.batch_info()
    sim.simulate_batch(batch)          # warm replay
    torch.cuda.synchronize()
    sim.reset_stats()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.batch_steps):
        sim.simulate_batch(batch)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.batch_steps
    st = sim.stats()
    fixed = sim.batch_info()              # counters of the last replay
    echoes = sum(int(sim.read_batch(i, beams=False)["n_echoes"].sum())
                 for i in range(len(bw.frames)))
    sim.close()
    del planes
    torch.cuda.empty_cache()
    # compulsory HBM bytes: every G-buffer read once (24 B per pixel), echoes
    # and counts written
    E = bw.params.max_echoes
    compulsory = sum(24 * f.gbuffer.depth.size + f.pattern.n_beams * (40 * E + 4) for f in bw.frames)
    gbs = compulsory / (ms * 1e-3) / 1e9
    return {"workload": bw.name, "frames": info["n_frames"], "beams": info["n_beams"],
            "samples": info["samples"], "work_items": info["n_items"],
            "wave_schedule_items": info["wave_items"], "direct_frames": info["direct_frames"],
            "fixed_point_beams": fixed["fixed_point_beams"], "fixed_point_redone": fixed["fixed_point_redone"],
            "short_run_frames": fixed["short_run_frames"],
            "grid": info["grid"], "ms_per_batch": ms,
            "compulsory_bytes": compulsory, "achieved_GBs": gbs, "peak_GBs": HBM_PEAK_GBS,
            "hbm_frac": gbs / HBM_PEAK_GBS,
            "graph_ms_profiled": st["batch_ms"] / max(1, st["batch_launches"]),
            "samples_per_s": info["samples"] / (ms * 1e-3),
            "beams_per_s": info["n_beams"] / (ms * 1e-3),
            "frames_per_s": info["n_frames"] / (ms * 1e-3),
            "echoes": echoes, "steps": args.batch_steps,
            "setup_s": setup_s, "autotune_ms": info["autotune_ms"], "generate_s": gen_s}


def prepass_bytes(w):
    """Algorithmic HBM bytes of one pre-pass launch: the depth plane for every
    pixel, the other five planes (reflectance, gain, normal) for pixels with a
    valid in-range depth, and the 4-column pixel records (8 B, plus 4 B of sun
    shading with the sun term) for every pixel of the padded width."""
    import numpy as np
    d = w.gbuffer.depth.astype(np.float64)
    H, W = d.shape
    to_bin = 2.0 / (299792458.0 * w.params.bin_ns * 1e-9)
    with np.errstate(invalid="ignore"):
        valid = np.isfinite(d) & (d > 0) & (np.floor(d * to_bin) < w.params.n_bins)
    W4 = (W + 3) // 4 * 4
    out = 8 + (4 if w.params.sun_irradiance != 0.0 else 0)
    return 4 * d.size + 20 * int(valid.sum()) + out * W4 * H


def touched_pixels(w):
    """Pixels of a frame inside some beam's truncated Gaussian footprint
    (host geometry: the containing pixel of each beam and the cells of the
    3-sigma ellipse on the pixel-offset grid)."""
    import numpy as np
    r = w.gbuffer.raster
    dphi = (r.az_max - r.az_min) / r.width
    de = (r.el_max - r.el_min) / r.height
    sx, sy = w.pattern.sigma_deg
    t = w.pattern.trunc_sigmas
    M, N = int(t * sx / dphi), int(t * sy / de)
    m, n = np.meshgrid(np.arange(-M, M + 1), np.arange(-N, N + 1))
    cell = (m * dphi / sx) ** 2 + (n * de / sy) ** 2 <= t * t
    mask = np.zeros((r.height, r.width), dtype=bool)
    u = np.floor((w.pattern.beam_az - r.az_min) / dphi).astype(np.int64)
    v = np.floor((r.el_max - w.pattern.beam_el) / de).astype(np.int64)
    mm, nn = m[cell], n[cell]
    for ub, vb in zip(u, v):
        uu, vv = ub + mm, vb + nn
        ok = (uu >= 0) & (uu < r.width) & (vv >= 0) & (vv < r.height)
        mask[vv[ok], uu[ok]] = True
    return int(mask.sum())


def replayed_small_report(args, n_frames=32, steps=20):
    """n_frames 1024x512 frames of i.i.d. surfaces, each with 1000 Gaussian
    beams of 89 cells, as one replayed graph.  Two byte counts against 8 TB/s:
    every G-buffer read once (24 B per pixel) with the echoes and counts
    written, and only the pixels some beam's kernel touches (the frames are
    gathered straight from their planes, so the rest is never read)."""
    import torch
    import scenes
    import paper_2512_05932_amd as lidar
    frames = [scenes.iid_frame(args.seed + i) for i in range(n_frames)]
    planes = [lidar.upload_gbuffer(f.gbuffer, "cuda:0") for f in frames]
    stream = torch.cuda.current_stream()
    sim = lidar.LidarSim(frames[0].params, stream=stream)
    batch = lidar.Batch([(f.gbuffer.raster, p) for f, p in zip(frames, planes)],
                        [f.pattern for f in frames])
    sim.simulate_batch(batch)
    sim.simulate_batch(batch)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        sim.simulate_batch(batch)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    info = sim.batch_info()
    sim.close()
    del planes
    torch.cuda.empty_cache()
    E = frames[0].params.max_echoes
    compulsory = sum(24 * f.gbuffer.depth.size + f.pattern.n_beams * (40 * E + 4) for f in frames)
    gbs = compulsory / (ms * 1e-3) / 1e9
    touched = sum(24 * touched_pixels(f) + f.pattern.n_beams * (40 * E + 4) for f in frames)
    return {"workload": f"{n_frames} x 1024x512 i.i.d. frames (40x25 beams), one graph replay",
            "ms_per_batch": ms, "compulsory_bytes": compulsory, "achieved_GBs": gbs,
            "peak_GBs": HBM_PEAK_GBS, "frac": gbs / HBM_PEAK_GBS,
            "touched_bytes": touched, "touched_GBs": touched / (ms * 1e-3) / 1e9,
            "touched_frac": touched / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "direct_frames": info["direct_frames"],
            "samples_per_s": info["samples"] / (ms * 1e-3),
            "beams_per_s": info["n_beams"] / (ms * 1e-3), "steps": steps}


def _timed(stream, fn, n):
    import torch
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(n):
        fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / n


def rows_report(args, steps=10):
    """The path's options on the scanning workload (range-corrected and
    interval ranges, raw and strongest echo selection), range stacking
    (Alg. 2) on its workload, and the reprojection of a pinhole rendering;
    per row the time per frame and the roofline of its dominant kernel."""
    from dataclasses import replace
    import numpy as np
    import torch
    import scenes
    import paper_2512_05932_amd as lidar
    stream = torch.cuda.current_stream()
    out = {}
    w = scenes.road_scan(args.seed)
    planes = lidar.upload_gbuffer(w.gbuffer, "cuda:0")
    sun = w.params.sun_irradiance != 0.0
    modes = (("range_corrected", dict(range_mode=lidar.LIDAR_RANGE_CORRECTED)),
             ("range_interval", dict(range_mode=lidar.LIDAR_RANGE_INTERVAL)),
             ("echo_strongest", dict(echo_select=lidar.LIDAR_ECHO_STRONGEST)),
             ("echo_raw_nearest", dict(echo_select=lidar.LIDAR_ECHO_RAW_NEAREST)))
    for name, kw in modes:
        prm = replace(w.params, **kw)
        sim = lidar.LidarSim(prm, stream=stream, profile=True)
        sim.set_pattern(w.pattern)
        sim.set_gbuffer(w.gbuffer.raster, planes)
        for _ in range(2):
            sim.simulate_frame()
        torch.cuda.synchronize()
        sim.reset_stats()
        ms = _timed(stream, sim.simulate_frame, steps)
        st = sim.stats()
        res = sim.read(beams=False)
        sim.close()
        fp = st["footprint_ms"] / max(1, st["footprint_launches"])
        samples = st["samples_per_frame"]
        flops = samples * (FLOPS_PER_SAMPLE + (FLOPS_PER_SAMPLE_SUN if sun else 0))
        rec = {"workload": w.name, "ms_per_frame": ms, "footprint_ms": fp,
               "samples_per_s": samples / (ms * 1e-3), "echoes_per_frame": int(res["n_echoes"].sum()),
               "roofline": {"bound": "alu", "kernel": "k_footprint_corr" if "corrected" in name
                            else "k_footprint", "achieved": flops / (fp * 1e-3) / 1e12,
                            "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                            "frac": flops / (fp * 1e-3) / 1e12 / FP32_PEAK_TFLOPS}}
        if "corrected" in name:
            f64 = samples * FP64_PER_CORRECTED_SAMPLE / (fp * 1e-3) / 1e12
            rec["roofline_fp64"] = {"bound": "alu", "achieved": f64, "peak": FP64_PEAK_TFLOPS,
                                    "unit": "TFLOP/s", "frac": f64 / FP64_PEAK_TFLOPS,
                                    "fp64_ops_per_sample": FP64_PER_CORRECTED_SAMPLE}
        out[name] = rec
    del planes
    # range stacking (Alg. 2) on the paper's setting
    sw = scenes.range_stacking_scene(args.seed)
    H, W = sw.gbuffer.depth.shape
    planes = lidar.upload_gbuffer(sw.gbuffer, "cuda:0")
    s_out = torch.empty((H, W), dtype=torch.int32, device="cuda")
    x_out = torch.empty((H, W), dtype=torch.float32, device="cuda")
    sim = lidar.LidarSim(sw.params, stream=stream)
    sim.set_gbuffer(sw.gbuffer.raster, planes)
    run = lambda: sim.range_stacking(sw.row_kernel, sw.col_kernel, sw.rho_min, s_out, x_out)
    run()
    ms = _timed(stream, run, steps)
    sim.close()
    s_np = s_out.cpu().numpy()
    d = sw.gbuffer.depth.astype(np.float64)
    with np.errstate(invalid="ignore"):
        b = np.floor(d * 2.0 / (299792458.0 * sw.params.bin_ns * 1e-9))
    present = np.unique(b[np.isfinite(b) & (b < sw.params.n_bins)]).size
    KW, KH = sw.row_kernel.size, sw.col_kernel.size
    ps = float(W * H) * present
    eff = ps * 2.0 * (KW + KH) / (ms * 1e-3) / 1e12
    out["range_stacking"] = {
        "workload": sw.name, "ms_per_frame": ms, "slices": int(sw.params.n_bins),
        "slices_present": int(present), "pixels_with_slice": float((s_np < sw.params.n_bins).mean()),
        "pixel_slices_per_s": ps / (ms * 1e-3),
        "roofline": {"bound": "alu", "kernel": "k_range_stacking", "achieved": eff,
                     "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": eff / FP32_PEAK_TFLOPS,
                     "note": "algorithmic: 2 (KW + KH) FLOP per pixel and present slice (separable "
                             "correlation of every present slice over the whole image); the kernel "
                             "skips tiles without the slice and stops tiles once resolved"},
        "paper_context": "Alg. 2: 4.3 s per frame (1200 slices), 0.8 s with slice skipping, "
                         "OpenCV on a 14-core i7-13800H"}
    del planes
    # reprojection of a pinhole rendering (z buffer, 24 bits) onto 4096 x 1024
    ph = scenes.pinhole_render(args.seed, width=1920, height=1080, hfov_deg=90.0, pitch_deg=-2.0,
                               fmt=4, near=0.3, far=1000.0, n_boxes=16)
    dev = [torch.from_numpy(np.ascontiguousarray(a).view(np.int32) if a.dtype == np.uint32
                            else np.ascontiguousarray(a)).to("cuda")
           for a in (ph.depth, ph.reflectance, ph.retro_gain, ph.normal[0], ph.normal[1], ph.normal[2])]
    r = scenes.Raster(4096, 1024, -45.0, 45.0, -22.5, 22.5)
    sim = lidar.LidarSim(w.params, stream=stream)
    run = lambda: sim.set_gbuffer_pinhole(ph, dev, r)
    run()
    ms = _timed(stream, run, steps)
    sim.close()
    nbytes = 24.0 * r.width * r.height * 2          # six planes written, six gathered
    gbs = nbytes / (ms * 1e-3) / 1e9
    out["reproject"] = {"workload": "pinhole 1920x1080 (90 deg, 24-bit z) -> 4096x1024 equiangular",
                        "ms": ms, "pixels_per_s": r.width * r.height / (ms * 1e-3),
                        "roofline": {"bound": "hbm", "kernel": "k_reproject", "achieved": gbs,
                                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                                     "bytes_per_launch": nbytes}}
    return out


def clopper_pearson(k, n, conf=0.95):
    """Exact two-sided binomial interval of a rate k / n."""
    from scipy.stats import beta
    if n == 0:
        return (None, None)
    a = 1.0 - conf
    lo = 0.0 if k == 0 else float(beta.ppf(a / 2, k, n - k + 1))
    hi = 1.0 if k == n else float(beta.ppf(1 - a / 2, k + 1, n - k))
    return (lo, hi)


SUR_FLOPS_PER_BEAM = 2 * (1056 * 256 + 2 * 256 * 256 + 256 * 16)   # the network's products
BF16_PEAK_TFLOPS = 2500.0


def surrogate_report(args, pattern="gauss", train_frames=None, steps=None, eval_frames=None,
                     oracle_sample=2000, gate=(0.95, 0.5)):
    """Surrogate on scanning frames (road + boxes, 8192x512, 64 x 2000 = 128k
    beams): the network is trained from scratch by the library's kernels on
    the plain path's echoes of ``train_frames`` frames (AdamW, batch 4096),
    then held-out frames are simulated in plain and in surrogate mode (gate
    c_min = 0.95, alpha = 0.5) with the G-buffers resident; reported: both
    times, speed-up, fallback fraction, agreement within one bin with the
    plain path (all beams) and with the FP64 oracle (a beam sample)."""
    import numpy as np
    import torch
    from concurrent.futures import ThreadPoolExecutor
    import scenes
    import paper_2512_05932_amd as lidar
    from paper_2512_05932_amd import surrogate as sur
    train_frames = train_frames or args.sur_train_frames
    steps = steps or args.sur_steps
    eval_frames = eval_frames or args.sur_eval_frames
    seeds = [1000 + i for i in range(train_frames)] + [args.seed + i for i in range(eval_frames)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(16) as ex:
        ws = list(ex.map(lambda s: scenes.surrogate_frame(s, pattern), seeds))
    gen_s = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    sim = lidar.LidarSim(ws[0].params, stream=stream, profile=True)
    planes = [lidar.upload_gbuffer(w.gbuffer, "cuda:0") for w in ws]
    t0 = time.perf_counter()
    X, L = sur.make_dataset(sim, [(w.gbuffer.raster, p, w.pattern)
                                  for w, p in zip(ws[:train_frames], planes)])
    torch.cuda.synchronize()
    data_s = time.perf_counter() - t0
    sim.set_weights(scenes.surrogate_init(0))
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    losses = sur.train(sim, X, L, steps, batch=4096, lr=2e-3, log_every=max(1, steps // 5))
    ev1.record(stream)
    torch.cuda.synchronize()
    train_ms = ev0.elapsed_time(ev1)
    n_rows = int(X.shape[0])
    del X, L
    sim.set_gate(*gate)
    res = []
    oracle_ok, oracle_acc, tail_dec = [], [], []
    nb = ws[-1].pattern.n_beams
    xbuf = torch.empty((nb, 1056), dtype=torch.int16, device="cuda")
    auxbuf = torch.empty((nb, 4), dtype=torch.float32, device="cuda")
    for w, p in zip(ws[train_frames:], planes[train_frames:]):
        sim.set_pattern(w.pattern)
        sim.set_gbuffer(w.gbuffer.raster, p)
        times = {}
        outs = {}
        for mode in (lidar.LIDAR_MODE_PLAIN, lidar.LIDAR_MODE_SURROGATE):
            for _ in range(2):
                sim.simulate_frame(mode)
            torch.cuda.synchronize()
            sim.reset_stats()
            ev0.record(stream)
            for _ in range(10):
                sim.simulate_frame(mode)
            ev1.record(stream)
            torch.cuda.synchronize()
            times[mode] = ev0.elapsed_time(ev1) / 10
            outs[mode] = sim.read()
            st = sim.stats()
        ag = sur.echo_agreement(outs[lidar.LIDAR_MODE_PLAIN], outs[lidar.LIDAR_MODE_SURROGATE])
        res.append({"seed": w.meta["seed"], "plain_ms": times[lidar.LIDAR_MODE_PLAIN],
                    "surrogate_ms": times[lidar.LIDAR_MODE_SURROGATE],
                    "fallback": st["fallback_beams"] / max(1, st["surrogate_beams"]),
                    "within_1_bin_vs_plain": ag["within_1_bin"]})
        if oracle_sample and not args.no_cpu_baseline:
            # a sample of every evaluated frame's beams against the FP64
            # oracle (with the pattern's tails, and for a table pattern also
            # without them: beams whose echoes change are decided by the tails)
            import oracle
            k = -(-oracle_sample // eval_frames)
            idx = np.sort(np.random.default_rng(w.meta["seed"] + 3).choice(w.pattern.n_beams, k,
                                                                           replace=False))
            sub = scenes.subset_beams(w, idx).pattern
            ref = oracle.simulate(w.gbuffer, sub, w.params, want_xi=False, want_xi_hat=False)
            got = outs[lidar.LIDAR_MODE_SURROGATE]
            acc = sur.echo_agreement({"n_echoes": ref.n_echoes, "echoes": ref.echoes},
                                     {"n_echoes": got["n_echoes"][idx], "echoes": got["echoes"][idx]},
                                     per_beam=True)
            # the gate's decisions of the last surrogate frame (aux column 3)
            sim.surrogate_features(xbuf, aux=auxbuf)
            accepted = auxbuf[:, 3].cpu().numpy()[idx] > 0.5
            oracle_ok.append(acc)
            oracle_acc.append(accepted)
            if pattern == "table":
                core = scenes.core_only_pattern(sub)
                ref0 = oracle.simulate(w.gbuffer, core, w.params, want_xi=False, want_xi_hat=False)
                tail_dec.append(~sur.echo_agreement({"n_echoes": ref.n_echoes, "echoes": ref.echoes},
                                                    {"n_echoes": ref0.n_echoes, "echoes": ref0.echoes},
                                                    per_beam=True))
    # the fused network kernel alone, on the last frame's inputs
    B = ws[-1].pattern.n_beams
    xin = xbuf
    yout = torch.empty((B, 16), dtype=torch.float32, device="cuda")
    sim.surrogate_features(xin)
    sim.surrogate_forward(xin, yout)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(10):
        sim.surrogate_forward(xin, yout)
    ev1.record(stream)
    torch.cuda.synchronize()
    mlp_ms = ev0.elapsed_time(ev1) / 10
    sim.close()
    del planes
    torch.cuda.empty_cache()
    tp = float(np.mean([r["plain_ms"] for r in res]))
    ts = float(np.mean([r["surrogate_ms"] for r in res]))
    orc = None
    if oracle_ok:
        ok = np.concatenate(oracle_ok)
        accd = np.concatenate(oracle_acc)
        lo, hi = clopper_pearson(int(ok.sum()), ok.size)
        orc = {"beams": int(ok.size), "within_1_bin": float(ok.mean()),
               "clopper_pearson_95": [lo, hi],
               "accepted_beams": int(accd.sum()),
               "within_1_bin_accepted": float(ok[accd].mean()) if accd.any() else None,
               "clopper_pearson_95_accepted": list(clopper_pearson(int(ok[accd].sum()), int(accd.sum())))
               if accd.any() else None}
        if tail_dec:
            td = np.concatenate(tail_dec)
            orc["tail_decided"] = float(td.mean())
            orc["tail_decided_among_fallback"] = float(td[~accd].mean()) if (~accd).any() else None
            orc["tail_decided_among_accepted"] = float(td[accd].mean()) if accd.any() else None
    mlp_tflops = SUR_FLOPS_PER_BEAM * B / (mlp_ms * 1e-3) / 1e12
    return {"workload": ws[-1].name, "beams_per_frame": B, "pattern": pattern,
            "train_frames": train_frames, "train_rows": n_rows, "train_steps": steps,
            "batch": 4096, "train_ms": train_ms, "train_rows_per_s": steps * 4096 / (train_ms * 1e-3),
            "losses": losses, "gate": {"c_min": gate[0], "alpha": gate[1]},
            "eval": res, "plain_ms": tp, "surrogate_ms": ts, "speedup": tp / ts,
            "beams_per_s_surrogate": B / (ts * 1e-3), "beams_per_s_plain": B / (tp * 1e-3),
            "fallback": float(np.mean([r["fallback"] for r in res])),
            "within_1_bin_vs_plain": float(np.min([r["within_1_bin_vs_plain"] for r in res])),
            "within_1_bin_vs_oracle": orc["within_1_bin"] if orc else None,
            "oracle": orc, "oracle_sample_beams": orc["beams"] if orc else 0,
            "mlp_ms": mlp_ms, "mlp_tflops": mlp_tflops, "mlp_frac_bf16_peak": mlp_tflops / BF16_PEAK_TFLOPS,
            "generate_s": gen_s, "dataset_s": data_s}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the engine "
              "has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    import numpy as np
    import torch
    import scenes
    import paper_2512_05932_amd as lidar

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.batch_only:
        print(json.dumps({"batch": batch_report(args)}), flush=True)
        return
    if args.surrogate_only:
        print(json.dumps({"surrogate": surrogate_report(args, oracle_sample=10000),
                          "surrogate_table_pattern": surrogate_report(args, "table", oracle_sample=10000)}),
              flush=True)
        return
    if args.rows_only:
        print(json.dumps({"rows": rows_report(args)}), flush=True)
        return
    w = scenes.road_scan(args.seed)
    stream = torch.cuda.current_stream()
    planes = lidar.upload_gbuffer(w.gbuffer, "cuda:0")
    sim = lidar.LidarSim(w.params, stream=stream, profile=True)
    sim.set_pattern(w.pattern)
    sim.set_gbuffer(w.gbuffer.raster, planes)
    for _ in range(args.warmup):
        sim.simulate_frame()
    torch.cuda.synchronize()
    sim.reset_stats()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        sim.simulate_frame()
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    st = sim.stats()
    out = sim.read(beams=True)
    sim.close()
    ms = total_ms / args.steps
    samples = st["samples_per_frame"]
    B = w.pattern.n_beams
    fp_ms = st["footprint_ms"] / max(1, st["footprint_launches"])
    sun = w.params.sun_irradiance != 0.0
    flops = samples * (FLOPS_PER_SAMPLE + (FLOPS_PER_SAMPLE_SUN if sun else 0))
    achieved = flops / (fp_ms * 1e-3) / 1e12
    traffic = measured_traffic(args.traffic)
    rec = {
        "metric": METRIC,
        "value": samples * args.steps / (total_ms * 1e-3),
        "unit": "beam-pixel samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "image": "8192x512", "fov_deg": "145x3.2",
                   "beams": B, "pattern": "table 256x256, FWHM 0.1x0.8 deg, 1e-4 tails to 2 deg",
                   "bins": w.params.n_bins, "bin_ns": w.params.bin_ns,
                   "max_echoes": w.params.max_echoes, "samples_per_frame": samples,
                   "seed": args.seed},
        "beams_per_s": B * args.steps / (total_ms * 1e-3),
        "echoes_per_frame": int(out["n_echoes"].sum()),
        "echo_stats": {"beams_with_echoes": float((out["n_echoes"] > 0).mean()),
                       "beams_floor_above_threshold": float(
                           (out["beams"]["floor"] > w.params.threshold).mean()),
                       "runs_touching_both_edges": float(
                           ((out["echoes"]["flags"][:, 0] == 3) & (out["n_echoes"] > 0)).mean())},
        "roofline": {"bound": "alu", "kernel": "k_footprint", "achieved": achieved,
                     "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS, "traffic": traffic,
                     "avg_launch_ms": fp_ms, "flops_per_launch": flops,
                     "flops_per_sample": FLOPS_PER_SAMPLE + (FLOPS_PER_SAMPLE_SUN if sun else 0),
                     "peak_unpacked": FP32_UNPACKED_TFLOPS,
                     "frac_unpacked": achieved / FP32_UNPACKED_TFLOPS,
                     "units": unit_figures(args.counters, fp_ms, samples)},
        "prepass_ms": st["prepass_ms"] / max(1, st["prepass_launches"]),
    }
    # the HBM-bound parts: the pre-pass streams the G-buffer once per frame,
    # and small frames replayed in a batch are bound by their compulsory bytes
    pp_ms = rec["prepass_ms"]
    pp_bytes = prepass_bytes(w)
    rec["hbm_roofline"] = {
        "prepass": {"kernel": "k_prepass", "bound": "hbm", "bytes_per_launch": pp_bytes,
                    "avg_launch_ms": pp_ms,
                    "achieved": pp_bytes / (pp_ms * 1e-3) / 1e9 if pp_ms > 0 else None,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": pp_bytes / (pp_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if pp_ms > 0 else None},
        "replayed_iid_frames": replayed_small_report(args) if not args.no_batch else None,
    }
    if not args.no_batch:
        rec["batch"] = batch_report(args)
    if not args.no_rows:
        rec["rows"] = rows_report(args)
    if not args.no_surrogate:
        rec["surrogate"] = surrogate_report(args, oracle_sample=10000)
        rec["surrogate_table_pattern"] = surrogate_report(args, "table", oracle_sample=10000)
    if not args.no_cpu_baseline:
        rec["precision"] = precision_report(w, planes)
        rec["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
