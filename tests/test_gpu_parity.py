"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Element-by-element on the workloads at sizes the oracle finishes in seconds
(many tiles, ragged tails), on sampled beams of the full-size scanning-sensor
frame in the launch configuration the benchmark times, and on edge cases.
"""
from dataclasses import replace
import math

import numpy as np
import pytest

import scenes
from scenes import Raster, Pattern, SensorParams, PATTERN_GAUSS, PATTERN_TABLE

from .parity import run_gpu, compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_05932_amd as lidar
    lidar.load()          # fails loudly if the HIP library is missing


def _report(name, rep):
    print(f"[parity] {name}: beams={rep.n_beams} ambiguous={rep.ambiguous} "
          f"max_wave_err={rep.max_wave_err:.2e} echoes={rep.echoes_compared} "
          f"peak+-1={rep.peak_off_by_one}", flush=True)


def test_iid_frame_full_frame(oracle_mod):
    w = scenes.iid_frame(0)
    ref = oracle_mod.simulate(w.gbuffer, w.pattern, w.params)
    got = run_gpu(w.gbuffer, w.pattern, w.params)
    rep = compare(got, ref, w.params)
    _report("iid_frame", rep)
    assert rep.echoes_compared > 2000
    assert got["stats"]["samples_per_frame"] == int(ref.samples.sum())


def test_scanning_sensor_reduced_raster(oracle_mod):
    """Same scene recipe on a 2048x128 raster, 16 x 300 beams: every beam
    compared; footprints span several 64-row strips and column chunks."""
    w = scenes.road_scan(0, width=2048, height=128, n_lines=16, n_cols=300)
    ref = oracle_mod.simulate(w.gbuffer, w.pattern, w.params)
    got = run_gpu(w.gbuffer, w.pattern, w.params)
    rep = compare(got, ref, w.params)
    _report("scan-2048x128", rep)
    assert rep.echoes_compared > 1000


def test_scanning_sensor_full_size_sampled_beams(oracle_mod):
    """Full 8192x512 frame with all 28,800 beams in the benchmark's launch
    configuration; 480 beams (every line, spread over azimuth) are checked
    against the oracle one by one."""
    w = scenes.road_scan(0)
    rng = np.random.default_rng(2)
    idx = np.sort(rng.choice(w.pattern.n_beams, size=480, replace=False))
    sub = scenes.subset_beams(w, idx)
    ref = oracle_mod.simulate(w.gbuffer, sub.pattern, sub.params)
    got = run_gpu(w.gbuffer, w.pattern, w.params)
    rep = compare(got, ref, w.params, beam_idx=idx)
    _report("scan-8192x512-sampled", rep)
    assert got["stats"]["samples_per_frame"] > 2.0e9
    # every beam has a count, sky beams included
    assert got["n_echoes"].shape == (w.pattern.n_beams,)


def _tiny_params(**kw):
    base = dict(n_bins=300, bin_ns=1.0, max_echoes=3, threshold=2e-6, emit_power=1.0,
                pulse_fwhm_ns=4.0, pulse_trunc_sigmas=4.0, ambient_const=1e-7,
                sun_irradiance=0.5, sun_dir=(0.3, -0.5, math.sqrt(1 - 0.34)))
    base.update(kw)
    return SensorParams(**base)


def _tiny(kind, W=37, H=23, seed=3):
    rng = np.random.default_rng(seed)
    raster = Raster(W, H, -6.0, 6.0 * (2 * W / 64), -2.0, 4.0)
    gb = scenes.random_gbuffer(raster, rng, depth_range=(3.0, 40.0), retro_frac=0.1)
    d = gb.depth.copy()
    d[rng.uniform(size=d.shape) < 0.05] = np.inf
    d[rng.uniform(size=d.shape) < 0.02] = np.nan
    d[rng.uniform(size=d.shape) < 0.02] = -1.0
    gb = replace(gb, depth=d)
    az = np.array([0.1, -5.9, 5.95, 2.0, 6.4, -1.3, -30.0, 0.0])
    el = np.array([1.0, 3.9, -1.9, 4.2, 0.5, -2.3, 0.0, -0.05])
    if kind == PATTERN_GAUSS:
        pat = Pattern(kind, az, el, sigma_deg=(0.6, 0.45), trunc_sigmas=3.0)
    else:
        t = rng.uniform(0.0, 1.0, size=(7, 9)).astype(np.float32)
        t[0, :4] = 0.0
        pat = Pattern(kind, az, el, table=t, half_deg=(1.6, 1.1))
    return gb, pat


@pytest.mark.parametrize("kind", [PATTERN_GAUSS, PATTERN_TABLE])
def test_tiny_images_edges_clipping_and_invalid_pixels(oracle_mod, kind):
    gb, pat = _tiny(kind)
    p = _tiny_params()
    ref = oracle_mod.simulate(gb, pat, p)
    got = run_gpu(gb, pat, p)
    rep = compare(got, ref, p)
    _report(f"tiny-{kind}", rep)
    assert ref.samples[6] == 0          # beam far outside: empty footprint


def test_all_sky_and_threshold_below_floor(oracle_mod):
    gb, pat = _tiny(PATTERN_GAUSS)
    sky = replace(gb, depth=np.full_like(gb.depth, np.inf))
    p = _tiny_params(sun_irradiance=0.0)
    got = run_gpu(sky, pat, p)
    assert np.all(got["n_echoes"] == 0)
    np.testing.assert_array_equal(got["waveforms"], np.float32(p.ambient_const))
    # T below the floor: one echo spanning every bin, both edge flags
    p2 = _tiny_params(sun_irradiance=0.0, threshold=0.5e-7)
    got = run_gpu(sky, pat, p2)
    assert np.all(got["n_echoes"] == 1)
    e = got["echoes"][:, 0]
    assert np.all(e["bin_first"] == 0) and np.all(e["bin_last"] == p2.n_bins - 1)
    assert np.all(e["flags"] == 3)
    np.testing.assert_allclose(e["pulse_width_ns"], p2.n_bins * p2.bin_ns, rtol=1e-6)


def test_many_echoes_are_counted_but_capped(oracle_mod):
    w = scenes.iid_frame(0)
    p = replace(w.params, threshold=w.params.ambient_const + 1e-6, max_echoes=2)
    sub = scenes.subset_beams(w, np.arange(0, 1000, 7))
    ref = oracle_mod.simulate(w.gbuffer, sub.pattern, p)
    assert ref.n_echoes.max() > 5
    got = run_gpu(w.gbuffer, sub.pattern, p)
    compare(got, ref, p)


@pytest.mark.parametrize("R,dt", [(1, 1.0), (7, 2.0), (8000, 0.1)])
def test_extreme_bin_counts(oracle_mod, R, dt):
    gb, pat = _tiny(PATTERN_GAUSS, W=64, H=64)
    gb = replace(gb, depth=np.where(np.isfinite(gb.depth), gb.depth * 0.1, gb.depth).astype(np.float32))
    p = _tiny_params(n_bins=R, bin_ns=dt, threshold=1e-5)
    ref = oracle_mod.simulate(gb, pat, p)
    got = run_gpu(gb, pat, p)
    compare(got, ref, p)


@pytest.mark.parametrize("R,dt,fwhm", [(8000, 0.06, 4.0), (2000, 0.0531, 4.0), (500, 1.0, 0.5),
                                        (333, 0.3, 1.2), (1000, 0.2, 2.0)])
def test_pulse_tap_counts(oracle_mod, R, dt, fwhm):
    """Pulse lengths from 1 to 128 taps each side (odd and even J), with the
    longest waveform: the convolution's zero padding, tap shift and block
    count, and the group size the LDS budget allows."""
    gb, pat = _tiny(PATTERN_TABLE, W=64, H=64)
    gb = replace(gb, depth=np.where(np.isfinite(gb.depth), gb.depth * 0.1, gb.depth).astype(np.float32))
    p = _tiny_params(n_bins=R, bin_ns=dt, pulse_fwhm_ns=fwhm, threshold=1e-5)
    sigma = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    J = math.ceil(p.pulse_trunc_sigmas * sigma / dt)
    assert 1 <= J <= 128
    ref = oracle_mod.simulate(gb, pat, p)
    got = run_gpu(gb, pat, p)
    rep = compare(got, ref, p)
    _report(f"taps-J{J}-R{R}", rep)


def test_single_pixel_image_and_single_beam(oracle_mod):
    raster = Raster(1, 1, -0.5, 0.5, -0.5, 0.5)
    gb = scenes.shell_gbuffer(raster, 12.0, 0.7)
    pat = Pattern(PATTERN_GAUSS, np.array([0.0]), np.array([0.0]), sigma_deg=(0.4, 0.4),
                  trunc_sigmas=3.0)
    p = _tiny_params(sun_irradiance=0.0, threshold=1e-4)
    ref = oracle_mod.simulate(gb, pat, p)
    got = run_gpu(gb, pat, p)
    compare(got, ref, p)
    assert got["beams"]["samples"][0] == 1


def test_row_pitch_larger_than_width(oracle_mod):
    import torch
    import paper_2512_05932_amd as lidar
    gb, pat = _tiny(PATTERN_TABLE, W=40, H=30)
    p = _tiny_params()
    ref = oracle_mod.simulate(gb, pat, p)
    pitch = 53
    planes = []
    for a in gb.planes():
        big = np.full((a.shape[0], pitch), np.nan, np.float32)
        big[:, :a.shape[1]] = a
        planes.append(torch.from_numpy(big).cuda())
    sim = lidar.LidarSim(p, stream=torch.cuda.current_stream(), keep_waveforms=True)
    sim.set_pattern(pat)
    sim.set_gbuffer(gb.raster, planes, pitch=pitch)
    sim.simulate_frame()
    got = sim.read(waveforms=True)
    sim.close()
    compare(got, ref, p)


def test_pattern_raster_and_scene_changes_between_frames(oracle_mod):
    import torch
    import paper_2512_05932_amd as lidar
    w = scenes.iid_frame(0)
    w_b = scenes.iid_frame(1)
    sub = scenes.subset_beams(w, np.arange(0, 1000, 3))
    sim = lidar.LidarSim(w.params, stream=torch.cuda.current_stream(), keep_waveforms=True)
    # frame 1: scene 0; frame 2: scene 1 (same raster); frame 3: new pattern
    for gbuf, pat in ((w.gbuffer, w.pattern), (w_b.gbuffer, w.pattern), (w_b.gbuffer, sub.pattern)):
        planes = lidar.upload_gbuffer(gbuf)
        sim.set_pattern(pat) if pat is not w.pattern or gbuf is w.gbuffer else None
        sim.set_gbuffer(gbuf.raster, planes)
        sim.simulate_frame()
        got = sim.read(waveforms=True)
        compare(got, oracle_mod.simulate(gbuf, pat, w.params), w.params)
    # frame 4: a different raster with the same pattern
    gb2, _ = _tiny(PATTERN_GAUSS, W=96, H=48)
    sim.set_gbuffer(gb2.raster, lidar.upload_gbuffer(gb2))
    sim.simulate_frame()
    got = sim.read(waveforms=True)
    compare(got, oracle_mod.simulate(gb2, sub.pattern, w.params), w.params)
    sim.close()


def test_device_destination_copies_and_profiling(oracle_mod):
    import torch
    import paper_2512_05932_amd as lidar
    w = scenes.iid_frame(0)
    planes = lidar.upload_gbuffer(w.gbuffer)
    sim = lidar.LidarSim(w.params, stream=torch.cuda.current_stream(), profile=True)
    sim.set_pattern(w.pattern)
    sim.set_gbuffer(w.gbuffer.raster, planes)
    for _ in range(3):
        sim.simulate_frame()
    cnt = torch.zeros(w.pattern.n_beams, dtype=torch.int32, device="cuda")
    sim.read_device(n_echoes=cnt)
    host = sim.read()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(cnt.cpu().numpy(), host["n_echoes"])
    st = sim.stats()
    assert st["frames"] == 3 and st["footprint_launches"] == 3 and st["footprint_ms"] > 0
    assert st["kernel_w"] == 11 and st["kernel_h"] == 11 and st["n_taps"] == 15
    sim.reset_stats()
    assert sim.stats()["frames"] == 0
    sim.close()


def test_error_paths_on_device():
    import torch
    import paper_2512_05932_amd as lidar
    w = scenes.iid_frame(0)
    sim = lidar.LidarSim(w.params, stream=torch.cuda.current_stream())
    with pytest.raises(lidar.LidarError) as e:
        sim.simulate_frame()
    assert e.value.status == lidar.LIDAR_E_STATE
    sim.set_pattern(w.pattern)
    with pytest.raises(lidar.LidarError) as e:
        sim.simulate_frame()
    assert e.value.status == lidar.LIDAR_E_STATE
    with pytest.raises(lidar.LidarError) as e:
        sim.read()
    assert e.value.status == lidar.LIDAR_E_STATE
    planes = lidar.upload_gbuffer(w.gbuffer)
    sim.set_gbuffer(w.gbuffer.raster, planes)
    with pytest.raises(lidar.LidarError) as e:
        sim.simulate_frame(mode=7)
    assert e.value.status == lidar.LIDAR_E_UNSUPPORTED
    with pytest.raises(lidar.LidarError) as e:
        sim.simulate_frame(mode=lidar.LIDAR_MODE_SURROGATE)      # no weights yet
    assert e.value.status == lidar.LIDAR_E_STATE
    sim.simulate_frame()
    with pytest.raises(lidar.LidarError) as e:
        sim.read(waveforms=True)
    assert e.value.status == lidar.LIDAR_E_INVALID
    bad = Pattern(PATTERN_TABLE, w.pattern.beam_az, w.pattern.beam_el,
                  table=np.zeros((4, 4), np.float32), half_deg=(1.0, 1.0))
    with pytest.raises(lidar.LidarError) as e:
        sim.set_pattern(bad)
    assert e.value.status == lidar.LIDAR_E_INVALID
    # a Gaussian narrower than a pixel: the grid holds only the centre cell,
    # which is still a valid kernel
    narrow = Pattern(PATTERN_GAUSS, w.pattern.beam_az, w.pattern.beam_el,
                     sigma_deg=(0.001, 0.001), trunc_sigmas=3.0)
    sim.set_pattern(narrow)
    sim.simulate_frame()
    assert np.all(sim.read()["beams"]["samples"] == 1)
    sim.close()
