"""Parity of the batched path (one persistent launch over many uneven frames,
replayed from a captured HIP graph) with the FP64 oracle, through the C-ABI.
"""
from dataclasses import replace
import math

import numpy as np
import pytest

import scenes
from scenes import PATTERN_TABLE, Pattern

from .parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_05932_amd as lidar
    lidar.load()


def _small_batch(seed=0, n_frames=12):
    """The batch recipe at test scale: 4 raster sizes (ragged, not multiples
    of 4 or 64), 150-1500 beams, footprints of 20-4000 pixels."""
    return scenes.frame_batch(seed, n_frames=n_frames,
                              sizes=((130, 66), (258, 129), (517, 250), (301, 301)),
                              beams=(150, 1500), footprint_px=(20.0, 4000.0))


def _upload(bw):
    import paper_2512_05932_amd as lidar
    return [lidar.upload_gbuffer(f.gbuffer, "cuda") for f in bw.frames]


def _check_all(sim, bw, params, oracle_mod, tag, waveforms=True, idx=None):
    reps = []
    for i, f in enumerate(bw.frames):
        got = sim.read_batch(i, waveforms=waveforms)
        pat = f.pattern if idx is None else scenes.subset_beams(f, idx[i]).pattern
        ref = oracle_mod.simulate(f.gbuffer, pat, params, want_xi=False)
        reps.append(compare(got, ref, params, beam_idx=None if idx is None else idx[i],
                            check_waveforms=waveforms))
    n = sum(r.n_beams for r in reps)
    e = sum(r.echoes_compared for r in reps)
    w = max(r.max_wave_err for r in reps)
    print(f"[batch] {tag}: frames={len(reps)} beams={n} echoes={e} max_wave_err={w:.2e}",
          flush=True)
    return reps


def test_batch_every_beam_matches_oracle(oracle_mod):
    import torch
    import paper_2512_05932_amd as lidar
    bw = _small_batch(0)
    planes = _upload(bw)
    sim = lidar.LidarSim(bw.params, stream=torch.cuda.current_stream(), keep_waveforms=True)
    try:
        batch = lidar.Batch([(f.gbuffer.raster, p) for f, p in zip(bw.frames, planes)],
                            [f.pattern for f in bw.frames])
        sim.simulate_batch(batch)
        info = sim.batch_info()
        assert info["n_frames"] == len(bw.frames) and info["graph"] == 1
        assert info["n_beams"] == sum(f.pattern.n_beams for f in bw.frames)
        reps = _check_all(sim, bw, bw.params, oracle_mod, "small-12")
        assert sum(r.echoes_compared for r in reps) > 3000
    finally:
        sim.close()


@pytest.mark.parametrize("sun", [False, True])
def test_batch_wave_schedule_single_beam_groups(oracle_mod, sun):
    """Frames whose beam groups all hold a single beam (three 1024x512
    i.i.d. frames, 1000 beams each, footprints far apart) go to the wave
    schedule and, touching few of their pixels, are gathered straight from
    the G-buffer planes; every beam is compared with the oracle, on two
    replays; with and without the sun term."""
    import torch
    import paper_2512_05932_amd as lidar
    frames = [scenes.iid_frame(s) for s in range(3)]
    params = frames[0].params
    if sun:
        se = math.sin(math.radians(35.0))
        params = replace(params, sun_irradiance=30.0,
                         sun_dir=(math.sqrt(1 - se * se) * 0.8, math.sqrt(1 - se * se) * 0.6, se))
    bw = scenes.BatchWorkload("iid-3", frames, params)
    planes = _upload(bw)
    sim = lidar.LidarSim(bw.params, stream=torch.cuda.current_stream(), keep_waveforms=True)
    try:
        batch = lidar.Batch([(f.gbuffer.raster, p) for f, p in zip(bw.frames, planes)],
                            [f.pattern for f in bw.frames])
        for rep in range(2):
            sim.simulate_batch(batch)
            info = sim.batch_info()
            assert info["wave_items"] == info["n_items"] == 3000
            # 89 samples per beam over 524288 pixels: gathered from the planes
            assert info["direct_frames"] == 3
            reps = _check_all(sim, bw, bw.params, oracle_mod, f"wave-iid-3 sun={sun} replay {rep}")
            assert sum(r.echoes_compared for r in reps) > 6000
        if sun:
            floors = np.concatenate([sim.read_batch(i)["beams"]["floor"] for i in range(3)])
            assert np.count_nonzero(floors > params.ambient_const) > 0.8 * floors.size
    finally:
        sim.close()


def test_batch_wave_schedule_from_pixel_records(oracle_mod):
    """Single-beam groups on frames that their beams cover densely enough
    (sigma 0.2 deg: about 314 samples per beam, more than one per two pixels)
    take the wave schedule over the pre-pass records, not the direct gather."""
    import torch
    import paper_2512_05932_amd as lidar
    frames = _wide_iid((8, 9), scenes.iid_frame(0).params)
    bw = scenes.BatchWorkload("iid-2-wide", frames, frames[0].params)
    planes = _upload(bw)
    sim = lidar.LidarSim(bw.params, stream=torch.cuda.current_stream(), keep_waveforms=True)
    try:
        batch = lidar.Batch([(f.gbuffer.raster, p) for f, p in zip(bw.frames, planes)],
                            [f.pattern for f in bw.frames])
        sim.simulate_batch(batch)
        info = sim.batch_info()
        print(f"[batch] wide iid: {info}", flush=True)
        assert info["wave_items"] == info["n_items"] == 2000
        assert info["direct_frames"] == 0
        reps = _check_all(sim, bw, bw.params, oracle_mod, "wave-iid-2 records")
        assert sum(r.echoes_compared for r in reps) > 3000
    finally:
        sim.close()


def _wide_iid(seeds, params):
    frames = []
    for s in seeds:
        f = scenes.iid_frame(s)
        frames.append(replace(f, pattern=replace(f.pattern, sigma_deg=(0.2, 0.2)), params=params))
    return frames


def test_batch_fixed_point_accumulation(oracle_mod):
    """Frames whose bins span at most half the waveform (i.i.d. depths of 5-60
    m in 2048 bins of 0.5 ns) accumulate their wave-schedule histograms in
    64-bit fixed point; every beam against the oracle.  Integer additions do
    not depend on their order, so two replays give the same bits."""
    import torch
    import paper_2512_05932_amd as lidar
    params = scenes.batch_params()
    frames = _wide_iid((10, 11), params)
    bw = scenes.BatchWorkload("iid-2-fixed", frames, params)
    planes = _upload(bw)
    sim = lidar.LidarSim(params, stream=torch.cuda.current_stream(), keep_waveforms=True)
    try:
        batch = lidar.Batch([(f.gbuffer.raster, p) for f, p in zip(bw.frames, planes)],
                            [f.pattern for f in bw.frames])
        outs = []
        for rep in range(2):
            sim.simulate_batch(batch)
            info = sim.batch_info()
            print(f"[batch] fixed point: {info}", flush=True)
            assert info["wave_items"] == info["n_items"] == 2000 and info["direct_frames"] == 0
            assert info["fixed_point_beams"] == 2000
            # i.i.d. depths: nearly every pixel starts a new bin, so both
            # frames add every sample on its own
            assert info["short_run_frames"] == 2
            reps = _check_all(sim, bw, params, oracle_mod, f"fixed-point replay {rep}")
            assert sum(r.echoes_compared for r in reps) > 1500
            outs.append([sim.read_batch(i, waveforms=True) for i in range(len(bw.frames))])
        for a, b in zip(*outs):
            assert a["waveforms"].tobytes() == b["waveforms"].tobytes()
            assert a["echoes"].tobytes() == b["echoes"].tobytes()
    finally:
        sim.close()


@pytest.mark.parametrize("select,n_echoes,n_bins,t_scale", [
    (scenes.ECHO_SELECT_ALL, 1, 2048, 1.0),
    (scenes.ECHO_SELECT_ALL, 8, 2048, 1.0),
    (scenes.ECHO_SELECT_NEAREST, 3, 2048, 1.0),
    (scenes.ECHO_SELECT_STRONGEST, 3, 2048, 1.0),
    (scenes.ECHO_SELECT_LONGEST, 2, 2048, 1.0),
    (scenes.ECHO_SELECT_RAW_STRONGEST, 3, 2048, 1.0),
    (scenes.ECHO_SELECT_RAW_NEAREST, 3, 2048, 1.0),
    (scenes.ECHO_SELECT_ALL, 3, 2048, 0.0),
    (scenes.ECHO_SELECT_ALL, 3, 700, 1.0),
])
def test_batch_wave_schedule_echo_modes(oracle_mod, select, n_echoes, n_bins, t_scale):
    """Echoes of the wave schedule (one beam per wave; the first runs of ALL
    and NEAREST found from the passes' above-threshold bits as they are
    written) for every selection, the raw ones included, on i.i.d. frames with
    ~10 runs per beam, a threshold below the floor (one run over every bin,
    both edge flags) and a waveform whose last pass is partial (700 bins);
    every beam against the oracle."""
    import torch
    import paper_2512_05932_amd as lidar
    from .parity import compare_selection
    params = replace(scenes.batch_params(), echo_select=select, max_echoes=n_echoes, n_bins=n_bins)
    if t_scale == 0.0:
        params = replace(params, threshold=0.5 * params.ambient_const)
    frames = _wide_iid((16,), params)
    bw = scenes.BatchWorkload("iid-1-echo-modes", frames, params)
    planes = _upload(bw)
    sim = lidar.LidarSim(params, stream=torch.cuda.current_stream(), keep_waveforms=True)
    try:
        batch = lidar.Batch([(f.gbuffer.raster, p) for f, p in zip(bw.frames, planes)],
                            [f.pattern for f in bw.frames])
        sim.simulate_batch(batch)
        info = sim.batch_info()
        print(f"[batch] echo modes {select}/{n_echoes}/{n_bins}/{t_scale}: {info}", flush=True)
        assert info["wave_items"] == info["n_items"] == 1000
        got = sim.read_batch(0, waveforms=True)
        ref = oracle_mod.simulate(frames[0].gbuffer, frames[0].pattern, params)
        if select == scenes.ECHO_SELECT_ALL:
            rep = compare(got, ref, params)
        else:
            rep = compare_selection(got, ref, params)
        print(f"[batch] echo modes: {rep.echoes_compared} echoes compared, counts "
              f"{int(ref.n_echoes.sum())}", flush=True)
        # one echo per beam where a single run is selected or kept (beams
        # with a bin within the tolerance of T are not compared)
        single = select != scenes.ECHO_SELECT_ALL or n_echoes == 1
        assert rep.echoes_compared > (200 if single else 500)
        if t_scale == 0.0:
            assert (got["n_echoes"] == 1).all()
            flags = got["echoes"][:, 0]["flags"]
            assert ((flags & 3) == 3).all()
        elif select == scenes.ECHO_SELECT_ALL and n_bins == 2048:
            assert (ref.n_echoes > n_echoes).sum() > 100
    finally:
        sim.close()


def test_batch_fixed_point_run_sums_on_smooth_frames(oracle_mod):
    """A frame whose depth changes slowly along its rows (a tilted plane with
    a gentle ripple: about 0.16 bins per pixel) keeps summing runs of equal
    bins in fixed point; every beam against the oracle."""
    import torch
    import paper_2512_05932_amd as lidar
    params = scenes.batch_params()
    frames = _wide_iid((15,), params)
    gb = frames[0].gbuffer
    H, W = gb.depth.shape
    u = np.arange(W)[None, :]
    v = np.arange(H)[:, None]
    depth = (20.0 + 10.0 * v / H + 2.0 * np.sin(2.0 * np.pi * u / W)).astype(np.float32)
    frames[0] = replace(frames[0], gbuffer=replace(gb, depth=depth))
    bw = scenes.BatchWorkload("smooth-1-fixed", frames, params)
    planes = _upload(bw)
    sim = lidar.LidarSim(params, stream=torch.cuda.current_stream(), keep_waveforms=True)
    try:
        batch = lidar.Batch([(f.gbuffer.raster, p) for f, p in zip(bw.frames, planes)],
                            [f.pattern for f in bw.frames])
        sim.simulate_batch(batch)
        info = sim.batch_info()
        print(f"[batch] smooth frame: {info}", flush=True)
        assert info["wave_items"] == info["n_items"] == 1000
        assert info["fixed_point_beams"] == 1000 and info["short_run_frames"] == 0
        reps = _check_all(sim, bw, params, oracle_mod, "fixed-point run sums")
        assert sum(r.echoes_compared for r in reps) > 500
    finally:
        sim.close()


def test_batch_fixed_point_in_the_group_schedule(oracle_mod):
    """Beams closer than a kernel width (sigma 0.5 deg) form groups of up to
    four on the group schedule; their histograms accumulate in fixed point
    too (one unit per group); every beam against the oracle."""
    import torch
    import paper_2512_05932_amd as lidar
    params = scenes.batch_params()
    frames = []
    for s in (13, 14):
        f = scenes.iid_frame(s)
        frames.append(replace(f, pattern=replace(f.pattern, sigma_deg=(0.5, 0.5)), params=params))
    bw = scenes.BatchWorkload("iid-2-groups", frames, params)
    planes = _upload(bw)
    sim = lidar.LidarSim(params, stream=torch.cuda.current_stream(), keep_waveforms=True)
    try:
        batch = lidar.Batch([(f.gbuffer.raster, p) for f, p in zip(bw.frames, planes)],
                            [f.pattern for f in bw.frames])
        sim.simulate_batch(batch)
        info = sim.batch_info()
        print(f"[batch] groups in fixed point: {info}", flush=True)
        assert info["wave_items"] == 0 and info["n_items"] < 2000
        assert info["fixed_point_beams"] == 2000
        reps = _check_all(sim, bw, params, oracle_mod, "fixed-point groups")
        assert sum(r.echoes_compared for r in reps) > 1500
    finally:
        sim.close()


def test_batch_fixed_point_falls_back_where_its_bound_is_loose(oracle_mod):
    """One pixel 10^15 times brighter than the rest sets a coarse fixed-point
    unit for every beam of its frame; without ambient light the beams that
    see only ordinary pixels fail the truncation bound and run again with
    FP32 atomics, and every beam still matches the oracle."""
    import torch
    import paper_2512_05932_amd as lidar
    params = replace(scenes.batch_params(), ambient_const=0.0)
    frames = _wide_iid((12,), params)
    gb = frames[0].gbuffer
    gain = gb.retro_gain.copy()
    gain[100, 100] = 1e15
    frames[0] = replace(frames[0], gbuffer=replace(gb, retro_gain=gain))
    bw = scenes.BatchWorkload("iid-1-bright", frames, params)
    planes = _upload(bw)
    sim = lidar.LidarSim(params, stream=torch.cuda.current_stream(), keep_waveforms=True)
    try:
        batch = lidar.Batch([(f.gbuffer.raster, p) for f, p in zip(bw.frames, planes)],
                            [f.pattern for f in bw.frames])
        sim.simulate_batch(batch)
        info = sim.batch_info()
        print(f"[batch] bright pixel: {info}", flush=True)
        assert info["fixed_point_beams"] == 1000 and info["fixed_point_redone"] > 900
        _check_all(sim, bw, params, oracle_mod, "fixed-point fallback")
    finally:
        sim.close()


@pytest.mark.parametrize("n_bins,bin_ns", [(700, 0.55), (1100, 0.35)])
def test_batch_wave_schedule_ragged_waveforms(oracle_mod, n_bins, bin_ns):
    """The wave schedule with waveform lengths that end inside a 512-bin
    output pass (and inside a 64-bin chunk), the last bin near the farthest
    depths so that echoes reach it: two i.i.d. frames."""
    import torch
    import paper_2512_05932_amd as lidar
    frames = [scenes.iid_frame(s) for s in (4, 5)]
    params = replace(frames[0].params, n_bins=n_bins, bin_ns=bin_ns)
    bw = scenes.BatchWorkload(f"iid-2-R{n_bins}", frames, params)
    planes = _upload(bw)
    sim = lidar.LidarSim(bw.params, stream=torch.cuda.current_stream(), keep_waveforms=True)
    try:
        batch = lidar.Batch([(f.gbuffer.raster, p) for f, p in zip(bw.frames, planes)],
                            [f.pattern for f in bw.frames])
        sim.simulate_batch(batch)
        info = sim.batch_info()
        assert info["wave_items"] == info["n_items"] == 2000
        reps = _check_all(sim, bw, bw.params, oracle_mod, f"wave-iid-2 R={n_bins}")
        assert sum(r.echoes_compared for r in reps) > 3000
    finally:
        sim.close()


def test_batch_mixed_schedules(oracle_mod):
    """One batch whose sparse frames (150 beams, 20-pixel footprints) take the
    wave schedule and whose dense frames (1500 beams, 4000-pixel footprints)
    take the group schedule: two persistent launches in one graph."""
    import torch
    import paper_2512_05932_amd as lidar
    sparse = scenes.frame_batch(6, n_frames=3, sizes=((517, 250), (301, 301)), beams=(150, 150),
                                footprint_px=(20.0, 20.0))
    dense = scenes.frame_batch(7, n_frames=3, sizes=((517, 250), (301, 301)), beams=(1500, 1500),
                               footprint_px=(4000.0, 4000.0))
    bw = scenes.BatchWorkload("mixed", sparse.frames + dense.frames, sparse.params)
    planes = _upload(bw)
    sim = lidar.LidarSim(bw.params, stream=torch.cuda.current_stream(), keep_waveforms=True)
    try:
        batch = lidar.Batch([(f.gbuffer.raster, p) for f, p in zip(bw.frames, planes)],
                            [f.pattern for f in bw.frames])
        sim.simulate_batch(batch)
        info = sim.batch_info()
        assert 0 < info["wave_items"] < info["n_items"]
        reps = _check_all(sim, bw, bw.params, oracle_mod, "mixed-schedules")
        assert sum(r.echoes_compared for r in reps) > 2000
    finally:
        sim.close()


def test_batch_graph_replays_follow_changed_gbuffers(oracle_mod):
    """The captured graph is replayed three times; between replays the
    G-buffer contents change in place (eager torch work and a synchronise):
    every replay must match the oracle on the current contents, without a new
    set-up."""
    import torch
    import paper_2512_05932_amd as lidar
    bw = _small_batch(1, n_frames=6)
    planes = _upload(bw)
    sim = lidar.LidarSim(bw.params, stream=torch.cuda.current_stream(), keep_waveforms=True,
                         profile=True)
    try:
        batch = lidar.Batch([(f.gbuffer.raster, p) for f, p in zip(bw.frames, planes)],
                            [f.pattern for f in bw.frames])
        for rep in range(3):
            scale = np.float32(1.0 + 0.15 * rep)
            for f, p in zip(bw.frames, planes):
                p[0].copy_(torch.from_numpy(f.gbuffer.depth * scale).cuda())
            torch.cuda.synchronize()
            sim.simulate_batch(batch)
            info = sim.batch_info()
            cur = scenes.BatchWorkload(bw.name, [
                replace(f, gbuffer=replace(f.gbuffer, depth=f.gbuffer.depth * scale))
                for f in bw.frames], bw.params)
            # the reference sees the same float32 depths as the device
            for f, p in zip(cur.frames, planes):
                assert np.array_equal(p[0].cpu().numpy(), f.gbuffer.depth)
            _check_all(sim, cur, bw.params, oracle_mod, f"replay{rep}")
        st = sim.stats()
        assert st["batch_launches"] == 3 and st["batch_ms"] > 0.0
        assert info["graph"] == 1
    finally:
        sim.close()


def test_batch_autotuned_tiles_and_table_patterns_with_sun(oracle_mod):
    """Autotuned strip heights; frames mixing Gaussian and tabulated
    patterns; the sun term on (every pre-pass of the graph writes sun
    shading)."""
    import torch
    import paper_2512_05932_amd as lidar
    bw = _small_batch(2, n_frames=8)
    rng = np.random.default_rng(5)
    frames = []
    for i, f in enumerate(bw.frames):
        if i % 2:
            t = rng.uniform(0.0, 1.0, size=(9, 11)).astype(np.float32)
            r = f.gbuffer.raster
            pat = Pattern(PATTERN_TABLE, f.pattern.beam_az, f.pattern.beam_el, table=t,
                          half_deg=(7.0 * r.dphi, 5.0 * r.de))
            f = replace(f, pattern=pat)
        frames.append(f)
    bw = replace(bw, frames=frames)
    se = math.sin(math.radians(40.0))
    params = replace(bw.params, sun_irradiance=0.02,
                     sun_dir=(math.sqrt(1 - se * se) * 0.6, math.sqrt(1 - se * se) * 0.8, se))
    planes = _upload(bw)
    sim = lidar.LidarSim(params, stream=torch.cuda.current_stream(), keep_waveforms=True,
                         autotune=True)
    try:
        batch = lidar.Batch([(f.gbuffer.raster, p) for f, p in zip(bw.frames, planes)],
                            [f.pattern for f in bw.frames])
        sim.simulate_batch(batch)
        info = sim.batch_info()
        assert info["autotuned"] == 1 and info["autotune_ms"] > 0.0
        _check_all(sim, bw, params, oracle_mod, "autotune-sun-table")
        floors = np.concatenate([sim.read_batch(i)["beams"]["floor"] for i in range(len(frames))])
        assert np.count_nonzero(floors > params.ambient_const) > 0.3 * floors.size
    finally:
        sim.close()


def test_batch_full_size_sampled_beams(oracle_mod):
    """The full batch workload (64 frames of 512x256 to 4096x2048, 5k-100k
    beams, footprints of 20-20,000 pixels) in one graph launch; 24 beams of
    every frame are checked against the oracle one by one."""
    import torch
    import paper_2512_05932_amd as lidar
    bw = scenes.frame_batch(0)
    print(f"[batch] full: generated {len(bw.frames)} frames", flush=True)
    planes = _upload(bw)
    sim = lidar.LidarSim(bw.params, stream=torch.cuda.current_stream(), keep_waveforms=False)
    try:
        batch = lidar.Batch([(f.gbuffer.raster, p) for f, p in zip(bw.frames, planes)],
                            [f.pattern for f in bw.frames])
        sim.simulate_batch(batch)
        torch.cuda.synchronize()
        info = sim.batch_info()
        print(f"[batch] full: {info}", flush=True)
        # footprints clipped at the image edges hold fewer samples
        nominal = sum(f.pattern.n_beams * f.meta["footprint_px"] for f in bw.frames)
        assert 0.8 * nominal < info["samples"] < 1.05 * nominal
        rng = np.random.default_rng(9)
        idx = [np.sort(rng.choice(f.pattern.n_beams, size=24, replace=False)) for f in bw.frames]
        reps = _check_all(sim, bw, bw.params, oracle_mod, "full-64", waveforms=False, idx=idx)
        assert sum(r.echoes_compared for r in reps) > 500
    finally:
        sim.close()
        del planes
        torch.cuda.empty_cache()


def test_batch_errors_name_the_frame():
    import torch
    import paper_2512_05932_amd as lidar
    bw = _small_batch(3, n_frames=3)
    planes = _upload(bw)
    sim = lidar.LidarSim(bw.params, stream=torch.cuda.current_stream())
    try:
        with pytest.raises(lidar.LidarError, match="before simulate_batch"):
            sim._batch = None
            sim._check(sim._lib.lidar_sim_read_batch(sim._h, 0, None, None, None, None, 0))
        bad = replace(bw.frames[2].pattern, sigma_deg=(0.0, 1.0))
        batch = lidar.Batch([(f.gbuffer.raster, p) for f, p in zip(bw.frames, planes)],
                            [f.pattern for f in bw.frames[:2]] + [bad])
        with pytest.raises(lidar.LidarError, match="frame 2: Gaussian pattern"):
            sim.simulate_batch(batch)
        good = lidar.Batch([(f.gbuffer.raster, p) for f, p in zip(bw.frames, planes)],
                           [f.pattern for f in bw.frames])
        sim.simulate_batch(good)
        with pytest.raises(lidar.LidarError, match="frame index out of range"):
            sim._check(sim._lib.lidar_sim_read_batch(sim._h, 3, None, None, None, None, 0))
        sim.reset_batch()
        with pytest.raises(lidar.LidarError, match="no batch"):
            sim.batch_info()
    finally:
        sim.close()
