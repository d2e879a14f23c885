"""The path's options on the GPU against the FP64 oracle, through the C-ABI:
a tabulated pulse, a collector-sensitivity table for the sun term, echo
selection (runs of xi_hat and raw-signal bins) and the two range modes
(normal-corrected ranges, pixel range intervals), single frames and
batches, plus the allocation-free entry point with a tabulated pulse and an
echo selection."""
from dataclasses import replace
import math

import numpy as np
import pytest

import scenes

from .parity import compare, compare_selection, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lidar():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_05932_amd as lidar
    lidar.load()
    return lidar


def _scan(seed=0):
    return scenes.road_scan(seed, width=2048, height=128, n_lines=16, n_cols=300)


def _iid(step=5):
    w = scenes.iid_frame(0)
    return scenes.subset_beams(w, np.arange(0, w.pattern.n_beams, step))


def _kappa(table_shape=(256, 256), half=2.0, sig=(0.5, 1.0)):
    ny, nx = table_shape
    x = -half + (np.arange(nx) + 0.5) * (2 * half / nx)
    y = half - (np.arange(ny) + 0.5) * (2 * half / ny)
    yy, xx = np.meshgrid(y, x, indexing="ij")
    return np.exp(-0.5 * ((xx / sig[0]) ** 2 + (yy / sig[1]) ** 2)).astype(np.float32)


def test_tabulated_pulse(lidar, oracle_mod):
    """An asymmetric 9-tap pulse (fast rise, slow decay) on workload-1 frames."""
    w = _iid()
    p = replace(w.params, pulse_taps=np.array([0.0, 0.3, 1.0, 0.8, 0.6, 0.45, 0.3, 0.2, 0.1]),
                pulse_fwhm_ns=0.0)
    got = run_gpu(w.gbuffer, w.pattern, p)
    ref = oracle_mod.simulate(w.gbuffer, w.pattern, p)
    rep = compare(got, ref, p)
    print(f"[opt] tabulated pulse: {rep.echoes_compared} echoes, max wave err {rep.max_wave_err:.2e}",
          flush=True)
    assert rep.echoes_compared > 300


def test_kappa_table_sun_floor(lidar, oracle_mod):
    """Scanning frame with a wide Gaussian kappa (0.5 x 1.0 deg) for the sun
    term: the floor follows kappa over its own support."""
    w = _scan()
    pat = replace(w.pattern, rx_table=_kappa())
    got = run_gpu(w.gbuffer, pat, w.params)
    ref = oracle_mod.simulate(w.gbuffer, pat, w.params)
    rep = compare(got, ref, w.params)
    base = oracle_mod.simulate(w.gbuffer, w.pattern, w.params, want_xi=False)
    print(f"[opt] kappa table: {rep.echoes_compared} echoes; floor/default median "
          f"{np.median(ref.floor[base.floor > 0] / base.floor[base.floor > 0]):.2f}", flush=True)
    assert not np.allclose(ref.floor, base.floor)


@pytest.mark.parametrize("mode", [scenes.ECHO_SELECT_STRONGEST, scenes.ECHO_SELECT_NEAREST,
                                  scenes.ECHO_SELECT_LONGEST, scenes.ECHO_SELECT_RAW_STRONGEST,
                                  scenes.ECHO_SELECT_RAW_NEAREST])
@pytest.mark.parametrize("which", ["iid", "scan"])
def test_echo_selection(lidar, oracle_mod, mode, which):
    w = _iid() if which == "iid" else _scan()
    p = replace(w.params, echo_select=mode)
    if mode >= scenes.ECHO_SELECT_RAW_STRONGEST:
        # the raw signal peaks higher than the convolved one: threshold at
        # a quarter of the median raw maximum
        base = oracle_mod.simulate(w.gbuffer, w.pattern, w.params, want_xi_hat=False)
        p = replace(p, threshold=0.25 * float(np.median(base.xi.max(axis=1))))
    got = run_gpu(w.gbuffer, w.pattern, p)
    ref = oracle_mod.simulate(w.gbuffer, w.pattern, p)
    rep = compare_selection(got, ref, p)
    print(f"[opt] select {mode} on {which}: {rep.echoes_compared} echoes, {rep.peak_off_by_one} "
          f"near-ties, {rep.ambiguous} ambiguous beams", flush=True)
    assert rep.echoes_compared > 100


@pytest.mark.parametrize("mode", [scenes.RANGE_INTERVAL, scenes.RANGE_CORRECTED])
def test_range_modes_on_the_scanning_frame(lidar, oracle_mod, mode):
    w = _scan()
    p = replace(w.params, range_mode=mode)
    got = run_gpu(w.gbuffer, w.pattern, p)
    ref = oracle_mod.simulate(w.gbuffer, w.pattern, p)
    rep = compare(got, ref, p)
    print(f"[opt] range mode {mode}: {rep.echoes_compared} echoes, max wave err "
          f"{rep.max_wave_err:.2e}", flush=True)
    assert rep.echoes_compared > 1000


@pytest.mark.parametrize("mode", [scenes.RANGE_INTERVAL, scenes.RANGE_CORRECTED])
def test_range_modes_on_a_tilted_plane(lidar, oracle_mod, mode):
    """Beams on a plane at 75 deg incidence (0.1 ns bins: several bins per
    pixel), Gaussian footprints, waveforms and echoes against the oracle."""
    from .test_oracle_options import plane_gbuffer
    r = scenes.Raster(256, 128, -8.0, 8.0, -4.0, 4.0)
    a = math.radians(75.0)
    gb, n, c = plane_gbuffer(r, (-math.cos(a), -math.sin(a), 0.0), (25.0, 0.0, 0.0))
    rng = np.random.default_rng(2)
    az, el = rng.uniform(-7.0, 7.0, 120), rng.uniform(-3.5, 3.5, 120)
    pat = scenes.Pattern(scenes.PATTERN_GAUSS, az, el, sigma_deg=(0.15, 0.1), trunc_sigmas=3.0)
    p = scenes.SensorParams(n_bins=4096, bin_ns=0.1, max_echoes=3, threshold=4e-7, emit_power=1.0,
                            pulse_fwhm_ns=1.0, range_mode=mode)
    got = run_gpu(gb, pat, p)
    ref = oracle_mod.simulate(gb, pat, p)
    rep = compare(got, ref, p)
    print(f"[opt] plane, range mode {mode}: {rep.echoes_compared} echoes", flush=True)
    assert rep.echoes_compared >= 60


def test_batch_with_interval_ranges_and_kappa(lidar, oracle_mod):
    """Two scanning frames and a workload-1 frame in one batch (graph replay)
    with pixel range intervals; the scanning frames carry a kappa table."""
    import torch
    p = replace(_scan(0).params, range_mode=scenes.RANGE_INTERVAL)
    ws = [_scan(0), _scan(1), _iid(3)]
    pats = [replace(ws[0].pattern, rx_table=_kappa()), ws[1].pattern, ws[2].pattern]
    planes = [lidar.upload_gbuffer(w.gbuffer, "cuda") for w in ws]
    sim = lidar.LidarSim(p, stream=torch.cuda.current_stream(), keep_waveforms=True)
    try:
        batch = lidar.Batch([(w.gbuffer.raster, pl) for w, pl in zip(ws, planes)], pats)
        sim.simulate_batch(batch)
        sim.simulate_batch(batch)
        outs = [sim.read_batch(i, waveforms=True) for i in range(3)]
    finally:
        sim.close()
    for i, (w, pat) in enumerate(zip(ws, pats)):
        ref = oracle_mod.simulate(w.gbuffer, pat, p)
        rep = compare(outs[i], ref, p)
        print(f"[opt] batch frame {i}: {rep.echoes_compared} echoes", flush=True)


def test_corrected_ranges_not_in_batches(lidar):
    import torch
    w = _iid(50)
    p = replace(w.params, range_mode=scenes.RANGE_CORRECTED)
    planes = lidar.upload_gbuffer(w.gbuffer, "cuda")
    sim = lidar.LidarSim(p, stream=torch.cuda.current_stream())
    try:
        batch = lidar.Batch([(w.gbuffer.raster, planes)], [w.pattern])
        with pytest.raises(lidar.LidarError) as e:
            sim.simulate_batch(batch)
        assert e.value.status == lidar.LIDAR_E_UNSUPPORTED
    finally:
        sim.close()


def test_static_path_with_tabulated_pulse_and_selection(lidar, oracle_mod):
    import torch
    w = _iid(4)
    p = replace(w.params, pulse_taps=np.array([0.2, 1.0, 0.5, 0.25]+[0.0]), pulse_fwhm_ns=0.0,
                echo_select=scenes.ECHO_SELECT_STRONGEST)
    B, E = w.pattern.n_beams, p.max_echoes
    planes = lidar.upload_gbuffer(w.gbuffer, "cuda")
    ech = torch.zeros((B, E * 40), dtype=torch.uint8, device="cuda")
    cnt = torch.zeros((B,), dtype=torch.int32, device="cuda")
    bi = torch.zeros((B, 24), dtype=torch.uint8, device="cuda")
    lidar.simulate_static(p, w.pattern, w.gbuffer.raster, planes, ech, cnt, bi,
                          stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    got = {"echoes": ech.cpu().numpy().view(lidar.ECHO_DTYPE).reshape(B, E),
           "n_echoes": cnt.cpu().numpy(), "beams": bi.cpu().numpy().view(lidar.BEAM_DTYPE).reshape(B)}
    ref = oracle_mod.simulate(w.gbuffer, w.pattern, p)
    rep = compare_selection(got, ref, p)
    assert rep.echoes_compared > 100
