"""Reprojection of pinhole renderings (z-buffer depth) on the GPU against the
FP64 oracle, through the C-ABI, and the plain path on the reprojected
G-buffer.

Bar: the nearest pinhole pixel is an FP64 decision on both sides, so
reflectance and gain are equal; the output depth is the FP32 rounding of
the same FP64 expression (contraction off on both sides) and must be equal
except where the correction's ratio, which uses the output direction's
cosines (device vs host libm), rounds to another FP32 value (at most one ulp,
on at most 0.1 % of the pixels); normals within 1e-7."""
import numpy as np
import pytest

import scenes
from oracle import pinhole as P

from .parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lidar():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_05932_amd as lidar
    lidar.load()
    return lidar


def _upload(lidar, src, pad=0):
    import torch
    h, w = src.height, src.width
    def plane(a):
        a = np.ascontiguousarray(a)
        if pad:
            b = np.zeros((h, w + pad), dtype=a.dtype)
            b[:, :w] = a
            a = b
        return torch.from_numpy(a.view(np.int16) if a.dtype == np.uint16 else
                                (a.view(np.int32) if a.dtype == np.uint32 else a)).to("cuda")
    return [plane(src.depth), plane(src.reflectance), plane(src.retro_gain),
            plane(src.normal[0]), plane(src.normal[1]), plane(src.normal[2])]


RASTER = scenes.Raster(512, 96, -36.0, 36.0, -9.0, 3.0)
PARAMS = scenes.SensorParams(n_bins=1024, bin_ns=0.5, max_echoes=3, threshold=2e-6, emit_power=1.0,
                             pulse_fwhm_ns=4.0, ambient_const=1e-8)


@pytest.mark.parametrize("correct", [False, True])
@pytest.mark.parametrize("fmt", [P.DEPTH_RANGE, P.DEPTH_EYE_Z, P.DEPTH_WINDOW_F32,
                                 P.DEPTH_WINDOW_U16, P.DEPTH_WINDOW_U24])
def test_reprojection_matches_oracle(lidar, fmt, correct):
    import torch
    src = scenes.pinhole_render(4, width=800, height=300, hfov_deg=70.0, yaw_deg=5.0, pitch_deg=-3.0,
                                fmt=fmt, near=0.3, far=800.0, n_boxes=12)
    planes = _upload(lidar, src, pad=24)
    sim = lidar.LidarSim(PARAMS, stream=torch.cuda.current_stream())
    try:
        sim.set_gbuffer_pinhole(src, planes, RASTER, correct=correct, pitch=src.width + 24)
        got = sim.read_gbuffer()
    finally:
        sim.close()
    ref = P.reproject(src.as_dict(), RASTER, correct=correct)
    depth = ref[0].astype(np.float32)
    fin = np.isfinite(depth)
    assert fin.mean() > 0.3
    np.testing.assert_array_equal(np.isfinite(got[0]), fin)
    diff = got[0][fin] != depth[fin]
    ulp = np.abs(got[0][fin].view(np.int32) - depth[fin].view(np.int32))
    print(f"[pinhole] fmt {fmt} correct {correct}: {fin.sum()} pixels, {diff.sum()} depths differ "
          f"(max {ulp.max()} ulp)", flush=True)
    assert ulp.max() <= 1 and diff.mean() <= (1e-3 if correct else 0.0)
    np.testing.assert_array_equal(got[1], ref[1].astype(np.float32))
    np.testing.assert_array_equal(got[2], ref[2].astype(np.float32))
    for k in range(3):
        np.testing.assert_allclose(got[3 + k], ref[3][k], atol=1e-7)


@pytest.mark.parametrize("fmt", [P.DEPTH_EYE_Z, P.DEPTH_WINDOW_U24])
def test_frame_on_a_reprojected_gbuffer(lidar, oracle_mod, fmt):
    """The plain path on the reprojected G-buffer against the oracle on the
    oracle's reprojection (Gaussian beams over the raster)."""
    import torch
    src = scenes.pinhole_render(5, width=800, height=300, hfov_deg=70.0, pitch_deg=-3.0, fmt=fmt,
                                near=0.3, far=800.0, n_boxes=12)
    planes = _upload(lidar, src)
    az, el = scenes.grid_beams(RASTER, 60, 12)
    pat = scenes.Pattern(scenes.PATTERN_GAUSS, az, el, sigma_deg=(0.2, 0.2), trunc_sigmas=3.0)
    sim = lidar.LidarSim(PARAMS, stream=torch.cuda.current_stream(), keep_waveforms=True)
    try:
        sim.set_pattern(pat)
        sim.set_gbuffer_pinhole(src, planes, RASTER)
        sim.simulate_frame()
        got = sim.read(waveforms=True)
    finally:
        sim.close()
    gb = P.to_gbuffer(RASTER, P.reproject(src.as_dict(), RASTER))
    ref = oracle_mod.simulate(gb, pat, PARAMS)
    rep = compare(got, ref, PARAMS)
    print(f"[pinhole] frame fmt {fmt}: {rep.echoes_compared} echoes", flush=True)
    assert rep.echoes_compared > 300


def test_pinhole_errors(lidar):
    import torch
    src = scenes.pinhole_render(0, width=64, height=32, fmt=P.DEPTH_RANGE, n_boxes=0)
    planes = _upload(lidar, src)
    sim = lidar.LidarSim(PARAMS, stream=torch.cuda.current_stream())
    try:
        buf = np.zeros(6, dtype=np.float32)
        assert sim._lib.lidar_sim_read_gbuffer(sim._h, buf.ctypes.data, 0) == lidar.LIDAR_E_STATE
        bad = scenes.Pinhole(**{**src.__dict__, "rot": src.rot * 1.1})
        with pytest.raises(lidar.LidarError) as e:
            sim.set_gbuffer_pinhole(bad, planes, RASTER)
        assert e.value.status == lidar.LIDAR_E_INVALID and "orthonormal" in str(e.value)
        win = scenes.Pinhole(**{**src.__dict__, "fmt": P.DEPTH_WINDOW_F32, "near": 5.0, "far": 1.0})
        with pytest.raises(lidar.LidarError) as e:
            sim.set_gbuffer_pinhole(win, planes, RASTER)
        assert e.value.status == lidar.LIDAR_E_INVALID
    finally:
        sim.close()
