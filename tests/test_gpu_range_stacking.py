"""Range stacking (Alg. 2) with a separable kernel on the GPU, through the
C-ABI, against the FP64 oracle.

Small images: every pixel against the oracle's Alg. 2 (library per-slice
2-D correlations of the FP64 intensities).  Larger images: sampled pixels
against the oracle's Alg. 1 (a beam centred on the pixel, the table pattern
equal to V[n] H[m] on the pixel offsets): the correlation of slice k at the
pixel is the beam's raw xi[k] / S_b, and the paper states that both
algorithms agree.  A pixel is ambiguous when some slice's correlation lies
within 2e-5 of its largest correlation from rho_min (FP32 sums of up to
KW + KH terms); elsewhere the nearest slice is exact and its value within
2e-5 relative."""
import math

import numpy as np
import pytest

import scenes
from oracle import range_stacking as RS
from oracle import surrogate as SUR

pytestmark = pytest.mark.gpu
TOL = 2e-5


@pytest.fixture(scope="module")
def lidar():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_05932_amd as lidar
    lidar.load()
    return lidar


def _gpu(lidar, gb, params, Hk, Vk, rho):
    import torch
    planes = lidar.upload_gbuffer(gb, "cuda")
    H, W = gb.depth.shape
    s_out = torch.full((H, W), -5, dtype=torch.int32, device="cuda")
    x_out = torch.full((H, W), -1.0, dtype=torch.float32, device="cuda")
    sim = lidar.LidarSim(params, stream=torch.cuda.current_stream())
    try:
        sim.set_gbuffer(gb.raster, planes)
        sim.range_stacking(Hk, Vk, rho, s_out, x_out)
        torch.cuda.synchronize()
    finally:
        sim.close()
    return s_out.cpu().numpy(), x_out.cpu().numpy()


def _gauss(half, sigma, shift=0.0):
    """Gaussian factor on offsets -half..half, centred at `shift` (a skewed
    factor makes a swapped or reversed factor visible)."""
    x = np.arange(-half, half + 1)
    return np.exp(-0.5 * ((x - shift) / sigma) ** 2).astype(np.float32)


@pytest.mark.parametrize("seed,half,n_bins", [(0, (4, 2), 96), (1, (9, 6), 96), (2, (0, 0), 96),
                                             (3, (127, 40), 4000)])
def test_every_pixel_of_small_images(lidar, oracle_mod, seed, half, n_bins):
    """Every pixel against Alg. 2.  The last case has the largest kernel
    (wider and taller than the image) and 4000 bins, so the per-row slice
    bitmaps do not fit the workgroup's LDS and every window row is staged."""
    rng = np.random.default_rng(seed)
    r = scenes.Raster(70, 37, -7.0, 7.0, -3.0, 4.4)
    gb = scenes.random_gbuffer(r, rng, depth_range=(3.0, 12.0), retro_frac=0.05)
    d = gb.depth.copy()
    d[rng.uniform(size=d.shape) < 0.1] = np.inf
    gb = scenes.GBuffer(r, d, gb.reflectance, gb.retro_gain, gb.normal)
    p = scenes.SensorParams(n_bins=n_bins, bin_ns=1.0, max_echoes=3, threshold=1e-6, emit_power=1.0,
                            pulse_fwhm_ns=4.0)
    Hk = _gauss(half[0], max(half[0], 1) / 2.0, 0.4 * half[0])
    Vk = _gauss(half[1], max(half[1], 1) / 2.0, -0.5 * half[1])
    t = SUR.pixel_terms(gb, p, lambda v: oracle_mod.row_solid_angle(r, v))
    inten, bins = t["shade"], t["kbin"].astype(np.int64)
    K = np.outer(Vk.astype(np.float64), Hk.astype(np.float64))
    corr = RS.slice_correlations(inten, bins, K, p.n_bins)
    top = np.max(np.stack(list(corr.values())), axis=0)
    rho = 0.4 * float(np.median(top[top > 0]))
    s_ref, x_ref = RS.nearest_above(inten, bins, K, p.n_bins, rho)
    amb = np.zeros(inten.shape, bool)
    for c in corr.values():
        amb |= np.abs(c - rho) <= TOL * top
    s_gpu, x_gpu = _gpu(lidar, gb, p, Hk, Vk, rho)
    ok = ~amb
    print(f"[rs] seed {seed}: {ok.sum()} of {ok.size} pixels unambiguous, "
          f"{(s_ref[ok] < p.n_bins).sum()} with a slice", flush=True)
    np.testing.assert_array_equal(s_gpu[ok], s_ref[ok])
    np.testing.assert_allclose(x_gpu[ok], x_ref[ok], rtol=TOL, atol=0)
    assert (s_ref[ok] < p.n_bins).sum() > 200


def test_sampled_pixels_of_a_road_scene_against_beam_iteration(lidar, oracle_mod):
    """2048 x 128 road scene (0.0625 x 0.03125 deg pixels), 69 x 41 separable
    Gaussian kernel, 2048 bins of 0.5 ns; 400 sampled pixels."""
    r = scenes.Raster(2048, 128, -64.0, 64.0, -2.0, 2.0)
    gb, boxes, obj = scenes.road_scene(r, np.random.default_rng(3))
    p = scenes.SensorParams(n_bins=2048, bin_ns=0.5, max_echoes=3, threshold=1e-12, emit_power=1.0,
                            pulse_fwhm_ns=4.0, echo_select=scenes.ECHO_SELECT_RAW_NEAREST)
    M, N = 34, 20
    Hk, Vk = _gauss(M, 11.0, 6.0), _gauss(N, 7.0, -4.0)
    # a table on the pixel offsets: cell centres at m dphi, n de
    table = np.outer(Vk, Hk).astype(np.float32)
    rng = np.random.default_rng(4)
    us = rng.integers(0, 2048, 400)
    vs = rng.integers(0, 128, 400)
    az = r.az_min + (us + 0.5) * r.dphi
    el = r.el_max - (vs + 0.5) * r.de
    pat = scenes.Pattern(scenes.PATTERN_TABLE, az, el, table=table,
                         half_deg=((2 * M + 1) * r.dphi / 2, (2 * N + 1) * r.de / 2))
    K = oracle_mod.kernel_grid(r, pat)
    np.testing.assert_allclose(K, np.outer(Vk, Hk), rtol=1e-12)
    ref = oracle_mod.simulate(gb, pat, p, want_xi_hat=False)
    assert np.array_equal(ref.pixel[:, 0], us) and np.array_equal(ref.pixel[:, 1], vs)
    corr = ref.xi / ref.scale[:, None]                      # slice correlations at the pixels
    top = corr.max(axis=1)
    rho = 0.3 * float(np.median(top[top > 0]))
    s_gpu, x_gpu = _gpu(lidar, gb, p, Hk, Vk, rho)
    checked = found = 0
    for b in range(400):
        if np.any(np.abs(corr[b] - rho) <= TOL * top[b]):
            continue
        checked += 1
        above = np.flatnonzero(corr[b] >= rho)
        g = s_gpu[vs[b], us[b]]
        if above.size:
            found += 1
            assert g == above[0], (b, g, above[0])
            assert x_gpu[vs[b], us[b]] == pytest.approx(corr[b, above[0]], rel=TOL)
        else:
            assert g == p.n_bins and x_gpu[vs[b], us[b]] == 0.0
    print(f"[rs] road: {checked} sampled pixels checked, {found} with a slice", flush=True)
    assert checked > 350 and found > 150


def test_nothing_reaches_a_high_rho_min(lidar):
    r = scenes.Raster(64, 32, -4.0, 4.0, -2.0, 2.0)
    gb = scenes.shell_gbuffer(r, 20.0, 0.5)
    p = scenes.SensorParams(n_bins=256, bin_ns=1.0, max_echoes=3, threshold=1e-6, emit_power=1.0,
                            pulse_fwhm_ns=4.0)
    s_gpu, x_gpu = _gpu(lidar, gb, p, _gauss(3, 1.5), _gauss(2, 1.0), 1e6)
    assert np.all(s_gpu == 256) and np.all(x_gpu == 0.0)
