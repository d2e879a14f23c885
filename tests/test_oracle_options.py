"""Pins of the oracle's options against closed forms, invariants and the
paper's second algorithm: the tabulated pulse, the collector-sensitivity
table of the sun term, the two range modes (normal-based range correction,
pixel range intervals) and echo selection."""
import math
from dataclasses import replace

import numpy as np
import pytest

import scenes
from scenes import Raster, Pattern, SensorParams, PATTERN_GAUSS, PATTERN_TABLE

from . import brute

C = 299792458.0


def _params(**kw):
    base = dict(n_bins=256, bin_ns=1.0, max_echoes=4, threshold=1e-3, emit_power=1.0,
                pulse_fwhm_ns=4.0, pulse_trunc_sigmas=4.0, ambient_const=0.0,
                sun_irradiance=0.0, sun_dir=(0.0, 0.0, 1.0))
    base.update(kw)
    return SensorParams(**base)


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def _dir(az_deg, el_deg):
    a, e = np.radians(az_deg), np.radians(el_deg)
    return np.array([np.cos(e) * np.cos(a), np.cos(e) * np.sin(a), np.sin(e)])


def plane_gbuffer(raster, normal, point, rho=0.5):
    """A plane n.x = n.point rendered exactly: every pixel-centre ray's
    distance to the plane (inf where the ray misses it), the plane normal
    everywhere."""
    n = _unit(normal)
    c = float(n @ np.asarray(point, dtype=np.float64))
    p = scenes.pixel_directions(raster)
    nd = np.einsum("i,ihw->hw", n, p)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = c / nd
    t = np.where((t > 0) & np.isfinite(t), t, np.inf)
    H, W = t.shape
    nrm = np.broadcast_to(n[:, None, None], (3, H, W)).astype(np.float32).copy()
    return scenes.GBuffer(raster, t.astype(np.float32), np.full((H, W), rho, np.float32),
                          np.ones((H, W), np.float32), nrm), n, c


# ---------------------------------------------------------------------------
# tabulated pulse
# ---------------------------------------------------------------------------

def _shell(R=256, dt=1.0, **kw):
    raster = Raster(160, 120, -8.0, 8.0, -6.0, 6.0)
    gb = scenes.shell_gbuffer(raster, 30.0, 0.5)
    pat = Pattern(PATTERN_GAUSS, np.array([0.03, -1.51]), np.array([0.02, 1.17]),
                  sigma_deg=(0.3, 0.2), trunc_sigmas=3.0)
    return gb, pat, _params(n_bins=R, bin_ns=dt, threshold=1e-5, **kw)


def test_tabulated_gaussian_pulse_equals_the_fwhm_path(oracle_mod):
    """A table of Gaussian samples (any scale) gives the FWHM path's taps
    and the same waveforms, to rounding."""
    gb, pat, p = _shell(ambient_const=3e-8)
    taps = oracle_mod.pulse_taps(p)
    J = len(taps) // 2
    sigma = 4.0 / (2 * math.sqrt(2 * math.log(2)))
    t = np.arange(-J, J + 1) * 1.0
    table = 3.7 * np.exp(-t * t / (2 * sigma * sigma))
    pt = replace(p, pulse_taps=table, pulse_fwhm_ns=0.0)
    np.testing.assert_allclose(oracle_mod.pulse_taps(pt), taps, rtol=1e-15, atol=1e-17)
    a = oracle_mod.simulate(gb, pat, p)
    b = oracle_mod.simulate(gb, pat, pt)
    np.testing.assert_allclose(b.xi_hat, a.xi_hat, rtol=1e-14, atol=1e-22)
    np.testing.assert_array_equal(b.n_echoes, a.n_echoes)


def test_asymmetric_tabulated_pulse_is_convolved_not_correlated(oracle_mod):
    """A single return a at bin k_d under the pulse (1, 2, 0, 0, 0) / 3: the
    convolution puts varpi(j dt) at bin k_d + j, i.e. a/3 at k_d - 2 and
    2a/3 at k_d - 1, nothing at or after k_d."""
    gb, pat, p = _shell()
    p = replace(p, pulse_taps=np.array([1.0, 2.0, 0.0, 0.0, 0.0]), pulse_fwhm_ns=0.0)
    res = oracle_mod.simulate(gb, pat, p)
    a = 0.5 / (math.pi * 30.0 ** 2)
    for b in range(pat.n_beams):
        xh = res.xi_hat[b]
        assert xh[198] == pytest.approx(a / 3, rel=1e-8)
        assert xh[199] == pytest.approx(2 * a / 3, rel=1e-8)
        assert np.all(np.delete(xh, [198, 199]) == 0.0)


def test_single_tap_pulse_leaves_the_raw_signal(oracle_mod):
    gb, pat, p = _shell(ambient_const=1e-9)
    p = replace(p, pulse_taps=np.array([0.25]), pulse_fwhm_ns=0.0)
    res = oracle_mod.simulate(gb, pat, p)
    np.testing.assert_allclose(res.xi_hat, res.xi + 1e-9, rtol=1e-15, atol=0)


# ---------------------------------------------------------------------------
# collector sensitivity kappa for the sun term
# ---------------------------------------------------------------------------

def _aligned_table_scene(sun_rho=math.pi):
    """0.0625-deg pixels and 129 x 129 tables whose cell centres fall on the
    kernel offsets (half extent 4.03125 deg, M = N = 64); a wall facing the
    sun (n = s) with rho = pi, so that A_b = E_sun sum kappa Omega."""
    raster = Raster(256, 256, -8.0, 8.0, -8.0, 8.0)
    n = np.zeros((3, 256, 256), np.float32)
    n[2] = 1.0
    gb = scenes.GBuffer(raster, np.full((256, 256), 10.0, np.float32),
                        np.full((256, 256), sun_rho, np.float32), np.ones((256, 256), np.float32), n)
    x = -4.0 + 0.0625 * np.arange(129)
    yy, xx = np.meshgrid(-x, x, indexing="ij")
    core = np.exp(-0.5 * ((xx / 0.1) ** 2 + (yy / 0.15) ** 2)).astype(np.float32)
    return raster, gb, xx, yy, core


def test_kappa_table_closed_form_sun_floor(oracle_mod):
    """With kappa a wide Gaussian (0.6 x 0.4 deg) and a narrow combined
    pattern, the sun floor is E_sun sum kappa Omega = E_sun 2 pi s_x s_y
    (rad^2, Poisson summation) times <cos e> ~ 1 - 3e-5: it follows kappa,
    not K / max K."""
    raster, gb, xx, yy, core = _aligned_table_scene()
    kappa = np.exp(-0.5 * ((xx / 0.6) ** 2 + (yy / 0.4) ** 2)).astype(np.float32)
    pat = Pattern(PATTERN_TABLE, np.array([0.03125]), np.array([-0.03125]), table=core,
                  half_deg=(4.03125, 4.03125), rx_table=kappa)
    p = _params(sun_irradiance=2.0, n_bins=128)
    res = oracle_mod.simulate(gb, pat, p)
    expect = 2.0 * 2 * math.pi * math.radians(0.6) * math.radians(0.4)
    assert res.floor[0] == pytest.approx(expect, rel=1e-4)
    plain = oracle_mod.simulate(gb, replace(pat, rx_table=None), p)
    assert plain.floor[0] == pytest.approx(2.0 * 2 * math.pi * math.radians(0.1) * math.radians(0.15),
                                           rel=1e-3)


def test_kappa_table_equal_to_normalised_pattern_reproduces_the_floor(oracle_mod):
    """kappa = K / max K given as a table gives the default floor; the floor
    is linear in kappa."""
    raster, gb, xx, yy, core = _aligned_table_scene(sun_rho=0.4)
    pat = Pattern(PATTERN_TABLE, np.array([0.03125, 1.3]), np.array([-0.03125, -2.2]), table=core,
                  half_deg=(4.03125, 4.03125))
    p = _params(sun_irradiance=0.7, n_bins=128, sun_dir=tuple(_unit([0.2, 0.1, 1.0])))
    K = oracle_mod.kernel_grid(raster, pat)
    base = oracle_mod.simulate(gb, pat, p)
    norm = (core / np.float32(K.max())).astype(np.float32)
    same = oracle_mod.simulate(gb, replace(pat, rx_table=norm), p)
    np.testing.assert_allclose(same.floor, base.floor, rtol=1e-7)
    half = oracle_mod.simulate(gb, replace(pat, rx_table=(0.5 * norm).astype(np.float32)), p)
    np.testing.assert_allclose(half.floor, 0.5 * same.floor, rtol=1e-12)
    np.testing.assert_array_equal(half.xi, base.xi)        # the laser signal is untouched


# ---------------------------------------------------------------------------
# range modes: normal-based correction and pixel range intervals
# ---------------------------------------------------------------------------

def test_plane_range_limits(oracle_mod):
    p = np.array([1.0, 0.0, 0.0])
    n = np.array([-1.0, 0.0, 0.0])
    w = _unit([1.0, 0.3, 0.0])
    assert oracle_mod.plane_range(10.0, p, w, n) == pytest.approx(10.0 * 1.0 / (w @ -n))
    # ratio above 2 (grazing), of the wrong sign (ray misses the facing side)
    # and below 1/2
    w2 = _unit([0.3, 1.0, 0.0])
    assert w2 @ n > -0.5 and oracle_mod.plane_range(10.0, p, w2, n) == 20.0
    assert oracle_mod.plane_range(10.0, p, np.array([-1.0, 0.0, 0.0]), n) == 20.0
    pg, ng = _unit([1.0, 0.0, 0.0]), _unit([-0.2, -1.0, 0.0])
    wg = _unit([0.2, 1.0, 0.0])
    q = (pg @ ng) / (wg @ ng)
    assert 0 < q < 0.5 and oracle_mod.plane_range(10.0, pg, wg, ng) == 5.0


def _tilted_plane(incidence_deg, dist=20.0, raster=None):
    """A plane at `dist` m along the forward axis whose normal leans
    `incidence_deg` from -x towards +y (the range grows along azimuth)."""
    raster = raster or Raster(64, 32, -2.0, 2.0, -1.0, 1.0)          # 0.0625 deg pixels
    a = math.radians(incidence_deg)
    return plane_gbuffer(raster, (-math.cos(a), -math.sin(a), 0.0), (dist, 0.0, 0.0))


def test_corrected_range_is_the_true_ray_plane_intersection(oracle_mod):
    """One-cell kernel (3 sigma below a pixel): in the corrected mode the
    single bin of each beam is the bin of the exact distance to the plane
    along the beam's own direction, in the centre mode the bin of its
    pixel-centre distance; both differ over the pixel (0.1 ns bins, 70 deg
    incidence: about 4 bins across a pixel)."""
    gb, n, c = _tilted_plane(70.0)
    rng = np.random.default_rng(5)
    az = rng.uniform(-1.5, 1.5, 40)
    el = rng.uniform(-0.8, 0.8, 40)
    pat = Pattern(PATTERN_GAUSS, az, el, sigma_deg=(0.01, 0.01), trunc_sigmas=3.0)
    p = _params(n_bins=2048, bin_ns=0.1, threshold=1e9)
    to_bin = 2.0 / (C * 0.1e-9)
    cen = oracle_mod.simulate(gb, pat, p)
    cor = oracle_mod.simulate(gb, pat, replace(p, range_mode=scenes.RANGE_CORRECTED))
    checked = moved = 0
    for b in range(40):
        x = c / (n @ _dir(az[b], el[b])) * to_bin
        if abs(x - round(x)) < 0.01:
            continue                      # float32 G-buffer inputs decide this bin
        checked += 1
        nz = np.flatnonzero(cor.xi[b])
        assert list(nz) == [math.floor(x)], (b, x, nz)
        kc = np.flatnonzero(cen.xi[b])
        assert list(kc) == [math.floor(float(gb.depth[cen.pixel[b, 1], cen.pixel[b, 0]]) * to_bin)]
        moved += kc[0] != nz[0]
        assert cor.xi[b].sum() == cen.xi[b].sum()
    assert checked >= 35 and moved >= 20


def test_corrected_range_moves_weight_between_bins_only(oracle_mod):
    """A 3-sigma Gaussian of several pixels on the tilted plane: the
    corrected waveform holds the same total as the centre-range one, spread
    over the bins of the cells' exact ray distances."""
    gb, n, c = _tilted_plane(60.0)
    pat = Pattern(PATTERN_GAUSS, np.array([0.01, -0.77]), np.array([0.02, 0.31]),
                  sigma_deg=(0.15, 0.1), trunc_sigmas=3.0)
    p = _params(n_bins=2048, bin_ns=0.1, threshold=1e9)
    cen = oracle_mod.simulate(gb, pat, p)
    cor = oracle_mod.simulate(gb, pat, replace(p, range_mode=scenes.RANGE_CORRECTED))
    np.testing.assert_allclose(cor.xi.sum(axis=1), cen.xi.sum(axis=1), rtol=1e-12)
    to_bin = 2.0 / (C * 0.1e-9)
    r = gb.raster
    for b in range(2):
        u, v = cor.pixel[b]
        M = int(math.floor(0.45 / r.dphi))
        N = int(math.floor(0.3 / r.de))
        bins = set()
        for m in range(-M, M + 1):
            for k in range(-N, N + 1):
                if (m * r.dphi / 0.15) ** 2 + (k * r.de / 0.1) ** 2 > 9:
                    continue
                x = c / (n @ _dir(pat.beam_az[b] + m * r.dphi, pat.beam_el[b] - k * r.de)) * to_bin
                bins.add(math.floor(x))
        got = set(np.flatnonzero(cor.xi[b]).tolist())
        assert got <= bins | {x + d for x in bins for d in (-1, 1)}
        assert len(got & bins) >= 0.9 * len(got)


def test_pixel_interval_of_a_tilted_plane(oracle_mod):
    """The interval of a pixel on a plane n.x = c: the smallest and largest
    of c / (n.w) over the pixel's centre and four corner rays w."""
    for inc in (0.0, 35.0, 70.0):
        gb, n, c = _tilted_plane(inc)
        r = gb.raster
        for (u, v) in ((3, 4), (31, 16), (60, 29)):
            ws = [_dir(r.az_min + (u + du) * r.dphi, r.el_max - (v + dv) * r.de)
                  for du in (0, 1) for dv in (0, 1)]
            ts = [c / (n @ w) for w in ws]
            d = c / (n @ _dir(r.az_min + (u + 0.5) * r.dphi, r.el_max - (v + 0.5) * r.de))
            r0, r1 = oracle_mod.pixel_interval(r, u, v, d, n)
            assert r0 == pytest.approx(min(ts + [d]), rel=1e-12)
            assert r1 == pytest.approx(max(ts + [d]), rel=1e-12)
            if inc == 0.0 and u == 31:
                # facing the sensor: second order in the pixel angle (20 m x 1.2e-6)
                assert r1 - r0 < 5e-5


def test_interval_mode_conserves_energy_and_widens_epw_with_tilt(oracle_mod):
    """Sharing each pixel's weight over the bins of its interval keeps every
    beam's total; at growing incidence the echo pulse width grows (section
    II-C: at flat incidence the EPW is dominated by the geometric range
    interval)."""
    epw = []
    for inc in (0.0, 40.0, 60.0, 70.0, 78.0):
        gb, n, c = _tilted_plane(inc, raster=Raster(96, 48, -3.0, 3.0, -1.5, 1.5))
        pat = Pattern(PATTERN_GAUSS, np.array([0.01]), np.array([0.02]), sigma_deg=(0.2, 0.2),
                      trunc_sigmas=3.0)
        p = _params(n_bins=1024, bin_ns=0.25, pulse_fwhm_ns=2.0, threshold=1e-12)
        cen = oracle_mod.simulate(gb, pat, p)
        itv = oracle_mod.simulate(gb, pat, replace(p, range_mode=scenes.RANGE_INTERVAL,
                                                   threshold=0.2 * float(cen.xi_hat.max())))
        np.testing.assert_allclose(itv.xi.sum(axis=1), cen.xi.sum(axis=1), rtol=1e-12)
        assert itv.n_echoes[0] == 1
        epw.append(float(itv.echoes[0, 0]["pulse_width_ns"]))
    assert all(b >= a for a, b in zip(epw, epw[1:])), epw
    assert epw[-1] > 2.0 * epw[0], epw


# ---------------------------------------------------------------------------
# echo selection
# ---------------------------------------------------------------------------

def _three_runs():
    xh = np.zeros(40)
    xh[5:8] = [2.0, 3.0, 2.0]          # crossings at 5.0 and 8.0: EPW 3
    xh[12:21] = 2.0                    # EPW 9
    xh[25:27] = [5.0, 5.0]             # crossings at 24.7 and 27.3: EPW 2.6, peak 5
    return xh


@pytest.mark.parametrize("mode,first,peak,epw", [
    (scenes.ECHO_SELECT_NEAREST, 5, 6, 3.0), (scenes.ECHO_SELECT_STRONGEST, 25, 25, 2.6),
    (scenes.ECHO_SELECT_LONGEST, 12, 12, 9.0)])
def test_echo_selection_of_hand_made_runs(oracle_mod, mode, first, peak, epw):
    xh = _three_runs()
    n, e = oracle_mod.select(xh, xh, 1.0, 0.5, 1.0, 3, mode)
    assert n == 3
    assert e[0]["bin_first"] == first and e[0]["bin_peak"] == peak
    assert e[0]["pulse_width_ns"] == pytest.approx(epw, abs=1e-12)
    assert e[0]["intensity"] == pytest.approx(xh[peak] - 0.5)
    assert np.all(e[1:]["bin_last"] == 0)
    # the selected echo is one of the echoes of the default mode
    n_all, e_all = oracle_mod.select(xh, xh, 1.0, 0.5, 1.0, 3, scenes.ECHO_SELECT_ALL)
    assert n_all == 3 and e[0] in e_all


def test_echo_selection_ties_take_the_first_run(oracle_mod):
    xh = np.zeros(30)
    xh[3:6] = [2.0, 4.0, 2.0]
    xh[15:18] = [2.0, 4.0, 2.0]
    for mode in (scenes.ECHO_SELECT_STRONGEST, scenes.ECHO_SELECT_LONGEST):
        n, e = oracle_mod.select(xh, xh, 1.0, 0.0, 1.0, 2, mode)
        assert n == 2 and e[0]["bin_peak"] == 4


def test_raw_selection_of_a_hand_made_signal(oracle_mod):
    """Without the pulse: the nearest bin at or above T (Alg. 2's >= rho_min)
    and the strongest bin (first of equal maxima), as one-bin echoes."""
    xi = np.array([0.0, 0.0, 0.5, 1.0, 3.0, 1.0, 0.0, 2.0, 3.0, 0.0])
    n, e = oracle_mod.select(xi, xi * 0, 1.0, 0.0, 0.5, 2, scenes.ECHO_SELECT_RAW_NEAREST)
    assert n == 1 and e[0]["bin_peak"] == e[0]["bin_first"] == e[0]["bin_last"] == 3
    assert e[0]["intensity"] == 1.0 and e[0]["pulse_width_ns"] == 0.0
    assert e[0]["time_ns"] == 1.75 and e[0]["range_m"] == pytest.approx(3.5 * 0.25 * C * 1e-9)
    n, e = oracle_mod.select(xi, xi * 0, 1.0, 0.0, 0.5, 2, scenes.ECHO_SELECT_RAW_STRONGEST)
    assert n == 1 and e[0]["bin_peak"] == 4 and e[0]["intensity"] == 3.0
    n, e = oracle_mod.select(xi, xi * 0, 3.5, 0.0, 0.5, 2, scenes.ECHO_SELECT_RAW_NEAREST)
    assert n == 0 and e[0]["bin_last"] == 0


def test_raw_nearest_is_range_stacking_at_the_beam_pixel(oracle_mod):
    """Alg. 2 (per-slice correlation, nearest slice at or above rho_min)
    sampled at a beam's pixel equals Alg. 1's raw nearest echo when rho_min
    is T over the beam's scale: the two algorithms correspond (section
    II-C)."""
    from oracle import range_stacking as rs
    rng = np.random.default_rng(4)
    raster = Raster(32, 16, -6.0, 6.0, -2.0, 4.0)
    gb = scenes.random_gbuffer(raster, rng, depth_range=(3.0, 40.0), retro_frac=0.1)
    az = np.array([0.1, -4.9, 4.95, 2.0, -1.3, 3.3])
    el = np.array([1.0, 3.2, -1.4, 0.2, -1.1, 2.5])
    pat = Pattern(PATTERN_GAUSS, az, el, sigma_deg=(0.6, 0.45), trunc_sigmas=3.0)
    p = _params(n_bins=300, bin_ns=1.0)
    plain = oracle_mod.simulate(gb, pat, p)
    T = 0.4 * float(np.median(plain.xi.max(axis=1)))
    res = oracle_mod.simulate(gb, pat, replace(p, threshold=T,
                                               echo_select=scenes.ECHO_SELECT_RAW_NEAREST))
    K = oracle_mod.kernel_grid(raster, pat)
    d = gb.depth.astype(np.float64)
    bins = np.floor(d * 2.0 / (C * 1e-9)).astype(np.int64)
    phi = np.radians(raster.az_min + (np.arange(32) + 0.5) * raster.dphi)
    el_c = np.radians(raster.el_max - (np.arange(16) + 0.5) * raster.de)
    view = np.stack([np.cos(el_c)[:, None] * np.cos(phi)[None, :],
                     np.cos(el_c)[:, None] * np.sin(phi)[None, :],
                     np.broadcast_to(np.sin(el_c)[:, None], d.shape)])
    cos_t = np.maximum(0.0, -(gb.normal.astype(np.float64) * view).sum(0))
    om = np.array([brute.row_solid_angle(raster, v) for v in range(16)])[:, None]
    inten = gb.retro_gain * gb.reflectance.astype(np.float64) / math.pi * cos_t / (d * d) * om
    found = 0
    for b in range(pat.n_beams):
        u, v = res.pixel[b]
        s_near, xi_near = rs.nearest_above(inten, bins, K, 300, T / res.scale[b])
        if s_near[v, u] < 300:
            found += 1
            assert res.n_echoes[b] == 1 and res.echoes[b, 0]["bin_peak"] == s_near[v, u]
            assert res.echoes[b, 0]["intensity"] == pytest.approx(xi_near[v, u] * res.scale[b],
                                                                  rel=1e-12)
        else:
            assert res.n_echoes[b] == 0
    assert found >= 4


def test_corrected_range_of_an_offset_cell(oracle_mod):
    """A table whose only non-zero cell sits at (m, n) = (+2, -1) (cell
    centres on the 0.0625-deg pixel offsets): the corrected sample lies on
    the ray through the beam centre shifted by 2 pixels in azimuth and one
    up, dir(az_b + 2 dphi, el_b + de), at the plane's exact distance along
    it; the centre mode uses the depth of pixel (u_b + 2, v_b - 1)."""
    # a plane leaning in azimuth and in elevation: the range changes along both
    gb, n, c = plane_gbuffer(Raster(64, 32, -2.0, 2.0, -1.0, 1.0), (-1.0, -2.0, -1.5), (20.0, 0.0, 0.0))
    r = gb.raster
    t = np.zeros((9, 9), np.float32)
    t[3, 6] = 1.0
    rng = np.random.default_rng(8)
    az = rng.uniform(-1.5, 1.5, 40)
    el = rng.uniform(-0.8, 0.8, 40)
    pat = Pattern(PATTERN_TABLE, az, el, table=t, half_deg=(0.28125, 0.28125))
    K = oracle_mod.kernel_grid(r, pat)
    assert K.shape == (9, 9) and K[3, 6] == 1.0 and K.sum() == 1.0
    p = _params(n_bins=2048, bin_ns=0.1, threshold=1e9)
    to_bin = 2.0 / (C * 0.1e-9)
    cen = oracle_mod.simulate(gb, pat, p)
    cor = oracle_mod.simulate(gb, pat, replace(p, range_mode=scenes.RANGE_CORRECTED))
    checked = 0
    for b in range(40):
        x = c / (n @ _dir(az[b] + 2 * r.dphi, el[b] + r.de)) * to_bin
        if abs(x - round(x)) < 0.01:
            continue
        checked += 1
        assert list(np.flatnonzero(cor.xi[b])) == [math.floor(x)], (b, x)
        u, v = cen.pixel[b]
        assert list(np.flatnonzero(cen.xi[b])) == [math.floor(float(gb.depth[v - 1, u + 2]) * to_bin)]
    assert checked >= 35


def test_range_stacking_with_a_separable_kernel():
    """For kappa eta = H * V (section III-B, Alg. 2's separable speed-up) the
    per-slice 2-D correlation with K[n][m] = V[n] H[m] equals a correlation
    along the rows with H followed by one along the columns with V (library
    1-D correlations); the nearest slice at or above rho_min follows."""
    from scipy import ndimage
    from oracle import range_stacking as rs
    rng = np.random.default_rng(9)
    inten = rng.uniform(0.0, 1.0, (40, 56)) * (rng.uniform(size=(40, 56)) < 0.6)
    bins = rng.integers(0, 12, (40, 56))
    Hk = rng.uniform(0.1, 1.0, 9)          # columns m = -4..4
    Vk = rng.uniform(0.1, 1.0, 5)          # rows n = -2..2
    K = np.outer(Vk, Hk)
    for s in (0, 5, 11):
        img = np.where(bins == s, inten, 0.0)
        two = ndimage.correlate1d(ndimage.correlate1d(img, Hk, axis=1, mode="constant"), Vk, axis=0,
                                  mode="constant")
        np.testing.assert_allclose(rs.slice_correlations(inten, bins, K, 12, [s])[s], two,
                                   rtol=1e-12, atol=1e-14)
    rho = 1.5
    s_near, xi_near = rs.nearest_above(inten, bins, K, 12, rho)
    stack = np.stack([ndimage.correlate1d(ndimage.correlate1d(np.where(bins == s, inten, 0.0), Hk, axis=1,
                                                              mode="constant"), Vk, axis=0, mode="constant")
                      for s in range(12)])
    above = stack >= rho
    first = np.where(above.any(0), above.argmax(0), 12)
    np.testing.assert_array_equal(s_near, first)
