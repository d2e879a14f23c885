"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, invariants, library routines, brute force on tiny images and the
paper's second algorithm.  A dropped term, a wrong sign or index, or a
transposed operand anywhere in the oracle fails at least one of them.
"""
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


# --------------------------------------------------------------------------
# a0-a1: kernel, quadrature, normalisation
# --------------------------------------------------------------------------

@pytest.mark.parametrize("sig,h", [((0.1, 0.1), (60 / 1024, 30 / 512)),
                                   ((0.07, 0.2), (0.03, 0.05))])
def test_gaussian_lattice_sum_is_2pi_sigma2(oracle_mod, sig, h):
    """Poisson summation: sum_{m,n} exp(-((mh_x/s_x)^2+(nh_y/s_y)^2)/2) h_x h_y
    = 2 pi s_x s_y up to 2 exp(-2 pi^2 s^2/h^2) (< 1e-20 here)."""
    raster = Raster(64, 64, 0.0, 64 * h[0], 0.0, 64 * h[1])
    pat = Pattern(PATTERN_GAUSS, np.zeros(1), np.zeros(1), sigma_deg=sig, trunc_sigmas=14.0)
    K = oracle_mod.kernel_grid(raster, pat)
    total = K.sum() * h[0] * h[1]
    assert total == pytest.approx(2 * math.pi * sig[0] * sig[1], rel=1e-13)


def test_gaussian_3sigma_support_has_89_cells(oracle_mod):
    """Workload 1 grid: the 3-sigma disc of sigma = 0.1 deg at 60/1024 deg per
    pixel holds the lattice points m^2 + n^2 <= (0.3 / (60/1024))^2: 89 cells."""
    w = scenes.iid_frame()
    K = oracle_mod.kernel_grid(w.gbuffer.raster, w.pattern)
    assert K.shape == (11, 11)
    r2 = (0.3 / (60 / 1024)) ** 2
    lattice = sum(1 for m in range(-6, 7) for n in range(-6, 7) if m * m + n * n <= r2)
    assert lattice == 89
    assert int((K > 0).sum()) == 89
    assert K[5, 5] == 1.0


def test_kernel_orientation_rows_go_down(oracle_mod):
    """Row offset n is downward (lower elevation): an asymmetric table with mass
    only above the centre must put its cells at negative n."""
    t = np.zeros((4, 4), np.float32)
    t[0, 1] = 1.0          # row 0 = top (+elevation), column 1 = left of centre
    raster = Raster(40, 40, 0.0, 4.0, 0.0, 4.0)        # 0.1 deg per pixel
    pat = Pattern(PATTERN_TABLE, np.zeros(1), np.zeros(1), table=t, half_deg=(0.2, 0.2))
    K = oracle_mod.kernel_grid(raster, pat)             # M = N = 2
    assert K.shape == (5, 5)
    # cell centre of t[0,1]: x = -0.2 + 1.5*0.1 = -0.05, y = 0.2 - 0.5*0.1 = 0.15
    # -> half-way between grid offsets; its mass lies at m <= 0, n <= -1
    nz = np.argwhere(K > 0)
    assert (nz[:, 0] - 2 <= -1).all() and (nz[:, 1] - 2 <= 0).all()


def test_table_bilinear_reproduces_linear_functions(oracle_mod):
    """Bilinear interpolation is exact for f = a + b x + c y between cell
    centres, returns the table values at cell centres and is zero far outside."""
    nx, ny, hx, hy = 16, 12, 2.0, 1.5
    x = -hx + (np.arange(nx) + 0.5) * (2 * hx / nx)
    y = hy - (np.arange(ny) + 0.5) * (2 * hy / ny)
    yy, xx = np.meshgrid(y, x, indexing="ij")
    f = lambda x, y: 3.0 + 0.5 * x - 0.25 * y
    t = f(xx, yy).astype(np.float32)
    pat = Pattern(PATTERN_TABLE, np.zeros(1), np.zeros(1), table=t, half_deg=(hx, hy))
    rng = np.random.default_rng(1)
    for _ in range(50):
        qx = rng.uniform(x[0], x[-1])
        qy = rng.uniform(y[-1], y[0])
        assert oracle_mod.pattern_value(pat, qx, qy) == pytest.approx(f(qx, qy), rel=1e-6)
    for j in (0, 5, 11):
        for i in (0, 7, 15):
            assert oracle_mod.pattern_value(pat, x[i], y[j]) == float(t[j, i])
    assert oracle_mod.pattern_value(pat, hx + 0.2, 0.0) == 0.0
    assert oracle_mod.pattern_value(pat, 0.0, -hy - 0.2) == 0.0


def test_row_solid_angles_tile_the_sphere(oracle_mod):
    """Rows of a full 360 x 180 deg raster add up to 4 pi sr; any raster's rows
    add up to the spherical-zone area dphi_total (sin e_max - sin e_min); a
    small pixel approaches cos(e) dphi de."""
    full = Raster(36, 90, -180.0, 180.0, -90.0, 90.0)
    tot = sum(oracle_mod.row_solid_angle(full, v) for v in range(90)) * 36
    assert tot == pytest.approx(4 * math.pi, rel=1e-14)
    r = Raster(100, 50, -20.0, 30.0, -7.0, 11.0)
    zone = math.radians(50.0) * (math.sin(math.radians(11.0)) - math.sin(math.radians(-7.0)))
    assert sum(oracle_mod.row_solid_angle(r, v) for v in range(50)) * 100 == \
        pytest.approx(zone, rel=1e-13)
    small = Raster(1000, 1000, 0.0, 1.0, 40.0, 41.0)
    e = math.radians(41.0 - 0.0005)
    assert oracle_mod.row_solid_angle(small, 0) == pytest.approx(
        math.cos(e) * math.radians(1e-3) ** 2, rel=1e-6)
    # rows outside the image continue the same zones (used by the normalisation)
    assert oracle_mod.row_solid_angle(r, -1) > 0 and oracle_mod.row_solid_angle(r, 50) > 0


def test_beam_pixel_is_the_containing_pixel(oracle_mod):
    r = Raster(40, 20, -10.0, 10.0, -5.0, 5.0)            # 0.5 deg pixels
    assert oracle_mod.beam_pixel(r, -10.0 + 0.25, 5.0 - 0.25) == (0, 0)
    assert oracle_mod.beam_pixel(r, 0.0, 0.0) == (20, 10)   # boundary -> higher index
    assert oracle_mod.beam_pixel(r, 9.99, -4.99) == (39, 19)
    assert oracle_mod.beam_pixel(r, 10.2, 0.1) == (40, 9)   # outside the image


# --------------------------------------------------------------------------
# a5: pulse
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dt,ntaps", [(1.0, 15), (0.5, 29)])
def test_pulse_taps_fwhm_sum_and_variance(oracle_mod, dt, ntaps):
    p = _params(bin_ns=dt)
    taps = oracle_mod.pulse_taps(p)
    assert taps.shape == (ntaps,)
    J = ntaps // 2
    assert taps.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_array_equal(taps, taps[::-1])
    # FWHM 4 ns: the samples 2 ns either side of the peak are at half maximum
    j_half = int(round(2.0 / dt))
    assert taps[J + j_half] / taps[J] == pytest.approx(0.5, rel=1e-14)
    # variance of the sampled Gaussian ~ sigma^2 (truncation at 4 sigma)
    sigma = 4.0 / (2 * math.sqrt(2 * math.log(2)))
    var = (((np.arange(ntaps) - J) * dt) ** 2 * taps).sum()
    assert var == pytest.approx(sigma ** 2, rel=2e-3)


# --------------------------------------------------------------------------
# a2-a6: closed forms on a constant-range shell
# --------------------------------------------------------------------------

def _shell_case(d=30.0, rho=0.5, Pe=1.0, A=0.0, T=None, dt=1.0, R=256):
    raster = Raster(160, 120, -8.0, 8.0, -6.0, 6.0)
    gb = scenes.shell_gbuffer(raster, d, rho)
    az = np.array([0.03, -1.51, 2.26])
    el = np.array([0.02, 1.17, -2.4])
    pat = Pattern(PATTERN_GAUSS, az, el, sigma_deg=(0.3, 0.2), trunc_sigmas=3.0)
    a = Pe * rho / (math.pi * d * d)
    if T is None:
        T = A + 0.3 * a * 0.2
    return gb, pat, _params(n_bins=R, bin_ns=dt, threshold=T, emit_power=Pe, ambient_const=A), a


def test_shell_single_bin_closed_form(oracle_mod):
    """Every footprint pixel at range d, facing the sensor, Lambertian rho:
    xi[k_d] = P_e rho / (pi d^2) exactly and every other bin is 0."""
    gb, pat, p, a = _shell_case()
    res = oracle_mod.simulate(gb, pat, p)
    kd = int(math.floor(30.0 * 2 / (C * 1e-9)))
    assert kd == 200
    for b in range(pat.n_beams):
        # float32 normals make cos(theta) = 1 only to ~1e-9
        assert res.xi[b, kd] == pytest.approx(a, rel=1e-8, abs=0)
        others = np.delete(res.xi[b], kd)
        assert np.all(others == 0.0)


def test_shell_echo_closed_form(oracle_mod):
    """Single target: peak xi_hat = a varpi[0] + A at bin k_d; the run is
    {k : a varpi[k-k_d] + A > T}; range within half a bin of d; the EPW is
    close to the continuous Gaussian width 2 sigma sqrt(2 ln(a varpi0/(T-A)))."""
    A = 2e-8
    gb, pat, p, a = _shell_case(A=A)
    taps = oracle_mod.pulse_taps(p)
    J = len(taps) // 2
    res = oracle_mod.simulate(gb, pat, p)
    kd = 200
    run = [kd + j for j in range(-J, J + 1) if a * taps[J + j] + A > p.threshold]
    sigma = 4.0 / (2 * math.sqrt(2 * math.log(2)))
    for b in range(pat.n_beams):
        assert res.n_echoes[b] == 1
        e = res.echoes[b, 0]
        assert e["bin_peak"] == kd
        assert e["bin_first"] == run[0] and e["bin_last"] == run[-1]
        assert e["intensity"] == pytest.approx(a * taps[J], rel=1e-8, abs=0)
        assert res.xi_hat[b, kd] == pytest.approx(a * taps[J] + A, rel=1e-8, abs=0)
        assert abs(e["range_m"] - 30.0) <= 0.25 * C * 1e-9
        assert e["time_ns"] == pytest.approx((kd + 0.5) * 1.0)
        # sampled pulse ~ Gaussian of area 1 per bin: amplitude a*varpi0
        w_cont = 2 * sigma * math.sqrt(2 * math.log(a * taps[J] / (p.threshold - A)))
        assert e["pulse_width_ns"] == pytest.approx(w_cont, abs=0.15)


def test_footprint_weights_sum_to_emitted_power(oracle_mod):
    """Sum over the footprint of the weights at unit shading (rho = pi,
    cos = 1, d = 1 m) equals P_e for an interior beam (the normalisation is the
    integral of the pattern times the pixel solid angles)."""
    raster = Raster(200, 100, -10.0, 10.0, -5.0, 5.0)
    gb = scenes.shell_gbuffer(raster, 1.0, math.pi)
    pat = Pattern(PATTERN_GAUSS, np.array([0.11, 3.3]), np.array([-0.3, 2.1]),
                  sigma_deg=(0.4, 0.25), trunc_sigmas=3.0)
    # the G-buffer holds rho = float32(pi) and float32 normals: the shading is
    # 1 to within ~1e-8, which bounds the comparison (any formula error is O(1))
    rho_f32 = float(np.float32(math.pi)) / math.pi
    for Pe in (1.0, 0.37):
        res = oracle_mod.simulate(gb, pat, _params(emit_power=Pe, bin_ns=1.0, n_bins=16))
        assert res.xi.sum(axis=1) == pytest.approx([Pe * rho_f32] * 2, rel=1e-8, abs=0)


def test_epw_monotone_intensity_linear_in_power(oracle_mod):
    widths, peaks = [], []
    for Pe in (1.0, 1.5, 2.0, 4.0, 8.0, 16.0):
        gb, pat, p, a = _shell_case(Pe=Pe, T=0.2 * 0.5 / (math.pi * 900) * 0.2)
        res = oracle_mod.simulate(gb, pat, p)
        widths.append(res.echoes[0, 0]["pulse_width_ns"])
        peaks.append(res.echoes[0, 0]["intensity"])
    assert all(b >= a for a, b in zip(widths, widths[1:]))
    assert widths[-1] > widths[0]
    ratios = np.array(peaks) / np.array([1.0, 1.5, 2.0, 4.0, 8.0, 16.0])
    assert ratios == pytest.approx(ratios[0], rel=1e-12)


# --------------------------------------------------------------------------
# invariants on the random and scanning workloads
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def w1():
    return scenes.iid_frame(0)


@pytest.fixture(scope="module")
def w1_res(oracle_mod, w1):
    return oracle_mod.simulate(w1.gbuffer, w1.pattern, w1.params)


def test_zero_emission_leaves_the_floor(oracle_mod, w1):
    p = replace(w1.params, emit_power=0.0)
    res = oracle_mod.simulate(w1.gbuffer, w1.pattern, p)
    assert np.all(res.xi == 0.0)
    assert np.all(res.xi_hat == w1.params.ambient_const)
    assert np.all(res.n_echoes == 0)


def test_energy_is_conserved_by_the_pulse(w1, w1_res):
    """Unit-sum pulse: sum_k (xi_hat - A) = sum_k xi when no signal is within
    J bins of either edge."""
    R, J = w1.params.n_bins, 7
    inner = (w1_res.xi[:, :J].sum(1) == 0) & (w1_res.xi[:, R - J:].sum(1) == 0)
    assert inner.sum() > 100
    lhs = (w1_res.xi_hat - w1_res.floor[:, None]).sum(1)[inner]
    rhs = w1_res.xi.sum(1)[inner]
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_linearity_in_power_and_scene_superposition(oracle_mod, w1, w1_res):
    p2 = replace(w1.params, emit_power=2.5)
    r2 = oracle_mod.simulate(w1.gbuffer, w1.pattern, p2)
    np.testing.assert_allclose(r2.xi, 2.5 * w1_res.xi, rtol=1e-13, atol=0)
    # split the scene into two disjoint halves (the other half is sky)
    gb = w1.gbuffer
    mask = np.random.default_rng(3).uniform(size=gb.depth.shape) < 0.5
    ga = replace(gb, depth=np.where(mask, gb.depth, np.inf).astype(np.float32))
    gbb = replace(gb, depth=np.where(mask, np.inf, gb.depth).astype(np.float32))
    ra = oracle_mod.simulate(ga, w1.pattern, w1.params)
    rb = oracle_mod.simulate(gbb, w1.pattern, w1.params)
    np.testing.assert_allclose(ra.xi + rb.xi, w1_res.xi, rtol=1e-12, atol=1e-25)


def test_invalid_pixels_contribute_nothing(oracle_mod, w1, w1_res):
    gb = w1.gbuffer
    rng = np.random.default_rng(5)
    bad = rng.uniform(size=gb.depth.shape) < 0.1
    results = []
    for fill in (np.inf, np.nan, -3.0, 0.0, 500.0):     # 500 m is beyond r_max
        g = replace(gb, depth=np.where(bad, fill, gb.depth).astype(np.float32))
        results.append(oracle_mod.simulate(g, w1.pattern, w1.params))
    for r in results[1:]:
        np.testing.assert_array_equal(r.xi, results[0].xi)
        np.testing.assert_array_equal(r.n_echoes, results[0].n_echoes)
    assert not np.array_equal(results[0].xi, w1_res.xi)


def test_azimuth_shift_invariance(oracle_mod, w1, w1_res):
    """Rotating scene (depths, normals) and beams about the vertical axis by a
    whole number of pixels leaves every waveform unchanged."""
    gb = w1.gbuffer
    s = 37
    ang = math.radians(s * gb.raster.dphi)
    c, sn = math.cos(ang), math.sin(ang)
    roll = lambda a: np.roll(a, s, axis=-1)
    n = gb.normal.astype(np.float64)
    nrot = np.stack([c * n[0] - sn * n[1], sn * n[0] + c * n[1], n[2]])
    g2 = scenes.GBuffer(gb.raster, roll(gb.depth), roll(gb.reflectance), roll(gb.retro_gain),
                        roll(nrot).astype(np.float32))
    # beams whose footprint stays inside the unwrapped part of the image
    keep = (w1.pattern.beam_az > gb.raster.az_min + 1.0) & \
        (w1.pattern.beam_az + s * gb.raster.dphi < gb.raster.az_max - 1.0)
    idx = np.nonzero(keep)[0]
    pat = replace(w1.pattern, beam_az=w1.pattern.beam_az[idx] + s * gb.raster.dphi,
                  beam_el=w1.pattern.beam_el[idx])
    res = oracle_mod.simulate(g2, pat, w1.params)
    np.testing.assert_allclose(res.xi, w1_res.xi[idx], rtol=2e-6, atol=1e-6 * w1_res.xi.max())
    np.testing.assert_array_equal(np.nonzero(res.xi)[1], np.nonzero(w1_res.xi[idx])[1])


def test_beam_permutation_permutes_outputs(oracle_mod, w1, w1_res):
    perm = np.random.default_rng(7).permutation(w1.pattern.n_beams)
    pat = replace(w1.pattern, beam_az=w1.pattern.beam_az[perm], beam_el=w1.pattern.beam_el[perm])
    res = oracle_mod.simulate(w1.gbuffer, pat, w1.params)
    np.testing.assert_array_equal(res.xi_hat, w1_res.xi_hat[perm])
    np.testing.assert_array_equal(res.echoes, w1_res.echoes[perm])


# --------------------------------------------------------------------------
# textbook routines: convolution and run-length encoding
# --------------------------------------------------------------------------

def test_pulse_is_numpy_convolve_plus_floor(oracle_mod, w1, w1_res):
    taps = oracle_mod.pulse_taps(w1.params)
    for b in range(0, w1.pattern.n_beams, 37):
        ref = np.convolve(w1_res.xi[b], taps, mode="same") + w1_res.floor[b]
        np.testing.assert_allclose(w1_res.xi_hat[b], ref, rtol=1e-13, atol=1e-20)


def _rle(mask):
    d = np.diff(np.concatenate([[0], mask.astype(np.int8), [0]]))
    return np.nonzero(d == 1)[0], np.nonzero(d == -1)[0] - 1


def test_echoes_are_run_length_encoding_of_threshold(w1, w1_res):
    T = w1.params.threshold
    for b in range(w1.pattern.n_beams):
        xh = w1_res.xi_hat[b]
        starts, ends = _rle(xh > T)
        assert w1_res.n_echoes[b] == len(starts)
        for e, (k0, k1) in zip(w1_res.echoes[b], list(zip(starts, ends))[:3]):
            assert (e["bin_first"], e["bin_last"]) == (k0, k1)
            assert e["bin_peak"] == k0 + int(np.argmax(xh[k0:k1 + 1]))
            assert e["intensity"] == xh[e["bin_peak"]] - w1_res.floor[b]


def test_echo_crossings_are_linear_interpolation(oracle_mod):
    """A triangle waveform crosses T at known times; an edge-touching run
    reports the edge time."""
    xh = np.zeros(20)
    xh[5:10] = [1.0, 3.0, 5.0, 3.0, 1.0]
    n, e = oracle_mod.detect(xh, 2.0, 0.0, 1.0, 4)
    assert n == 1
    # up: between bin centres 5.5 (1.0) and 6.5 (3.0) -> 6.0; down: 8.5 -> 9.0
    assert e[0]["pulse_width_ns"] == pytest.approx(3.0, abs=1e-15)
    assert (e[0]["bin_first"], e[0]["bin_peak"], e[0]["bin_last"]) == (6, 7, 8)
    xh2 = np.zeros(10)
    xh2[:3] = [5.0, 4.0, 1.0]
    n, e = oracle_mod.detect(xh2, 2.0, 0.0, 0.5, 4)
    assert n == 1 and e[0]["flags"] & 1
    # bin centres at 0.25, 0.75, 1.25 ns: from 0 to the crossing between
    # 0.75 ns (4.0) and 1.25 ns (1.0), i.e. 0.75 + 0.5 * 2/3
    assert e[0]["pulse_width_ns"] == pytest.approx(0.75 + 0.5 * 2 / 3, abs=1e-15)


# --------------------------------------------------------------------------
# brute force on tiny images, and the second algorithm
# --------------------------------------------------------------------------

def _tiny(kind, seed=11):
    rng = np.random.default_rng(seed)
    raster = Raster(32, 16, -6.0, 6.0, -2.0, 4.0)          # 0.375 deg pixels
    gb = scenes.random_gbuffer(raster, rng, depth_range=(3.0, 40.0), retro_frac=0.1)
    d = gb.depth.copy()
    d[rng.uniform(size=d.shape) < 0.05] = np.inf
    gb = replace(gb, depth=d)
    az = np.array([0.1, -5.9, 5.95, 2.0, 6.4, -1.3])        # interior, edges, outside
    el = np.array([1.0, 3.9, -1.9, 4.2, 0.5, -2.3])
    if kind == PATTERN_GAUSS:
        pat = Pattern(kind, az, el, sigma_deg=(0.6, 0.45), trunc_sigmas=3.0)
    else:
        t = rng.uniform(0.0, 1.0, size=(7, 9)).astype(np.float32)
        t[0, 0] = 0.0
        pat = Pattern(kind, az, el, table=t, half_deg=(1.6, 1.1))
    params = _params(n_bins=300, bin_ns=1.0, sun_irradiance=0.7,
                     sun_dir=(0.3, -0.5, math.sqrt(1 - 0.34)))
    return gb, pat, params


@pytest.mark.parametrize("kind", [PATTERN_GAUSS, PATTERN_TABLE])
def test_brute_force_tiny_images(oracle_mod, kind):
    gb, pat, params = _tiny(kind)
    res = oracle_mod.simulate(gb, pat, params)
    xi_ref, a_ref = brute.brute_xi(gb, pat, params)
    scale = np.abs(xi_ref).max()
    assert scale > 0
    np.testing.assert_allclose(res.xi, xi_ref, rtol=1e-12, atol=1e-13 * scale)
    np.testing.assert_allclose(res.floor, params.sun_irradiance * a_ref, rtol=1e-12,
                               atol=1e-15)


@pytest.mark.parametrize("kind", [PATTERN_GAUSS, PATTERN_TABLE])
def test_range_stacking_agrees_with_beam_iteration(oracle_mod, kind):
    """Alg. 2 (per-slice 2-D correlation, library routine) sampled at a beam's
    pixel equals Alg. 1's bin divided by the beam scale; the nearest slice at
    or above rho_min agrees too (the paper: both algorithms correspond to
    floating-point limits)."""
    from oracle import range_stacking as rs
    gb, pat, params = _tiny(kind, seed=4)
    # keep only beams whose pixel is inside the image
    res = oracle_mod.simulate(gb, pat, params)
    r = gb.raster
    inside = [b for b in range(pat.n_beams)
              if 0 <= res.pixel[b, 0] < r.width and 0 <= res.pixel[b, 1] < r.height]
    assert len(inside) >= 3
    # per-pixel rendered intensity rho_hat * Omega and the time bin of every pixel
    xi_ref, _ = brute.brute_xi(gb, pat, params)   # only used for scale
    K = oracle_mod.kernel_grid(r, pat)
    d = gb.depth.astype(np.float64)
    valid = np.isfinite(d) & (d > 0)
    dd = np.where(valid, d, 1.0)
    bins = np.where(valid, np.floor(dd * 2.0 / (C * params.bin_ns * 1e-9)), -1).astype(np.int64)
    phi = np.radians(r.az_min + (np.arange(r.width) + 0.5) * r.dphi)
    el = np.radians(r.el_max - (np.arange(r.height) + 0.5) * r.de)
    view = np.stack([np.cos(el)[:, None] * np.cos(phi)[None, :],
                     np.cos(el)[:, None] * np.sin(phi)[None, :],
                     np.broadcast_to(np.sin(el)[:, None], d.shape)])
    cos_t = np.maximum(0.0, -(gb.normal.astype(np.float64) * view).sum(0))
    om = np.array([brute.row_solid_angle(r, v) for v in range(r.height)])[:, None]
    g64 = gb.retro_gain.astype(np.float64)
    rho64 = gb.reflectance.astype(np.float64)
    inten = np.where(valid, g64 * rho64 / math.pi * cos_t / (dd * dd), 0.0) * om
    corr = rs.slice_correlations(inten, bins, K, params.n_bins)
    for b in inside:
        u, v = res.pixel[b]
        for s, img in corr.items():
            assert img[v, u] * res.scale[b] == pytest.approx(res.xi[b, s], rel=1e-12,
                                                              abs=1e-14 * xi_ref.max())
    rho_min = 0.3 * np.median([res.xi[b].max() / res.scale[b] for b in inside])
    s_near, xi_near = rs.nearest_above(inten, bins, K, params.n_bins, rho_min)
    for b in inside:
        u, v = res.pixel[b]
        scaled = res.xi[b] / res.scale[b]
        above = np.nonzero(scaled >= rho_min * (1 - 1e-12))[0]
        if above.size:
            assert s_near[v, u] == above[0]
            assert xi_near[v, u] == pytest.approx(scaled[above[0]], rel=1e-12)
        else:
            assert s_near[v, u] == params.n_bins


def test_sun_floor_closed_form(oracle_mod):
    """A Lambertian wall facing the sun (n = s, rho = pi) under a wide
    untruncated Gaussian collector: A_b = E_sun * sum kappa Omega which, for a
    beam on the horizon, is the lattice sum 2 pi s_x s_y (rad^2) times cos e
    averaged over the footprint (1 - O(s^2))."""
    raster = Raster(240, 240, -6.0, 6.0, -6.0, 6.0)       # 0.05 deg pixels
    sdir = (0.0, 0.0, 1.0)
    n = np.zeros((3, 240, 240), np.float32)
    n[2] = 1.0
    gb = scenes.GBuffer(raster, np.full((240, 240), 10.0, np.float32),
                        np.full((240, 240), math.pi, np.float32),
                        np.ones((240, 240), np.float32), n)
    sx, sy = 0.3, 0.2
    pat = Pattern(PATTERN_GAUSS, np.array([0.025]), np.array([0.025]),
                  sigma_deg=(sx, sy), trunc_sigmas=8.0)
    p = _params(sun_irradiance=2.0, sun_dir=sdir, n_bins=128)
    res = oracle_mod.simulate(gb, pat, p)
    expect = 2.0 * 2 * math.pi * math.radians(sx) * math.radians(sy)
    assert res.floor[0] == pytest.approx(expect, rel=3e-5)
