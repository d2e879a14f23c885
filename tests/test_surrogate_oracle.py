"""Pins of the surrogate oracle (``oracle/surrogate.py``) against library
routines, closed forms and finite differences."""
import math

import numpy as np
import pytest

import scenes
from oracle import surrogate as S


def test_bf16_rounding_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = rng.standard_normal(20000).astype(np.float32) * np.float32(3.0)
    u = x.view(np.uint32).copy()
    u[:5000] = (u[:5000] & np.uint32(0xFFFF0000)) | np.uint32(0x8000)     # exact ties
    u[5000:6000] = (u[5000:6000] & np.uint32(0xFFFF0000)) | np.uint32(0x7FFF)
    x = u.view(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(S.bf16_round(x), ref)


def test_gelu_closed_forms_and_library():
    torch = pytest.importorskip("torch")
    x = np.linspace(-6, 6, 1201)
    assert S.gelu(np.array([0.0]))[0] == 0.0
    # z Phi(z) - (-z) Phi(-z) = z (Phi(z) + Phi(-z) = 1)
    np.testing.assert_allclose(S.gelu(x) - S.gelu(-x), x, rtol=0, atol=1e-14)
    ref = torch.nn.functional.gelu(torch.from_numpy(x), approximate="none").numpy()
    np.testing.assert_allclose(S.gelu(x), ref, rtol=0, atol=1e-15)
    h = 1e-6
    fd = (S.gelu(x + h) - S.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(S.gelu_prime(x), fd, rtol=0, atol=1e-9)


def test_forward_matches_a_library_mlp():
    torch = pytest.importorskip("torch")
    flat = scenes.surrogate_init(3).astype(np.float64)
    flat += np.random.default_rng(1).standard_normal(flat.size) * 1e-2   # non-zero biases too
    p = S.unpack(flat)
    X = np.random.default_rng(2).standard_normal((7, S.IN))
    net = torch.nn.Sequential(
        torch.nn.Linear(S.IN, S.HID), torch.nn.GELU(), torch.nn.Linear(S.HID, S.HID),
        torch.nn.GELU(), torch.nn.Linear(S.HID, S.HID), torch.nn.GELU(),
        torch.nn.Linear(S.HID, S.OUT)).double()
    with torch.no_grad():
        for i, l in enumerate((0, 2, 4, 6)):
            net[l].weight.copy_(torch.from_numpy(p[f"W{i + 1}"].T.copy()))
            net[l].bias.copy_(torch.from_numpy(p[f"b{i + 1}"].copy()))
        ref = net(torch.from_numpy(X)).numpy()
    got = S.forward(X, flat, rounded=False).Y
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_loss_closed_form_at_zero_logits():
    Y = np.zeros((4, S.OUT))
    lab = np.zeros((4, 16))
    # every BCE at logit 0 is ln 2; all predicted and true existences are 0,
    # so the confidence target is 1
    L, G = S.loss_and_grad(Y, lab)
    assert L == pytest.approx(4 * math.log(2.0), rel=1e-15)
    np.testing.assert_allclose(G[:, :3], 0.5 / 4)
    np.testing.assert_allclose(G[:, 12], -0.5 / 4)
    # an existing echo one bin off is not "ok"
    lab[:, 0] = 1.0
    Y[:, 0] = 2.0
    Y[:, 3] = 1.0 / 16.0
    assert np.all(S.confidence_target(Y, lab) == 0.0)
    Y[:, 3] = 0.4 / 16.0
    assert np.all(S.confidence_target(Y, lab) == 1.0)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(4)
    flat = scenes.surrogate_init(5).astype(np.float64)
    flat += rng.standard_normal(flat.size) * 1e-2
    X = rng.standard_normal((6, S.IN)) * 0.5
    X[:, S.IN_USED:] = 0.0
    lab = np.zeros((6, 16))
    lab[:, :3] = rng.integers(0, 2, size=(6, 3))
    lab[:, 3:12] = rng.standard_normal((6, 9)) * 0.3

    def loss(f):
        return S.loss_and_grad(S.forward(X, f, rounded=False).Y, lab)[0]

    c = S.forward(X, flat, rounded=False)
    _, dY = S.loss_and_grad(c.Y, lab)
    g = S.backward(c, dY, flat, rounded=False)
    idx = np.concatenate([rng.choice(S.N_PARAMS, 300, replace=False),
                          np.arange(S.N_PARAMS - 16, S.N_PARAMS)])     # b4 included
    h = 1e-5
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        fd = (loss(fp) - loss(fm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_adamw_matches_torch_optimizer():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(6)
    theta = rng.standard_normal(S.N_PARAMS)
    hp = dict(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.01)
    mask = S.decay_mask().astype(bool)
    tw = torch.tensor(theta[mask], dtype=torch.float64, requires_grad=True)
    tb = torch.tensor(theta[~mask], dtype=torch.float64, requires_grad=True)
    opt = torch.optim.AdamW([{"params": [tw], "weight_decay": hp["weight_decay"]},
                             {"params": [tb], "weight_decay": 0.0}],
                            lr=hp["lr"], betas=(hp["beta1"], hp["beta2"]), eps=hp["eps"])
    m = np.zeros(S.N_PARAMS)
    v = np.zeros(S.N_PARAMS)
    th = theta.copy()
    for t in range(1, 4):
        g = rng.standard_normal(S.N_PARAMS)
        tw.grad = torch.from_numpy(g[mask].copy())
        tb.grad = torch.from_numpy(g[~mask].copy())
        opt.step()
        th, m, v = S.adamw_step(th, g, m, v, t, **hp)
    np.testing.assert_allclose(th[mask], tw.detach().numpy(), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(th[~mask], tb.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_initial_weights_layout():
    flat = scenes.surrogate_init(0)
    assert flat.size == S.N_PARAMS == 406288
    p = S.unpack(flat)
    assert np.all(p["W1"][S.IN_USED:] == 0) and np.all(p["W4"][:, S.OUT_USED:] == 0)
    assert abs(p["W1"][:S.IN_USED].std() * math.sqrt(S.IN_USED) - 1.0) < 0.01


# ---- the surrogate's inputs (oracle) against closed forms -------------------

def _shell_inputs(depth=40.0, rho=0.6, sun=0.0):
    import oracle as O
    r = scenes.Raster(96, 64, -12.0, 12.0, -8.0, 8.0)
    gb = scenes.shell_gbuffer(r, depth, rho)
    az = np.array([0.0, 3.3, -5.1])
    el = np.array([0.0, 1.7, -2.2])
    pat = scenes.Pattern(scenes.PATTERN_GAUSS, az, el, sigma_deg=(0.5, 0.4), trunc_sigmas=3.0)
    p = scenes.SensorParams(n_bins=512, bin_ns=1.0, max_echoes=3, threshold=1e-5, emit_power=1.0,
                            pulse_fwhm_ns=4.0, pulse_trunc_sigmas=4.0, ambient_const=1e-7,
                            sun_irradiance=sun, sun_dir=(-1.0, 0.0, 0.0))
    O._load()
    K = O.kernel_grid(r, pat)
    ref = O.simulate(gb, pat, p, want_xi=False)
    out = S.features(gb, pat, p, K, ref.pixel, ref.scale, lambda v: O.row_solid_angle(r, v))
    return gb, pat, p, ref, out


def test_inputs_of_a_constant_range_shell():
    """Every pixel at 40 m facing the sensor: cell means are the shell's
    values, the reference bin is the shell's bin, the first channel is the
    offset of the shell's depth from that bin's centre, there is no tail
    (the 3-sigma Gaussian's core box spans its window)."""
    gb, pat, p, ref, (X, kref, et, ae, geo) = _shell_inputs()
    to_bin = 2.0 / (299792458.0 * 1e-9)
    k = math.floor(np.float32(40.0) * to_bin)
    assert np.all(kref == k)
    np.testing.assert_allclose(X[:, :256], (40.0 * to_bin - (k + 0.5)) / 64.0, rtol=1e-12)
    np.testing.assert_allclose(X[:, 256:512], np.float32(0.6), rtol=1e-6)     # reflectance cover
    np.testing.assert_allclose(X[:, 512:768], 0.0, atol=1e-15)                # log10(g = 1)
    np.testing.assert_allclose(X[:, 768:1024], 1.0, atol=1e-6)                # cos(theta)
    np.testing.assert_allclose(X[:, 1029], k / 512.0)
    assert np.all(et == 0.0)
    np.testing.assert_allclose(ae, 1e-7)                                      # no sun


def test_floor_estimate_of_a_sunlit_shell():
    """With the sun behind the sensor the shell's sun floor is E_sun (rho/pi)
    sum K Omega (n.s) / max K; the coarse-cell estimate (kernel at cell
    centres) must agree with the plain oracle's exact floor to 2 %."""
    gb, pat, p, ref, (X, kref, et, ae, geo) = _shell_inputs(sun=0.5)
    inside = ref.samples > 0
    np.testing.assert_allclose(ae[inside], ref.floor[inside], rtol=0.02)


def test_labels_closed_form():
    echoes = np.zeros((2, 3), dtype=[("bin_peak", "i4"), ("intensity", "f8"),
                                     ("pulse_width_ns", "f8")])
    echoes["bin_peak"] = [[100, 300, 0], [5, 0, 0]]
    echoes["intensity"] = [[2e-5, 1e-9, 0], [1e-5, 0, 0]]
    echoes["pulse_width_ns"] = [[4.0, 8.0, 0], [2.0, 0, 0]]
    p = scenes.SensorParams(n_bins=512, bin_ns=1.0, max_echoes=3, threshold=1e-5, emit_power=1.0,
                            pulse_fwhm_ns=4.0)
    lab = S.labels(np.array([96, 5]), echoes, np.array([2, 5]), p)
    np.testing.assert_allclose(lab[0], [1, 1, 0, 0.25, 4.0, 0, math.log10(2.0), -3.0, 0,
                                        1.0, 2.0, 0, 0, 0, 0, 0])
    # more echoes than stored: existence only for the three slots
    np.testing.assert_allclose(lab[1, :3], [1, 1, 1])


# ---- tail energy and reference bin against hand-computed values -------------
#
# A 256 x 128 raster of 0.125-deg pixels and a 33 x 33 table whose cell
# centres fall on the kernel's pixel offsets (half extent 2.0625 deg, so that
# K[n][m] is exactly table[n + 16][m + 16]): a core of 1 at the centre and 0.5
# on the 5 x 3 cells around it, and a flat tail of 1e-4 elsewhere (below the
# 2e-4 core fraction).  The core box is then m in [-2, 2], n in [-1, 1];
# coarse cells are single pixels and super-cells 3 x 3 pixels.  One beam sits
# at pixel (128, 64).  Every other pixel is sky unless a test places a
# surface, always facing the sensor (cos(theta) = 1) with gain 1.

_HALF = 2.0625
_TAIL = float(np.float32(1e-4))     # the table's float32 tail level
_C = 299792458.0


def _tail_table():
    t = np.full((33, 33), _TAIL, np.float32)
    t[15:18, 14:19] = 0.5
    t[16, 16] = 1.0
    return t


def _sky_scene():
    r = scenes.Raster(256, 128, -16.0, 16.0, -8.0, 8.0)
    n = -scenes.pixel_directions(r)
    gb = scenes.GBuffer(r, np.full((128, 256), np.inf, np.float32),
                        np.zeros((128, 256), np.float32), np.ones((128, 256), np.float32),
                        n.astype(np.float32))
    pat = scenes.Pattern(scenes.PATTERN_TABLE, np.array([0.0625]), np.array([-0.0625]),
                         table=_tail_table(), half_deg=(_HALF, _HALF))
    p = scenes.SensorParams(n_bins=512, bin_ns=1.0, max_echoes=3, threshold=1e-9, emit_power=1.0,
                            pulse_fwhm_ns=4.0, pulse_trunc_sigmas=4.0, ambient_const=1e-12)
    return r, gb, pat, p


def _depth_of_bin(k):
    """A radial range whose time bin (1 ns bins) is k: the bin centre."""
    return np.float32((k + 0.5) * _C * 1e-9 / 2.0)


def _shade(r, v, d, rho):
    """Omega(v) (rho / pi) / d^2 of a pixel facing the sensor, Omega the
    exact pixel solid angle dphi (sin e_top - sin e_bot)."""
    d2r = math.pi / 180.0
    e_top = r.el_max - v * 0.125
    e_bot = e_top - 0.125
    om = 0.125 * d2r * (math.sin(e_top * d2r) - math.sin(e_bot * d2r))
    return om * (rho / math.pi) / (float(d) ** 2)


def _features(r, gb, pat, p):
    import oracle as O
    O._load()
    K = O.kernel_grid(r, pat)
    assert K.shape == (33, 33) and K[16, 16] == 1.0 and K[16, 18] == 0.5 and K[16, 19] == _TAIL
    ref = O.simulate(gb, pat, p, want_xi=False)
    assert tuple(ref.pixel[0]) == (128, 64)
    out = S.features(gb, pat, p, K, ref.pixel, ref.scale, lambda v: O.row_solid_angle(r, v))
    return ref, out


def test_tail_energy_of_two_tail_super_cells():
    """Super-cell A (columns 138-140, rows 63-65; centre offset m = 11, n = 0)
    holds pixels in bins 14..17, super-cell B (columns 141-143; m = 14) pixels
    in bins 16..21.  Each spreads K (1e-4) times its shade sum evenly over its
    bin range; with 8 bins per coarse tail bin, A covers coarse bins 1 and 2,
    B coarse bin 2 only, so E_tail = S_b 1e-4 (shade_A / 4 + shade_B / 6)."""
    r, gb, pat, p = _sky_scene()
    bins_a, bins_b = [14, 15, 16, 17], [16, 17, 18, 19, 20, 21]
    shade = {"A": 0.0, "B": 0.0}
    i = 0
    for name, cols, bins in (("A", range(138, 141), bins_a), ("B", range(141, 144), bins_b)):
        for v in range(63, 66):
            for u in cols:
                k = bins[i % len(bins)]
                i += 1
                rho = 0.3 + 0.05 * (i % 5)
                gb.depth[v, u] = _depth_of_bin(k)
                gb.reflectance[v, u] = rho
                shade[name] += _shade(r, v, gb.depth[v, u], float(np.float32(rho)))
    ref, (X, kref, et, ae, geo) = _features(r, gb, pat, p)
    assert (geo["cm"], geo["cn"], geo["cw"], geo["ch"], geo["sw"], geo["sh"]) == (2, 1, 1, 1, 3, 3)
    expect = ref.scale[0] * _TAIL * (shade["A"] / 4.0 + shade["B"] / 6.0)
    assert et[0] == pytest.approx(expect, rel=1e-6)
    # the patches lie outside the 16 x 16 coarse patch and the core box: no
    # reference-bin contribution, no floor
    assert ae[0] == pytest.approx(1e-12)


def test_reference_bin_smoothed_first_maximum():
    """Core-box cells put K x shade into bins k = 300 (centre pixel, K = 1),
    k + 1 (the two pixels at m = +-1, K = 0.5) and k + 3 (the pixel at m = 2,
    n = 0, K = 0.5).  Smoothing with (1, 2, 3, 2, 1) gives, at bin j,
    h(j-2) + 2 h(j-1) + 3 h(j) + 2 h(j+1) + h(j+2); with h = (1, 1.1, 0, 1.5)
    x w0 the smoothed values at k .. k+3 are 5.2, 7.1, 6.2, 5.6 (times w0),
    so k_ref = k + 1, while the unsmoothed maximum sits at k + 3."""
    r, gb, pat, p = _sky_scene()
    k = 300
    w0 = 1e-3
    cells = {(128, 64): (k, 1.0, 1.0), (127, 64): (k + 1, 0.5, 0.55), (129, 64): (k + 1, 0.5, 0.55),
             (130, 64): (k + 3, 0.5, 1.5)}
    h = {}
    for (u, v), (kb, kv, rel) in cells.items():
        gb.depth[v, u] = _depth_of_bin(kb)
        # reflectance chosen so that K x shade = rel x w0
        rho = rel * w0 / (kv * _shade(r, v, gb.depth[v, u], 1.0))
        gb.reflectance[v, u] = rho
        h[kb] = h.get(kb, 0.0) + kv * _shade(r, v, gb.depth[v, u], float(np.float32(rho)))
    assert h[k] == pytest.approx(w0, rel=1e-6) and h[k + 1] == pytest.approx(1.1 * w0, rel=1e-6)
    assert h[k + 3] == pytest.approx(1.5 * w0, rel=1e-6)
    ref, (X, kref, et, ae, geo) = _features(r, gb, pat, p)
    assert kref[0] == k + 1
    # the first channel is each cell's mean-depth offset from k_ref's centre
    d = float(gb.depth[64, 128])
    assert X[0, 8 * 16 + 8] == pytest.approx((d * 2.0 / (_C * 1e-9) - (k + 1.5)) / 64.0, rel=1e-9)


def test_reference_bin_first_of_equal_maxima_and_fallback():
    """Two equal weights w two bins apart (k and k + 2) smooth to 3w + w at k,
    2w + 2w at k + 1 and w + 3w at k + 2: three equal maxima, of which the
    first (bin k) is taken.  Without a core-box cell the reference bin is
    the bin of the nearest cell mean depth in the patch."""
    r, gb, pat, p = _sky_scene()
    k = 200
    for (u, v), kb in (((128, 64), k), ((130, 64), k + 2)):
        gb.depth[v, u] = _depth_of_bin(kb)
        kv = 1.0 if u == 128 else 0.5
        gb.reflectance[v, u] = 1e-3 / (kv * _shade(r, v, gb.depth[v, u], 1.0))
    ref, (X, kref, et, ae, geo) = _features(r, gb, pat, p)
    assert kref[0] == k
    # no core cell: only a pixel outside the core box but inside the patch
    r, gb, pat, p = _sky_scene()
    gb.depth[64, 133] = _depth_of_bin(77)
    gb.depth[60, 124] = _depth_of_bin(90)
    gb.reflectance[64, 133] = gb.reflectance[60, 124] = 0.5
    ref, (X, kref, et, ae, geo) = _features(r, gb, pat, p)
    assert kref[0] == 77
