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
