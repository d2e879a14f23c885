"""The synthetic workloads have the properties their recipes promise.

The threshold and sun-irradiance literals of the scanning-sensor workload are
re-derived here with the oracle; the echo statistics of both workloads are
checked against their recipes; blooming (echoes from retroreflectors outside
the beam centre) must arise from the pattern tails on its own.
"""
import math

import numpy as np
import pytest

import scenes


@pytest.fixture(scope="module")
def w2():
    return scenes.road_scan(0)


def test_iid_frame_recipe_and_echo_statistics(oracle_mod):
    w = scenes.iid_frame(0)
    gb = w.gbuffer
    assert gb.depth.shape == (512, 1024)
    assert 5.0 <= gb.depth.min() and gb.depth.max() <= 60.0
    assert abs((gb.retro_gain > 1).mean() - 0.02) < 0.002
    assert w.pattern.n_beams == 1000
    res = oracle_mod.simulate(gb, w.pattern, w.params, want_xi=False)
    assert np.all(res.samples == 89)
    # recipe: 1-5 mean echoes per beam and under half the beams without echo
    assert 1.0 <= res.n_echoes.mean() <= 5.0
    assert (res.n_echoes == 0).mean() < 0.5


def test_road_scan_threshold_literal(oracle_mod, w2):
    """T = 5 % of the pulse-convolved peak of a rho = 0.5 face at 100 m filling
    the beam: that face gives xi = P_e rho / (pi d^2) in one bin."""
    taps = oracle_mod.pulse_taps(w2.params)
    peak = w2.params.emit_power * 0.5 / (math.pi * 100.0 ** 2) * taps[len(taps) // 2]
    assert w2.params.threshold == pytest.approx(0.05 * peak, rel=1e-3)


def test_road_scan_recipe_sun_floor_and_blooming(oracle_mod, w2):
    gb = w2.gbuffer
    assert gb.depth.shape == (512, 8192)
    assert 0.01 <= (gb.retro_gain > 1).mean() < 0.013
    assert w2.pattern.n_beams == 16 * 1800
    idx = np.arange(0, w2.pattern.n_beams, 11)
    sub = scenes.subset_beams(w2, idx)
    res = oracle_mod.simulate(gb, sub.pattern, sub.params, want_xi=False, want_xi_hat=False)
    # sun floor: its 95th percentile at 0.75 T, so that the echo stage sees
    # real returns (a floor above T would make the whole waveform one run)
    r = res.floor / w2.params.threshold
    assert 0.70 < np.quantile(r, 0.95) < 0.80
    assert (r >= 1.0).mean() < 0.05
    assert (res.n_echoes > 0).mean() > 0.6
    assert not np.any((res.echoes["flags"][:, 0] == 3) & (res.n_echoes > 0))
    # blooming: an echo whose bin matches a retroreflective pixel of the
    # footprint while the beam's own pixel is neither retroreflective nor at
    # that range
    C = 299792458.0
    to_bin = 2.0 / (C * w2.params.bin_ns * 1e-9)
    d = gb.depth
    bins = np.where(np.isfinite(d), np.floor(d.astype(np.float64) * to_bin), -1)
    retro = gb.retro_gain > 1
    H, W = d.shape
    bloom = 0
    for i, b in enumerate(idx):
        u, v = res.pixel[i]
        if not (0 <= u < W and 0 <= v < H):
            continue
        u0, u1 = max(0, u - 113), min(W, u + 114)
        rb = bins[:, u0:u1][retro[:, u0:u1]]
        if rb.size == 0 or retro[v, u]:
            continue
        for e in res.echoes[i][:min(res.n_echoes[i], 3)]:
            kp = e["bin_peak"]
            if abs(bins[v, u] - kp) > 4 and np.any(np.abs(rb - kp) <= 2):
                bloom += 1
                break
    assert bloom / len(idx) >= 0.01
