"""Comparison of the HIP path with the FP64 oracle (test helper).

Tolerances (written out here, derived in the design doc):
  * waveform: per beam, max_k |xi_hat_gpu - xi_hat_ref| <= WAVE_TOL * max_k xi_hat_ref
    (FP32 accumulation; the bound the method's precision policy states);
  * a beam is threshold-ambiguous when some bin has |xi_hat_ref - T| <=
    WAVE_TOL * max_k xi_hat_ref: there FP32 may legitimately decide a run
    differently, so only non-ambiguous beams must match echo counts exactly;
  * on non-ambiguous beams every kept echo has the same first and last bin,
    a peak bin within +-1 (exact where the run's maximum is unambiguous) and
    the FP64 range of its peak bin (bit-identical when the peak bins agree);
  * intensity within WAVE_TOL * max xi_hat_ref of the oracle's waveform at the
    GPU's peak bin; EPW within the interpolation error bound
    dt * sum over both crossings of 3 WAVE_TOL max / |slope| + 1e-5 ns;
  * floor A_b within WAVE_TOL * max(A_b, max xi_hat_ref) relative; scale S_b
    within 1e-6 relative (FP64 rounded to FP32); pixel and sample counts exact.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

WAVE_TOL = 1e-5
C = 299792458.0


def run_gpu(gbuffer, pattern, params, keep_waveforms=True, stream=None):
    import torch
    import paper_2512_05932_amd as lidar
    planes = lidar.upload_gbuffer(gbuffer, "cuda")
    sim = lidar.LidarSim(params, stream=stream or torch.cuda.current_stream(),
                         keep_waveforms=keep_waveforms)
    try:
        sim.set_pattern(pattern)
        sim.set_gbuffer(gbuffer.raster, planes)
        sim.simulate_frame()
        out = sim.read(waveforms=keep_waveforms)
        out["stats"] = sim.stats()
    finally:
        sim.close()
    return out


@dataclass
class Report:
    n_beams: int
    ambiguous: int
    max_wave_err: float
    count_mismatch: int
    echoes_compared: int
    peak_off_by_one: int


def compare(gpu, ref, params, beam_idx=None, check_waveforms=True) -> Report:
    """Assert the parity rules; ``beam_idx`` maps GPU rows to oracle rows."""
    g_ech, g_cnt, g_beams = gpu["echoes"], gpu["n_echoes"], gpu["beams"]
    if beam_idx is not None:
        g_ech, g_cnt, g_beams = g_ech[beam_idx], g_cnt[beam_idx], g_beams[beam_idx]
        g_wav = gpu["waveforms"][beam_idx] if gpu.get("waveforms") is not None else None
    else:
        g_wav = gpu.get("waveforms")
    B = ref.xi_hat.shape[0]
    T, dt, R, E = params.threshold, params.bin_ns, params.n_bins, params.max_echoes
    half_c_dt = 0.5 * C * (dt * 1e-9)
    peak = ref.xi_hat.max(axis=1)
    # per-beam inputs of the path
    np.testing.assert_array_equal(g_beams["pixel_u"], ref.pixel[:, 0])
    np.testing.assert_array_equal(g_beams["pixel_v"], ref.pixel[:, 1])
    np.testing.assert_array_equal(g_beams["samples"], ref.samples)
    np.testing.assert_allclose(g_beams["scale"], ref.scale, rtol=1e-6)
    floor_err = np.abs(g_beams["floor"].astype(np.float64) - ref.floor)
    floor_tol = WAVE_TOL * np.maximum(peak, ref.floor) + 1e-30
    assert np.all(floor_err <= floor_tol), \
        f"floor error {(floor_err / floor_tol).max():.2f} x tolerance"

    max_err = 0.0
    if check_waveforms and g_wav is not None:
        err = np.abs(g_wav.astype(np.float64) - ref.xi_hat).max(axis=1) / peak
        max_err = float(err.max())
        bad = np.nonzero(err > WAVE_TOL)[0]
        assert bad.size == 0, f"waveform error {err[bad[0]]:.3e} > {WAVE_TOL} at beam {bad[0]}"
    ambiguous = (np.abs(ref.xi_hat - T) <= WAVE_TOL * peak[:, None]).any(axis=1)
    count_mismatch = int(((g_cnt != ref.n_echoes) & ~ambiguous).sum())
    assert count_mismatch == 0, \
        f"{count_mismatch} non-ambiguous beams with a different echo count"
    compared = off1 = 0
    for b in np.nonzero(~ambiguous)[0]:
        xh = ref.xi_hat[b]
        for i in range(min(int(ref.n_echoes[b]), E)):
            ge, re = g_ech[b, i], ref.echoes[b, i]
            compared += 1
            assert ge["bin_first"] == re["bin_first"] and ge["bin_last"] == re["bin_last"], \
                (b, i, ge, re)
            dk = int(ge["bin_peak"]) - int(re["bin_peak"])
            assert abs(dk) <= 1, (b, i, ge, re)
            if dk:
                off1 += 1
                # only a near-tie may move the peak
                assert abs(xh[ge["bin_peak"]] - xh[re["bin_peak"]]) <= 2 * WAVE_TOL * peak[b]
                assert abs(ge["range_m"] - re["range_m"]) <= half_c_dt * (1 + 1e-12)
            else:
                assert ge["range_m"] == re["range_m"] and ge["time_ns"] == re["time_ns"]
            assert ge["flags"] == re["flags"]
            ref_int = xh[ge["bin_peak"]] - ref.floor[b]
            assert abs(ge["intensity"] - ref_int) <= WAVE_TOL * peak[b] * 1.01, (b, i)
            k0, k1 = int(re["bin_first"]), int(re["bin_last"])
            tol = 1e-5
            if k0 > 0:
                tol += dt * 3 * WAVE_TOL * peak[b] / abs(xh[k0] - xh[k0 - 1])
            if k1 < R - 1:
                tol += dt * 3 * WAVE_TOL * peak[b] / abs(xh[k1] - xh[k1 + 1])
            assert abs(ge["pulse_width_ns"] - re["pulse_width_ns"]) <= tol, (b, i, ge, re, tol)
        # unused slots are zeroed
        for i in range(min(int(g_cnt[b]), E), E):
            assert g_ech[b, i]["bin_last"] == 0 and g_ech[b, i]["range_m"] == 0.0
    return Report(B, int(ambiguous.sum()), max_err, count_mismatch, compared, off1)


def _beam_checks(g_beams, ref, peak):
    np.testing.assert_array_equal(g_beams["pixel_u"], ref.pixel[:, 0])
    np.testing.assert_array_equal(g_beams["pixel_v"], ref.pixel[:, 1])
    np.testing.assert_array_equal(g_beams["samples"], ref.samples)
    np.testing.assert_allclose(g_beams["scale"], ref.scale, rtol=1e-6)
    floor_err = np.abs(g_beams["floor"].astype(np.float64) - ref.floor)
    assert np.all(floor_err <= WAVE_TOL * np.maximum(peak, ref.floor) + 1e-30)


def compare_selection(gpu, ref, params) -> Report:
    """Parity of one selected echo per beam (echo_select != ALL).

    Runs of xi_hat (STRONGEST, NEAREST, LONGEST): on non-ambiguous beams the
    counts of all runs agree, and slot 0 is the oracle's selected run (same
    bins, FP64 range, intensity and EPW within the rules of ``compare``)
    unless the oracle's selection is a near-tie: two runs whose peaks differ
    by at most 2 WAVE_TOL max (STRONGEST) or whose pulse widths differ by at
    most the EPW interpolation bound (LONGEST); then the GPU's run must be
    one of the tied runs.  Raw modes: the waveform is the raw S_b xi, a beam
    is ambiguous when some bin lies within WAVE_TOL max of T, and the chosen
    bin is the oracle's or (RAW_STRONGEST) a bin within 2 WAVE_TOL max of the
    maximum."""
    import oracle as O
    mode, T, dt, R = params.echo_select, params.threshold, params.bin_ns, params.n_bins
    raw = mode >= 4
    sig = ref.xi if raw else ref.xi_hat
    peak = np.abs(sig).max(axis=1) + 1e-300
    _beam_checks(gpu["beams"], ref, ref.xi_hat.max(axis=1))
    max_err = 0.0
    if gpu.get("waveforms") is not None:
        err = np.abs(gpu["waveforms"].astype(np.float64) - sig).max(axis=1) / peak
        max_err = float(err.max())
        assert max_err <= WAVE_TOL, f"waveform error {max_err:.3e}"
    amb = (np.abs(sig - T) <= WAVE_TOL * peak[:, None]).any(axis=1)
    g_cnt, g_ech = gpu["n_echoes"], gpu["echoes"]
    mism = int(((g_cnt != ref.n_echoes) & ~amb).sum())
    assert mism == 0, f"{mism} non-ambiguous beams with another count"
    compared = ties = 0
    for b in np.nonzero(~amb & (ref.n_echoes > 0))[0]:
        ge, re = g_ech[b, 0], ref.echoes[b, 0]
        compared += 1
        assert np.all(g_ech[b, 1:]["bin_last"] == 0)
        if raw:
            k = int(ge["bin_peak"])
            assert ge["bin_first"] == ge["bin_last"] == k and ge["pulse_width_ns"] == 0.0
            if k != re["bin_peak"]:
                ties += 1
                assert mode == 4 and abs(sig[b, k] - sig[b, re["bin_peak"]]) <= 2 * WAVE_TOL * peak[b]
            assert abs(ge["intensity"] - sig[b, k]) <= WAVE_TOL * peak[b]
            continue
        if ge["bin_first"] != re["bin_first"]:
            # a near-tie of the selection: the GPU's run must be tied with the
            # oracle's choice
            ties += 1
            n_all, runs = O.detect(ref.xi_hat[b], T, ref.floor[b], dt, R)
            match = [e for e in runs if e["bin_first"] == ge["bin_first"]]
            assert match, (b, ge, re)
            other = match[0]
            if mode == 1:
                assert abs(other["intensity"] - re["intensity"]) <= 2 * WAVE_TOL * peak[b], (b, ge, re)
            elif mode == 3:
                assert abs(other["pulse_width_ns"] - re["pulse_width_ns"]) <= 1e-3 * dt, (b, ge, re)
            else:
                raise AssertionError((b, ge, re))
            re = other
        assert ge["bin_first"] == re["bin_first"] and ge["bin_last"] == re["bin_last"]
        assert abs(int(ge["bin_peak"]) - int(re["bin_peak"])) <= 1
        if ge["bin_peak"] == re["bin_peak"]:
            assert ge["range_m"] == re["range_m"]
        xh = ref.xi_hat[b]
        assert abs(ge["intensity"] - (xh[ge["bin_peak"]] - ref.floor[b])) <= WAVE_TOL * peak[b] * 1.01
        assert abs(ge["pulse_width_ns"] - re["pulse_width_ns"]) <= 1e-3 * dt + 1e-5
    return Report(len(g_cnt), int(amb.sum()), max_err, mism, compared, ties)
