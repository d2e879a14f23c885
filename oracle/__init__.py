"""FP64 CPU oracle of the single-bounce beam-iteration LiDAR model.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the benchmark's measuring legs (the CPU baseline, and the reference for the
per-field error of the precision report and the surrogate's range error),
never by the product path: no result the library returns comes from here.  It is
independent of the HIP library (no shared code, headers or constants); the
only thing both consume is the seeded input arrays from ``scenes``.

``simulate`` wraps ``lidar_oracle.c`` (plain C, FP64, OpenMP over beams).
``range_stacking`` (module ``oracle.range_stacking``) is the paper's second
algorithm (Alg. 2), used as an independent cross-check of the first and as
the reference of the GPU's range stacking.  ``oracle.pinhole`` reprojects a
pinhole rendering with a z buffer onto the equiangular raster.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblidar_oracle.so")


class _Raster(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32),
                ("az_min", C.c_double), ("az_max", C.c_double),
                ("el_min", C.c_double), ("el_max", C.c_double)]


class _Pattern(C.Structure):
    _fields_ = [("kind", C.c_int32), ("sigma_az", C.c_double), ("sigma_el", C.c_double),
                ("trunc_sigmas", C.c_double), ("table", C.POINTER(C.c_float)),
                ("nx", C.c_int32), ("ny", C.c_int32),
                ("half_az", C.c_double), ("half_el", C.c_double),
                ("rx_table", C.POINTER(C.c_float))]


class _Params(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("max_echoes", C.c_int32),
                ("bin_ns", C.c_double), ("threshold", C.c_double),
                ("emit_power", C.c_double), ("pulse_fwhm_ns", C.c_double),
                ("pulse_trunc_sigmas", C.c_double), ("ambient_const", C.c_double),
                ("sun_irradiance", C.c_double), ("sun_dir", C.c_double * 3),
                ("pulse_taps", C.POINTER(C.c_double)), ("n_pulse_taps", C.c_int32),
                ("echo_select", C.c_int32), ("range_mode", C.c_int32)]


ECHO_DTYPE = np.dtype([("range_m", "f8"), ("time_ns", "f8"), ("intensity", "f8"),
                       ("pulse_width_ns", "f8"), ("bin_peak", "i4"), ("bin_first", "i4"),
                       ("bin_last", "i4"), ("flags", "i4")])

_lib = None


def build(force: bool = False) -> str:
    """Compile lidar_oracle.c with gcc (FP64, no FMA contraction, OpenMP)."""
    from . import compile as _c
    return _c.build(force=force)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = C.CDLL(LIB_PATH)
        P = C.POINTER
        lib.orc_simulate.restype = C.c_int
        lib.orc_simulate.argtypes = [
            P(_Raster)] + [P(C.c_float)] * 6 + [
            P(_Pattern), C.c_int32, P(C.c_double), P(C.c_double), P(_Params),
            P(C.c_double), P(C.c_double), P(C.c_double), C.c_void_p, P(C.c_int32),
            P(C.c_int64), P(C.c_double), P(C.c_int64), C.c_int]
        lib.orc_kernel_extent.argtypes = [P(_Raster), P(_Pattern), P(C.c_int32), P(C.c_int32)]
        lib.orc_kernel_grid.argtypes = [P(_Raster), P(_Pattern), P(C.c_double)]
        lib.orc_pattern_value.restype = C.c_double
        lib.orc_pattern_value.argtypes = [P(_Pattern), C.c_double, C.c_double]
        lib.orc_row_solid_angle.restype = C.c_double
        lib.orc_row_solid_angle.argtypes = [P(_Raster), C.c_int64]
        lib.orc_beam_pixel.argtypes = [P(_Raster), C.c_double, C.c_double,
                                       P(C.c_int64), P(C.c_int64)]
        lib.orc_pulse_half_taps.restype = C.c_int32
        lib.orc_pulse_half_taps.argtypes = [P(_Params)]
        lib.orc_pulse_taps.argtypes = [P(_Params), P(C.c_double)]
        lib.orc_detect.restype = C.c_int32
        lib.orc_detect.argtypes = [P(C.c_double), C.c_int32, C.c_double, C.c_double,
                                   C.c_double, C.c_int32, C.c_void_p]
        lib.orc_select.restype = C.c_int32
        lib.orc_select.argtypes = [P(C.c_double), P(C.c_double), C.c_int32, C.c_double,
                                   C.c_double, C.c_double, C.c_int32, C.c_int32, C.c_void_p]
        lib.orc_plane_range.restype = C.c_double
        lib.orc_plane_range.argtypes = [C.c_double, P(C.c_double), P(C.c_double), P(C.c_double)]
        lib.orc_pixel_interval.argtypes = [P(_Raster), C.c_int64, C.c_int64, C.c_double,
                                           P(C.c_double), P(C.c_double), P(C.c_double)]
        _lib = lib
    return _lib


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _raster(r) -> _Raster:
    return _Raster(r.width, r.height, r.az_min, r.az_max, r.el_min, r.el_max)


def _pattern(p, keep):
    if p.table is not None:
        t = np.ascontiguousarray(p.table, dtype=np.float32)
        keep.append(t)
        rx = None
        if getattr(p, "rx_table", None) is not None:
            rxa = np.ascontiguousarray(p.rx_table, dtype=np.float32)
            assert rxa.shape == t.shape
            keep.append(rxa)
            rx = _fptr(rxa)
        return _Pattern(p.kind, 0.0, 0.0, 0.0, _fptr(t), t.shape[1], t.shape[0],
                        float(p.half_deg[0]), float(p.half_deg[1]), rx)
    return _Pattern(p.kind, float(p.sigma_deg[0]), float(p.sigma_deg[1]),
                    float(p.trunc_sigmas), None, 0, 0, 0.0, 0.0, None)


def _params(q, keep=None) -> _Params:
    taps = getattr(q, "pulse_taps", None)
    tp, nt = None, 0
    if taps is not None:
        ta = np.ascontiguousarray(taps, dtype=np.float64)
        if keep is None:
            raise ValueError("a tabulated pulse needs a keep list")
        keep.append(ta)
        tp, nt = _dptr(ta), int(ta.shape[0])
    return _Params(q.n_bins, q.max_echoes, q.bin_ns, q.threshold, q.emit_power,
                   q.pulse_fwhm_ns, q.pulse_trunc_sigmas, q.ambient_const,
                   q.sun_irradiance, (C.c_double * 3)(*q.sun_dir), tp, nt,
                   int(getattr(q, "echo_select", 0)), int(getattr(q, "range_mode", 0)))


@dataclass
class OracleResult:
    xi: np.ndarray | None        # [B][R] raw binned signal (before the pulse)
    xi_hat: np.ndarray | None    # [B][R] pulse-convolved signal plus floor
    floor: np.ndarray            # [B] ambient floor A_b
    echoes: np.ndarray           # [B][E] ECHO_DTYPE
    n_echoes: np.ndarray         # [B] int32, all runs (uncapped)
    samples: np.ndarray          # [B] int64 in-image kernel cells with K > 0
    scale: np.ndarray            # [B] S_b
    pixel: np.ndarray            # [B][2] (u_b, v_b)


def simulate(gbuffer, pattern, params, want_xi=True, want_xi_hat=True,
             n_threads: int = 0) -> OracleResult:
    """Run the FP64 oracle over every beam of ``pattern`` on ``gbuffer``."""
    lib = _load()
    keep = []
    planes = [np.ascontiguousarray(a, dtype=np.float32) for a in gbuffer.planes()]
    r = _raster(gbuffer.raster)
    pat = _pattern(pattern, keep)
    prm = _params(params, keep)
    B, R, E = pattern.n_beams, params.n_bins, params.max_echoes
    az = np.ascontiguousarray(pattern.beam_az, dtype=np.float64)
    el = np.ascontiguousarray(pattern.beam_el, dtype=np.float64)
    xi = np.zeros((B, R)) if want_xi else None
    xh = np.zeros((B, R)) if want_xi_hat else None
    fl = np.zeros(B)
    ech = np.zeros((B, E), dtype=ECHO_DTYPE)
    ne = np.zeros(B, dtype=np.int32)
    ns = np.zeros(B, dtype=np.int64)
    sc = np.zeros(B)
    px = np.zeros((B, 2), dtype=np.int64)
    rc = lib.orc_simulate(C.byref(r), *[_fptr(a) for a in planes], C.byref(pat), B,
                          _dptr(az), _dptr(el), C.byref(prm),
                          _dptr(xi) if xi is not None else None,
                          _dptr(xh) if xh is not None else None,
                          _dptr(fl), ech.ctypes.data_as(C.c_void_p),
                          ne.ctypes.data_as(C.POINTER(C.c_int32)),
                          ns.ctypes.data_as(C.POINTER(C.c_int64)), _dptr(sc),
                          px.ctypes.data_as(C.POINTER(C.c_int64)), int(n_threads))
    if rc != 0:
        raise RuntimeError(f"oracle failed ({rc})")
    return OracleResult(xi, xh, fl, ech, ne, ns, sc, px)


def kernel_grid(raster, pattern) -> np.ndarray:
    """K[n + N][m + M] in FP64 (rows: downward pixel offset n; columns: m)."""
    lib = _load()
    keep = []
    r, p = _raster(raster), _pattern(pattern, keep)
    M, N = C.c_int32(), C.c_int32()
    lib.orc_kernel_extent(C.byref(r), C.byref(p), C.byref(M), C.byref(N))
    K = np.zeros((2 * N.value + 1, 2 * M.value + 1))
    lib.orc_kernel_grid(C.byref(r), C.byref(p), _dptr(K))
    return K


def pattern_value(pattern, x_deg: float, y_deg: float) -> float:
    lib = _load()
    keep = []
    p = _pattern(pattern, keep)
    return lib.orc_pattern_value(C.byref(p), float(x_deg), float(y_deg))


def row_solid_angle(raster, v: int) -> float:
    lib = _load()
    r = _raster(raster)
    return lib.orc_row_solid_angle(C.byref(r), int(v))


def beam_pixel(raster, az: float, el: float):
    lib = _load()
    r = _raster(raster)
    u, v = C.c_int64(), C.c_int64()
    lib.orc_beam_pixel(C.byref(r), float(az), float(el), C.byref(u), C.byref(v))
    return u.value, v.value


def pulse_taps(params) -> np.ndarray:
    lib = _load()
    keep = []
    q = _params(params, keep)
    J = lib.orc_pulse_half_taps(C.byref(q))
    taps = np.zeros(2 * J + 1)
    lib.orc_pulse_taps(C.byref(q), _dptr(taps))
    return taps


def detect(xi_hat: np.ndarray, threshold: float, floor: float, bin_ns: float,
           max_echoes: int):
    """Echo detection on one waveform; returns (n_runs, echoes[:min(n, E)])."""
    lib = _load()
    xh = np.ascontiguousarray(xi_hat, dtype=np.float64)
    out = np.zeros(max(1, max_echoes), dtype=ECHO_DTYPE)
    n = lib.orc_detect(_dptr(xh), xh.shape[0], threshold, floor, bin_ns, max_echoes,
                       out.ctypes.data_as(C.c_void_p))
    return n, out[:min(n, max_echoes)]


def select(xi: np.ndarray, xi_hat: np.ndarray, threshold: float, floor: float, bin_ns: float,
           max_echoes: int, mode: int):
    """Echoes of one beam under an echo-selection mode; returns (count,
    echoes[max_echoes])."""
    lib = _load()
    a = np.ascontiguousarray(xi, dtype=np.float64)
    b = np.ascontiguousarray(xi_hat, dtype=np.float64)
    out = np.zeros(max(1, max_echoes), dtype=ECHO_DTYPE)
    n = lib.orc_select(_dptr(a), _dptr(b), a.shape[0], threshold, floor, bin_ns, max_echoes,
                       int(mode), out.ctypes.data_as(C.c_void_p))
    return n, out[:max_echoes]


def plane_range(d: float, p, w, n) -> float:
    """d (p.n)/(w.n) with the ratio limited to [1/2, 2]."""
    lib = _load()
    arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (p, w, n)]
    return lib.orc_plane_range(float(d), *[_dptr(x) for x in arr])


def pixel_interval(raster, u: int, v: int, d: float, normal):
    """(r0, r1): the range interval of pixel (u, v) of range d and normal n."""
    lib = _load()
    r = _raster(raster)
    nn = np.ascontiguousarray(normal, dtype=np.float64)
    r0, r1 = C.c_double(), C.c_double()
    lib.orc_pixel_interval(C.byref(r), int(u), int(v), float(d), _dptr(nn), C.byref(r0), C.byref(r1))
    return r0.value, r1.value
