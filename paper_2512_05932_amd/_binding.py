"""ctypes binding of ``liblidar_sim.so`` (argument marshalling only).

The names mirror ``include/lidar_sim.h``.  Device memory comes from torch
tensors (``data_ptr()``); every step of the model runs in the HIP kernels.
The binding raises if the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblidar_sim.so")

LIDAR_OK = 0
LIDAR_E_INVALID = -1
LIDAR_E_STATE = -2
LIDAR_E_HIP = -3
LIDAR_E_NOMEM = -4
LIDAR_E_UNSUPPORTED = -5

LIDAR_KEEP_WAVEFORMS = 1
LIDAR_PROFILE = 2
LIDAR_AUTOTUNE = 4
LIDAR_DETERMINISTIC = 8
LIDAR_PATTERN_GAUSS = 1
LIDAR_PATTERN_TABLE = 2
LIDAR_MODE_PLAIN = 0
LIDAR_MODE_SURROGATE = 1
LIDAR_ECHO_SURROGATE = 4
LIDAR_ECHO_ALL, LIDAR_ECHO_STRONGEST, LIDAR_ECHO_NEAREST, LIDAR_ECHO_LONGEST = 0, 1, 2, 3
LIDAR_ECHO_RAW_STRONGEST, LIDAR_ECHO_RAW_NEAREST = 4, 5
LIDAR_RANGE_CENTRE, LIDAR_RANGE_CORRECTED, LIDAR_RANGE_INTERVAL = 0, 1, 2

# every function the header declares
EXPORTED = ["lidar_sim_create", "lidar_sim_destroy", "lidar_sim_set_pattern",
            "lidar_sim_set_gbuffer", "lidar_sim_simulate_frame", "lidar_sim_read_echoes",
            "lidar_sim_simulate_batch", "lidar_sim_read_batch", "lidar_sim_batch_info",
            "lidar_sim_reset_batch", "lidar_sim_surrogate_set_weights",
            "lidar_sim_surrogate_get_weights", "lidar_sim_surrogate_forward",
            "lidar_sim_surrogate_gradients", "lidar_sim_surrogate_train_step",
            "lidar_sim_surrogate_train",
            "lidar_sim_surrogate_set_gate", "lidar_sim_surrogate_features", "lidar_sim_get_stats",
            "lidar_sim_reset_stats", "lidar_sim_simulate_static", "lidar_sim_set_gbuffer_pinhole",
            "lidar_sim_read_gbuffer", "lidar_sim_range_stacking", "lidar_sim_last_error"]

SUR_IN, SUR_OUT, SUR_PARAMS = 1056, 16, 406288


class lidar_sim_params(C.Structure):
    _fields_ = [("n_bins", C.c_uint32), ("max_echoes", C.c_uint32), ("bin_ns", C.c_double),
                ("threshold", C.c_double), ("emit_power", C.c_double),
                ("pulse_fwhm_ns", C.c_double), ("pulse_trunc_sigmas", C.c_double),
                ("ambient_const", C.c_double), ("sun_irradiance", C.c_double),
                ("sun_dir", C.c_double * 3), ("flags", C.c_uint32), ("echo_select", C.c_uint32),
                ("range_mode", C.c_uint32), ("n_pulse_taps", C.c_uint32),
                ("pulse_taps", C.POINTER(C.c_float))]


class lidar_pattern_desc(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("n_beams", C.c_uint32), ("sigma_deg", C.c_double * 2),
                ("trunc_sigmas", C.c_double), ("table", C.POINTER(C.c_float)),
                ("nx", C.c_uint32), ("ny", C.c_uint32), ("half_deg", C.c_double * 2),
                ("beam_az_deg", C.POINTER(C.c_double)), ("beam_el_deg", C.POINTER(C.c_double)),
                ("rx_table", C.POINTER(C.c_float))]


class lidar_gbuffer_desc(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("pitch", C.c_uint64),
                ("az_min_deg", C.c_double), ("az_max_deg", C.c_double),
                ("el_min_deg", C.c_double), ("el_max_deg", C.c_double),
                ("depth", C.c_void_p), ("reflectance", C.c_void_p), ("retro_gain", C.c_void_p),
                ("normal_x", C.c_void_p), ("normal_y", C.c_void_p), ("normal_z", C.c_void_p)]


class lidar_pinhole_desc(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("pitch", C.c_uint64),
                ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("rot", C.c_double * 9), ("depth_format", C.c_uint32), ("normal_correct", C.c_uint32),
                ("z_near", C.c_double), ("z_far", C.c_double), ("depth", C.c_void_p),
                ("reflectance", C.c_void_p), ("retro_gain", C.c_void_p), ("normal_x", C.c_void_p),
                ("normal_y", C.c_void_p), ("normal_z", C.c_void_p)]


class lidar_stats(C.Structure):
    _fields_ = [("frames", C.c_uint64), ("n_beams", C.c_uint64),
                ("samples_per_frame", C.c_uint64), ("kernel_w", C.c_uint32),
                ("kernel_h", C.c_uint32), ("n_taps", C.c_uint32), ("reserved", C.c_uint32),
                ("footprint_ms", C.c_double), ("footprint_launches", C.c_uint64),
                ("prepass_ms", C.c_double), ("prepass_launches", C.c_uint64),
                ("batch_ms", C.c_double), ("batch_launches", C.c_uint64),
                ("surrogate_beams", C.c_uint64), ("fallback_beams", C.c_uint64),
                ("surrogate_ms", C.c_double), ("surrogate_frames", C.c_uint64)]


class lidar_train_hparams(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("weight_decay", C.c_double)]


class lidar_batch_info(C.Structure):
    _fields_ = [("n_frames", C.c_uint32), ("group_size", C.c_uint32), ("n_beams", C.c_uint64),
                ("n_items", C.c_uint64), ("samples", C.c_uint64), ("grid", C.c_uint32),
                ("graph", C.c_uint32), ("autotuned", C.c_uint32), ("wave_items", C.c_uint32),
                ("autotune_ms", C.c_double), ("direct_frames", C.c_uint32), ("fixed_point_beams", C.c_uint32),
                ("fixed_point_redone", C.c_uint32), ("short_run_frames", C.c_uint32)]


ECHO_DTYPE = np.dtype([("range_m", "<f8"), ("time_ns", "<f8"), ("intensity", "<f4"),
                       ("pulse_width_ns", "<f4"), ("bin_peak", "<i4"), ("bin_first", "<i4"),
                       ("bin_last", "<i4"), ("flags", "<u4")])
BEAM_DTYPE = np.dtype([("pixel_u", "<i4"), ("pixel_v", "<i4"), ("scale", "<f4"),
                       ("floor", "<f4"), ("samples", "<u4"), ("reserved", "<u4")])
assert ECHO_DTYPE.itemsize == 40 and BEAM_DTYPE.itemsize == 24

_lib = None


class LidarError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"lidar_sim error {status}: {message}")
        self.status = status


def load():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    P, V = C.POINTER, C.c_void_p
    lib.lidar_sim_create.argtypes = [P(lidar_sim_params), V, P(V)]
    lib.lidar_sim_destroy.argtypes = [V]
    lib.lidar_sim_set_pattern.argtypes = [V, P(lidar_pattern_desc)]
    lib.lidar_sim_set_gbuffer.argtypes = [V, P(lidar_gbuffer_desc)]
    lib.lidar_sim_simulate_frame.argtypes = [V, C.c_uint32]
    lib.lidar_sim_read_echoes.argtypes = [V, V, V, V, V, C.c_int]
    lib.lidar_sim_simulate_batch.argtypes = [V, P(lidar_gbuffer_desc), P(lidar_pattern_desc),
                                             C.c_uint32]
    lib.lidar_sim_read_batch.argtypes = [V, C.c_uint32, V, V, V, V, C.c_int]
    lib.lidar_sim_batch_info.argtypes = [V, P(lidar_batch_info)]
    lib.lidar_sim_reset_batch.argtypes = [V]
    lib.lidar_sim_surrogate_set_weights.argtypes = [V, V, C.c_uint64]
    lib.lidar_sim_surrogate_get_weights.argtypes = [V, V, C.c_uint64]
    lib.lidar_sim_surrogate_forward.argtypes = [V, V, V, C.c_uint32]
    lib.lidar_sim_surrogate_gradients.argtypes = [V, V, V, C.c_uint32, V, V]
    lib.lidar_sim_surrogate_train_step.argtypes = [V, V, V, C.c_uint32, P(lidar_train_hparams), V]
    lib.lidar_sim_surrogate_train.argtypes = [V, V, V, C.c_uint64, C.c_uint32, C.c_uint32,
                                              P(lidar_train_hparams), C.c_double, C.c_uint64, V,
                                              C.c_uint32]
    lib.lidar_sim_surrogate_set_gate.argtypes = [V, C.c_double, C.c_double]
    lib.lidar_sim_surrogate_features.argtypes = [V, V, V, V]
    lib.lidar_sim_get_stats.argtypes = [V, P(lidar_stats)]
    lib.lidar_sim_reset_stats.argtypes = [V]
    lib.lidar_sim_simulate_static.argtypes = [P(lidar_sim_params), P(lidar_pattern_desc),
                                              P(lidar_gbuffer_desc), V, V, V, V]
    lib.lidar_sim_set_gbuffer_pinhole.argtypes = [V, P(lidar_pinhole_desc), C.c_uint32, C.c_uint32,
                                                  C.c_double, C.c_double, C.c_double, C.c_double]
    lib.lidar_sim_read_gbuffer.argtypes = [V, V, C.c_int]
    lib.lidar_sim_range_stacking.argtypes = [V, V, C.c_uint32, V, C.c_uint32, C.c_double, V, V]
    lib.lidar_sim_last_error.argtypes = [V]
    lib.lidar_sim_last_error.restype = C.c_char_p
    for name in EXPORTED[:-1]:
        getattr(lib, name).restype = C.c_int32
    _lib = lib
    return lib


def make_params(p, flags: int = 0, keep: list | None = None) -> lidar_sim_params:
    """lidar_sim_params from any object with the fields of the C struct
    (optional: pulse_taps, echo_select, range_mode); a tabulated pulse array
    goes into `keep`, which must outlive the call that reads it."""
    taps = getattr(p, "pulse_taps", None)
    tp, nt = None, 0
    if taps is not None:
        t = np.ascontiguousarray(taps, dtype=np.float32)
        if keep is None:
            raise ValueError("a tabulated pulse needs a keep list")
        keep.append(t)
        tp, nt = t.ctypes.data_as(C.POINTER(C.c_float)), int(t.shape[0])
    return lidar_sim_params(int(p.n_bins), int(p.max_echoes), float(p.bin_ns),
                            float(p.threshold), float(p.emit_power), float(p.pulse_fwhm_ns),
                            float(p.pulse_trunc_sigmas), float(p.ambient_const),
                            float(p.sun_irradiance), (C.c_double * 3)(*map(float, p.sun_dir)),
                            int(flags), int(getattr(p, "echo_select", 0)),
                            int(getattr(p, "range_mode", 0)), nt, tp)


def pattern_desc(pattern, keep: list) -> lidar_pattern_desc:
    """Descriptor of a pattern; the host arrays it points to go into `keep`."""
    az = np.ascontiguousarray(pattern.beam_az, dtype=np.float64)
    el = np.ascontiguousarray(pattern.beam_el, dtype=np.float64)
    d = lidar_pattern_desc()
    d.kind = int(pattern.kind)
    d.n_beams = az.shape[0]
    d.beam_az_deg = az.ctypes.data_as(C.POINTER(C.c_double))
    d.beam_el_deg = el.ctypes.data_as(C.POINTER(C.c_double))
    keep += [az, el]
    if pattern.kind == LIDAR_PATTERN_GAUSS:
        d.sigma_deg = (C.c_double * 2)(*map(float, pattern.sigma_deg))
        d.trunc_sigmas = float(pattern.trunc_sigmas)
    else:
        table = np.ascontiguousarray(pattern.table, dtype=np.float32)
        d.table = table.ctypes.data_as(C.POINTER(C.c_float))
        d.ny, d.nx = table.shape
        d.half_deg = (C.c_double * 2)(*map(float, pattern.half_deg))
        keep.append(table)
        rx = getattr(pattern, "rx_table", None)
        if rx is not None:
            rxa = np.ascontiguousarray(rx, dtype=np.float32)
            if rxa.shape != table.shape:
                raise ValueError("rx_table must have the table's shape")
            d.rx_table = rxa.ctypes.data_as(C.POINTER(C.c_float))
            keep.append(rxa)
    return d


def gbuffer_desc(raster, planes, pitch: int | None = None) -> lidar_gbuffer_desc:
    """Descriptor of six float32 device planes [H][pitch] (torch tensors)."""
    ptrs = [int(t.data_ptr()) for t in planes]
    return lidar_gbuffer_desc(int(raster.width), int(raster.height),
                              int(pitch if pitch is not None else raster.width),
                              float(raster.az_min), float(raster.az_max),
                              float(raster.el_min), float(raster.el_max), *ptrs)


class Batch:
    """Descriptor arrays of a batch of frames, built once so that repeated
    simulate_batch calls pass identical descriptors (and replay the captured
    graph).  frames: list of (raster, planes) or (raster, planes, pitch);
    patterns: one pattern per frame (the same object may repeat)."""

    def __init__(self, frames, patterns):
        if len(frames) != len(patterns) or not frames:
            raise ValueError("need one pattern per frame and at least one frame")
        n = len(frames)
        self.n_frames = n
        self.gb = (lidar_gbuffer_desc * n)()
        self.pd = (lidar_pattern_desc * n)()
        self._keep: list = []
        cache = {}
        for i, (fr, pat) in enumerate(zip(frames, patterns)):
            raster, planes = fr[0], fr[1]
            pitch = fr[2] if len(fr) > 2 else None
            self.gb[i] = gbuffer_desc(raster, planes, pitch)
            self._keep.append(planes)
            if id(pat) not in cache:
                cache[id(pat)] = pattern_desc(pat, self._keep)
            self.pd[i] = cache[id(pat)]
        self.n_beams = [int(self.pd[i].n_beams) for i in range(n)]


STATIC_SCRATCH_BYTES = 64 << 20


def simulate_static(params, pattern, raster, planes, echoes, n_echoes, beams, stream=None,
                    pitch: int | None = None):
    """lidar_sim_simulate_static: one plain frame with no device allocation.
    echoes / n_echoes / beams: device tensors of [B][E] lidar_echo bytes
    (uint8 [B][E*40]), int32 [B] and lidar_beam_info bytes (uint8 [B][24])."""
    lib = load()
    keep: list = []
    prm = make_params(params, 0, keep)
    pd = pattern_desc(pattern, keep)
    gd = gbuffer_desc(raster, planes, pitch)
    s = C.c_void_p(stream.cuda_stream if stream is not None else 0)
    rc = lib.lidar_sim_simulate_static(C.byref(prm), C.byref(pd), C.byref(gd), s,
                                       C.c_void_p(echoes.data_ptr()), C.c_void_p(n_echoes.data_ptr()),
                                       C.c_void_p(beams.data_ptr()))
    if rc != LIDAR_OK:
        raise LidarError(rc, lib.lidar_sim_last_error(None).decode())


class LidarSim:
    """One engine handle on one HIP stream."""

    def __init__(self, params, stream=None, keep_waveforms: bool = False,
                 profile: bool = False, autotune: bool = False, deterministic: bool = False):
        self._lib = load()
        self.params = params
        flags = (LIDAR_KEEP_WAVEFORMS if keep_waveforms else 0) | \
            (LIDAR_PROFILE if profile else 0) | (LIDAR_AUTOTUNE if autotune else 0) | \
            (LIDAR_DETERMINISTIC if deterministic else 0)
        keep: list = []
        self._prm = make_params(params, flags, keep)
        self._h = C.c_void_p()
        s = C.c_void_p(stream.cuda_stream if stream is not None else 0)
        rc = self._lib.lidar_sim_create(C.byref(self._prm), s, C.byref(self._h))
        if rc != LIDAR_OK:
            raise LidarError(rc, self._lib.lidar_sim_last_error(None).decode())
        self.n_beams = 0
        self.keep_waveforms = keep_waveforms
        self._keep = []

    def _check(self, rc):
        if rc != LIDAR_OK:
            raise LidarError(rc, self._lib.lidar_sim_last_error(self._h).decode())

    def close(self):
        if self._h:
            self._lib.lidar_sim_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_pattern(self, pattern):
        keep: list = []
        d = pattern_desc(pattern, keep)
        self._check(self._lib.lidar_sim_set_pattern(self._h, C.byref(d)))
        self.n_beams = d.n_beams

    def set_gbuffer(self, raster, planes, pitch: int | None = None):
        """planes: (depth, reflectance, retro_gain, normal_x, normal_y, normal_z),
        float32 device tensors [H][pitch] (kept alive by this object until the
        next call)."""
        d = gbuffer_desc(raster, planes, pitch)
        self._check(self._lib.lidar_sim_set_gbuffer(self._h, C.byref(d)))
        self._keep = list(planes)

    def set_gbuffer_pinhole(self, src, dev_planes, raster, correct: bool = False, pitch=None):
        """src: an object with the pinhole fields (width, height, fx, fy, cx,
        cy, rot, fmt, near, far); dev_planes: (depth, reflectance, retro_gain,
        normal_x, normal_y, normal_z) device tensors [h][pitch]."""
        rot = (C.c_double * 9)(*[float(x) for x in np.asarray(src.rot, dtype=np.float64).ravel()])
        ptrs = [int(t.data_ptr()) for t in dev_planes]
        d = lidar_pinhole_desc(int(src.width), int(src.height),
                               int(pitch if pitch is not None else src.width), float(src.fx),
                               float(src.fy), float(src.cx), float(src.cy), rot, int(src.fmt),
                               1 if correct else 0, float(src.near), float(src.far), *ptrs)
        self._check(self._lib.lidar_sim_set_gbuffer_pinhole(
            self._h, C.byref(d), int(raster.width), int(raster.height), float(raster.az_min),
            float(raster.az_max), float(raster.el_min), float(raster.el_max)))
        self._keep = list(dev_planes)
        self._gb_shape = (int(raster.height), int(raster.width))

    def range_stacking(self, row_kernel, col_kernel, rho_min, s_nearest, xi_nearest):
        """Alg. 2 on the current G-buffer with K[n][m] = col_kernel[n] *
        row_kernel[m]; s_nearest / xi_nearest: device tensors [H][W] int32 /
        float32 (enqueued)."""
        hk = np.ascontiguousarray(row_kernel, dtype=np.float32)
        vk = np.ascontiguousarray(col_kernel, dtype=np.float32)
        self._check(self._lib.lidar_sim_range_stacking(
            self._h, hk.ctypes.data, (hk.size - 1) // 2, vk.ctypes.data, (vk.size - 1) // 2,
            float(rho_min), int(s_nearest.data_ptr()), int(xi_nearest.data_ptr())))

    def read_gbuffer(self) -> np.ndarray:
        """The reprojected planes [6][H][W] (synchronises)."""
        H, W = self._gb_shape
        out = np.zeros((6, H, W), dtype=np.float32)
        self._check(self._lib.lidar_sim_read_gbuffer(self._h, out.ctypes.data, 0))
        return out

    def simulate_frame(self, mode: int = LIDAR_MODE_PLAIN):
        self._check(self._lib.lidar_sim_simulate_frame(self._h, int(mode)))

    def read(self, waveforms: bool = False, beams: bool = True):
        """Copy the last frame's results to host numpy arrays (synchronises)."""
        B, E, R = self.n_beams, int(self.params.max_echoes), int(self.params.n_bins)
        ech = np.zeros((B, E), dtype=ECHO_DTYPE)
        cnt = np.zeros(B, dtype=np.int32)
        wav = np.zeros((B, R), dtype=np.float32) if waveforms else None
        bi = np.zeros(B, dtype=BEAM_DTYPE) if beams else None
        self._check(self._lib.lidar_sim_read_echoes(
            self._h, ech.ctypes.data, cnt.ctypes.data,
            wav.ctypes.data if wav is not None else None,
            bi.ctypes.data if bi is not None else None, 0))
        return {"echoes": ech, "n_echoes": cnt, "waveforms": wav, "beams": bi}

    def read_device(self, echoes=None, n_echoes=None, waveforms=None, beams=None):
        """Enqueue device-to-device copies into torch tensors (no sync)."""
        p = lambda t: int(t.data_ptr()) if t is not None else None
        self._check(self._lib.lidar_sim_read_echoes(self._h, p(echoes), p(n_echoes),
                                                    p(waveforms), p(beams), 1))

    def simulate_batch(self, batch: Batch):
        self._check(self._lib.lidar_sim_simulate_batch(self._h, batch.gb, batch.pd,
                                                       batch.n_frames))
        self._batch = batch

    def read_batch(self, frame: int, waveforms: bool = False, beams: bool = True):
        """Frame `frame` of the last batch as host numpy arrays (synchronises)."""
        B, E, R = self._batch.n_beams[frame], int(self.params.max_echoes), int(self.params.n_bins)
        ech = np.zeros((B, E), dtype=ECHO_DTYPE)
        cnt = np.zeros(B, dtype=np.int32)
        wav = np.zeros((B, R), dtype=np.float32) if waveforms else None
        bi = np.zeros(B, dtype=BEAM_DTYPE) if beams else None
        self._check(self._lib.lidar_sim_read_batch(
            self._h, int(frame), ech.ctypes.data, cnt.ctypes.data,
            wav.ctypes.data if wav is not None else None,
            bi.ctypes.data if bi is not None else None, 0))
        return {"echoes": ech, "n_echoes": cnt, "waveforms": wav, "beams": bi}

    def batch_info(self) -> dict:
        s = lidar_batch_info()
        self._check(self._lib.lidar_sim_batch_info(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in s._fields_ if f != "reserved"}

    def reset_batch(self):
        self._check(self._lib.lidar_sim_reset_batch(self._h))

    # ---- surrogate network (device tensors: x int16 [n][1056] holding bfloat16
    # bit patterns, labels / outputs float32 [n][16]) ----
    def set_weights(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._check(self._lib.lidar_sim_surrogate_set_weights(self._h, p.ctypes.data, p.size))

    def get_weights(self) -> np.ndarray:
        p = np.zeros(SUR_PARAMS, dtype=np.float32)
        self._check(self._lib.lidar_sim_surrogate_get_weights(self._h, p.ctypes.data, p.size))
        return p

    def surrogate_forward(self, x, y):
        self._check(self._lib.lidar_sim_surrogate_forward(self._h, x.data_ptr(), y.data_ptr(),
                                                          x.shape[0]))

    def surrogate_gradients(self, x, labels, grads=None, loss=None):
        p = lambda t: int(t.data_ptr()) if t is not None else None
        self._check(self._lib.lidar_sim_surrogate_gradients(
            self._h, x.data_ptr(), labels.data_ptr(), x.shape[0], p(grads), p(loss)))

    def train_step(self, x, labels, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                   weight_decay=1e-4, loss=None):
        hp = lidar_train_hparams(lr, beta1, beta2, eps, weight_decay)
        self._check(self._lib.lidar_sim_surrogate_train_step(
            self._h, x.data_ptr(), labels.data_ptr(), x.shape[0], C.byref(hp),
            int(loss.data_ptr()) if loss is not None else None))

    def train(self, x, labels, steps: int, batch: int = 4096, lr: float = 1e-3,
              lr_final: float | None = None, weight_decay: float = 1e-4, seed: int = 0,
              losses=None, log_every: int = 0, beta1=0.9, beta2=0.999, eps=1e-8):
        """The library's training loop (lidar_sim_surrogate_train); losses: a
        float32 device tensor of ceil(steps / log_every) entries or None."""
        hp = lidar_train_hparams(lr, beta1, beta2, eps, weight_decay)
        self._check(self._lib.lidar_sim_surrogate_train(
            self._h, x.data_ptr(), labels.data_ptr(), x.shape[0], batch, steps, C.byref(hp),
            lr / 10 if lr_final is None else lr_final, seed & (2 ** 64 - 1),
            int(losses.data_ptr()) if losses is not None else None, log_every))

    def set_gate(self, c_min: float = 0.5, alpha: float = 0.5):
        self._check(self._lib.lidar_sim_surrogate_set_gate(self._h, float(c_min), float(alpha)))

    def surrogate_features(self, x, labels=None, aux=None):
        """x: int16 device tensor [n_beams][1056] (bfloat16 bits); labels,
        aux: float32 device tensors [n_beams][16] / [n_beams][4] or None."""
        p = lambda t: int(t.data_ptr()) if t is not None else None
        self._check(self._lib.lidar_sim_surrogate_features(self._h, x.data_ptr(), p(labels), p(aux)))

    def stats(self) -> dict:
        s = lidar_stats()
        self._check(self._lib.lidar_sim_get_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in s._fields_ if f != "reserved"}

    def reset_stats(self):
        self._check(self._lib.lidar_sim_reset_stats(self._h))

    def last_error(self) -> str:
        return self._lib.lidar_sim_last_error(self._h).decode()
