"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module only *produces inputs*: G-buffer planes on an equiangular
azimuth/elevation raster, beam steering patterns, the beam x receiver pattern
table and the sensor parameters.  It contains none of the method's
arithmetic (no footprint weights, no time binning, no pulse shaping, no echo
detection); both sides of every parity test consume exactly the arrays made
here.

Raster convention (shared input format, see ``include/lidar_sim.h``):
  * ``W x H`` pixels, row-major ``[H][W]`` float32 planes;
  * column ``u`` covers azimuth ``[az_min + u*dphi, az_min + (u+1)*dphi)`` with
    ``dphi = (az_max - az_min) / W`` (degrees);
  * row ``v`` covers elevation ``[el_max - (v+1)*de, el_max - v*de)`` with
    ``de = (el_max - el_min) / H``; row 0 is the top of the image;
  * the unit direction of azimuth ``phi`` and elevation ``e`` in the sensor
    frame (x forward, y left, z up) is ``(cos e cos phi, cos e sin phi, sin e)``;
  * ``depth`` is the radial range in metres along the pixel-centre ray; sky is
    ``+inf``; normals are unit vectors in the sensor frame.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import math

import numpy as np

C_LIGHT = 299792458.0


@dataclass
class Raster:
    width: int
    height: int
    az_min: float
    az_max: float
    el_min: float
    el_max: float

    @property
    def dphi(self) -> float:
        return (self.az_max - self.az_min) / self.width

    @property
    def de(self) -> float:
        return (self.el_max - self.el_min) / self.height


@dataclass
class GBuffer:
    raster: Raster
    depth: np.ndarray        # [H][W] float32, radial range (m); inf = no hit
    reflectance: np.ndarray  # [H][W] float32, diffuse albedo rho
    retro_gain: np.ndarray   # [H][W] float32, g (1 = not retroreflective)
    normal: np.ndarray       # [3][H][W] float32, unit surface normal

    def planes(self):
        return (self.depth, self.reflectance, self.retro_gain,
                self.normal[0], self.normal[1], self.normal[2])


PATTERN_GAUSS = 1
PATTERN_TABLE = 2


@dataclass
class Pattern:
    kind: int
    beam_az: np.ndarray                  # [B] float64, degrees
    beam_el: np.ndarray                  # [B] float64, degrees
    sigma_deg: tuple = (0.0, 0.0)        # GAUSS: sigma along az, el
    trunc_sigmas: float = 3.0            # GAUSS: elliptical cut radius in sigmas
    table: np.ndarray | None = None      # TABLE: [ny][nx] float32, row 0 = +el
    half_deg: tuple = (0.0, 0.0)         # TABLE: half extent along az, el
    rx_table: np.ndarray | None = None   # TABLE: collector sensitivity kappa on the same grid

    @property
    def n_beams(self) -> int:
        return int(self.beam_az.shape[0])


@dataclass
class SensorParams:
    n_bins: int
    bin_ns: float
    max_echoes: int
    threshold: float
    emit_power: float
    pulse_fwhm_ns: float
    pulse_trunc_sigmas: float = 4.0
    ambient_const: float = 0.0
    sun_irradiance: float = 0.0
    sun_dir: tuple = (0.0, 0.0, 1.0)
    pulse_taps: np.ndarray | None = None  # tabulated pulse: 2J+1 samples at the bin pitch
    echo_select: int = 0                  # ECHO_SELECT_* (0: the first max_echoes runs)
    range_mode: int = 0                   # RANGE_* (0: each pixel at its centre range)


# echo selection and range modes (values of the C-ABI's enums)
ECHO_SELECT_ALL, ECHO_SELECT_STRONGEST, ECHO_SELECT_NEAREST, ECHO_SELECT_LONGEST = 0, 1, 2, 3
ECHO_SELECT_RAW_STRONGEST, ECHO_SELECT_RAW_NEAREST = 4, 5
RANGE_CENTRE, RANGE_CORRECTED, RANGE_INTERVAL = 0, 1, 2


@dataclass
class Workload:
    name: str
    gbuffer: GBuffer
    pattern: Pattern
    params: SensorParams
    meta: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------
# geometry helpers (input generation only)
# ----------------------------------------------------------------------------

def pixel_directions(r: Raster) -> np.ndarray:
    """Unit pixel-centre directions, [3][H][W] float64."""
    dphi, de = r.dphi, r.de
    phi = np.deg2rad(r.az_min + (np.arange(r.width) + 0.5) * dphi)
    el = np.deg2rad(r.el_max - (np.arange(r.height) + 0.5) * de)
    ce, se = np.cos(el)[:, None], np.sin(el)[:, None]
    cp, sp = np.cos(phi)[None, :], np.sin(phi)[None, :]
    return np.stack([ce * cp, ce * sp, np.broadcast_to(se, (r.height, r.width))])


def _orthonormal_basis(a: np.ndarray):
    """Two unit vectors orthogonal to the unit vectors a ([3][...])."""
    helper = np.zeros_like(a)
    use_z = np.abs(a[2]) < 0.9
    helper[2][use_z] = 1.0
    helper[0][~use_z] = 1.0
    t1 = np.cross(a, helper, axis=0)
    t1 /= np.linalg.norm(t1, axis=0, keepdims=True)
    t2 = np.cross(a, t1, axis=0)
    return t1, t2


# ----------------------------------------------------------------------------
# Workload 1: uniform random G-buffer, grid of Gaussian beams
# ----------------------------------------------------------------------------

def random_gbuffer(raster: Raster, rng: np.random.Generator, depth_range=(5.0, 60.0),
                   refl_range=(0.05, 0.9), max_tilt_deg=60.0, retro_frac=0.02,
                   retro_gain=100.0) -> GBuffer:
    """i.i.d. per-pixel surfaces: depth U(depth_range), reflectance U(refl_range),
    normals uniform on the cap of half-angle ``max_tilt_deg`` around -view (so
    cos(theta) ~ U(cos max_tilt, 1)), retroreflective with probability
    ``retro_frac`` (gain ``retro_gain``, else 1)."""
    H, W = raster.height, raster.width
    depth = rng.uniform(depth_range[0], depth_range[1], size=(H, W))
    refl = rng.uniform(refl_range[0], refl_range[1], size=(H, W))
    cmin = math.cos(math.radians(max_tilt_deg))
    cos_t = rng.uniform(cmin, 1.0, size=(H, W))
    psi = rng.uniform(0.0, 2.0 * math.pi, size=(H, W))
    retro = rng.uniform(size=(H, W)) < retro_frac
    view = pixel_directions(raster)
    a = -view
    t1, t2 = _orthonormal_basis(a)
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    n = a * cos_t + t1 * (sin_t * np.cos(psi)) + t2 * (sin_t * np.sin(psi))
    n /= np.linalg.norm(n, axis=0, keepdims=True)
    gain = np.where(retro, retro_gain, 1.0)
    return GBuffer(raster, depth.astype(np.float32), refl.astype(np.float32),
                   gain.astype(np.float32), n.astype(np.float32))


def grid_beams(raster: Raster, n_az: int, n_el: int, az_range=None, el_range=None):
    """Beams at the centres of an n_az x n_el grid of cells over the FOV."""
    a0, a1 = az_range if az_range else (raster.az_min, raster.az_max)
    e0, e1 = el_range if el_range else (raster.el_min, raster.el_max)
    az = a0 + (np.arange(n_az) + 0.5) * ((a1 - a0) / n_az)
    el = e0 + (np.arange(n_el) + 0.5) * ((e1 - e0) / n_el)
    ee, aa = np.meshgrid(el, az, indexing="ij")   # line-major: [el][az]
    return aa.ravel().astype(np.float64), ee.ravel().astype(np.float64)


def iid_frame(seed: int = 0) -> Workload:
    """1024x512 px over 60x30 deg, i.i.d. surfaces, 40x25 grid of Gaussian
    beams (sigma 0.1 deg, cut at 3 sigma), 512 bins of 1 ns, 4 ns FWHM pulse,
    constant ambient, fixed threshold."""
    rng = np.random.default_rng(seed)
    raster = Raster(1024, 512, -30.0, 30.0, -15.0, 15.0)
    gb = random_gbuffer(raster, rng)
    az, el = grid_beams(raster, 40, 25)
    pat = Pattern(PATTERN_GAUSS, az, el, sigma_deg=(0.1, 0.1), trunc_sigmas=3.0)
    ambient = 1e-7
    params = SensorParams(n_bins=512, bin_ns=1.0, max_echoes=3,
                          threshold=ambient + 5e-6, emit_power=1.0,
                          pulse_fwhm_ns=4.0, pulse_trunc_sigmas=4.0,
                          ambient_const=ambient, sun_irradiance=0.0)
    return Workload("plain-1frame-1024x512-1000beams-gauss", gb, pat, params,
                    {"seed": seed})


# ----------------------------------------------------------------------------
# Workload 2: scanning sensor, road + boxes, tabulated elliptic pattern
# ----------------------------------------------------------------------------

SENSOR_HEIGHT = 0.5

# Threshold and sun irradiance of the scanning-sensor workload.  T is 5 % of
# the pulse-convolved peak return of a rho = 0.5 Lambertian face at 100 m
# that fills the beam at normal incidence.  The per-beam sun floor is
# bimodal (a quarter of the beams see only sky through their core, the
# beams whose core sees the sunlit road collect 20-50 times more than the
# median), so E_sun is set by its upper end: the 95th percentile of the
# floor is 0.75 T, which keeps every beam's floor below T (the median floor
# is then 0.004 T).  Both literals were derived with the FP64 oracle and are
# re-derived by the test suite (tests/test_workloads.py).
ROAD_THRESHOLD = 9.345e-08
ROAD_SUN_IRRADIANCE = 0.02841


def elliptic_table(nx=256, ny=256, half_deg=(2.0, 2.0), fwhm_deg=(0.1, 0.8),
                   tail=1e-4, tail_radius_deg=2.0) -> np.ndarray:
    """Combined beam x receiver pattern on a [ny][nx] grid of cell centres over
    +-half_deg: elliptic Gaussian core plus a flat tail of relative level
    ``tail`` inside a disc (blooming tails).  Row 0 is the top (+elevation)."""
    hx, hy = half_deg
    x = -hx + (np.arange(nx) + 0.5) * (2.0 * hx / nx)
    y = hy - (np.arange(ny) + 0.5) * (2.0 * hy / ny)
    sx = fwhm_deg[0] / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    sy = fwhm_deg[1] / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    yy, xx = np.meshgrid(y, x, indexing="ij")
    core = np.exp(-0.5 * ((xx / sx) ** 2 + (yy / sy) ** 2))
    disc = (xx * xx + yy * yy) <= tail_radius_deg ** 2
    t = core + tail * disc
    t[t < 1e-30] = 0.0          # no float32 denormals in the table
    return t.astype(np.float32)


@dataclass
class Box:
    center: np.ndarray   # (x, y) on the road plane, metres
    yaw: float           # radians
    length: float
    width: float
    height: float
    rho: float


def _ray_box(dirs, box: Box, z0: float):
    """Ray-OBB slab intersection for rays from the origin.  Returns (t, normal)
    with t = inf for misses.  dirs: [3][N]."""
    c, s = math.cos(box.yaw), math.sin(box.yaw)
    # box frame: x along length, y along width, z up; origin at box centre
    cz = z0 + 0.5 * box.height
    o = np.array([-box.center[0], -box.center[1], -cz])
    o_l = np.array([c * o[0] + s * o[1], -s * o[0] + c * o[1], o[2]])
    d_l = np.stack([c * dirs[0] + s * dirs[1], -s * dirs[0] + c * dirs[1], dirs[2]])
    half = np.array([0.5 * box.length, 0.5 * box.width, 0.5 * box.height])
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d_l
        t1 = (-half[:, None] - o_l[:, None]) * inv
        t2 = (half[:, None] - o_l[:, None]) * inv
    tmin = np.minimum(t1, t2)
    tmax = np.maximum(t1, t2)
    tmin = np.where(np.isnan(tmin), -np.inf, tmin)
    tmax = np.where(np.isnan(tmax), np.inf, tmax)
    t_near = tmin.max(axis=0)
    t_far = tmax.min(axis=0)
    axis = tmin.argmax(axis=0)
    hit = (t_near <= t_far) & (t_near > 1e-6)
    t = np.where(hit, t_near, np.inf)
    # outward normal of the entry face, in the box frame then rotated back
    sign = -np.sign(np.take_along_axis(d_l, axis[None, :], axis=0)[0])
    n_l = np.zeros((3, dirs.shape[1]))
    n_l[axis, np.arange(dirs.shape[1])] = sign
    n = np.stack([c * n_l[0] - s * n_l[1], s * n_l[0] + c * n_l[1], n_l[2]])
    return t, n, axis, o_l, d_l


def road_scene(raster: Raster, rng: np.random.Generator, n_boxes=24,
               range_lim=(5.0, 140.0), lateral_lim=(-15.0, 15.0), retro_frac=0.01,
               retro_gain=500.0):
    """FP64 ray cast of a road plane (SENSOR_HEIGHT below the sensor) and
    ``n_boxes`` vehicle-like boxes standing on it (longitudinal position
    U(range_lim), lateral U(lateral_lim), heading within +-17 deg of the road);
    sky = inf.  Rectangular retroreflective patches (plates / signs) are added
    on the box faces until at least ``retro_frac`` of the pixels are
    retroreflective."""
    H, W = raster.height, raster.width
    dirs = pixel_directions(raster)                      # [3][H][W]
    z0 = -SENSOR_HEIGHT
    with np.errstate(divide="ignore", invalid="ignore"):
        t_road = np.where(dirs[2] < 0.0, z0 / dirs[2], np.inf)
    depth = t_road.copy()
    normal = np.zeros((3, H, W))
    normal[2] = 1.0
    obj = np.where(np.isfinite(t_road), 0, -1).astype(np.int64)
    rho_road = rng.uniform(0.05, 0.9)
    boxes = []
    for i in range(n_boxes):
        b = Box(center=np.array([rng.uniform(*range_lim), rng.uniform(*lateral_lim)]),
                yaw=rng.uniform(-0.3, 0.3), length=rng.uniform(4.0, 12.0),
                width=rng.uniform(1.8, 2.6), height=rng.uniform(1.4, 3.5),
                rho=rng.uniform(0.05, 0.9))
        boxes.append(b)
    # cast each box only over the pixel block spanned by its corners
    blocks = []
    for i, b in enumerate(boxes):
        c, s = math.cos(b.yaw), math.sin(b.yaw)
        corners = []
        for sl in (-0.5, 0.5):
            for sw in (-0.5, 0.5):
                for sh in (0.0, 1.0):
                    x = b.center[0] + c * sl * b.length - s * sw * b.width
                    y = b.center[1] + s * sl * b.length + c * sw * b.width
                    corners.append((x, y, z0 + sh * b.height))
        corners = np.array(corners)
        if np.any(corners[:, 0] <= 0.1):
            blocks.append(None)
            continue
        az = np.degrees(np.arctan2(corners[:, 1], corners[:, 0]))
        el = np.degrees(np.arctan2(corners[:, 2], np.hypot(corners[:, 0], corners[:, 1])))
        u0 = max(0, int(math.floor((az.min() - raster.az_min) / raster.dphi)) - 2)
        u1 = min(W, int(math.ceil((az.max() - raster.az_min) / raster.dphi)) + 2)
        v0 = max(0, int(math.floor((raster.el_max - el.max()) / raster.de)) - 2)
        v1 = min(H, int(math.ceil((raster.el_max - el.min()) / raster.de)) + 2)
        if u0 >= u1 or v0 >= v1:
            blocks.append(None)
            continue
        d = dirs[:, v0:v1, u0:u1].reshape(3, -1)
        t, n, axis, o_l, d_l = _ray_box(d, b, z0)
        shape = (v1 - v0, u1 - u0)
        t = t.reshape(shape)
        cur = depth[v0:v1, u0:u1]
        closer = t < cur
        cur[closer] = t[closer]
        nn = normal[:, v0:v1, u0:u1]
        nn[:, closer] = n.reshape(3, *shape)[:, closer]
        obj[v0:v1, u0:u1][closer] = i + 1
        blocks.append((v0, v1, u0, u1, axis.reshape(shape), o_l, d_l.reshape(3, *shape)))
    rho = np.where(obj == 0, rho_road, 0.0)
    for i, b in enumerate(boxes):
        rho = np.where(obj == i + 1, b.rho, rho)
    gain = np.ones((H, W))
    # retroreflective patches on box faces, in face-local coordinates
    target = int(math.ceil(retro_frac * H * W))
    n_retro = 0
    visible = [i for i in range(n_boxes) if blocks[i] is not None
               and np.any(obj[blocks[i][0]:blocks[i][1], blocks[i][2]:blocks[i][3]] == i + 1)]
    guard = 0
    while n_retro < target and visible and guard < 20000:
        guard += 1
        bi = visible[int(rng.integers(0, len(visible)))]
        b = boxes[bi]
        v0, v1, u0, u1, axis, o_l, d_l = blocks[bi]
        mine = obj[v0:v1, u0:u1] == bi + 1
        dd = depth[v0:v1, u0:u1]
        p = o_l[:, None, None] + d_l * np.where(mine, dd, 0.0)[None]
        side = axis[mine]
        if not np.any(side != 2):
            continue
        face = int(rng.choice(side[side != 2]))
        s_coord = p[1] if face == 0 else p[0]
        h_coord = p[2] + 0.5 * b.height
        face_len = b.width if face == 0 else b.length
        pw = rng.uniform(0.3, 1.2)
        ph = rng.uniform(0.1, 0.6)
        s0 = rng.uniform(-0.5 * face_len, max(-0.5 * face_len, 0.5 * face_len - pw))
        h0 = rng.uniform(0.2, max(0.25, b.height - ph - 0.1))
        inside = mine & (axis == face) & (s_coord >= s0) & (s_coord <= s0 + pw) & \
            (h_coord >= h0) & (h_coord <= h0 + ph)
        g = gain[v0:v1, u0:u1]
        newly = inside & (g == 1.0)
        if n_retro > 0 and n_retro + int(newly.sum()) > 1.2 * target:
            continue            # keep the retroreflective fraction near the target
        g[newly] = retro_gain
        n_retro += int(newly.sum())
    gb = GBuffer(raster, depth.astype(np.float32), rho.astype(np.float32),
                 gain.astype(np.float32), normal.astype(np.float32))
    return gb, boxes, obj


def road_scan(seed: int = 0, width: int = 8192, height: int = 512,
            n_lines: int = 16, n_cols: int = 1800) -> Workload:
    """Scanning sensor: 8192x512 px over 145 x 3.2 deg, road + 24 boxes, 1 %
    retroreflective patches with gain 500, 16 x 1800 beams, tabulated 256x256
    elliptic pattern (FWHM 0.1 x 0.8 deg, 1e-4 tails to 2 deg), 2048 bins of
    0.5 ns, sun ambient, up to 3 echoes.  ``width``/``height``/``n_lines``/
    ``n_cols`` shrink the same scene for quick tests (FOV unchanged)."""
    rng = np.random.default_rng(seed)
    raster = Raster(width, height, -72.5, 72.5, -1.6, 1.6)
    gb, boxes, obj = road_scene(raster, rng)
    az, el = grid_beams(raster, n_cols, n_lines)
    pat = Pattern(PATTERN_TABLE, az, el, table=elliptic_table(),
                  half_deg=(2.0, 2.0))
    se, ce = math.sin(math.radians(30.0)), math.cos(math.radians(30.0))
    sun = (ce * math.cos(math.radians(45.0)), ce * math.sin(math.radians(45.0)), se)
    params = SensorParams(n_bins=2048, bin_ns=0.5, max_echoes=3,
                          threshold=ROAD_THRESHOLD, emit_power=1.0,
                          pulse_fwhm_ns=4.0, pulse_trunc_sigmas=4.0,
                          ambient_const=0.0,
                          sun_irradiance=ROAD_SUN_IRRADIANCE, sun_dir=sun)
    name = f"plain-scan-{width}x{height}-{n_lines}x{n_cols}beams-table256"
    return Workload(name, gb, pat, params, {"seed": seed, "boxes": boxes,
                                            "object_id": obj})


def subset_beams(w: Workload, idx) -> Workload:
    """The same workload restricted to the beams ``idx`` (beams are independent)."""
    idx = np.asarray(idx)
    pat = replace(w.pattern, beam_az=w.pattern.beam_az[idx].copy(),
                  beam_el=w.pattern.beam_el[idx].copy())
    return replace(w, pattern=pat)


# ----------------------------------------------------------------------------
# small hand-built inputs for closed-form and edge-case tests
# ----------------------------------------------------------------------------

def shell_gbuffer(raster: Raster, depth_m: float, rho: float, gain: float = 1.0) -> GBuffer:
    """Every pixel at the same radial range, facing the sensor (n = -view)."""
    H, W = raster.height, raster.width
    n = -pixel_directions(raster)
    return GBuffer(raster, np.full((H, W), depth_m, np.float32),
                   np.full((H, W), rho, np.float32),
                   np.full((H, W), gain, np.float32), n.astype(np.float32))


# ----------------------------------------------------------------------------
# Workload 3: a batch of uneven frames
# ----------------------------------------------------------------------------

@dataclass
class BatchWorkload:
    name: str
    frames: list            # of Workload, all with the same SensorParams
    params: SensorParams
    meta: dict = field(default_factory=dict)


def lissajous_beams(raster: Raster, n: int, p: int, q: int, fill: float = 0.95):
    """n beams along a Lissajous figure over the FOV: az = A_az sin(2 pi p t +
    pi/2), el = A_el sin(2 pi q t), t = i / n (centred on the FOV)."""
    t = np.arange(n, dtype=np.float64) / n
    ca = 0.5 * (raster.az_min + raster.az_max)
    cel = 0.5 * (raster.el_min + raster.el_max)
    A_az = 0.5 * fill * (raster.az_max - raster.az_min)
    A_el = 0.5 * fill * (raster.el_max - raster.el_min)
    az = ca + A_az * np.sin(2.0 * math.pi * p * t + 0.5 * math.pi)
    el = cel + A_el * np.sin(2.0 * math.pi * q * t)
    return az, el


def jitter_beams(raster: Raster, n_az: int, n_el: int, rng: np.random.Generator):
    """Grid beams moved by U(-1/2, 1/2) of the grid spacing in each angle."""
    az, el = grid_beams(raster, n_az, n_el)
    da = (raster.az_max - raster.az_min) / n_az
    de = (raster.el_max - raster.el_min) / n_el
    az = az + rng.uniform(-0.5, 0.5, az.shape) * da
    el = el + rng.uniform(-0.5, 0.5, el.shape) * de
    return az, el


BATCH_SIZES = ((512, 256), (1024, 512), (2048, 1024), (4096, 2048))


def batch_params() -> SensorParams:
    """Sensor of the batch workload: the scanning sensor's waveform (2048 bins
    of 0.5 ns, 4 ns pulse, threshold) with a constant ambient term instead of
    the sun (the sun floor grows with the footprint's solid angle, which here
    spans three decades)."""
    return SensorParams(n_bins=2048, bin_ns=0.5, max_echoes=3,
                        threshold=ROAD_THRESHOLD, emit_power=1.0,
                        pulse_fwhm_ns=4.0, pulse_trunc_sigmas=4.0,
                        ambient_const=1e-8, sun_irradiance=0.0)


def frame_batch(seed: int = 0, n_frames: int = 64, sizes=BATCH_SIZES,
            beams=(5000, 100000), footprint_px=(20.0, 20000.0),
            fov=(60.0, 30.0), threads: int = 8) -> BatchWorkload:
    """Batch of ``n_frames`` frames: sizes cycled through ``sizes`` (equal
    counts, shuffled), scenes alternating between i.i.d. surfaces (as the
    1-frame workload) and the road + boxes ray cast (as the scanning sensor)
    over a ``fov`` (deg) field of view, steering cycling through grid,
    Lissajous (coprime p, q) and jittered grid, beam count ~ log-U(``beams``)
    and Gaussian footprints of F ~ log-U(``footprint_px``) pixels (radius
    sqrt(F / pi) px = 3 sigma).  Smaller ``sizes``/``beams``/``footprint_px``
    give the same recipe at test scale."""
    rng = np.random.default_rng(seed)
    params = batch_params()
    size_idx = np.repeat(np.arange(len(sizes)), int(math.ceil(n_frames / len(sizes))))[:n_frames]
    rng.shuffle(size_idx)

    def frame(i):
        W, H = sizes[size_idx[i]]
        raster = Raster(W, H, -0.5 * fov[0], 0.5 * fov[0], -0.5 * fov[1], 0.5 * fov[1])
        frng = np.random.default_rng([seed, i])
        if i % 2 == 0:
            gb = random_gbuffer(raster, frng)
            style = "iid"
        else:
            gb = road_scene(raster, frng)[0]
            style = "road"
        B = int(round(math.exp(frng.uniform(math.log(beams[0]), math.log(beams[1])))))
        F = math.exp(frng.uniform(math.log(footprint_px[0]), math.log(footprint_px[1])))
        sigma_px = math.sqrt(F / math.pi) / 3.0
        steer = ("grid", "lissajous", "jitter")[i % 3]
        n_el = max(1, int(round(math.sqrt(B * H / W))))
        n_az = max(1, int(round(B / n_el)))
        if steer == "grid":
            az, el = grid_beams(raster, n_az, n_el)
        elif steer == "jitter":
            az, el = jitter_beams(raster, n_az, n_el, frng)
        else:
            p = int(frng.integers(50, 400))
            q = int(frng.integers(int(0.6 * p), int(0.9 * p)))
            while math.gcd(p, q) != 1:
                q += 1
            az, el = lissajous_beams(raster, B, p, q)
        pat = Pattern(PATTERN_GAUSS, az, el,
                      sigma_deg=(sigma_px * raster.dphi, sigma_px * raster.de),
                      trunc_sigmas=3.0)
        return Workload(f"frame{i}-{W}x{H}-{style}-{steer}", gb, pat, params,
                        {"footprint_px": F, "steering": steer, "scene": style})

    # every frame draws from its own seeded generator: threads do not change
    # the result
    if threads > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(threads) as ex:
            frames = list(ex.map(frame, range(n_frames)))
    else:
        frames = [frame(i) for i in range(n_frames)]
    return BatchWorkload(f"batch-{n_frames}frames-uneven", frames, params,
                         {"seed": seed, "sizes": [sizes[k] for k in size_idx]})


# ----------------------------------------------------------------------------
# surrogate network: seeded initial weights (an input of training)
# ----------------------------------------------------------------------------

SURROGATE_LAYERS = ((1056, 1030, 256), (256, 256, 256), (256, 256, 256), (256, 256, 16))
SURROGATE_OUT_USED = 13


def surrogate_init(seed: int = 0) -> np.ndarray:
    """Flat FP32 parameters [W1 (1056x256, row-major in x out), b1, W2, b2, W3,
    b3, W4 (256x16), b4]: weights U(-sqrt(3/fan_in), sqrt(3/fan_in)) (unit
    variance per unit-variance input), zero biases; the padding rows of W1
    (inputs 1030..1055) and columns of W4 (outputs 13..15) are zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (n_in, fan_in, n_out) in enumerate(SURROGATE_LAYERS):
        a = math.sqrt(3.0 / fan_in)
        W = rng.uniform(-a, a, size=(n_in, n_out))
        W[fan_in:, :] = 0.0
        if li == len(SURROGATE_LAYERS) - 1:
            W[:, SURROGATE_OUT_USED:] = 0.0
        parts += [W.ravel(), np.zeros(n_out)]
    return np.concatenate(parts).astype(np.float32)


def random_bf16_bits(seed: int, n: int, cols: int = 1056, used: int = 1030,
                     scale: float = 1.0) -> np.ndarray:
    """[n][cols] bfloat16 bit patterns (uint16) of N(0, scale^2) draws
    truncated to bfloat16 (the low 16 bits of the binary32 value dropped);
    columns from ``used`` on are zero."""
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal((n, cols)) * scale).astype(np.float32)
    x[:, used:] = 0.0
    return (x.view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def bf16_bits_to_float(b: np.ndarray) -> np.ndarray:
    """The float32 values of bfloat16 bit patterns (exact)."""
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def random_surrogate_labels(seed: int, n: int) -> np.ndarray:
    """[n][16] label rows: random existence flags and targets of moderate size."""
    rng = np.random.default_rng(seed)
    lab = np.zeros((n, 16), dtype=np.float32)
    lab[:, :3] = rng.integers(0, 2, size=(n, 3))
    lab[:, 3:12] = (rng.standard_normal((n, 9)) * 0.5).astype(np.float32)
    lab[:, 3:12] *= np.tile(lab[:, :3], 3)
    return lab


# ----------------------------------------------------------------------------
# Workloads 4 and 5: frames for the surrogate (training data and inference)
# ----------------------------------------------------------------------------

def surrogate_frame(seed: int, pattern: str = "gauss", n_lines: int = 64,
                    n_cols: int = 2000) -> Workload:
    """A scanning-sensor scene (8192x512 px over 145 x 3.2 deg, road + 24
    boxes, 1 % retroreflective patches) scanned by n_lines x n_cols beams.
    pattern "gauss": Gaussian beams with the scanning pattern's core (sigma
    0.0425 x 0.34 deg, cut at 3 sigma) and the batch workload's sensor
    (constant ambient, no sun); "table": the tabulated pattern with its 1e-4
    tails and the scanning sensor's parameters (sun floor)."""
    w = road_scan(seed, n_lines=n_lines, n_cols=n_cols)
    if pattern == "table":
        return replace(w, name=f"surrogate-scan-{n_lines}x{n_cols}-table256")
    pat = Pattern(PATTERN_GAUSS, w.pattern.beam_az, w.pattern.beam_el,
                  sigma_deg=(0.0425, 0.34), trunc_sigmas=3.0)
    return replace(w, pattern=pat, params=batch_params(),
                   name=f"surrogate-scan-{n_lines}x{n_cols}-gauss")


def core_only_pattern(pattern: Pattern) -> Pattern:
    """The scanning workload's tabulated pattern without its 1e-4 tails (the
    same beams and elliptic core), to tell which echoes the tails decide."""
    return Pattern(PATTERN_TABLE, pattern.beam_az, pattern.beam_el,
                   table=elliptic_table(tail=0.0), half_deg=(2.0, 2.0))


# ----------------------------------------------------------------------------
# Pinhole renderings (the renderer's side of a z buffer)
# ----------------------------------------------------------------------------

@dataclass
class Pinhole:
    """A pinhole rendering: intrinsics (image x = fx X/Z + cx, y = fy Y/Z + cy,
    camera frame x right, y down, z forward; pixel (i, j) covers [i, i+1) x
    [j, j+1)), camera-to-sensor rotation, depth in one of the formats of
    ``oracle.pinhole`` (DEPTH_*), and reflectance, retro gain and normals
    (camera frame) as [h][w] planes."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    rot: np.ndarray
    fmt: int
    near: float
    far: float
    depth: np.ndarray          # float32 (RANGE, EYE_Z, WINDOW_F32), uint16 or uint32
    reflectance: np.ndarray
    retro_gain: np.ndarray
    normal: np.ndarray         # [3][h][w] float32, camera frame

    def as_dict(self):
        return dict(width=self.width, height=self.height, fx=self.fx, fy=self.fy, cx=self.cx,
                    cy=self.cy, rot=self.rot, fmt=self.fmt, near=self.near, far=self.far,
                    depth=self.depth, reflectance=self.reflectance, retro_gain=self.retro_gain,
                    normal=self.normal)


def yaw_pitch_rotation(yaw_deg: float = 0.0, pitch_deg: float = 0.0) -> np.ndarray:
    """Camera-to-sensor rotation of a camera turned by yaw (to the left, about
    z) and pitch (upwards) from looking along the sensor's x axis."""
    fwd = np.array([[0.0, 0.0, 1.0], [-1.0, 0.0, 0.0], [0.0, -1.0, 0.0]])
    a, b = math.radians(yaw_deg), math.radians(pitch_deg)
    rz = np.array([[math.cos(a), -math.sin(a), 0.0], [math.sin(a), math.cos(a), 0.0], [0.0, 0.0, 1.0]])
    ry = np.array([[math.cos(b), 0.0, -math.sin(b)], [0.0, 1.0, 0.0], [math.sin(b), 0.0, math.cos(b)]])
    return rz @ ry @ fwd


def encode_window_depth(z, near: float, far: float):
    """Window depth of eye-space distances z (> 0) under an OpenGL
    perspective projection: clip-space z / w mapped from [-1, 1] to [0, 1];
    non-finite z (no hit) is the cleared far value 1."""
    z = np.asarray(z, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        # projection matrix row 3 applied to (.., .., -z, 1), divided by w = z
        clip_z = (-(far + near) / (far - near)) * (-z) + (-2.0 * far * near / (far - near))
        ndc = clip_z / z
    w = np.clip(0.5 * ndc + 0.5, 0.0, 1.0)          # depth buffers clamp to [0, 1]
    return np.where(np.isfinite(z) & (z > 0), w, 1.0)


def pinhole_render(seed: int = 0, width: int = 640, height: int = 360, hfov_deg: float = 60.0,
                   yaw_deg: float = 0.0, pitch_deg: float = 0.0, fmt: int = 0,
                   near: float = 0.5, far: float = 500.0, n_boxes: int = 10,
                   retro_frac: float = 0.02) -> Pinhole:
    """Road plane (SENSOR_HEIGHT below the sensor) and boxes ray cast in FP64
    through a pinhole camera; per object reflectance U(0.05, 0.9); a random
    fraction of pixels retroreflective (gain 100); depth stored in format
    ``fmt`` (0 radial range, 1 eye-space z, 2/3/4 window depth as float32 /
    uint16 / 24 bits in uint32 between the near and far planes)."""
    rng = np.random.default_rng(seed)
    f = 0.5 * width / math.tan(math.radians(0.5 * hfov_deg))
    cx, cy = 0.5 * width, 0.5 * height
    R = yaw_pitch_rotation(yaw_deg, pitch_deg)
    jj, ii = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
    ray_c = np.stack([(ii + 0.5 - cx) / f, (jj + 0.5 - cy) / f, np.ones((height, width))])
    norm = np.sqrt((ray_c ** 2).sum(0))
    dirs = np.einsum("ij,jhw->ihw", R, ray_c / norm)                    # unit, sensor frame
    z0 = -SENSOR_HEIGHT
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(dirs[2] < 0.0, z0 / dirs[2], np.inf)
    normal = np.zeros((3, height, width))
    normal[2] = 1.0
    rho = np.full((height, width), rng.uniform(0.05, 0.9))
    flat = dirs.reshape(3, -1)
    for _ in range(n_boxes):
        b = Box(center=np.array([rng.uniform(6.0, 80.0), rng.uniform(-12.0, 12.0)]),
                yaw=rng.uniform(-0.4, 0.4), length=rng.uniform(3.0, 10.0),
                width=rng.uniform(1.8, 2.6), height=rng.uniform(1.2, 3.0), rho=rng.uniform(0.05, 0.9))
        tb, nb, _, _, _ = _ray_box(flat, b, z0)
        tb = tb.reshape(height, width)
        closer = tb < t
        t = np.where(closer, tb, t)
        normal[:, closer] = nb.reshape(3, height, width)[:, closer]
        rho = np.where(closer, b.rho, rho)
    hit = np.isfinite(t)
    rho = np.where(hit, rho, 0.0)
    gain = np.where(hit & (rng.uniform(size=t.shape) < retro_frac), 100.0, 1.0)
    n_cam = np.einsum("ji,jhw->ihw", R, normal)                         # R^T n
    z_eye = t / norm
    if fmt == 0:
        depth = t.astype(np.float32)
    elif fmt == 1:
        depth = z_eye.astype(np.float32)
    else:
        w = encode_window_depth(np.where(hit, z_eye, np.inf), near, far)
        if fmt == 2:
            depth = w.astype(np.float32)
        elif fmt == 3:
            depth = np.clip(np.rint(w * 65535.0), 0, 65535).astype(np.uint16)
        else:
            depth = np.clip(np.rint(w * 16777215.0), 0, 16777215).astype(np.uint32)
    return Pinhole(width, height, f, f, cx, cy, R, fmt, near, far, depth,
                   rho.astype(np.float32), gain.astype(np.float32), n_cam.astype(np.float32))


# ----------------------------------------------------------------------------
# Range stacking (Alg. 2) workload
# ----------------------------------------------------------------------------

@dataclass
class StackWorkload:
    name: str
    gbuffer: GBuffer
    params: SensorParams
    row_kernel: np.ndarray     # H over columns m = -M..M
    col_kernel: np.ndarray     # V over rows n = -N..N
    rho_min: float


def range_stacking_scene(seed: int = 0) -> StackWorkload:
    """The paper's range-stacking setting (a 4096-pixel-wide rendering,
    68-pixel-wide beam kernels, 1200 range slices): the road + boxes scene
    ray cast on 4096 x 512 pixels over 145 x 12.8 deg; a separable kernel
    H * V standing in for the scanning pattern: H an elliptic core of sigma
    0.0425 deg (1.2 px) with a 1e-4 tail over 69 columns, V a Gaussian of
    sigma 0.34 deg (13.6 px) over 83 rows; 1200 slices of 1 ns; rho_min is
    5 % of the correlation of a rho = 0.5 face at 100 m that fills the
    kernel."""
    rng = np.random.default_rng(seed)
    raster = Raster(4096, 512, -72.5, 72.5, -6.4, 6.4)
    gb, boxes, obj = road_scene(raster, rng)
    x = np.arange(-34, 35) * raster.dphi
    H = (np.exp(-0.5 * (x / 0.0425) ** 2) + 1e-4).astype(np.float32)
    y = np.arange(-41, 42) * raster.de
    V = np.exp(-0.5 * (y / 0.34) ** 2).astype(np.float32)
    om = math.radians(raster.dphi) * math.radians(raster.de)
    rho_min = 0.05 * float(H.astype(np.float64).sum() * V.astype(np.float64).sum()) * om * 0.5 / (
        math.pi * 100.0 ** 2)
    params = SensorParams(n_bins=1200, bin_ns=1.0, max_echoes=3, threshold=rho_min, emit_power=1.0,
                          pulse_fwhm_ns=4.0)
    return StackWorkload(f"range-stacking-4096x512-69x83-1200slices", gb, params, H, V, rho_min)
