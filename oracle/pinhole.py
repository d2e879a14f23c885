"""Reprojection of a pinhole rendering onto the equiangular raster, in FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): it shares no code with
the HIP library.

A rasterising renderer gives a pinhole (perspective) image; the beam
iteration needs an image whose pixels are equal steps of azimuth and
elevation, so that one kernel serves every beam (section II-C: reproject the
rendered image).  Depth may come from the z buffer, which stores a window
depth spaced reciprocally between the near and far clipping planes (section
II-D, z buffer resolution).  For every output pixel:

  1. its centre direction v (sensor frame: x forward, y left, z up) is turned
     into the camera frame (x right, y down, z forward): c = R^T v, R the
     camera-to-sensor rotation;
  2. if c_z > 0 it projects to image coordinates x = f_x c_x / c_z + c_x0,
     y = f_y c_y / c_z + c_y0; the pinhole pixel containing that point
     (floor of both; pixel (i, j) covers [i, i+1) x [j, j+1)) is taken as it
     is: no depth interpolation, which would create ranges between targets
     (section II-D, rasterization);
  3. the depth of that pixel is decoded to the radial range r_p along its
     centre ray: a radial range as given; an eye-space z times |ray| / ray_z;
     a window depth w in [0, 1) (float, 16 or 24 bits normalised) first to
     z = n f / (f - w (f - n)); values outside the valid range (non-finite,
     <= 0, w >= 1 or w < 0) are sky;
  4. the output range is r_p, or with the normal-based correction (section
     II-D) r_p (p.n) / (v.n), p the pinhole pixel's centre direction, the
     ratio limited to [1/2, 2] (2 where v misses the plane's facing side);
  5. reflectance and retro gain are copied, the normal is turned into the
     sensor frame (n_s = R n_c).
Output pixels that see no pinhole pixel are sky (range +inf, reflectance 0,
gain 1, normal 0).
"""
from __future__ import annotations

import math

import numpy as np

DEPTH_RANGE, DEPTH_EYE_Z, DEPTH_WINDOW_F32, DEPTH_WINDOW_U16, DEPTH_WINDOW_U24 = 0, 1, 2, 3, 4

# camera-to-sensor rotation of a camera looking along the sensor's x axis:
# camera x (right) = sensor -y, camera y (down) = sensor -z, camera z = sensor x
FORWARD = np.array([[0.0, 0.0, 1.0], [-1.0, 0.0, 0.0], [0.0, -1.0, 0.0]])


def window_depth_to_z(w, near: float, far: float):
    """Eye-space z of a window depth w (perspective depth between the clip
    planes): z = n f / (f - w (f - n)); NaN where w is not in [0, 1)."""
    w = np.asarray(w, dtype=np.float64)
    ok = (w >= 0.0) & (w < 1.0)
    z = near * far / (far - np.where(ok, w, 0.0) * (far - near))
    return np.where(ok, z, np.nan)


def decode_depth(values, fmt: int, near: float = 0.0, far: float = 0.0):
    """Eye-space z (formats EYE_Z and WINDOW_*) or radial range (RANGE) of the
    stored depth values, FP64; NaN marks sky."""
    v = np.asarray(values)
    if fmt == DEPTH_RANGE or fmt == DEPTH_EYE_Z:
        d = v.astype(np.float64)
        return np.where(np.isfinite(d) & (d > 0.0), d, np.nan)
    if fmt == DEPTH_WINDOW_F32:
        w = v.astype(np.float64)
    elif fmt == DEPTH_WINDOW_U16:
        w = v.astype(np.float64) / 65535.0
    elif fmt == DEPTH_WINDOW_U24:
        w = (v.astype(np.uint64) & 0xFFFFFF).astype(np.float64) / 16777215.0
    else:
        raise ValueError(fmt)
    with np.errstate(invalid="ignore"):
        return window_depth_to_z(np.where(np.isfinite(w), w, -1.0), near, far)


def reproject(src: dict, raster, correct: bool = False):
    """src: width, height, fx, fy, cx, cy, rot (3x3 camera-to-sensor), fmt,
    near, far, depth [h][w], reflectance, retro_gain, normal [3][h][w]
    (camera frame).  Returns (depth, reflectance, gain, normal[3]) on the
    equiangular raster (FP64)."""
    R = np.asarray(src["rot"], dtype=np.float64)
    W, H = raster.width, raster.height
    sw, sh = src["width"], src["height"]
    az = np.radians(raster.az_min + (np.arange(W) + 0.5) * (raster.az_max - raster.az_min) / W)
    el = np.radians(raster.el_max - (np.arange(H) + 0.5) * (raster.el_max - raster.el_min) / H)
    vs = np.stack([np.cos(el)[:, None] * np.cos(az)[None, :],
                   np.cos(el)[:, None] * np.sin(az)[None, :],
                   np.broadcast_to(np.sin(el)[:, None], (H, W))])      # [3][H][W]
    # R^T v, each component summed in the order j = 0, 1, 2
    c = [R[0, i] * vs[0] + R[1, i] * vs[1] + R[2, i] * vs[2] for i in range(3)]
    front = c[2] > 0.0
    cz = np.where(front, c[2], 1.0)
    x = src["fx"] * c[0] / cz + src["cx"]
    y = src["fy"] * c[1] / cz + src["cy"]
    i = np.floor(x)
    j = np.floor(y)
    inside = front & (i >= 0) & (i < sw) & (j >= 0) & (j < sh)
    ii = np.where(inside, i, 0).astype(np.int64)
    jj = np.where(inside, j, 0).astype(np.int64)
    dec = decode_depth(src["depth"], src["fmt"], src.get("near", 0.0), src.get("far", 0.0))[jj, ii]
    # centre ray of the pinhole pixel, camera frame, and its radial range
    rx = (ii + 0.5 - src["cx"]) / src["fx"]
    ry = (jj + 0.5 - src["cy"]) / src["fy"]
    norm = np.sqrt(rx * rx + ry * ry + 1.0)
    rng = dec if src["fmt"] == DEPTH_RANGE else dec * norm
    nc = [src["normal"][k].astype(np.float64)[jj, ii] for k in range(3)]
    ns = np.stack([R[i, 0] * nc[0] + R[i, 1] * nc[1] + R[i, 2] * nc[2] for i in range(3)])
    if correct:
        pc = [rx / norm, ry / norm, 1.0 / norm]
        ps = [R[i, 0] * pc[0] + R[i, 1] * pc[1] + R[i, 2] * pc[2] for i in range(3)]
        pn = ps[0] * ns[0] + ps[1] * ns[1] + ps[2] * ns[2]
        vn = vs[0] * ns[0] + vs[1] * ns[1] + vs[2] * ns[2]
        with np.errstate(divide="ignore", invalid="ignore"):
            q = pn / vn
        q = np.where(q > 0.0, q, 2.0)
        q = np.clip(q, 0.5, 2.0)
        rng = rng * q
    valid = inside & np.isfinite(rng)
    depth = np.where(valid, rng, np.inf)
    refl = np.where(valid, src["reflectance"].astype(np.float64)[jj, ii], 0.0)
    gain = np.where(valid, src["retro_gain"].astype(np.float64)[jj, ii], 1.0)
    normal = np.where(valid[None], ns, 0.0)
    return depth, refl, gain, normal


def to_gbuffer(raster, planes):
    """A scenes.GBuffer (float32 planes) from reproject's output."""
    import scenes
    depth, refl, gain, normal = planes
    return scenes.GBuffer(raster, depth.astype(np.float32), refl.astype(np.float32),
                          gain.astype(np.float32), normal.astype(np.float32))
