"""Pins of the pinhole reprojection oracle (z-buffer decoding, nearest
pinhole pixel, normal-based range correction) against closed forms."""
import math

import numpy as np
import pytest

import scenes
from oracle import pinhole as P


def test_window_depth_round_trip_and_endpoints():
    """The OpenGL window depth of eye distance z decodes back to z; the near
    plane maps to 0, the far plane to 1 (sky), and w grows with z."""
    n, f = 0.5, 500.0
    z = np.geomspace(n, f * 0.999, 400)
    w = scenes.encode_window_depth(z, n, f)
    assert w[0] == pytest.approx(0.0, abs=1e-15) and np.all(np.diff(w) > 0)
    assert scenes.encode_window_depth(np.array([f]), n, f)[0] == pytest.approx(1.0)
    np.testing.assert_allclose(P.window_depth_to_z(w, n, f), z, rtol=1e-9)
    assert np.isnan(P.window_depth_to_z(np.array([1.0, -0.1]), n, f)).all()


@pytest.mark.parametrize("fmt,levels", [(P.DEPTH_WINDOW_U16, 65535.0), (P.DEPTH_WINDOW_U24, 16777215.0)])
def test_quantised_window_depth_error_bound(fmt, levels):
    """Rounding w to q / levels moves z by at most dz/dw / (2 levels), with
    dz/dw = z^2 (f - n) / (n f): the error grows with z^2 and shrinks as the
    near plane moves out (section II-D: most resolution sits near the near
    plane)."""
    errs = {}
    for n in (0.1, 1.0):
        f = 1000.0
        z = np.geomspace(1.0, 300.0, 500)
        q = np.rint(scenes.encode_window_depth(z, n, f) * levels)
        q = q.astype(np.uint16 if fmt == P.DEPTH_WINDOW_U16 else np.uint32)
        dec = P.decode_depth(q, fmt, n, f)
        bound = z * z * (f - n) / (n * f) / (2 * levels)
        assert np.all(np.abs(dec - z) <= bound * (1 + 1e-6) + 1e-9 * z)
        errs[n] = np.abs(dec - z).max()
    assert errs[1.0] < 0.2 * errs[0.1]


def _plane_src(fmt=P.DEPTH_RANGE, yaw=0.0, pitch=-2.0, near=0.5, far=500.0):
    return scenes.pinhole_render(0, width=320, height=180, hfov_deg=50.0, yaw_deg=yaw,
                                 pitch_deg=pitch, fmt=fmt, near=near, far=far, n_boxes=0,
                                 retro_frac=0.0)


def _independent_projection(src, v):
    """Image coordinates of sensor direction v: intersect v with the image
    plane at distance f along the optical axis and measure the hit along the
    camera's right and down axes (columns of the rotation)."""
    right, down, axis = src.rot[:, 0], src.rot[:, 1], src.rot[:, 2]
    s = v @ axis
    hit = v / s
    return src.cx + src.fx * (hit @ right), src.cy + src.fy * (hit @ down), s


def test_reprojected_road_plane_closed_form():
    """The road plane z = -h seen through a camera pitched down: each output
    pixel takes the range along its nearest pinhole pixel's centre ray,
    -h / ray_z; with the correction, the range along its own direction,
    -h / v_z."""
    src = _plane_src()
    r = scenes.Raster(200, 60, -20.0, 20.0, -10.0, 1.0)
    dirs = scenes.pixel_directions(r)
    plain = P.reproject(src.as_dict(), r)[0]
    corr = P.reproject(src.as_dict(), r, correct=True)[0]
    h = scenes.SENSOR_HEIGHT
    checked = 0
    for v in range(0, 60, 3):
        for u in range(0, 200, 7):
            d = dirs[:, v, u]
            x, y, s = _independent_projection(src, d)
            if not (s > 0 and 0 <= x < src.width and 0 <= y < src.height):
                assert np.isinf(plain[v, u])
                continue
            i, j = int(math.floor(x)), int(math.floor(y))
            ray = src.rot @ np.array([(i + 0.5 - src.cx) / src.fx, (j + 0.5 - src.cy) / src.fy, 1.0])
            ray /= np.linalg.norm(ray)
            if ray[2] >= 0:
                assert np.isinf(plain[v, u])
                continue
            checked += 1
            assert plain[v, u] == pytest.approx(-h / ray[2], rel=2e-7)
            if d[2] < 0 and 0.5 <= ray[2] / d[2] <= 2.0:
                assert corr[v, u] == pytest.approx(-h / d[2], rel=2e-7)
    assert checked > 150


def test_depth_formats_agree():
    """The same scene stored as radial range, eye-space z and float window
    depth reprojects to the same ranges (to the precision of the format)."""
    r = scenes.Raster(160, 48, -22.0, 22.0, -8.0, 2.0)
    out = {fmt: P.reproject(scenes.pinhole_render(3, width=320, height=180, hfov_deg=50.0,
                                                  pitch_deg=-2.0, fmt=fmt, n_boxes=6).as_dict(), r)
           for fmt in (P.DEPTH_RANGE, P.DEPTH_EYE_Z, P.DEPTH_WINDOW_F32)}
    a = out[P.DEPTH_RANGE][0]
    fin = np.isfinite(a)
    assert fin.mean() > 0.3
    np.testing.assert_array_equal(np.isfinite(out[P.DEPTH_EYE_Z][0]), fin)
    np.testing.assert_allclose(out[P.DEPTH_EYE_Z][0][fin], a[fin], rtol=3e-7)
    # float32 window depth: dz = z^2 (f - n)/(n f) * 2^-24 at most
    b = out[P.DEPTH_WINDOW_F32][0]
    tol = a[fin] ** 2 * (500.0 - 0.5) / (0.5 * 500.0) * 2.0 ** -23 + 1e-6 * a[fin]
    assert np.all(np.abs(b[fin] - a[fin]) <= tol)
    for k in (1, 2):
        np.testing.assert_array_equal(out[P.DEPTH_EYE_Z][k], out[P.DEPTH_RANGE][k])


def test_nearest_pinhole_pixel_under_a_rotated_camera():
    """Pixel ids stored as reflectance: every output pixel takes the pinhole
    pixel containing its direction's projection (yaw 30, pitch 5 deg); the
    output pixel holding the direction of the optical axis takes the centre
    pixel; normals turn into the sensor frame."""
    src = scenes.pinhole_render(1, width=96, height=64, hfov_deg=40.0, yaw_deg=30.0,
                                pitch_deg=5.0, fmt=P.DEPTH_RANGE, n_boxes=0, retro_frac=0.0)
    ids = (np.arange(96 * 64, dtype=np.float64) / (96 * 64)).reshape(64, 96).astype(np.float32)
    src.reflectance[:] = ids
    src.depth[:] = 10.0
    r = scenes.Raster(240, 120, 0.0, 60.0, -15.0, 25.0)
    depth, refl, gain, normal = P.reproject(src.as_dict(), r)
    dirs = scenes.pixel_directions(r)
    seen = 0
    for v in range(0, 120, 2):
        for u in range(0, 240, 3):
            x, y, s = _independent_projection(src, dirs[:, v, u])
            if s > 0 and 0 <= x < 96 and 0 <= y < 64:
                seen += 1
                k = int(round(float(refl[v, u]) * 96 * 64))
                assert (k % 96, k // 96) == (int(math.floor(x)), int(math.floor(y)))
                assert depth[v, u] == 10.0
            else:
                assert np.isinf(depth[v, u]) and refl[v, u] == 0.0 and gain[v, u] == 1.0
    assert seen > 300
    axis = src.rot[:, 2]
    az, el = math.degrees(math.atan2(axis[1], axis[0])), math.degrees(math.asin(axis[2]))
    u = int((az - r.az_min) / r.dphi)
    v = int((r.el_max - el) / r.de)
    k = int(round(float(refl[v, u]) * 96 * 64))
    assert abs(k % 96 - 48) <= 1 and abs(k // 96 - 32) <= 1
    # the camera-frame normal (0, 0, -1) faces the camera: in the sensor frame
    # it points against the optical axis
    src.normal[:] = np.array([0.0, 0.0, -1.0], np.float32)[:, None, None]
    n_s = P.reproject(src.as_dict(), r)[3]
    np.testing.assert_allclose(n_s[:, v, u], -axis, atol=1e-12)
