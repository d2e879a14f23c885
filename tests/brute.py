"""Brute-force evaluation of Eq. 5 on tiny images (test helper).

Every pixel of the image is visited for every beam; the kernel is evaluated
directly at the pixel-minus-beam-pixel offset (Gaussian in closed form, tables
by scipy's zero-padded linear ``map_coordinates``), the row solid angle by
numerical quadrature of cos(e), and the normalisation over a window wider than
any kernel support.  No footprint bookkeeping, clipping or kernel-extent logic
is shared with the oracle.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, ndimage

C = 299792458.0


def kernel_at(pattern, x_deg, y_deg):
    x = np.asarray(x_deg, dtype=np.float64)
    y = np.asarray(y_deg, dtype=np.float64)
    if pattern.kind == 1:
        sx, sy = pattern.sigma_deg
        q = (x / sx) ** 2 + (y / sy) ** 2
        return np.where(q <= pattern.trunc_sigmas ** 2, np.exp(-0.5 * q), 0.0)
    t = pattern.table.astype(np.float64)
    ny, nx = t.shape
    hx, hy = pattern.half_deg
    fx = (x + hx) / (2 * hx / nx) - 0.5
    fy = (hy - y) / (2 * hy / ny) - 0.5
    coords = np.stack([fy.ravel(), fx.ravel()])
    v = ndimage.map_coordinates(t, coords, order=1, mode="grid-constant", cval=0.0)
    inside = (np.abs(x) <= hx) & (np.abs(y) <= hy)
    return np.where(inside, v.reshape(x.shape), 0.0)


def row_solid_angle(raster, v):
    de = raster.de
    e_top = raster.el_max - v * de
    e_bot = raster.el_max - (v + 1) * de
    val, _ = integrate.quad(lambda e: math.cos(math.radians(e)), e_bot, e_top,
                            epsabs=0.0, epsrel=1e-13)
    return math.radians(raster.dphi) * math.radians(1.0) * val


def brute_xi(gbuffer, pattern, params, pad=8):
    """Raw binned signal xi [B][R] and the sun sum a [B] by brute force."""
    r = gbuffer.raster
    W, H, R = r.width, r.height, params.n_bins
    dphi, de = r.dphi, r.de
    us = np.arange(W)
    vs = np.arange(H)
    phi = np.radians(r.az_min + (us + 0.5) * dphi)
    el = np.radians(r.el_max - (vs + 0.5) * de)
    view = np.stack([np.cos(el)[:, None] * np.cos(phi)[None, :],
                     np.cos(el)[:, None] * np.sin(phi)[None, :],
                     np.broadcast_to(np.sin(el)[:, None], (H, W))])
    n = gbuffer.normal.astype(np.float64)
    d = gbuffer.depth.astype(np.float64)
    rho = gbuffer.reflectance.astype(np.float64)
    g = gbuffer.retro_gain.astype(np.float64)
    cos_t = np.maximum(0.0, -(n * view).sum(0))
    valid = np.isfinite(d) & (d > 0)
    dd = np.where(valid, d, 1.0)
    kbin = np.where(valid, np.floor(dd * 2.0 / (C * params.bin_ns * 1e-9)), -1).astype(np.int64)
    valid &= (kbin >= 0) & (kbin < R)
    shade = np.where(valid, g * rho / math.pi * cos_t / (dd * dd), 0.0)
    sun = np.asarray(params.sun_dir, dtype=np.float64)
    sun_shade = np.where(valid, rho / math.pi * np.maximum(0.0, np.tensordot(sun, n, 1)), 0.0)
    # support of the kernel in pixels, padded generously
    if pattern.kind == 1:
        ext_x = pattern.trunc_sigmas * pattern.sigma_deg[0]
        ext_y = pattern.trunc_sigmas * pattern.sigma_deg[1]
    else:
        ext_x, ext_y = pattern.half_deg
    Mw = int(ext_x / dphi) + pad
    Nw = int(ext_y / de) + pad
    # kernel peak for the collector sensitivity kappa = K / max K, over the
    # same offsets the beam kernel uses
    mm, nn = np.meshgrid(np.arange(-Mw, Mw + 1), np.arange(-Nw, Nw + 1))
    kmax = kernel_at(pattern, mm * dphi, -nn * de).max()
    B = pattern.n_beams
    xi = np.zeros((B, R))
    a = np.zeros(B)
    for b in range(B):
        ub = math.floor((pattern.beam_az[b] - r.az_min) / dphi)
        vb = math.floor((r.el_max - pattern.beam_el[b]) / de)
        # normalisation: every kernel cell, on or off the image
        nb = 0.0
        for nrow in range(-Nw, Nw + 1):
            kr = kernel_at(pattern, np.arange(-Mw, Mw + 1) * dphi,
                           np.full(2 * Mw + 1, -nrow * de))
            if kr.any():
                nb += kr.sum() * row_solid_angle(r, vb + nrow)
        Sb = params.emit_power / nb
        # every pixel of the image
        K = kernel_at(pattern, (us[None, :] - ub) * dphi + 0.0 * vs[:, None],
                      -(vs[:, None] - vb) * de + 0.0 * us[None, :])
        om = np.array([row_solid_angle(r, v) for v in vs])[:, None]
        w = Sb * K * om * shade
        np.add.at(xi[b], kbin[valid], w[valid])
        a[b] = ((K / kmax) * om * sun_shade).sum()
    return xi, a
