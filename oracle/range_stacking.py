"""Range stacking (paper section II-C, Alg. 2) in FP64 with library correlations.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The rendered per-pixel intensity image is split into depth slices of one time
bin each; every slice is correlated with the centred kernel (one 2-D
correlation per slice, ``scipy.ndimage.correlate``), and the slices are
visited from far to near, keeping per pixel the nearest slice whose
correlated intensity reaches the threshold.  The paper states that with equal
parameters both algorithms agree to floating-point limits; at a beam's pixel
the slice correlation equals the beam-iteration signal of that bin divided by
the beam's scale factor.

The loop visits every slice 0 .. R-1 (the paper's loop bound stops at 1; the
0-based reading visits every bin).
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage


def slice_correlations(intensity: np.ndarray, bins: np.ndarray, kernel: np.ndarray,
                       n_bins: int, slices=None) -> dict:
    """{s: correlate(intensity * [bins == s], kernel)} for the requested slices
    (default: every slice that holds at least one pixel)."""
    if slices is None:
        slices = np.unique(bins[(bins >= 0) & (bins < n_bins)])
    out = {}
    for s in slices:
        img = np.where(bins == s, intensity, 0.0)
        out[int(s)] = ndimage.correlate(img, kernel, mode="constant", cval=0.0)
    return out


def nearest_above(intensity: np.ndarray, bins: np.ndarray, kernel: np.ndarray,
                  n_bins: int, rho_min: float):
    """Alg. 2: (S_nearest, xi_nearest) per pixel; S_nearest = n_bins where no
    slice reaches rho_min."""
    H, W = intensity.shape
    s_near = np.full((H, W), n_bins, dtype=np.int64)
    xi_near = np.zeros((H, W))
    present = np.unique(bins[(bins >= 0) & (bins < n_bins)])
    for s in sorted(present.tolist(), reverse=True):
        img = np.where(bins == s, intensity, 0.0)
        corr = ndimage.correlate(img, kernel, mode="constant", cval=0.0)
        hit = corr >= rho_min
        xi_near[hit] = corr[hit]
        s_near[hit] = s
    return s_near, xi_near
