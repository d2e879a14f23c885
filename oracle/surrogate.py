"""FP64 oracle of the learned surrogate (MLP 1056 -> 256 -> 256 -> 256 -> 16).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): it shares no code with
the HIP library.  The paper has no learned component; this module follows the
surrogate as the method's extension defines it: a multilayer perceptron with
GELU activations, trained by AdamW on echoes that the plain method produced.

Network (inputs padded from 1030 to 1056 with zeros, outputs padded from 13 to
16):
    Z1 = X W1 + b1,  H1 = gelu(Z1)
    Z2 = H1 W2 + b2, H2 = gelu(Z2)
    Z3 = H2 W3 + b3, H3 = gelu(Z3)
    Y  = H3 W4 + b4
with gelu(z) = z/2 (1 + erf(z / sqrt 2)).  The GPU computes every product in
BF16 with FP32 accumulation and stores X, the weights, H1..H3 and the
backward operands dY, dZ3..dZ1 in BF16; with ``rounded=True`` this oracle
rounds the same quantities to BF16 (round to nearest even) and does every
other operation in FP64.  With ``rounded=False`` it is the plain FP64
network, whose gradients are pinned against central finite differences.

Outputs y[0..2]: existence logits of echoes 1..3; y[3..5]: peak bin relative
to the beam's reference bin, in units of 16 bins; y[6..8]: log10(intensity /
T); y[9..11]: echo pulse width / 4 ns; y[12]: confidence logit.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

IN, IN_USED, HID, OUT, OUT_USED = 1056, 1030, 256, 16, 13
SHAPES = [("W1", (IN, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, HID)), ("b3", (HID,)), ("W4", (HID, OUT)), ("b4", (OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
BIN_SCALE = 16.0          # y[3..5] are in units of 16 bins
DK_CLIP = 4.0             # labels of peak offsets are clipped to +-64 bins
W_BIN, W_INT, W_EPW = 64.0, 1.0, 1.0


def unpack(flat: np.ndarray) -> dict:
    """Views of the flat parameter vector (W row-major [in][out])."""
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    return out


def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    bfloat16 keeps the sign, the 8 exponent bits and the top 7 fraction bits
    of a binary32 value; rounding adds half an ulp of the kept part (plus one
    when the kept part is odd) before truncating the low 16 bits."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _erf(x):
    return np.vectorize(math.erf, otypes=[np.float64])(x)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    """d/dz of z Phi(z) = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


@dataclass
class Cache:
    X: np.ndarray
    Z: list
    H: list
    Y: np.ndarray


def forward(X, flat, rounded: bool = True) -> Cache:
    p = unpack(np.asarray(flat, dtype=np.float64))
    r = bf16_round if rounded else (lambda a: np.asarray(a, dtype=np.float64))
    A = r(X)
    Z, H = [], [A]
    for l in (1, 2, 3):
        z = H[-1] @ r(p[f"W{l}"]) + p[f"b{l}"]
        Z.append(z)
        H.append(r(gelu(z)))
    Y = H[-1] @ r(p["W4"]) + p["b4"]
    return Cache(A, Z, H, Y)


def _bce(z, t):
    return np.maximum(z, 0.0) - z * t + np.log1p(np.exp(-np.abs(z)))


def _sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def confidence_target(Y, lab) -> np.ndarray:
    """1 where the prediction has every existence right and every existing
    echo in the right bin, its offset label not clipped (decided in FP32, as
    the device does)."""
    y = np.asarray(Y, dtype=np.float32)
    l = np.asarray(lab, dtype=np.float32)
    ok = np.ones(y.shape[0], dtype=bool)
    for e in range(3):
        te = l[:, e] > np.float32(0.5)
        ok &= (y[:, e] > 0) == te
        ok &= ~(te & (np.abs(y[:, 3 + e] - l[:, 3 + e]) * np.float32(BIN_SCALE) > np.float32(0.5)))
        ok &= ~(te & (np.abs(l[:, 3 + e]) >= np.float32(DK_CLIP)))
    return ok.astype(np.float64)


def loss_and_grad(Y, lab):
    """Mean over rows of the per-row loss
        sum_e BCE(y_e, exists_e)
      + sum_e exists_e (64 (dk_e' - dk_e)^2 + (li_e' - li_e)^2 + (w_e' - w_e)^2)
      + BCE(y_12, ok)
    and its gradient with respect to Y (zero in the padding columns)."""
    Y = np.asarray(Y, dtype=np.float64)
    lab = np.asarray(lab, dtype=np.float64)
    n = Y.shape[0]
    ok = confidence_target(Y, lab)
    L = np.zeros(n)
    G = np.zeros_like(Y)
    for e in range(3):
        ex = lab[:, e]
        L += _bce(Y[:, e], ex)
        G[:, e] = _sigmoid(Y[:, e]) - ex
        for off, w in ((3, W_BIN), (6, W_INT), (9, W_EPW)):
            d = Y[:, off + e] - lab[:, off + e]
            L += ex * w * d * d
            G[:, off + e] = ex * 2.0 * w * d
    L += _bce(Y[:, 12], ok)
    G[:, 12] = _sigmoid(Y[:, 12]) - ok
    return float(L.mean()), G / n


def backward(cache: Cache, dY, flat, rounded: bool = True) -> np.ndarray:
    """Gradient of the loss with respect to the flat parameters (FP32 biases
    and weights), given dL/dY."""
    p = unpack(np.asarray(flat, dtype=np.float64))
    r = bf16_round if rounded else (lambda a: np.asarray(a, dtype=np.float64))
    g = {}
    d = r(dY)                                   # operand of the products
    g["W4"] = cache.H[3].T @ d
    g["b4"] = d.sum(axis=0)
    for l in (3, 2, 1):
        dh = d @ r(p[f"W{l + 1}"]).T
        dz = r(dh * gelu_prime(cache.Z[l - 1]))
        g[f"W{l}"] = cache.H[l - 1].T @ dz
        g[f"b{l}"] = dz.sum(axis=0)
        d = dz
    return np.concatenate([g[name].ravel() for name, _ in SHAPES])


def decay_mask() -> np.ndarray:
    """1 for weights (decayed), 0 for biases."""
    return np.concatenate([np.full(int(np.prod(s)), 1.0 if n.startswith("W") else 0.0)
                           for n, s in SHAPES])


def adamw_step(theta, grad, m, v, t: int, lr, beta1, beta2, eps, weight_decay):
    """One AdamW step (Loshchilov and Hutter's decoupled weight decay, with
    bias correction): theta <- theta (1 - lr wd mask); m, v moving moments;
    theta <- theta - lr m_hat / (sqrt(v_hat) + eps).  Returns new copies."""
    theta = np.asarray(theta, dtype=np.float64) * (1.0 - lr * weight_decay * decay_mask())
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * grad
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ----------------------------------------------------------------------------
# Inputs of the network: coarse maps, per-beam patches, tail and floor
# estimates (FP64; the device rounds the inputs to BF16)
# ----------------------------------------------------------------------------

C_LIGHT = 299792458.0
CORE_FRACTION = 2e-4      # the core box holds every kernel cell with K >= 2e-4 max K
PATCH = 16
TAIL_BINS = 64            # coarse time bins of the tail-energy estimate


def geometry(K: np.ndarray, width: int, height: int) -> dict:
    """Cell sizes from the kernel grid K[n + N][m + M]: coarse cells tile the
    core box (cells with K >= 2e-4 max K) 16 x 16 times; super-cells tile
    the whole kernel window 16 x 16 times."""
    KH, KW = K.shape
    N, M = (KH - 1) // 2, (KW - 1) // 2
    rows, cols = np.nonzero(K >= CORE_FRACTION * K.max())
    cn, cm = int(np.abs(rows - N).max()), int(np.abs(cols - M).max())
    cw = max(1, -(-(2 * cm + 1) // PATCH))
    ch = max(1, -(-(2 * cn + 1) // PATCH))
    sw = max(1, -(-KW // PATCH))
    sh = max(1, -(-KH // PATCH))
    return dict(M=M, N=N, KW=KW, KH=KH, cm=cm, cn=cn, cw=cw, ch=ch, sw=sw, sh=sh,
                CW=-(-width // cw), CH=-(-height // ch), SW=-(-width // sw), SH=-(-height // sh),
                kmax=float(K.max()))


def pixel_terms(gbuffer, params, row_omega) -> dict:
    """Per-pixel FP64 quantities of the plain method: validity (finite depth
    > 0 whose time bin floor(2 d / (c dt)) is below R), cos(theta) =
    max(0, -n.v) with v the pixel-centre direction, the shade Omega (g rho /
    pi) cos(theta) / d^2 and the sun shading Omega (rho / pi) max(0, n.s)."""
    r = gbuffer.raster
    W, H = r.width, r.height
    dphi = (r.az_max - r.az_min) / W
    de = (r.el_max - r.el_min) / H
    az = np.deg2rad(r.az_min + (np.arange(W) + 0.5) * dphi)[None, :]
    el = np.deg2rad(r.el_max - (np.arange(H) + 0.5) * de)[:, None]
    vx, vy, vz = np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el) + 0 * az
    d = gbuffer.depth.astype(np.float64)
    rho = gbuffer.reflectance.astype(np.float64)
    g = gbuffer.retro_gain.astype(np.float64)
    n = [a.astype(np.float64) for a in gbuffer.normal]
    to_bin = 2.0 / (C_LIGHT * (params.bin_ns * 1e-9))
    with np.errstate(invalid="ignore", over="ignore"):
        ok = np.isfinite(d) & (d > 0)
        kb = np.where(ok, np.floor(np.where(ok, d, 0.0) * to_bin), np.inf)
    valid = ok & (kb < params.n_bins)
    kbin = np.where(valid, kb, -1.0)
    dv = np.where(valid, d, 1.0)
    cos = np.maximum(0.0, -(n[0] * vx + n[1] * vy + n[2] * vz))
    om = np.array([row_omega(v) for v in range(H)])[:, None]
    shade = np.where(valid, om * (g * rho / math.pi) * cos / (dv * dv), 0.0)
    s = params.sun_dir
    sun = np.where(valid, om * (rho / math.pi) * np.maximum(0.0, n[0] * s[0] + n[1] * s[1] + n[2] * s[2]), 0.0)
    return dict(valid=valid, d=np.where(valid, d, 0.0), rho=np.where(valid, rho, 0.0),
                g=np.where(valid, g, 0.0), cos=np.where(valid, cos, 0.0), shade=shade, sun=sun,
                kbin=kbin, to_bin=to_bin)


def _block_sum(a, bw, bh, nx, ny):
    H, W = a.shape
    pad = np.zeros((ny * bh, nx * bw))
    pad[:H, :W] = a
    return pad.reshape(ny, bh, nx, bw).sum(axis=(1, 3))


def _block_bin_range(kbin, bw, bh, nx, ny):
    """Per block: smallest and largest time bin of its valid pixels (0, -1
    for blocks without valid pixels)."""
    H, W = kbin.shape
    lo = np.full((ny * bh, nx * bw), np.inf)
    hi = np.full((ny * bh, nx * bw), -np.inf)
    lo[:H, :W] = np.where(kbin >= 0, kbin, np.inf)
    hi[:H, :W] = np.where(kbin >= 0, kbin, -np.inf)
    lo = lo.reshape(ny, bh, nx, bw).min(axis=(1, 3))
    hi = hi.reshape(ny, bh, nx, bw).max(axis=(1, 3))
    has = np.isfinite(lo)
    return np.where(has, lo, 0.0).astype(np.int64), np.where(has, hi, -1.0).astype(np.int64)


def coarse_maps(t: dict, geo: dict) -> dict:
    """Coarse cells (cw x ch pixels, clipped at the image edge): mean depth,
    retro gain and cos(theta) over valid pixels, reflectance summed over valid
    pixels divided by all pixels of the cell, sums of shade and sun shading;
    super-cells: sums of shade and sun shading, range of time bins."""
    cw, ch, CW, CH = geo["cw"], geo["ch"], geo["CW"], geo["CH"]
    ones = np.ones_like(t["d"])
    nall = _block_sum(ones, cw, ch, CW, CH)
    nval = _block_sum(t["valid"].astype(np.float64), cw, ch, CW, CH)
    safe = np.maximum(nval, 1.0)
    return dict(nval=nval,
                dmean=_block_sum(t["d"], cw, ch, CW, CH) / safe,
                rho=_block_sum(t["rho"], cw, ch, CW, CH) / nall,
                gmean=_block_sum(t["g"], cw, ch, CW, CH) / safe,
                cmean=_block_sum(t["cos"], cw, ch, CW, CH) / safe,
                sunc=_block_sum(t["sun"], cw, ch, CW, CH),
                shadec=_block_sum(t["shade"], cw, ch, CW, CH),
                shade=_block_sum(t["shade"], geo["sw"], geo["sh"], geo["SW"], geo["SH"]),
                binrange=_block_bin_range(t["kbin"], geo["sw"], geo["sh"], geo["SW"], geo["SH"]),
                sun=_block_sum(t["sun"], geo["sw"], geo["sh"], geo["SW"], geo["SH"]))


REF_WINDOW = 512          # time bins of the reference-bin histogram
REF_SMOOTH = (1.0, 2.0, 3.0, 2.0, 1.0)


def reference_bin(K, geo, maps, Ib, Jb, u, v, nval, dmean, Ic, Jc, inside, to_bin) -> int:
    """A coarse estimate of the beam's strongest return: the patch cells
    whose centre lies in the core box add K(centre) * (shade sum) at the time
    bin of their mean depth into a histogram of REF_WINDOW bins from the
    smallest such bin; the first maximum of the histogram smoothed with
    (1, 2, 3, 2, 1) is the reference bin.  Without such cells: the bin of the
    nearest cell mean depth in the patch, else 0."""
    M, N, cm, cn = geo["M"], geo["N"], geo["cm"], geo["cn"]
    cw, ch = geo["cw"], geo["ch"]
    ks, ws = [], []
    for j in range(PATCH):
        J = Jb - PATCH // 2 + j
        n = (2 * J * ch + ch - 2 * v) // 2
        for i in range(PATCH):
            I = Ib - PATCH // 2 + i
            m = (2 * I * cw + cw - 2 * u) // 2
            if not inside[j, i] or nval[j, i] <= 0 or abs(m) > cm or abs(n) > cn:
                continue
            w = K[n + N, m + M] * maps["shadec"][Jc[j, 0], Ic[0, i]]
            if w > 0:
                ks.append(int(math.floor(dmean[j, i] * to_bin)))
                ws.append(w)
    if ks:
        kmin = min(ks)
        hist = np.zeros(REF_WINDOW + 4)
        for k, w in zip(ks, ws):
            if k - kmin < REF_WINDOW:
                hist[k - kmin + 2] += w
        sm = np.zeros(REF_WINDOW)
        for d, c in enumerate(REF_SMOOTH):
            sm += c * hist[d:d + REF_WINDOW]
        return kmin + int(np.argmax(sm))
    if np.any(nval > 0):
        return int(math.floor(dmean[nval > 0].min() * to_bin))
    return 0


def beam_features(K, geo, maps, t, u, v, scale, az_deg, el_deg, params):
    """Network input (1056 values, FP64 before rounding) and (k_ref, E_tail,
    A_est) of one beam whose pixel is (u, v)."""
    W = t["d"].shape[1]
    H = t["d"].shape[0]
    cw, ch, CW, CH = geo["cw"], geo["ch"], geo["CW"], geo["CH"]
    Ib, Jb = u // cw, v // ch
    I = Ib - PATCH // 2 + np.arange(PATCH)[None, :]
    J = Jb - PATCH // 2 + np.arange(PATCH)[:, None]
    inside = (I >= 0) & (I < CW) & (J >= 0) & (J < CH)
    Ic, Jc = np.clip(I, 0, CW - 1), np.clip(J, 0, CH - 1)
    nval = np.where(inside, maps["nval"][Jc, Ic], 0.0)
    dmean = maps["dmean"][Jc, Ic]
    to_bin = t["to_bin"]
    M, N, cm, cn = geo["M"], geo["N"], geo["cm"], geo["cn"]
    k_ref = reference_bin(K, geo, maps, Ib, Jb, u, v, nval, dmean, Ic, Jc, inside, to_bin)
    x = np.zeros(IN)
    ch0 = np.where(nval > 0, np.clip((dmean * to_bin - (k_ref + 0.5)) / 64.0, -1.0, 1.0), 1.0)
    ch1 = np.where(inside, maps["rho"][Jc, Ic], 0.0)
    ch2 = np.where(nval > 0, np.log10(np.where(nval > 0, maps["gmean"][Jc, Ic], 1.0)) / 3.0, 0.0)
    ch3 = np.where(nval > 0, maps["cmean"][Jc, Ic], 0.0)
    for c, a in enumerate((ch0, ch1, ch2, ch3)):
        x[c * 256:(c + 1) * 256] = a.ravel()
    # the kernel is taken at each cell's centre (nearest kernel cell):
    # sun floor of the core box from the coarse cells, tail energy and the
    # tail's sun floor from the super-cells outside the core box
    a_sum = 0.0
    for j in range(PATCH):
        Jc_ = Jb - PATCH // 2 + j
        n = (2 * Jc_ * ch + ch - 2 * v) // 2
        if not (0 <= Jc_ < CH) or abs(n) > cn:
            continue
        for i in range(PATCH):
            Ic_ = Ib - PATCH // 2 + i
            m = (2 * Ic_ * cw + cw - 2 * u) // 2
            if not (0 <= Ic_ < CW) or abs(m) > cm:
                continue
            a_sum += K[n + N, m + M] * maps["sunc"][Jc_, Ic_]
    sw, sh = geo["sw"], geo["sh"]
    I0, I1 = max(0, (u - M) // sw), min(geo["SW"] - 1, (u + M) // sw)
    J0, J1 = max(0, (v - N) // sh), min(geo["SH"] - 1, (v + N) // sh)
    # tail energy per time bin: each tail super-cell spreads K * (its shade
    # sum) evenly over its bin range; the densities are summed per coarse bin
    # of TAIL_BIN bins (as if they met in one bin), and E_tail is the largest
    lo, hi = maps["binrange"]
    nb = -(-params.n_bins // TAIL_BINS)
    hist = np.zeros(TAIL_BINS)
    for Js in range(J0, J1 + 1):
        n = (2 * Js * sh + sh - 2 * v) // 2
        if abs(n) > N:
            continue
        for Is in range(I0, I1 + 1):
            m = (2 * Is * sw + sw - 2 * u) // 2
            if abs(m) > M or (abs(m) <= cm and abs(n) <= cn):
                continue
            w = K[n + N, m + M]
            a_sum += w * maps["sun"][Js, Is]
            if hi[Js, Is] >= lo[Js, Is]:
                dens = w * maps["shade"][Js, Is] / (hi[Js, Is] - lo[Js, Is] + 1)
                hist[lo[Js, Is] // nb:hi[Js, Is] // nb + 1] += dens
    et = hist.max()
    e_tail = scale * et
    a_est = params.ambient_const + params.sun_irradiance / geo["kmax"] * a_sum
    T = params.threshold
    x[1024] = ((u - Ib * cw) + 0.5) / cw - 0.5
    x[1025] = ((v - Jb * ch) + 0.5) / ch - 0.5
    x[1026] = el_deg / 90.0
    x[1027] = az_deg / 180.0
    x[1028] = (min(2.0, max(-4.0, math.log10(max(a_est, 1e-30) / T))) / 4.0) if T > 0 else 0.0
    x[1029] = k_ref / params.n_bins
    return x, k_ref, e_tail, a_est


def features(gbuffer, pattern, params, K, pixels, scales, row_omega):
    """Inputs of every beam: X [B][1056] (FP64), k_ref [B], E_tail [B],
    A_est [B], and the geometry."""
    geo = geometry(K, gbuffer.raster.width, gbuffer.raster.height)
    t = pixel_terms(gbuffer, params, row_omega)
    maps = coarse_maps(t, geo)
    B = len(scales)
    X = np.zeros((B, IN))
    kref = np.zeros(B, dtype=np.int64)
    et = np.zeros(B)
    ae = np.zeros(B)
    for b in range(B):
        X[b], kref[b], et[b], ae[b] = beam_features(
            K, geo, maps, t, int(pixels[b, 0]), int(pixels[b, 1]), float(scales[b]),
            float(pattern.beam_az[b]), float(pattern.beam_el[b]), params)
    return X, kref, et, ae, geo


def labels(kref, echoes, n_echoes, params) -> np.ndarray:
    """Training targets of beams from their plain-path echoes: existence of
    echoes 1..3, (peak bin - k_ref) / 16 clipped to +-4, log10(max(intensity,
    1e-3 T) / T), pulse width / 4 ns."""
    B = len(kref)
    lab = np.zeros((B, 16))
    T = params.threshold
    for e in range(3):
        ex = np.asarray(n_echoes) > e
        lab[:, e] = ex
        dk = np.clip((echoes["bin_peak"][:, e] - kref) / BIN_SCALE, -DK_CLIP, DK_CLIP)
        lab[:, 3 + e] = np.where(ex, dk, 0.0)
        inten = np.maximum(echoes["intensity"][:, e].astype(np.float64), 1e-3 * T)
        lab[:, 6 + e] = np.where(ex, np.log10(inten / T), 0.0)
        lab[:, 9 + e] = np.where(ex, echoes["pulse_width_ns"][:, e] / 4.0, 0.0)
    return lab
