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
    echo in the right bin (decided in FP32, as the device does)."""
    y = np.asarray(Y, dtype=np.float32)
    l = np.asarray(lab, dtype=np.float32)
    ok = np.ones(y.shape[0], dtype=bool)
    for e in range(3):
        te = l[:, e] > np.float32(0.5)
        ok &= (y[:, e] > 0) == te
        ok &= ~(te & (np.abs(y[:, 3 + e] - l[:, 3 + e]) * np.float32(BIN_SCALE) > np.float32(0.5)))
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
