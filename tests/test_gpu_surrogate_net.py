"""The surrogate network on the GPU (BF16 MFMA products, FP32 accumulation)
against the FP64 oracle that mirrors its BF16 roundings, through the C-ABI.

Tolerances (derived in the design doc): both sides round the same operands to
BF16; they differ by the FP32 vs FP64 accumulation of the products and by
the rare BF16 re-rounding of an activation that lies next to a rounding
boundary, which moves that activation by one BF16 ulp (2^-8 relative).
Outputs and per-tensor gradients agree to 3e-3 of the tensor's largest
magnitude; rows where the loss's discrete decisions (existence sign, peak
bin within half a bin) lie within 0.05 of their boundary are left out of the
gradient comparison, since there either decision is correct."""
import numpy as np
import pytest

import scenes
from oracle import surrogate as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lidar():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_05932_amd as lidar
    lidar.load()
    return lidar


def _sim(lidar):
    import torch
    w = scenes.iid_frame(0)
    return lidar.LidarSim(w.params, stream=torch.cuda.current_stream())


def _weights(seed):
    flat = scenes.surrogate_init(seed)
    rng = np.random.default_rng(seed + 100)
    p = S.unpack(flat)
    for b in ("b1", "b2", "b3", "b4"):
        p[b][:] = rng.standard_normal(p[b].shape).astype(np.float32) * np.float32(0.1)
    p["b4"][S.OUT_USED:] = 0.0
    return flat


def _dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _x(seed, n):
    import torch
    bits = scenes.random_bf16_bits(seed, n, scale=1.0)
    return bits, torch.from_numpy(bits.view(np.int16).copy()).cuda()


def _per_tensor(got, ref, tol, what):
    for name, shape in S.SHAPES:
        g = S.unpack(got)[name]
        r = S.unpack(ref)[name]
        scale = np.abs(r).max()
        err = np.abs(g - r).max()
        print(f"[sur] {what} {name}: max err {err:.3e} of max {scale:.3e}", flush=True)
        assert err <= tol * scale + 1e-12, (what, name, err, scale)


def test_forward_matches_oracle(lidar):
    import torch
    sim = _sim(lidar)
    try:
        flat = _weights(1)
        sim.set_weights(flat)
        np.testing.assert_array_equal(sim.get_weights(), flat)
        bits, x = _x(2, 300)                       # ragged: 300 rows
        y = torch.zeros((300, 16), dtype=torch.float32, device="cuda")
        sim.surrogate_forward(x, y)
        got = y.cpu().numpy().astype(np.float64)
        ref = S.forward(scenes.bf16_bits_to_float(bits), flat, rounded=True).Y
        err = np.abs(got - ref).max()
        print(f"[sur] forward max err {err:.3e} of max {np.abs(ref).max():.3e}", flush=True)
        assert err <= 3e-3 * np.abs(ref).max()
        assert np.all(got[:, S.OUT_USED:] == 0.0)
    finally:
        sim.close()


def _clear_rows(Y, lab, margin=0.05):
    keep = np.ones(Y.shape[0], dtype=bool)
    for e in range(3):
        keep &= np.abs(Y[:, e]) > margin
        te = lab[:, e] > 0.5
        keep &= ~te | (np.abs(np.abs(Y[:, 3 + e] - lab[:, 3 + e]) * 16.0 - 0.5) > margin)
    return keep


def test_gradients_match_oracle(lidar):
    import torch
    sim = _sim(lidar)
    try:
        flat = _weights(3)
        sim.set_weights(flat)
        bits, _ = _x(4, 700)
        lab = scenes.random_surrogate_labels(5, 700)
        X = scenes.bf16_bits_to_float(bits)
        keep = _clear_rows(S.forward(X, flat).Y, lab)
        bits, lab, X = bits[keep][:512], lab[keep][:512], X[keep][:512]
        n = bits.shape[0]
        assert n > 300
        x = torch.from_numpy(bits.view(np.int16).copy()).cuda()
        g = torch.zeros(S.N_PARAMS, dtype=torch.float32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        sim.surrogate_gradients(x, _dev(lab, torch.float32), g, loss)
        c = S.forward(X, flat)
        L, dY = S.loss_and_grad(c.Y, lab)
        ref = S.backward(c, dY, flat)
        assert loss.item() == pytest.approx(L, rel=1e-3)
        _per_tensor(g.cpu().numpy().astype(np.float64), ref, 3e-3, "grad")
    finally:
        sim.close()


def test_adamw_steps_match_oracle(lidar):
    import torch
    sim = _sim(lidar)
    try:
        flat = _weights(6)
        sim.set_weights(flat)
        hp = dict(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.01)
        theta = flat.astype(np.float64)
        m = np.zeros(S.N_PARAMS)
        v = np.zeros(S.N_PARAMS)
        for t in (1, 2):
            bits, x = _x(10 + t, 400)
            lab = scenes.random_surrogate_labels(20 + t, 400)
            X = scenes.bf16_bits_to_float(bits)
            c = S.forward(X, theta)
            _, dY = S.loss_and_grad(c.Y, lab)
            g = S.backward(c, dY, theta)
            theta, m, v = S.adamw_step(theta, g, m, v, t, **hp)
            sim.train_step(x, _dev(lab, torch.float32), **hp)
            got = sim.get_weights().astype(np.float64)
            # elements whose gradient is well above the noise of the
            # comparison move by about lr per step on both sides
            strong = np.abs(g) > 0.05 * np.abs(g).max()
            err = np.abs(got - theta)[strong].max()
            print(f"[sur] adamw step {t}: {strong.sum()} strong elements, max err {err:.3e}",
                  flush=True)
            assert err <= 0.1 * hp["lr"] * t
            # weight decay alone on elements without gradient (padding rows)
            pad = S.unpack(np.arange(S.N_PARAMS))["W1"][S.IN_USED:].ravel()
            np.testing.assert_allclose(got[pad], theta[pad], atol=1e-12)
    finally:
        sim.close()


def test_training_fits_a_learnable_task(lidar):
    """Labels that are a fixed function of the inputs (existence from the
    sign of linear read-outs, targets from smooth functions): the loss must
    fall well below its starting value within a few hundred steps."""
    import torch
    sim = _sim(lidar)
    try:
        sim.set_weights(scenes.surrogate_init(7))
        n = 4096
        bits, x = _x(30, n)
        X = scenes.bf16_bits_to_float(bits)
        rng = np.random.default_rng(31)
        R = rng.standard_normal((S.IN_USED, 6)) / np.sqrt(S.IN_USED)
        P = X[:, :S.IN_USED] @ R
        lab = np.zeros((n, 16), dtype=np.float32)
        lab[:, :3] = (P[:, :3] > 0)
        lab[:, 3:6] = np.tanh(P[:, 3:6]) * 0.5 * lab[:, :3]
        lab[:, 6:9] = 0.3 * P[:, :3] * lab[:, :3]
        lab[:, 9:12] = 0.2 * lab[:, :3]
        labd = _dev(lab, torch.float32)
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        losses = []
        for step in range(300):
            sim.train_step(x, labd, lr=1e-3, loss=loss)
            if step % 50 == 0 or step == 299:
                losses.append(loss.item())
        print(f"[sur] training losses {['%.3f' % l for l in losses]}", flush=True)
        assert losses[-1] < 0.5 * losses[0]
    finally:
        sim.close()
