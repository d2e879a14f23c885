"""Training and evaluation driver of the learned surrogate (argument
marshalling around the C-ABI: every step runs in the library's kernels).

``make_dataset`` runs the plain path on frames and collects the network
inputs and labels on the device; ``train`` runs AdamW steps over shuffled
minibatches; ``echo_agreement`` compares the echoes of two runs beam by beam.
"""
from __future__ import annotations

import numpy as np

from . import _binding as B


def make_dataset(sim, frames, device="cuda"):
    """frames: iterable of (raster, planes, pattern) with device G-buffer
    planes.  Returns (X int16 [N][1056] BF16 bits, labels float32 [N][16])
    on the device, N = total beams."""
    import torch
    xs, ls = [], []
    for raster, planes, pattern in frames:
        sim.set_pattern(pattern)
        sim.set_gbuffer(raster, planes)
        sim.simulate_frame(B.LIDAR_MODE_PLAIN)
        n = sim.n_beams
        x = torch.empty((n, B.SUR_IN), dtype=torch.int16, device=device)
        lab = torch.empty((n, 16), dtype=torch.float32, device=device)
        sim.surrogate_features(x, lab)
        xs.append(x)
        ls.append(lab)
    return torch.cat(xs), torch.cat(ls)


def train(sim, X, L, steps: int, batch: int = 4096, lr: float = 1e-3, weight_decay: float = 1e-4,
          seed: int = 0, lr_final: float | None = None, log_every: int = 0):
    """AdamW over shuffled minibatches of (X, L); returns the loss of every
    ``log_every``-th step (device values read at the end).  The learning rate
    decays linearly to ``lr_final`` (default lr / 10)."""
    import torch
    n = X.shape[0]
    g = torch.Generator(device=X.device)
    g.manual_seed(seed)
    lr_final = lr / 10 if lr_final is None else lr_final
    losses = []
    loss = torch.zeros(max(1, steps // max(1, log_every) + 1) if log_every else 1,
                       dtype=torch.float32, device=X.device)
    perm = torch.randperm(n, generator=g, device=X.device)
    pos = 0
    for step in range(steps):
        if pos + batch > n:
            perm = torch.randperm(n, generator=g, device=X.device)
            pos = 0
        idx = perm[pos:pos + min(batch, n)]
        pos += batch
        xb = X.index_select(0, idx)
        lb = L.index_select(0, idx)
        f = step / max(1, steps - 1)
        out = None
        if log_every and step % log_every == 0:
            out = loss[step // log_every:step // log_every + 1]
        sim.train_step(xb, lb, lr=lr + (lr_final - lr) * f, weight_decay=weight_decay, loss=out)
    if log_every:
        losses = loss.cpu().numpy().tolist()[:(steps - 1) // log_every + 1]
    return losses


def echo_agreement(ref: dict, got: dict, max_echoes: int = 3) -> dict:
    """Per-beam agreement of two results (read() dicts): the same number of
    echoes among the first ``max_echoes`` and every such echo's peak bin
    within one bin.  Returns the fraction of agreeing beams and its parts."""
    n_r = np.minimum(ref["n_echoes"], max_echoes)
    n_g = np.minimum(got["n_echoes"], max_echoes)
    same_n = n_r == n_g
    ok = same_n.copy()
    for e in range(max_echoes):
        has = same_n & (n_r > e)
        d = np.abs(ref["echoes"]["bin_peak"][:, e].astype(np.int64) -
                   got["echoes"]["bin_peak"][:, e].astype(np.int64))
        ok &= ~has | (d <= 1)
    return {"within_1_bin": float(ok.mean()), "count_agree": float(same_n.mean()),
            "beams": int(len(ok))}
