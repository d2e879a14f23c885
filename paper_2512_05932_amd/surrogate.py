"""Training and evaluation driver of the learned surrogate (argument
marshalling around the C-ABI: every step runs in the library's kernels).

``make_dataset`` runs the plain path on frames and collects the network
inputs and labels on the device; ``train`` calls the library's training loop
(AdamW steps over shuffled minibatches); ``echo_agreement`` compares the
echoes of two runs beam by beam.
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
    """AdamW over shuffled minibatches of (X, L) by the library's training
    loop; returns the loss of every ``log_every``-th step (device values read
    at the end).  The learning rate decays linearly to ``lr_final`` (default
    lr / 10)."""
    import torch
    losses = None
    if log_every:
        losses = torch.zeros((steps + log_every - 1) // log_every, dtype=torch.float32, device=X.device)
    sim.train(X, L, steps, batch=batch, lr=lr, lr_final=lr_final, weight_decay=weight_decay,
              seed=seed, losses=losses, log_every=log_every)
    return losses.cpu().numpy().tolist() if log_every else []


def echo_agreement(ref: dict, got: dict, max_echoes: int = 3, per_beam: bool = False):
    """Per-beam agreement of two results (read() dicts): the same number of
    echoes among the first ``max_echoes`` and every such echo's peak bin
    within one bin.  Returns the fraction of agreeing beams and its parts, or
    with ``per_beam`` the boolean agreement of every beam."""
    n_r = np.minimum(ref["n_echoes"], max_echoes)
    n_g = np.minimum(got["n_echoes"], max_echoes)
    same_n = n_r == n_g
    ok = same_n.copy()
    for e in range(max_echoes):
        has = same_n & (n_r > e)
        d = np.abs(ref["echoes"]["bin_peak"][:, e].astype(np.int64) -
                   got["echoes"]["bin_peak"][:, e].astype(np.int64))
        ok &= ~has | (d <= 1)
    if per_beam:
        return ok
    return {"within_1_bin": float(ok.mean()), "count_agree": float(same_n.mean()),
            "beams": int(len(ok))}
