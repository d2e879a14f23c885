"""What the trained surrogate gains over the plain method alone, on
Gaussian-beam scanning frames (road + boxes, 64 x 2000 beams): trained on
eight frames of the plain path's echoes by the library's own forward,
backward and AdamW kernels, it must keep >= 99 % of the beams of a held-out
frame within one bin of the FP64 oracle's echoes (sampled beams) and of the
plain path's (all beams) with the gate at c_min = 0.95, while simulating
that frame faster than the plain path does."""
import time

import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lidar():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_05932_amd as lidar
    lidar.load()
    return lidar


def _frames(seeds):
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(8) as ex:
        return list(ex.map(lambda s: scenes.surrogate_frame(s, "gauss"), seeds))


def _time(sim, mode, reps=10):
    import torch
    sim.simulate_frame(mode)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sim.simulate_frame(mode)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def test_trained_surrogate_is_faster_at_one_bin(lidar, oracle_mod):
    import torch
    from paper_2512_05932_amd import surrogate as sur
    ws = _frames([200, 201, 202, 203, 204, 205, 206, 207, 7])
    train, held = ws[:8], ws[8]
    sim = lidar.LidarSim(held.params, stream=torch.cuda.current_stream())
    try:
        planes = [lidar.upload_gbuffer(w.gbuffer, "cuda") for w in ws]
        X, L = sur.make_dataset(sim, [(w.gbuffer.raster, p, w.pattern)
                                      for w, p in zip(train, planes[:8])])
        sim.set_weights(scenes.surrogate_init(0))
        losses = sur.train(sim, X, L, steps=2500, batch=4096, lr=2e-3, log_every=250)
        print(f"[sur-train] {X.shape[0]} rows, losses {['%.3f' % l for l in losses]}", flush=True)
        assert losses[-1] < 0.1 * losses[0]
        sim.set_pattern(held.pattern)
        sim.set_gbuffer(held.gbuffer.raster, planes[8])
        sim.set_gate(0.95, 0.5)
        t_plain = _time(sim, lidar.LIDAR_MODE_PLAIN)
        plain = sim.read()
        t_sur = _time(sim, lidar.LIDAR_MODE_SURROGATE)
        got = sim.read()
        st = sim.stats()
        ag = sur.echo_agreement(plain, got)
        fb = st["fallback_beams"] / st["surrogate_beams"]
        print(f"[sur-train] held-out: fallback {fb:.3f}, within one bin of the plain path "
              f"{ag['within_1_bin']:.4f}, plain {t_plain * 1e3:.3f} ms, surrogate "
              f"{t_sur * 1e3:.3f} ms", flush=True)
        assert ag["within_1_bin"] >= 0.99
        assert fb < 0.3
        assert t_sur < t_plain
        # against the FP64 oracle on a beam sample
        idx = np.sort(np.random.default_rng(3).choice(held.pattern.n_beams, 2000, replace=False))
        ref = oracle_mod.simulate(held.gbuffer, scenes.subset_beams(held, idx).pattern,
                                  held.params, want_xi=False, want_xi_hat=False)
        ora = {"n_echoes": ref.n_echoes, "echoes": ref.echoes}
        sub = {"n_echoes": got["n_echoes"][idx], "echoes": got["echoes"][idx]}
        ago = sur.echo_agreement(ora, sub)
        print(f"[sur-train] within one bin of the oracle on {len(idx)} beams: "
              f"{ago['within_1_bin']:.4f}", flush=True)
        assert ago["within_1_bin"] >= 0.99
    finally:
        sim.close()
