"""The minibatch order of ``lidar_sim_surrogate_train`` written out from its
definition in the header (test helper): epoch e visits row P_e(p) at
position p, P_e a four-round Feistel network on 2h-bit values (2^(2h) >= n),
cycle-walked below n; round r maps (L, R) to (R, L ^ (mix(key_r ^ R) & mask))
with key_r = seed ^ ((4e + r + 1) * 0x9e3779b97f4a7c15 mod 2^64) and mix the
SplitMix64 output function."""
import numpy as np

M64 = (1 << 64) - 1


def mix64(z: int) -> int:
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def feistel(x: int, half: int, seed: int, epoch: int) -> int:
    mask = (1 << half) - 1
    L, R = x >> half, x & mask
    for r in range(4):
        key = seed ^ (((4 * epoch + r + 1) * 0x9E3779B97F4A7C15) & M64)
        L, R = R, L ^ (mix64(key ^ R) & mask)
    return (L << half) | R


def epoch_rows(n: int, seed: int, epoch: int) -> np.ndarray:
    half = 1
    while (1 << (2 * half)) < n:
        half += 1
    out = np.empty(n, dtype=np.int64)
    for p in range(n):
        x = feistel(p, half, seed, epoch)
        while x >= n:
            x = feistel(x, half, seed, epoch)
        out[p] = x
    return out
