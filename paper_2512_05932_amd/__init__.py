"""MI355X (gfx950) engine of the single-bounce beam-iteration LiDAR model.

The compute path is ``liblidar_sim.so`` (hand-written HIP kernels behind the
C-ABI of ``include/lidar_sim.h``); this package is its thin ctypes binding.
"""
from ._binding import (LidarSim, LidarError, Batch, load, ECHO_DTYPE, BEAM_DTYPE, EXPORTED,  # noqa: F401
                       LIDAR_OK, LIDAR_E_INVALID, LIDAR_E_STATE, LIDAR_E_HIP, LIDAR_E_NOMEM,
                       LIDAR_E_UNSUPPORTED, LIDAR_PATTERN_GAUSS, LIDAR_PATTERN_TABLE,
                       LIDAR_MODE_PLAIN, LIDAR_MODE_SURROGATE, LIDAR_ECHO_SURROGATE, LIDAR_AUTOTUNE,
                       LIDAR_DETERMINISTIC,
                       LIB_PATH, simulate_static, STATIC_SCRATCH_BYTES, LIDAR_ECHO_ALL,
                       LIDAR_ECHO_STRONGEST, LIDAR_ECHO_NEAREST, LIDAR_ECHO_LONGEST,
                       LIDAR_ECHO_RAW_STRONGEST, LIDAR_ECHO_RAW_NEAREST, LIDAR_RANGE_CENTRE,
                       LIDAR_RANGE_CORRECTED, LIDAR_RANGE_INTERVAL)


def upload_gbuffer(gbuffer, device="cuda"):
    """The six float32 planes of a host G-buffer as contiguous device tensors."""
    import torch
    return tuple(torch.from_numpy(__import__("numpy").ascontiguousarray(p)).to(device)
                 for p in gbuffer.planes())
