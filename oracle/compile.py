"""Build step of the oracle: gcc, FP64, no FMA contraction, OpenMP.

Test infrastructure only (see ``oracle/__init__.py``).
"""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "lidar_oracle.c")
OUT = os.path.join(_HERE, "liblidar_oracle.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(force: bool = True) -> str:
    if not force and os.path.exists(OUT):
        return OUT
    tmp = OUT + ".tmp"
    subprocess.run(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
