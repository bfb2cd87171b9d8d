"""Build libcgkmc.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "cgkmc.hip")
LIB = os.path.join(HERE, "libcgkmc.so")
PROBE_SRC = os.path.join(HERE, "csrc", "lds_probe.hip")
PROBE = os.path.join(HERE, "lds_probe")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # every rounding on the FP64 decision path happens where the source says
    "-ffp-contract=off",
    # no packed FP32 instructions in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the hop kernels' LDS atomics come from single lanes: no wave-level reduction around them
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{r.stderr[-6000:]}")
    os.replace(tmp, LIB)
    return LIB


def build_probe(verbose: bool = False) -> str:
    """The unit-throughput probe behind the roofline denominators (a standalone program, run
    as ./paper_1407_5026_amd/lds_probe; not part of the library build)."""
    tmp = PROBE + ".tmp"
    flags = [f for f in FLAGS if f not in ("-fPIC", "-shared")]
    cmd = [HIPCC, *flags, "-o", tmp, PROBE_SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{r.stderr[-6000:]}")
    os.replace(tmp, PROBE)
    return PROBE


if __name__ == "__main__":
    import sys

    if sys.argv[1:] == ["probe"]:
        print(build_probe(verbose=True))
    else:
        print(build(verbose=True))
