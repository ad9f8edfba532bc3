"""Builds libnvr.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libnvr.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["abi.cpp", "grid.hip", "march.hip", "warp.hip", "mlp.cpp", "mlp_plain.hip",
           "mlp_mfma.hip", "scatter.hip", "composite.hip", "optim.hip", "step.cpp",
           "occupancy.hip", "lut.hip", "keyframe.hip", "deform.hip", "probe.hip"]

ROCM_LIB = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")

FLAGS = ["-std=c++17", "-O3", "--offload-arch=gfx950", "-fPIC", "-I" + INCLUDE, "-I" + CSRC,
         # no packed-fp32 instructions anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # matrix-core results straight into ordinary registers (no copies out
         # of the accumulation registers between chained layers)
         "-mllvm", "-amdgpu-mfma-vgpr-form=1",
         "-munsafe-fp-atomics", "-Wno-unused-result"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-x", "hip", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{p.stderr}")
    return obj


def build(jobs: int = 8, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    p = subprocess.run([HIPCC, "-shared", "--offload-arch=gfx950", "-fPIC", "-o", tmp, *objs,
                        "-L" + ROCM_LIB, "-Wl,-rpath," + ROCM_LIB],
                       capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"link failed:\n{p.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
