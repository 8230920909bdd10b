"""Build libnqs.so (hand-written HIP for gfx950) in-tree with hipcc.

Every .hip file under csrc/ is compiled to an object in parallel, then linked
into one shared library next to this file.  Packed FP32 instructions are
disabled for the device code.  The matrix-core kernels whose accumulators
the compiler would otherwise place in AGPRs are built with the VGPR form of
the MFMA instructions: with accumulators in AGPRs it copies them to and from
VGPRs inside the loops.
"""
from __future__ import annotations

import glob
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnqs.so")
BUILD_DIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


# extra flags per source file
FILE_FLAGS = {
    "k_conv_f64mma.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "k_cnn1.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "k_cnn2.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "calib.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "k_conv_mfma.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "k_x3.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "k_net_cone64.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, *FILE_FLAGS.get(os.path.basename(src), []), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link libnqs.so; returns the library path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
