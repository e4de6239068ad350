"""Builds libsimus.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libsimus.so")
BUILD = os.path.join(PKG, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
          "-Wall", "-Wno-unused-function"]
# Packed FP32 instructions stay off: ordinary float code only.
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-fno-gpu-rdc", "-munsafe-fp-atomics"]

SOURCES = [("kernels.hip", True), ("synth_mfma.hip", True), ("tables.hip", True), ("adjoint.hip", True),
           ("adjoint_mfma.hip", True), ("pfield.hip", True), ("noalloc.hip", True),
           ("abi.cpp", False), ("plan.cpp", False)]


def _compile(src: str, device: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
    if device:
        cmd[1:1] = ["-x", "hip", *DEVICE]
    else:
        # host code only (hipcc would otherwise add a device pass for its default target)
        cmd[1:1] = ["-D__HIP_PLATFORM_AMD__", "--offload-host-only"]
    subprocess.check_call(cmd)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    # a failed build must not leave an older library behind to be loaded
    if os.path.exists(OUT):
        os.remove(OUT)
    srcs = [(s, d) for s, d in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = list(ex.map(lambda sd: _compile(*sd), srcs))
    tmp = OUT + ".tmp"
    subprocess.check_call([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs])
    os.replace(tmp, OUT)
    diag = os.path.join(PKG, "diag", "valu_rate.hip")
    if os.path.exists(diag):
        subprocess.check_call([HIPCC, "-O3", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
                               "-Xclang", "-packed-fp32-ops", "-o", os.path.join(PKG, "diag", "valu_rate"),
                               diag])
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
