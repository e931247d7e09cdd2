"""Builds the HIP library libsim.so for gfx950, in place next to this file.

    python -m paper_2404_11631_amd.build

Every HIP source is compiled with packed-FP32 instruction selection disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsim.so")
SOURCES = ["csrc/fw_paths.hip", "csrc/fw_batch.hip", "csrc/fw_dense.hip", "csrc/mlp.hip", "csrc/sim_api.hip", "csrc/sim_batch.hip", "csrc/cv_api.hip", "csrc/fw_wide.hip", "csrc/wide_api.hip", "csrc/fw_newsvendor.hip", "csrc/nv_api.hip",
           "csrc/fw_sqn.hip", "csrc/sqn_api.hip",
           "csrc/host_core.cpp"]
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False) -> str:
    objs = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc()] + flags() + lang + ["-c", os.path.join(HERE, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    subprocess.check_call([hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    # stand-alone issue-rate probe behind the ALU roofline figures
    probe = os.path.join(HERE, "valu_rate_probe")
    subprocess.check_call([hipcc()] + flags() + ["-o", probe + ".tmp", os.path.join(HERE, "csrc", "valu_rate_probe.hip")])
    os.replace(probe + ".tmp", probe)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
