"""Builds the HIP library libsim.so for gfx950, in place next to this file.

    python -m paper_2404_11631_amd.build            the library
    python -m paper_2404_11631_amd.build --probe    also the stand-alone VALU issue-rate probe

Every HIP source is compiled with packed-FP32 instruction selection disabled. Translation units
compile in parallel (one hipcc process per source, at most 8 at once).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsim.so")
SOURCES = ["csrc/fw_paths.hip", "csrc/fw_batch.hip", "csrc/fw_dense.hip", "csrc/mlp.hip", "csrc/sim_api.hip", "csrc/sim_batch.hip", "csrc/sim_noalloc.hip", "csrc/cv_api.hip", "csrc/fw_wide.hip", "csrc/wide_api.hip", "csrc/fw_newsvendor.hip", "csrc/nv_api.hip",
           "csrc/fw_sqn.hip", "csrc/fw_sqn_split.hip", "csrc/sqn_api.hip",
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


def _jobs() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(8, n))


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)

    def compile_one(src: str) -> str:
        obj = os.path.join(HERE, "_build", os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc()] + flags() + lang + ["-c", os.path.join(HERE, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        return obj

    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    subprocess.check_call([hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


def build_probe() -> list:
    """The stand-alone probes behind the roofline figures (not part of the library): VALU issue
    rates, and the cost of a dependent kernel launch."""
    out = []
    for name in ("valu_rate_probe", "launch_floor_probe"):
        probe = os.path.join(HERE, name)
        subprocess.check_call([hipcc()] + flags() + ["-o", probe + ".tmp", os.path.join(HERE, "csrc", name + ".hip")])
        os.replace(probe + ".tmp", probe)
        out.append(probe)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
    if "--probe" in sys.argv:
        print(build_probe())
