"""The split SQN kernels (fw_sqn_split.hip: one replication over many one-wavefront workgroups) in a
CPU emulation of the device, vs the oracle (Algorithms 3-4, Section 3.3).

The device source and the library's launch sequence (sqn_split_sequence) are compiled for the host
against tests/emu/shim (each workgroup runs as lockstep threads, workgroups one after another,
highest index first). This checks the kernels' logic without a GPU: the partial sums over slices
and their reduction in the next launch, the parity-buffered row dot products, the ring of pairs
(filling, wrapping), the window launches, the small-matrix rebuild, the snapshots, binary32 pairs,
ragged last slices, several replications. The iterates match the oracle to 1e-9 relative in the
2-norm (binary64 pairs; 1e-7 with binary32 pairs, where a value at a rounding boundary may round
differently on the two sides); pair counts exactly; the loss at each emulated checkpoint iterate
equals the oracle's checkpoint loss to 1e-10.
"""
import ctypes
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from paper_2404_11631_amd import sim, workloads

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def emu():
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    d = tempfile.mkdtemp(prefix="sqn_split_emu_")
    so = os.path.join(d, "libemusqn.so")
    subprocess.check_call([gxx, "-std=c++20", "-O2", "-fPIC", "-shared", "-I", os.path.join(HERE, "emu", "shim"),
                           "-I", os.path.join(ROOT, "include"), "-o", so, os.path.join(HERE, "emu", "emu_sqn_split.cpp"),
                           os.path.join(ROOT, "paper_2404_11631_amd", "csrc", "host_core.cpp"), "-lpthread"])
    L = ctypes.CDLL(so)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    L.emu_run_sqn_split.argtypes = [u8p, u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(sim.SimSqnParams),
                                    ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
    L.emu_sqn_split_out.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    L.emu_sqn_split_error.restype = ctypes.c_char_p
    yield L
    shutil.rmtree(d, ignore_errors=True)


CASES = [  # n, N, R, K, L, M, b, bH, ckpt, fp32
    dict(n=50, N=400, R=1, K=40, L=3, M=4, b=20, bH=30, ckpt=(7, 22), fp32=False),      # ring wraps (12 pairs, M = 4)
    dict(n=300, N=500, R=1, K=20, L=2, M=3, b=16, bH=24, ckpt=(5, 13), fp32=False),     # two slices, the second ragged
    dict(n=130, N=300, R=2, K=25, L=3, M=5, b=12, bH=18, ckpt=(), fp32=True),           # binary32 pairs, two replications
    dict(n=600, N=700, R=1, K=12, L=2, M=2, b=70, bH=100, ckpt=(12,), fp32=False),      # rows over several passes
    dict(n=37, N=200, R=1, K=7, L=4, M=3, b=9, bH=11, ckpt=(3,), fp32=False),           # K < 2L: no pair
    dict(n=1, N=64, R=1, K=15, L=2, M=2, b=5, bH=7, ckpt=(), fp32=False),               # one feature
]


def run(L, X, z, c, seed):
    N, n = X.shape
    sp = sim.sqn_params(L=c["L"], M=c["M"], b=c["b"], bH=c["bH"], beta=2.0, checkpoints=c["ckpt"], instance_id=3,
                        pairs_fp32=c["fp32"])
    u8p = ctypes.POINTER(ctypes.c_uint8)
    rc = L.emu_run_sqn_split(X.ctypes.data_as(u8p), z.ctypes.data_as(u8p), N, n, ctypes.byref(sp), c["R"], c["K"], seed)
    assert rc == 0, (rc, L.emu_sqn_split_error())
    nc = len(c["ckpt"])
    w = np.zeros((nc + 1, c["R"], n))
    pairs = np.zeros(c["R"], np.uint32)
    L.emu_sqn_split_out(w.ctypes.data, pairs.ctypes.data)
    return w, pairs


@pytest.mark.parametrize("c", CASES, ids=[f"n{c['n']}_R{c['R']}_K{c['K']}_M{c['M']}{'_f32' if c['fp32'] else ''}"
                                          for c in CASES])
def test_split_kernels_match_oracle(emu, c):
    X, z = workloads.sqn_dataset(5, c["n"], c["N"])
    seed = 17
    w, pairs = run(emu, X, z, c, seed)
    O = oracle.SqnOracle(X, z, L=c["L"], M=c["M"], b=c["b"], bH=c["bH"], beta=2.0, seed=seed, instance=3,
                         ckpt=c["ckpt"], pairs_fp32=c["fp32"])
    rtol = 1e-7 if c["fp32"] else 1e-9
    for r in range(c["R"]):
        o = O.run(r, c["K"])
        assert int(pairs[r]) == o["pairs"]
        err = np.linalg.norm(w[-1, r] - o["w"]) / max(np.linalg.norm(o["w"]), 1e-300)
        assert err <= rtol, (r, err)
        for k in range(len(c["ckpt"])):
            assert abs(O.loss(w[k, r]) - o["F_ckpt"][k]) <= 1e-10 * o["F_ckpt"][k], (r, k)
