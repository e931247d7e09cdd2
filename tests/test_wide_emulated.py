"""The wide path's kernels (fw_wide.hip) in a CPU emulation of the device, vs the oracle.

The device source and the library's launch sequence (wide_sequence) are compiled for the host
against tests/emu/shim (each workgroup runs as lockstep threads, workgroups one after another,
highest index first); the oracle for this shape replays the decisions under its binary32 rounding
bound, as the GPU tests do. This checks the kernels' logic (the step folded into the next sample
launch or taken on its own, the cross-workgroup dot products, the parity buffers, ragged last
workgroups, sample-size schedules) without a GPU; it says nothing about device timing.
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
    d = tempfile.mkdtemp(prefix="wide_emu_")
    so = os.path.join(d, "libemuw.so")
    subprocess.check_call([gxx, "-std=c++20", "-O2", "-fPIC", "-shared", "-I", os.path.join(HERE, "emu", "shim"),
                           "-I", os.path.join(ROOT, "include"), "-o", so, os.path.join(HERE, "emu", "emu_wide.cpp"),
                           os.path.join(ROOT, "paper_2404_11631_amd", "csrc", "host_core.cpp"), "-lpthread"])
    L = ctypes.CDLL(so)
    L.emu_run_wide.argtypes = [ctypes.POINTER(sim.SimParams), ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
    L.emu_wide_paths.argtypes = [ctypes.c_void_p] * 6
    L.emu_wide_error.restype = ctypes.c_char_p
    yield L
    shutil.rmtree(d, ignore_errors=True)


def run(L, p, R, T, seed):
    sp, keep = sim.Sim.params(p)
    rc = L.emu_run_wide(ctypes.byref(sp), R, T, seed)
    assert rc == 0, (rc, L.emu_wide_error())
    d, nc = len(p.mu), len(p.checkpoints)
    out = {"y": np.zeros(R), "f_ckpt": np.zeros((nc, R)), "cnt": np.zeros((R, d + 1), np.uint32),
           "wsum": np.zeros((R, d), np.uint64), "tau": np.zeros(R, np.uint32), "decisions": np.zeros((R, T), np.uint32)}
    L.emu_wide_paths(*(out[k].ctypes.data for k in ("y", "f_ckpt", "cnt", "wsum", "tau", "decisions")))
    return out


def close(a, b, rtol, atol):
    return abs(a - b) <= atol + rtol * abs(b)


CASES = [  # d, N, M, T, R, w0, schedule
    dict(d=4, N=2, M=1, T=14, R=2, w0=False, sched=None),
    dict(d=128, N=9, M=1, T=10, R=2, w0=False, sched=None),
    dict(d=520, N=5, M=3, T=9, R=1, w0=True, sched=None),           # 130 quads: five workgroups, ragged
    dict(d=264, N=6, M=2, T=8, R=2, w0=False, sched="grow"),        # N_k = 2 + k: the epoch changes every 2
    dict(d=1032, N=70, M=1, T=4, R=1, w0=False, sched=None),         # N > 64
]


@pytest.mark.parametrize("case", CASES, ids=[f"d{c['d']}_N{c['N']}_M{c['M']}" for c in CASES])
def test_wide_kernels_match_oracle(emu, case):
    d, N, M, T, R = case["d"], case["N"], case["M"], case["T"], case["R"]
    mu, sig = workloads.diag_instance(31, 0, d, "paper")
    sch = None
    if case["sched"] == "grow":
        sch = tuple(2 + k for k in range((T + M - 1) // M))
    p = sim.Problem(mu=mu, sigma=sig, N=N, M=M, w0=np.full(d, 0.5 / d) if case["w0"] else None,
                    checkpoints=(T // 2, T), gap_eps=1e-2, n_schedule=sch)
    g = run(emu, p, R, T, 23)
    W = oracle.WideOracle(p.mu, p.sigma, N=p.N, M=p.M, lam=p.lam, w0=p.w0, seed=23, instance=p.instance_id,
                          ckpt=p.checkpoints, gap_eps=p.gap_eps, n_sched=p.n_schedule)
    for r in range(R):
        o = W.path(r, T, replay=g["decisions"][r], uroff=oracle.U32)
        assert o["n_mismatch"] == 0, f"rep {r}: {o['n_mismatch']} mismatches, first at {o['first_mismatch']}"
        assert np.array_equal(g["decisions"][r], o["decisions"])
        assert np.array_equal(g["cnt"][r], o["cnt"])
        assert np.array_equal(g["wsum"][r], o["wsum"])
        assert close(g["y"][r], o["y"], 1e-11, 1e-14)
        for c in range(len(p.checkpoints)):
            assert close(g["f_ckpt"][c, r], o["f_ckpt"][c], 1e-11, 1e-14)
        assert o["tau_lo"] <= int(g["tau"][r]) <= o["tau_hi"]


def test_wide_zero_noise_emulated(emu):
    """sigma = 0: every decision is the asset of largest mean (closed form)."""
    d = 256
    mu, _ = workloads.diag_instance(2, 0, d, "paper")
    g = run(emu, sim.Problem(mu=mu, sigma=np.zeros(d), N=4), 1, 6, 1)
    assert (g["decisions"] == int(np.argmax(mu)) + 1).all()
    assert g["y"][0] == pytest.approx(-mu.max(), abs=1e-15)
