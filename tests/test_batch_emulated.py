"""The batched tile kernels (fw_batch.hip) in a CPU emulation of the device, vs the oracle.

The device source is compiled for the host against tests/emu/shim (each workgroup runs as lockstep
threads; shuffles, atomics and LDS are emulated), with the library's own planner. This checks the
kernel logic (sample splitting across lanes, butterfly sums, LDS signatures, tile partials and the
per-instance reduction) against the oracle without a GPU; it says nothing about device timing.
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
from tests import parity

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CASES = [  # (d, N, T, R, lanes per replication, noise)
    (2, 2, 40, 20, 1, 0),
    (5, 7, 30, 12, 4, 0),
    (13, 9, 20, 6, 16, 0),
    (20, 11, 16, 3, 64, 0),
    (32, 6, 12, 10, 8, 0),
    (17, 5, 10, 7, 4, 1),
    (4, 6, 20, 8, 4, 1),
    (7, 3, 30, 5, 0, 0),
]


@pytest.fixture(scope="module")
def emu():
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    d = tempfile.mkdtemp(prefix="batch_emu_")
    so = os.path.join(d, "libemu.so")
    subprocess.check_call([gxx, "-std=c++20", "-O2", "-fPIC", "-shared", "-I", os.path.join(HERE, "emu", "shim"),
                           "-I", os.path.join(ROOT, "include"), "-o", so, os.path.join(HERE, "emu", "emu.cpp"),
                           os.path.join(ROOT, "paper_2404_11631_amd", "csrc", "host_core.cpp"), "-lpthread"])
    L = ctypes.CDLL(so)
    L.emu_run_batch.argtypes = [ctypes.c_uint32, ctypes.POINTER(sim.SimParams), ctypes.POINTER(ctypes.c_uint64),
                                ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint64,
                                ctypes.POINTER(sim.SimBatchConfig), ctypes.c_int]
    L.emu_batch_stats.argtypes = [ctypes.c_uint32, ctypes.POINTER(sim.SimStats)]
    L.emu_philox_row_check.argtypes = [ctypes.c_uint64, ctypes.c_int]
    L.emu_philox.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
    L.emu_batch_paths.argtypes = [ctypes.c_uint32, ctypes.POINTER(sim.SimPathView),
                                  ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)]
    yield L
    shutil.rmtree(d, ignore_errors=True)


def _arr(ptr, dtype, n):
    ct = np.ctypeslib.as_ctypes_type(dtype)
    return np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ct)), shape=(n,)).copy()


def _paths(L, i):
    v = sim.SimPathView()
    P = ctypes.c_uint32()
    nt = ctypes.c_uint32()
    L.emu_batch_paths(i, ctypes.byref(v), ctypes.byref(P), ctypes.byref(nt))
    R, d, nc = v.R, v.d, v.n_checkpoints
    return {"y": _arr(v.y, np.float64, R), "tau": _arr(v.tau, np.uint32, R),
            "cnt": _arr(v.cnt, np.uint32, (d + 1) * R).reshape(d + 1, R),
            "wsum": _arr(v.wsum, np.uint64, d * R).reshape(d, R),
            "f_ckpt": np.stack([_arr(v.f_ckpt + 8 * c * v.f_ckpt_stride, np.float64, R) for c in range(nc)]),
            "decisions": _arr(v.decisions, np.uint8, v.T * v.log_rep_count).reshape(v.T, v.log_rep_count),
            "lanes_per_rep": P.value}


def test_tile_kernels_match_oracle(emu):
    probs, R, T, P = [], [], [], []
    for i, (d, N, t, r, p, noise) in enumerate(CASES):
        mu, sigma = workloads.diag_instance(77, i, d)
        w0 = np.full(d, 0.5 / d) if i == 1 else None
        probs.append(sim.Problem(mu=mu, sigma=sigma, N=N, noise=noise, nu=4 if noise else 3,
                                 checkpoints=(5, t), gap_eps=0.05, w0=w0, instance_id=i, log_reps=(0, r)))
        R.append(r)
        T.append(t)
        P.append(p)
    n, a, Ra, Ta, cfg, keep = sim._batch_args(probs, R, T, lanes_per_rep=P, keep_paths=True)
    assert emu.emu_run_batch(n, a, Ra, Ta, 99, ctypes.byref(cfg), 1) == 0
    for i, p in enumerate(probs):
        st = sim.SimStats()
        emu.emu_batch_stats(i, ctypes.byref(st))
        g = _paths(emu, i)
        if P[i]:
            assert g["lanes_per_rep"] == P[i]
        op = parity.oracle_problem(p, 99)
        outs = (oracle.PathOut * R[i])()
        for r in range(R[i]):
            outs[r] = parity.check_rep(op, g, r, T[i], oracle.U32, decisions=g["decisions"][:, r])
        parity.check_stats(st, op.reduce(outs, T[i]), len(p.checkpoints), len(p.mu), g["tau"])


def test_philox_row_equals_full_generator(emu):
    """The per-stream shortcut of the device generator (rounds 1-2 shared by the blocks of one
    (epoch, replication) row) gives the words of Philox4x32-10 run in full, and the full device
    generator gives the oracle's words."""
    assert emu.emu_philox_row_check(12345, 200000) == 0
    assert emu.emu_philox_row_check(2**64 - 99, 200000) == 0
    rng = np.random.default_rng(7)
    for _ in range(200):
        ctr = [int(v) for v in rng.integers(0, 2**32, 4)]
        key = [int(v) for v in rng.integers(0, 2**32, 2)]
        out = (ctypes.c_uint32 * 4)()
        emu.emu_philox((ctypes.c_uint32 * 4)(*ctr), (ctypes.c_uint32 * 2)(*key), out)
        assert list(out) == list(oracle.philox(ctr, key))


def test_plan_without_device():
    """sim_plan_batch: heavy instances get more lanes per replication; tiles cover every replication."""
    light = sim.Problem(mu=np.full(2, 0.5), sigma=np.full(2, 0.5), N=2)
    heavy = sim.Problem(mu=np.full(32, 0.5), sigma=np.full(32, 0.5), N=50)
    P, nt = sim.plan_batch([light, heavy], [4096, 4096], [100, 100_000], n_cu=256)
    assert P[0] == 1 and P[1] > 1
    assert nt[0] == 4096 // 64 and nt[1] == 4096 // (64 // P[1])
    P2, _ = sim.plan_batch([light, heavy], [4096, 4096], [100, 100_000], lanes_per_rep=[8, 4])
    assert P2 == [8, 4]
    with pytest.raises(sim.SimError):
        sim.plan_batch([light, heavy], [4096, 4096], [100, 100_000], lanes_per_rep=[8, 2])
    with pytest.raises(sim.SimError):
        sim.plan_batch([light], [10], [10], lanes_per_rep=[3])


def test_plan_checks_full_uneven_workload():
    """The uneven workload at full size (256 instances x 4,096 replications) passes the host-side
    checks of every bound the tile kernels read; T above the 33-bit signature and a normal count
    past 2^32 are refused before any launch."""
    w = workloads.WORKLOADS["uneven"]
    batch = workloads.uneven_batch(w["seed"], w["n_instances"], w["R"], w["d_range"], w["n_range"], w["t_range"])
    probs = [sim.Problem(mu=b.mu, sigma=b.sigma, N=b.N, instance_id=b.instance) for b in batch]
    P, nt = sim.plan_batch(probs, [b.R for b in batch], [b.T for b in batch], n_cu=256)
    for b, p, n in zip(batch, P, nt):
        assert p in (1, 2, 4, 8, 16, 32, 64)
        assert n == -(-b.R // (64 // p))
    pa = [1 if b.d <= 8 else 2 if b.d <= 16 else 4 for b in batch]
    for forced in (pa, [64] * len(batch)):
        P, _ = sim.plan_batch(probs, [b.R for b in batch], [b.T for b in batch], lanes_per_rep=forced)
        assert P == forced
    one = sim.Problem(mu=np.full(4, 0.5), sigma=np.full(4, 0.5), N=4)
    sim.plan_batch([one], [64], [131_071])
    with pytest.raises(sim.SimError) as e:
        sim.plan_batch([one], [64], [131_072])
    assert e.value.code == -5
    big = sim.Problem(mu=np.full(32, 0.5), sigma=np.full(32, 0.5), N=1 << 24, noise=sim.NOISE_T, nu=1000)
    with pytest.raises(sim.SimError) as e:
        sim.plan_batch([big], [64], [10])
    assert e.value.code == -1


WAVE_CASES = [  # (d, N, T, R, M): every instance at 64 lanes per replication, Gaussian noise
    (10, 10, 40, 3, 1),
    (2, 100, 25, 2, 2),       # N > 64: a lane forms two samples' dot products
    (32, 65, 12, 2, 1),       # d = 32 (the largest), N d + 3 = 2083 of the 2112 staged floats
    (7, 9, 30, 3, 3),         # d not a multiple of 4: Philox blocks span samples
]


def test_wave_kernel_matches_oracle(emu):
    """The one-wavefront form (fw_wave_kernel: a replication per wavefront, an asset per lane), chosen
    when every instance asks for 64 lanes per replication with Gaussian noise and N d within the
    staging area, against the oracle under the same replay protocol."""
    probs, R, T = [], [], []
    for i, (d, N, t, r, M) in enumerate(WAVE_CASES):
        mu, sigma = workloads.diag_instance(78, i, d)
        w0 = np.full(d, 0.5 / d) if i == 3 else None
        probs.append(sim.Problem(mu=mu, sigma=sigma, N=N, M=M, checkpoints=(5, t), gap_eps=0.05, w0=w0,
                                 instance_id=20 + i, log_reps=(0, r)))
        R.append(r)
        T.append(t)
    n, a, Ra, Ta, cfg, keep = sim._batch_args(probs, R, T, lanes_per_rep=[64] * len(probs), keep_paths=True)
    assert emu.emu_run_batch(n, a, Ra, Ta, 41, ctypes.byref(cfg), 1) == 0
    for i, p in enumerate(probs):
        st = sim.SimStats()
        emu.emu_batch_stats(i, ctypes.byref(st))
        g = _paths(emu, i)
        assert g["lanes_per_rep"] == 64
        op = parity.oracle_problem(p, 41)
        outs = (oracle.PathOut * R[i])()
        for r in range(R[i]):
            outs[r] = parity.check_rep(op, g, r, T[i], oracle.U32, decisions=g["decisions"][:, r])
        parity.check_stats(st, op.reduce(outs, T[i]), len(p.checkpoints), len(p.mu), g["tau"])
